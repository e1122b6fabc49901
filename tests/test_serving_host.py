"""Host-side logic of the serving module (no GPU): the transform split factor a
group takes for a given number of live cells (the table of measured step times
it encodes), and that a factor is set on the plan only when it changes."""

import pytest

from paper_2103_14890_amd import serving as sv


class _FakePlan:
    def __init__(self, tile, precision):
        self._tile, self.precision, self.calls = tile, precision, []

    def tile(self):
        return (self._tile, 0)

    def set_split(self, s):
        self.calls.append(s)


@pytest.mark.parametrize("tile,precision,table", [
    (64, "fx16", [(1, 8), (8, 8), (9, 4), (48, 4), (49, 2), (112, 2), (113, 1), (5000, 1)]),
    (64, "fp32", [(1, 8), (48, 4), (100, 2), (200, 1)]),
    (32, "fx16", [(1, 4), (640, 4), (641, 1)]),
    (32, "fp32", [(1, 1), (100, 1)]),
    (16, "fx16", [(1, 1), (100, 1)]),
])
def test_split_factor_follows_group_size(tile, precision, table):
    plan = _FakePlan(tile, precision)
    g = sv._Group(plan, {64: 64, 32: 32, 16: 16}[tile], device=None)
    for cells, want in table:
        g.set_split_for(cells)
        assert g.split == want, (cells, g.split, want)
    # the plan sees a call only when the factor changes
    changes = [table[0][1]] if table[0][1] != 1 else []
    for (_, a), (_, b) in zip(table, table[1:]):
        if b != a:
            changes.append(b)
    assert plan.calls == changes
