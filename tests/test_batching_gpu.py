"""GPU tests of the batched paths: one launch over several plans (cells of
different velocity grids), hipGraph capture and replay, and the launch-shape
autotuner. The operator is cell-local, so every variant must reproduce the
single-plan results bitwise."""

import json
import os

import numpy as np
import pytest

import workloads as wl

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import qcoll
    return qcoll


SLOTS = [(32, 8.0, "hard_sphere", 8, "fx16", False, 37), (16, 8.0, "maxwell", 16, "fx16", False, 9),
         (24, 8.0, "hard_sphere", 8, "fp32", False, 13), (32, 8.0, "maxwell", 8, "fx16", True, 5),
         (12, 5.0, "hard_sphere", 8, "fp32", True, 3), (48, 8.0, "hard_sphere", 8, "fx16", False, 4),
         (64, 8.0, "maxwell", 8, "fx16", True, 3)]


def _setup(qc, seed=0):
    plans, fs = [], []
    for i, (N, L, kern, M, prec, cons, cells) in enumerate(SLOTS):
        plans.append(qc.Plan(2, N, L, kern, M, precision=prec, conserve=cons))
        fs.append(torch.tensor(wl.mixture_cells(2, N, L, cells, 100 + i + seed), dtype=torch.float32, device="cuda"))
    return plans, fs


def test_eval_multi_bitwise_equals_single_launches(qc):
    plans, fs = _setup(qc)
    singles = [p.eval(f) for p, f in zip(plans, fs)]
    outs = [torch.full_like(s, float("nan")) for s in singles]
    qc.eval_multi(plans, fs, outs)
    torch.cuda.synchronize()
    for a, b in zip(singles, outs):
        assert torch.equal(a, b)
    for p in plans:
        p.close()


def test_concurrent_launches_stay_ordered_on_the_callers_stream(qc):
    """Two launches in one call (ten slots: a full slot table of eight, tile-64
    and N <= 32 plans mixed, and a second table) run on the caller's stream and
    a side stream; work queued on the caller's stream after the call (no host
    synchronisation in between) sees every result."""
    cfg = [(64, 8.0, "hard_sphere", 8, 3), (48, 8.0, "maxwell", 8, 2), (64, 10.0, "maxwell", 16, 2),
           (40, 8.0, "hard_sphere", 8, 1), (48, 6.0, "hard_sphere", 8, 3), (32, 8.0, "hard_sphere", 8, 70),
           (16, 8.0, "maxwell", 16, 5), (24, 8.0, "hard_sphere", 8, 4), (64, 8.0, "hard_sphere", 8, 2),
           (20, 8.0, "maxwell", 8, 6)]
    plans, fs = [], []
    for i, (N, L, kern, M, cells) in enumerate(cfg):
        plans.append(qc.Plan(2, N, L, kern, M, precision="fx16"))
        fs.append(torch.tensor(wl.mixture_cells(2, N, L, cells, 300 + i), dtype=torch.float32, device="cuda"))
    singles = [p.eval(f) for p, f in zip(plans, fs)]
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        outs = [torch.full_like(x, float("nan")) for x in singles]
        qc.eval_multi(plans, fs, outs, stream=side)
        copies = [o.clone() for o in outs]          # queued behind the call on the same stream
    torch.cuda.synchronize()
    for a, b in zip(singles, copies):
        assert torch.equal(a, b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_step_multi_bitwise_equals_single_launches(qc, scheme):
    plans, fs = _setup(qc, seed=7)
    ref = [f.clone() for f in fs]
    for p, f in zip(plans, ref):
        p.step(f, 0.02, 0.5, scheme)
    st = [torch.full((f.shape[0],), -1, dtype=torch.int32, device="cuda") for f in fs]
    qc.step_multi(plans, fs, 0.02, 0.5, scheme, st)
    torch.cuda.synchronize()
    for a, b, s in zip(ref, fs, st):
        assert torch.equal(a, b)
        assert (s == 0).all()
    for p in plans:
        p.close()


def test_graph_capture_and_replay(qc):
    """Capture single and batched launches in one graph; every replay (with eager
    work and synchronisation in between) equals the eager result bitwise."""
    plans, fs = _setup(qc, seed=3)
    eager = [p.eval(f) for p, f in zip(plans, fs)]
    torch.cuda.synchronize()
    q_single = torch.empty_like(eager[0])
    q_multi = [torch.empty_like(e) for e in eager]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up on the side stream before capture
        plans[0].eval(fs[0], q_single)
        qc.eval_multi(plans, fs, q_multi)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plans[0].eval(fs[0], q_single)
        qc.eval_multi(plans, fs, q_multi)
    for r in range(3):
        q_single.fill_(float("nan"))
        for q in q_multi:
            q.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(q_single, eager[0])
        for a, b in zip(q_multi, eager):
            assert torch.equal(a, b)
        other = plans[1].eval(fs[1])          # eager work between replays
        torch.cuda.synchronize()
        assert torch.equal(other, eager[1])
    for p in plans:
        p.close()


def test_autotune_keeps_results_and_caches(qc, tmp_path):
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    f = torch.tensor(wl.mixture_cells(2, 32, 8.0, 1024, 9), dtype=torch.float32, device="cuda")
    before = plan.eval(f)
    cache = str(tmp_path / "tune.json")
    best = plan.autotune(f, reps=2, cache=cache)
    assert best["tile"] == 32 and best["waves_per_block"] in (1, 2, 4, 8) and best["max_blocks"] >= 1
    after = plan.eval(f)
    torch.cuda.synchronize()
    assert torch.equal(before, after)
    data = json.load(open(cache))
    assert data[plan.key] == best
    other = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    assert other.load_tuning(cache) and other.shape() == best
    for ws in (1, 2, 4, 8):
        other.set_launch(ws, 64)
        assert torch.equal(other.eval(f), before)
    with pytest.raises(qc.QcollError):
        other.set_tile(16)                  # 18..32-point grids have one tile family
    plan.close()
    other.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
def test_autotune_tile_family(qc, tmp_path, precision):
    """A 16x16 plan runs on either tile family (the 16x16 kernels, or the 32x32
    kernels on the zero-padded grid): both stay within the precision's bound of
    the oracle, the autotuner picks among tiles x cells per workgroup x grid
    caps, the cached choice reproduces its results bitwise, and the batched
    call follows the plan's selected tile."""
    from oracle import spectral as sp
    tol = {"fx16": 1e-5, "fp32": 2e-4}[precision]
    f64 = wl.mixture_cells(2, 16, 8.0, 600, 19)
    f = torch.tensor(f64, dtype=torch.float32, device="cuda")
    ref = sp.q_fast(f64.astype(np.float32).astype(np.float64), sp.Setup(d=2, N=16, L=8.0, kernel="maxwell", M=16))
    plan = qc.Plan(2, 16, 8.0, "maxwell", 16, precision=precision)
    assert plan.tile() == (16, 32)
    outs = {}
    for t in (16, 32):
        plan.set_tile(t)
        assert plan.tile() == (t, 48 - t)
        q = plan.eval(f)
        torch.cuda.synchronize()
        outs[t] = q
        err = np.linalg.norm(q.cpu().double().numpy() - ref) / np.linalg.norm(ref)
        print(f"16x16 {precision} on the {t}x{t} tile kernels: rel L2 {err:.3e}")
        assert err < tol
    cache = str(tmp_path / "tune.json")
    best = plan.autotune(f, reps=2, cache=cache)
    assert best["tile"] in (16, 32) and plan.tile()[0] == best["tile"]
    tuned = plan.eval(f)
    other = qc.Plan(2, 16, 8.0, "maxwell", 16, precision=precision)
    assert other.load_tuning(cache) and other.shape() == best
    again = other.eval(f)
    out_m = torch.empty_like(again)
    qc.eval_multi([other], [f], [out_m])
    torch.cuda.synchronize()
    assert torch.equal(tuned, outs[best["tile"]]) and torch.equal(again, tuned) and torch.equal(out_m, tuned)
    with pytest.raises(qc.QcollError):
        other.set_tile(64)
    plan.close()
    other.close()


def test_more_slots_than_one_table(qc):
    """Ten plans in one call (the slot table holds eight; the call spreads them
    over several launches on the same stream) still match the single launches."""
    specs = [(N, kern) for N in (16, 24, 32, 20, 48) for kern in ("maxwell", "hard_sphere")]
    plans = [qc.Plan(2, N, 8.0, kern, 8, precision="fx16") for N, kern in specs]
    fs = [torch.tensor(wl.mixture_cells(2, N, 8.0, 3 + i, 300 + i), dtype=torch.float32, device="cuda")
          for i, (N, _) in enumerate(specs)]
    singles = [p.eval(f) for p, f in zip(plans, fs)]
    outs = [torch.full_like(s, float("nan")) for s in singles]
    qc.eval_multi(plans, fs, outs)
    ref = [f.clone() for f in fs]
    for p, f in zip(plans, ref):
        p.step(f, 0.01, 1.0, "explicit")
    qc.step_multi(plans, fs, 0.01, 1.0, "explicit")
    torch.cuda.synchronize()
    for a, b in zip(singles, outs):
        assert torch.equal(a, b)
    for a, b in zip(ref, fs):
        assert torch.equal(a, b)
    for p in plans:
        p.close()


@pytest.mark.parametrize("cells", [1, 37, 4100])
def test_pingpong_shape_matches_default_shape(qc, cells):
    """Eight wavefronts per workgroup (the ping-pong FX16 32x32 kernel) give the
    default shape's results bitwise, for eval, the projection, both single-stage
    steps and a multi-stage step, including a partly filled last workgroup."""
    f0 = torch.tensor(wl.mixture_cells(2, 32, 8.0, cells, 50 + cells), dtype=torch.float32, device="cuda")
    outs = {}
    for ws in (4, 8):
        plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
        cons = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
        for p in (plan, cons):
            p.set_launch(ws, 2048 if ws == 8 else 1024)
        fe, fi, fr = f0.clone(), f0.clone(), f0.clone()
        st = torch.full((cells,), -1, dtype=torch.int32, device="cuda")
        plan.step(fe, 0.02, 0.5, "explicit", st)
        plan.step(fi, 0.02, 0.5, "imex")
        plan.step_rk(fr, 0.02, 0.5, "ars222")
        outs[ws] = [plan.eval(f0), cons.eval(f0), fe, fi, fr, st]
        plan.close()
        cons.close()
    torch.cuda.synchronize()
    for a, b in zip(outs[4], outs[8]):
        assert torch.equal(a, b)
    assert (outs[8][5] == 0).all()


@pytest.mark.parametrize("scheme", ["ars222", "bpr343"])
@pytest.mark.parametrize("N,precision", [(32, "fx16"), (32, "fp32"), (16, "fx16")])
def test_step_rk_grid_stride_matches_default_shape(qc, N, precision, scheme):
    """Three one-wavefront workgroups walk 37 cells (about twelve each): the
    moments of f^n that the first stage launch keeps per cell, and the later
    launches read back, belong to that cell whatever wavefront computed it, so
    two steps match the default launch shape's bitwise."""
    cells = 37
    f0 = torch.tensor(wl.mixture_cells(2, N, 8.0, cells, 90 + N), dtype=torch.float32, device="cuda")
    out = []
    for shape in (None, (1, 3)):
        plan = qc.Plan(2, N, 8.0, "hard_sphere", 8, precision=precision)
        if shape is not None:
            plan.set_launch(*shape)
        f = f0.clone()
        for _ in range(2):
            plan.step_rk(f, 0.02, 0.5, scheme)
        out.append(f)
        plan.close()
    torch.cuda.synchronize()
    assert torch.equal(out[0], out[1])


def test_calls_on_a_side_stream_with_library_allocated_buffers(qc):
    """Calls queued on a stream other than the current one, with the binding
    allocating the output and work buffers: the buffers are recorded on that
    stream, and the results equal the same calls on the current stream."""
    f0 = wl.mixture_cells(2, 32, 8.0, 12, 21)
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    ref_f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    ref_q = plan.eval(ref_f)
    plan.step_rk(ref_f, 0.01, 1.0, "ars222")
    side = torch.cuda.Stream()
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    side.wait_stream(torch.cuda.current_stream())
    q = plan.eval(f, stream=side)
    plan.step_rk(f, 0.01, 1.0, "ars222", stream=side)
    # allocations on the current stream while the side stream may still run
    junk = [torch.full((12, 32, 32), 7.0, device="cuda") for _ in range(4)]
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert torch.equal(q, ref_q)
    assert torch.equal(f, ref_f)
    del junk
    plan.close()
