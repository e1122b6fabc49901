"""GPU tests of the transform split (qcoll_plan_set_split): one cell's gain
transforms shared out over the wavefronts of a workgroup (FX16 32x32 tiles) or
over several workgroups (tile-64 plans). The operator is a sum over the
transforms (section 3.3), so the split changes the order of that FP64 sum only:
the results match the oracle at the precision's bound, agree with the unsplit
results to FP64 rounding, and are deterministic."""

import ctypes

import numpy as np
import pytest

import workloads as wl
from oracle import spectral as sp
from oracle import stepping

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fx16": 1e-5, "fp32": 2e-4}


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import qcoll
    return qcoll


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# (N, L, kernel, M, precision, split, cells): 32x32 FX16 (exact and padded
# grids), tile-64 FX16 and FP32 with 2 to 16 parts (the Maxwell plan with 16:
# four gain transforms, so most parts have none and part 4 only the loss); cell
# counts not multiples of anything the launch groups by
CASES = [(32, 8.0, "hard_sphere", 8, "fx16", 4, 37), (24, 8.0, "maxwell", 16, "fx16", 4, 5),
         (64, 10.0, "hard_sphere", 16, "fx16", 4, 6), (64, 10.0, "maxwell", 8, "fx16", 2, 5),
         (48, 8.0, "hard_sphere", 8, "fp32", 2, 3), (40, 8.0, "maxwell", 8, "fp32", 4, 4),
         (64, 8.0, "hard_sphere", 8, "fx16", 8, 3), (56, 8.0, "maxwell", 8, "fx16", 16, 2)]


@pytest.mark.parametrize("N,L,kernel,M,precision,split,cells", CASES)
def test_split_eval_matches_oracle_and_unsplit(qc, N, L, kernel, M, precision, split, cells):
    f = wl.mixture_cells(2, N, L, cells, 500 + N)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan = qc.Plan(2, N, L, kernel, M, precision=precision)
    base = plan.eval(ft)
    plan.set_split(split)
    assert plan.split() == split
    q1 = plan.eval(ft)
    q2 = plan.eval(ft)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)                       # deterministic (fixed summation order)
    qn, bn = q1.cpu().double().numpy(), base.cpu().double().numpy()
    ref = sp.q_fast(f.astype(np.float32).astype(np.float64), sp.Setup(d=2, N=N, L=L, kernel=kernel, M=M))
    err, dsplit = _rel(qn, ref), _rel(qn, bn)
    print(f"N={N} {precision} split {split}: rel L2 vs oracle {err:.3e}, vs unsplit {dsplit:.3e}")
    assert err < TOL[precision]
    assert dsplit < 1e-10                            # the FP64 gain sum in another order
    plan.close()


@pytest.mark.parametrize("N,split", [(32, 4), (64, 4), (48, 2)])
def test_split_conserve_and_step(qc, N, split):
    """FP64 projection and the single-stage update run in the split form too
    (the epilogue of the part that adds the partial sums)."""
    L, M = 8.0, 8
    f = wl.noisy_mixture_cells(2, N, L, 5, 77, 0.01)
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=M)
    f32 = f.astype(np.float32).astype(np.float64)
    ref = sp.q_fast(f32, s)
    plan = qc.Plan(2, N, L, "hard_sphere", M, precision="fx16", conserve=True)
    plan.set_split(split)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    assert q.dtype == torch.float64
    mass = (np.abs(qn.sum(axis=(1, 2))) / np.abs(qn).sum(axis=(1, 2))).max()
    assert _rel(qn, sp.project_conservative(ref, 2, L)) < 1e-5 and mass < 1e-12
    plan.close()
    plan = qc.Plan(2, N, L, "hard_sphere", M, precision="fx16")
    plan.set_split(split)
    for scheme, fn in (("explicit", stepping.explicit_euler), ("imex", stepping.imex_euler_penalized)):
        ft = torch.tensor(f, dtype=torch.float32, device="cuda")
        st = torch.full((5,), -1, dtype=torch.int32, device="cuda")
        plan.step(ft, 0.02, 1.0, scheme, st)
        torch.cuda.synchronize()
        want = fn(f32, ref, 0.02, 1.0, 2, L) if scheme == "imex" else fn(f32, ref, 0.02, 1.0)
        assert np.abs(ft.cpu().double().numpy() - want).max() <= 2e-6 * np.abs(want).max()
        assert (st.cpu().numpy() == 0).all()
    plan.close()


def test_split_batched_slots_of_one_plan_and_buffer_growth(qc):
    """A split tile-64 plan in several slots of one batched launch (each slot
    takes its own range of the plan's buffers), mixed with unsplit and split
    32x32 plans; then growth of the buffers (a larger batch) and a smaller one
    again. Every result equals the single-call result of its plan bitwise."""
    p64 = qc.Plan(2, 64, 8.0, "hard_sphere", 8, precision="fx16")
    p32 = qc.Plan(2, 32, 8.0, "maxwell", 8, precision="fx16")
    p16 = qc.Plan(2, 16, 8.0, "hard_sphere", 8, precision="fx16")
    p64.set_split(4)
    p32.set_split(4)
    for k, (c1, c2) in enumerate([(3, 2), (70, 41), (2, 5)]):
        fs = [torch.tensor(wl.mixture_cells(2, n, 8.0, c, 900 + 10 * k + i), dtype=torch.float32, device="cuda")
              for i, (n, c) in enumerate([(64, c1), (32, 9), (64, c2), (16, 4)])]
        plans = [p64, p32, p64, p16]
        singles = [p.eval(f) for p, f in zip(plans, fs)]
        outs = [torch.full_like(s, float("nan")) for s in singles]
        qc.eval_multi(plans, fs, outs)
        torch.cuda.synchronize()
        for a, b in zip(singles, outs):
            assert torch.equal(a, b)
        st = [torch.full((f.shape[0],), -1, dtype=torch.int32, device="cuda") for f in fs]
        ref = [f.clone() for f in fs]
        for p, f in zip(plans, ref):
            p.step(f, 0.01, 1.0, "explicit")
        qc.step_multi(plans, fs, 0.01, 1.0, "explicit", st)
        torch.cuda.synchronize()
        for a, b, s in zip(ref, fs, st):
            assert torch.equal(a, b) and (s == 0).all()
    assert p64.info()["device_bytes"] >= 111 * 4 * 32768     # grown for 111 cells of four parts
    for p in (p64, p32, p16):
        p.close()


def test_split_rules_and_rk_ignores_split(qc):
    """Which plans take which factors; the multi-stage step ignores the split."""
    p16 = qc.Plan(2, 16, 8.0, "hard_sphere", 8, precision="fx16")
    assert qc.LIB.qcoll_plan_set_split(p16._h, 4) == qc.EINVAL       # 16x16 tile
    p16.set_tile(32)
    p16.set_split(4)
    p16.set_tile(16)                                                 # no split on this family: reset
    assert p16.split() == 1
    p16.close()
    fp = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fp32")
    assert qc.LIB.qcoll_plan_set_split(fp._h, 4) == qc.EINVAL        # FP32 32x32 tile
    fp.close()
    p3 = qc.Plan(3, 8, 4.0, "hard_sphere", 8, precision="fp32")
    assert qc.LIB.qcoll_plan_set_split(p3._h, 2) == qc.EINVAL
    p3.close()
    p = qc.Plan(2, 64, 8.0, "hard_sphere", 8, precision="fx16")
    for bad in (3, 32, 0):
        assert qc.LIB.qcoll_plan_set_split(p._h, bad) == qc.EINVAL
    f = torch.tensor(wl.mixture_cells(2, 64, 8.0, 3, 4), dtype=torch.float32, device="cuda")
    a, b = f.clone(), f.clone()
    p.step_rk(a, 0.02, 1.0, "ars222")
    p.set_split(2)
    p.step_rk(b, 0.02, 1.0, "ars222")
    empty = torch.empty((0, 64, 64), dtype=torch.float32, device="cuda")
    p.eval(empty)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    p.close()


def test_split_graph_capture_and_replay(qc):
    """Split plans captured in a graph (their buffers exist before the capture;
    growing them under capture is refused): every replay, with eager work and
    synchronisation in between, equals the eager split result bitwise, so the
    arrival counters are back at zero after each launch."""
    p64 = qc.Plan(2, 64, 8.0, "hard_sphere", 8, precision="fx16")
    p32 = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    p64.set_split(4)
    p32.set_split(4)
    f64 = torch.tensor(wl.mixture_cells(2, 64, 8.0, 6, 71), dtype=torch.float32, device="cuda")
    f32 = torch.tensor(wl.mixture_cells(2, 32, 8.0, 9, 72), dtype=torch.float32, device="cuda")
    e64, e32 = p64.eval(f64), p32.eval(f32)          # also sizes the tile-64 buffers
    torch.cuda.synchronize()
    q64, q32 = torch.empty_like(e64), torch.empty_like(e32)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        qc.eval_multi([p64, p32], [f64, f32], [q64, q32])
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        qc.eval_multi([p64, p32], [f64, f32], [q64, q32])
    for r in range(3):
        q64.fill_(float("nan"))
        q32.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(q64, e64) and torch.equal(q32, e32)
        other = p64.eval(f64)                        # eager split work between replays
        torch.cuda.synchronize()
        assert torch.equal(other, e64)
    # growing the buffers under capture is refused before any device work (the
    # raw call: no exception inside the capture)
    big = torch.tensor(wl.mixture_cells(2, 64, 8.0, 80, 73), dtype=torch.float32, device="cuda")
    qb = torch.empty(big.shape, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g2):
        rc = qc.LIB.qcoll_eval(p64._h, ctypes.c_void_p(big.data_ptr()), ctypes.c_void_p(qb.data_ptr()), 80,
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert rc == qc.EINVAL
    q_after = p64.eval(f64)                          # the plan still works outside the capture
    torch.cuda.synchronize()
    assert torch.equal(q_after, e64)
    p64.close()
    p32.close()
