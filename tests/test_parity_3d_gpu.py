"""GPU parity of the 3D path (FP32 MFMA, through the C ABI) against the FP64
oracle: hard spheres on 3D grids (16^3 and 32^3 tiles, zero-padded sizes),
the FP64 conservation projection, the stage updates, and the two-resolution
batched launch of the 3D workload (32^3 and 16^3 cells in one launch).

Tolerance: the plain-FP32 bound of the 2D tests (relative L2 2e-4 over the
batch, 1e-3 per cell); the projection leaves mass, momentum and energy at FP64
rounding (1e-12 relative). The FX16 variant (split-FP16 DFT-GEMMs on 16^3 and
32^3 tiles; spectrum, work fields and filters still stored in FP32): the
mixed-operator target 1e-5 over the batch, 1e-4 per cell.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import spectral as sp
from oracle import stepping

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL, CELL_TOL = 2e-4, 1e-3
FX_TOL, FX_CELL_TOL = 1e-5, 1e-4


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import qcoll
    return qcoll


def _ref(f64, N, L, M):
    s = sp.Setup(d=3, N=N, L=L, kernel="hard_sphere", M=M)
    return sp.q_fast(f64.astype(np.float32).astype(np.float64), s, sp.filter_bank(s))


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cell_rel(a, b):
    n = a.shape[0]
    return (np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)).max()


def _eval(plan, f64, conserve=False):
    f = torch.tensor(f64, dtype=torch.float32, device="cuda")
    q = plan.eval(f)
    torch.cuda.synchronize()
    return q.cpu().double().numpy()


@pytest.mark.parametrize("N,L,M,cells", [(16, 8.0, 8, 6), (16, 8.0, 32, 5), (12, 6.0, 8, 5), (8, 4.0, 8, 7),
                                         (32, 8.0, 8, 3), (24, 8.0, 8, 3)])
def test_parity_3d(qc, N, L, M, cells):
    f = wl.mixture_cells(3, N, L, cells, 40 + N)
    plan = qc.Plan(3, N, L, "hard_sphere", M, precision="fp32")
    q = _eval(plan, f)
    ref = _ref(f, N, L, M)
    err, cerr = _rel(q, ref), _cell_rel(q, ref)
    print(f"3D N={N} M={M}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < TOL and cerr < CELL_TOL
    plan.close()


@pytest.mark.parametrize("N,M,cells", [(32, 8, 8), (24, 8, 8), (20, 8, 8), (32, 32, 8), (16, 8, 8), (16, 32, 8),
                                       (12, 8, 8), (8, 8, 8)])
def test_parity_3d_fx16(qc, N, M, cells):
    f = wl.mixture_cells(3, N, 8.0, cells, 40 + N)
    plan = qc.Plan(3, N, 8.0, "hard_sphere", M, precision="fx16")
    q = _eval(plan, f)
    ref = _ref(f, N, 8.0, M)
    err, cerr = _rel(q, ref), _cell_rel(q, ref)
    print(f"3D FX16 N={N} M={M}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < FX_TOL and cerr < FX_CELL_TOL
    plan.close()


def test_parity_3d_fx16_every_even_grid(qc):
    """Every even grid from 8^3 to 32^3 (M = 8, batches of 8 cells): the batch
    stays within the mixed-operator target. Single cells near equilibrium,
    where gain and loss cancel most, carry the FP32 storage floor of this
    variant's spectrum, filters and work fields: up to about 1e-4 of their own
    norm."""
    for N in range(8, 33, 2):
        f = wl.mixture_cells(3, N, 8.0, 8, 40 + N)
        plan = qc.Plan(3, N, 8.0, "hard_sphere", 8, precision="fx16")
        q = _eval(plan, f)
        ref = _ref(f, N, 8.0, 8)
        err, cerr = _rel(q, ref), _cell_rel(q, ref)
        print(f"3D FX16 N={N}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
        assert err < FX_TOL and cerr < 2 * FX_CELL_TOL, N
        plan.close()


@pytest.mark.parametrize("N", [16, 32])
@pytest.mark.parametrize("e2", [-120, -100, 90])
def test_fx16_3d_extreme_magnitudes(qc, N, e2):
    """Small (max |f| ~ 2^-101, ~2^-121) and large (~2^89) cells on the 3D FX16
    path: the tile scales stay finite at every magnitude, and Q keeps the
    accuracy it has at unit scale while the FP32 spectra and work fields stay in
    the FP32 normal range (at 2^-121 their tails are subnormal: finite results,
    fewer digits)."""
    f1 = wl.mixture_cells(3, N, 8.0, 8, 78).astype(np.float32)
    s = sp.Setup(d=3, N=N, L=8.0, kernel="hard_sphere", M=8)
    bank = sp.filter_bank(s)
    plan = qc.Plan(3, N, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    errs = []
    for f in (f1, (f1 * np.float32(2.0 ** e2)).astype(np.float32)):
        q = plan.eval(torch.tensor(f, device="cuda"))
        torch.cuda.synchronize()
        qn = q.cpu().numpy()
        assert np.isfinite(qn).all()
        errs.append(_rel(qn, sp.project_conservative(sp.q_fast(f.astype(np.float64), s, bank), 3, 8.0)))
    print(f"3D FX16 N={N} scale 2^{e2}: rel L2 {errs[1]:.3e} (unit scale {errs[0]:.3e})")
    assert errs[0] < FX_TOL
    if e2 > -110:
        assert errs[1] < FX_TOL and errs[1] < 1.5 * errs[0] + 1e-7
    else:
        assert errs[1] < 1e-3
    plan.close()


def test_fx16_and_fp32_slots_in_one_call(qc):
    """FX16 plans of 32^3, 24^3 and 16^3 and an FP32 16^3 plan in one batched
    call equal their single-plan calls bitwise (eval with the projection, the
    IMEX step); FX16 plans of different grids in one launch use their own DFT
    tables."""
    fa = wl.mixture_cells(3, 32, 8.0, 8, 81)
    fc = wl.mixture_cells(3, 24, 8.0, 8, 82)
    fd = wl.mixture_cells(3, 16, 8.0, 8, 84)
    fb = wl.mixture_cells(3, 16, 8.0, 5, 83)
    pa = qc.Plan(3, 32, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    pc = qc.Plan(3, 24, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    pd = qc.Plan(3, 16, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    pb = qc.Plan(3, 16, 8.0, "hard_sphere", 8, precision="fp32", conserve=True)
    plans = (pa, pc, pd, pb)
    xs = [torch.tensor(x, dtype=torch.float32, device="cuda") for x in (fa, fc, fd, fb)]
    qs = [torch.empty(x.shape, dtype=torch.float64, device="cuda") for x in xs]
    qc.eval_multi(list(plans), xs, qs)
    singles = [p.eval(x) for p, x in zip(plans, xs)]
    torch.cuda.synchronize()
    for a, b in zip(qs, singles):
        assert torch.equal(a, b)
    ys = [x.clone() for x in xs]
    qc.step_multi(list(plans), xs, 0.01, 1.0, "imex")
    for p, y in zip(plans, ys):
        p.step(y, 0.01, 1.0, "imex")
    torch.cuda.synchronize()
    for a, b in zip(xs, ys):
        assert torch.equal(a, b)
    for q, f, N in ((qs[0], fa, 32), (qs[1], fc, 24), (qs[2], fd, 16)):
        ref = sp.project_conservative(_ref(f, N, 8.0, 8), 3, 8.0)
        err = _rel(q.cpu().numpy(), ref)
        print(f"mixed call: FX16 {N}^3 rel L2 {err:.3e}")
        assert err < FX_TOL
    for p in plans:
        p.close()


@pytest.mark.parametrize("N", [16, 32])
def test_conservation_3d(qc, N):
    cells = 4
    f = wl.mixture_cells(3, N, 8.0, cells, 7)
    plan = qc.Plan(3, N, 8.0, "hard_sphere", 8, precision="fp32", conserve=True)
    qd = torch.empty((cells, N, N, N), dtype=torch.float64, device="cuda")
    plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"), qd)
    torch.cuda.synchronize()
    q = qd.cpu().numpy()
    mom = sp.moments(q, 3, 8.0)
    scale = sp.moments(np.abs(q), 3, 8.0)
    print(f"3D N={N} conserve: worst |moment| / scale {(np.abs(mom) / scale[:, [0, 0, 0, 0, 4]]).max():.3e}")
    assert (np.abs(mom) <= 1e-12 * scale[:, [0, 0, 0, 0, 4]] + 1e-14).all()
    ref = sp.project_conservative(_ref(f, N, 8.0, 8), 3, 8.0)
    assert _rel(q, ref) < TOL
    plan.close()


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_step_3d(qc, scheme):
    N, L, cells = 16, 8.0, 5
    f0 = wl.mixture_cells(3, N, L, cells, 9)
    plan = qc.Plan(3, N, L, "hard_sphere", 8, precision="fp32")
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((cells,), -1, dtype=torch.int32, device="cuda")
    dt, eps = 0.05, 0.5
    plan.step(f, dt, eps, scheme, status)
    torch.cuda.synchronize()
    f32 = f0.astype(np.float32).astype(np.float64)
    q = _ref(f0, N, L, 8)
    want = (stepping.explicit_euler(f32, q, dt, eps) if scheme == "explicit"
            else stepping.imex_euler_penalized(f32, q, dt, eps, 3, L))
    got = f.cpu().double().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"3D step {scheme}: max rel {err:.3e}")
    assert err <= 1e-5
    assert (status.cpu().numpy() == 0).all()
    plan.close()


def test_step_3d_flags_nonfinite_cell_only(qc):
    f0 = wl.mixture_cells(3, 16, 8.0, 4, 10)
    f0[2, 3, 4, 5] = np.nan
    plan = qc.Plan(3, 16, 8.0, "hard_sphere", 8, precision="fp32")
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((4,), -1, dtype=torch.int32, device="cuda")
    plan.step(f, 0.01, 1.0, "explicit", status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[2] == 1 and (np.delete(st, 2) == 0).all()
    assert np.isfinite(f.cpu().numpy()[[0, 1, 3]]).all()
    plan.close()


def test_two_resolutions_one_launch(qc):
    """32^3 and 16^3 cells in one batched call equal the single-plan calls
    bitwise, for eval with the projection and for the step."""
    f32c = wl.mixture_cells(3, 32, 8.0, 3, 21)
    f16c = wl.mixture_cells(3, 16, 8.0, 7, 22)
    p32 = qc.Plan(3, 32, 8.0, "hard_sphere", 32, precision="fp32", conserve=True)
    p16 = qc.Plan(3, 16, 8.0, "hard_sphere", 32, precision="fp32", conserve=True)
    a = torch.tensor(f32c, dtype=torch.float32, device="cuda")
    b = torch.tensor(f16c, dtype=torch.float32, device="cuda")
    qa = torch.empty(a.shape, dtype=torch.float64, device="cuda")
    qb = torch.empty(b.shape, dtype=torch.float64, device="cuda")
    qc.eval_multi([p32, p16], [a, b], [qa, qb])
    sa, sb = p32.eval(a), p16.eval(b)
    torch.cuda.synchronize()
    assert torch.equal(qa, sa) and torch.equal(qb, sb)
    fa, fb = a.clone(), b.clone()
    qc.step_multi([p32, p16], [a, b], 0.01, 1.0, "imex")
    p32.step(fa, 0.01, 1.0, "imex")
    p16.step(fb, 0.01, 1.0, "imex")
    torch.cuda.synchronize()
    assert torch.equal(a, fa) and torch.equal(b, fb)
    ref = sp.project_conservative(_ref(f16c, 16, 8.0, 32), 3, 8.0)
    err = _rel(qb.cpu().numpy(), ref)
    print(f"two resolutions: 16^3 rel L2 {err:.3e}")
    assert err < TOL
    p32.close()
    p16.close()


@pytest.mark.parametrize("precision", ["fp32", "fx16"])
@pytest.mark.parametrize("name,N", [("hs3d_32", 32), ("hs3d_16", 16)])
def test_3d_workload_sampled_cells(qc, precision, name, N):
    """Each resolution of the 3D workload at 1024 cells in the launch shape of
    the benchmark: 32 cells spread over the batch against the oracle (batch
    and per-cell bounds), and the projection's moments on all cells."""
    f = wl.config_inputs(name, cells=1024)
    plan = qc.Plan(3, N, 8.0, "hard_sphere", 32, precision=precision, conserve=True)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    q = plan.eval(ft)
    torch.cuda.synchronize()
    idx = np.linspace(0, 1023, 32).astype(int)
    got = q[idx].cpu().numpy()
    ref = sp.project_conservative(_ref(f[idx], N, 8.0, 32), 3, 8.0)
    err, cerr = _rel(got, ref), _cell_rel(got, ref)
    print(f"{name} 1024 cells ({precision}): 32 sampled cells rel L2 {err:.3e}, worst cell {cerr:.3e}")
    if precision == "fx16":
        assert err < FX_TOL and cerr < FX_CELL_TOL
    else:
        assert err < TOL and cerr < CELL_TOL
    qa = q.cpu().numpy()
    mass = np.abs(qa.sum(axis=(1, 2, 3))) / np.abs(qa).sum(axis=(1, 2, 3))
    assert mass.max() <= 1e-12
    plan.close()


def test_3d_stage_graph_replay(qc):
    """One hipGraph-captured launch per stage over both resolutions (32^3 and
    16^3): every replay advances the state exactly like the eager batched step."""
    a0 = torch.tensor(wl.mixture_cells(3, 32, 8.0, 2, 61), dtype=torch.float32, device="cuda")
    b0 = torch.tensor(wl.mixture_cells(3, 16, 8.0, 5, 62), dtype=torch.float32, device="cuda")
    p32 = qc.Plan(3, 32, 8.0, "hard_sphere", 8, precision="fp32")
    p16 = qc.Plan(3, 16, 8.0, "hard_sphere", 8, precision="fp32")
    ea, eb = a0.clone(), b0.clone()          # eager reference trajectory
    ga, gb = a0.clone(), b0.clone()          # graph-owned state
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):               # warm-up on the side stream
        wa, wb = a0.clone(), b0.clone()
        qc.step_multi([p32, p16], [wa, wb], 0.01, 1.0, "imex")
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        qc.step_multi([p32, p16], [ga, gb], 0.01, 1.0, "imex")
    ga.copy_(a0)
    gb.copy_(b0)
    for _ in range(3):
        g.replay()
        qc.step_multi([p32, p16], [ea, eb], 0.01, 1.0, "imex")
        torch.cuda.synchronize()
        assert torch.equal(ga, ea) and torch.equal(gb, eb)
    p32.close()
    p16.close()


@pytest.mark.parametrize("scheme,N,precision", [("ars222", 16, "fp32"), ("bpr343", 16, "fp32"),
                                                ("bpr343", 24, "fx16")])
def test_step_rk_3d(qc, scheme, N, precision):
    """Multi-stage penalised IMEX step on a 3D grid against the oracle's stage
    recursion with the FP64 operator."""
    L, cells, dt, eps = 8.0, 3, 0.05, 0.5
    f0 = wl.mixture_cells(3, N, L, cells, 71)
    plan = qc.Plan(3, N, L, "hard_sphere", 8, precision=precision)
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((cells,), -1, dtype=torch.int32, device="cuda")
    plan.step_rk(f, dt, eps, scheme, status)
    torch.cuda.synchronize()
    s = sp.Setup(d=3, N=N, L=L, kernel="hard_sphere", M=8)
    bank = sp.filter_bank(s)
    want = stepping.imex_rk_penalized(f0.astype(np.float32).astype(np.float64),
                                      lambda F: sp.q_fast(F, s, bank), dt, eps, 3, L, scheme)
    got = f.cpu().double().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"3D step_rk {scheme} N={N} {precision}: max rel {err:.3e}")
    assert err <= 3e-5
    assert (status.cpu().numpy() == 0).all()
    plan.close()


@pytest.mark.parametrize("precision", ["fp32", "fx16"])
def test_workspace_calls_run_concurrently_on_one_plan(qc, precision):
    """One 3D plan, two streams, two caller workspaces (qcoll_eval_ws /
    qcoll_step_ws): concurrent calls equal the plan-scratch calls bitwise; a
    workspace smaller than one workgroup's scratch is refused; 2D plans take
    none."""
    N = 16
    plan = qc.Plan(3, N, 8.0, "hard_sphere", 8, precision=precision, conserve=True)
    sb = plan.scratch_bytes()
    assert sb == 144 * 16 ** 3
    fa = torch.tensor(wl.mixture_cells(3, N, 8.0, 40, 91), dtype=torch.float32, device="cuda")
    fb = torch.tensor(wl.mixture_cells(3, N, 8.0, 24, 92), dtype=torch.float32, device="cuda")
    ra, rb = plan.eval(fa), plan.eval(fb)
    torch.cuda.synchronize()
    wa = torch.empty(3 * sb, dtype=torch.uint8, device="cuda")     # three workgroups in flight
    wb = torch.empty(sb, dtype=torch.uint8, device="cuda")         # one
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s1.wait_stream(torch.cuda.current_stream())
    s2.wait_stream(torch.cuda.current_stream())
    qa = plan.eval_ws(fa, wa, stream=s1)
    qb = plan.eval_ws(fb, wb, stream=s2)
    torch.cuda.current_stream().wait_stream(s1)
    torch.cuda.current_stream().wait_stream(s2)
    torch.cuda.synchronize()
    assert torch.equal(qa, ra) and torch.equal(qb, rb)
    step_plan = qc.Plan(3, N, 8.0, "hard_sphere", 8, precision=precision)
    x, y = fa.clone(), fa.clone()
    step_plan.step(x, 0.01, 1.0, "imex")
    step_plan.step_ws(y, 0.01, wa, 1.0, "imex")
    torch.cuda.synchronize()
    assert torch.equal(x, y)
    small = torch.empty(sb - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(qc.QcollError):
        plan.eval_ws(fa, small)
    with pytest.raises(qc.QcollError):          # misaligned
        plan.eval_ws(fa, wa[16:16 + 2 * sb])
    p2 = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision=precision)
    assert p2.scratch_bytes() == 0
    f2 = torch.tensor(wl.mixture_cells(2, 32, 8.0, 5, 93), dtype=torch.float32, device="cuda")
    assert torch.equal(p2.eval_ws(f2, small), p2.eval(f2))
    for p in (plan, step_plan, p2):
        p.close()
