"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Metric (A11 reading): relative L2 over the whole batch, ||Q_gpu - Q_oracle|| /
||Q_oracle||, plus a per-cell bound. Tolerances: the mixed FX16 path 1e-5
(the target stated for the mixed path), plain FP32 2e-4 (FP32 DFT-GEMMs lose
about 5 significant digits to the gain/loss cancellation of these inputs).
"""

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


def _gpu_eval(plan, f64):
    f = torch.tensor(f64, dtype=torch.float32, device="cuda")
    q = plan.eval(f)
    torch.cuda.synchronize()
    return q.cpu().double().numpy()


def _ref(f64, kernel, M, N=32, L=8.0):
    s = sp.Setup(d=2, N=N, L=L, kernel=kernel, M=M)
    return sp.q_fast(f64.astype(np.float32).astype(np.float64), s)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cell_rel(a, b):
    n = a.shape[0]
    return (np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)).max()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
@pytest.mark.parametrize("kernel,M", [("hard_sphere", 8), ("maxwell", 8), ("hard_sphere", 16)])
def test_parity_small_batch(qc, precision, kernel, M):
    f = wl.mixture_cells(2, 32, 8.0, 37, 11)          # 37 cells: not a multiple of the 4 cells per workgroup
    plan = qc.Plan(2, 32, 8.0, kernel, M, precision=precision)
    q = _gpu_eval(plan, f)
    ref = _ref(f, kernel, M)
    err, cerr = _rel(q, ref), _cell_rel(q, ref)
    print(f"{precision} {kernel} M={M}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < TOL[precision] and cerr < 5 * TOL[precision]
    plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
def test_parity_noisy_input(qc, precision):
    """Mixture plus 1% additive noise clipped at 0: fills the high modes."""
    f = wl.noisy_mixture_cells(2, 32, 8.0, 16, 5, 0.01)
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision=precision)
    q = _gpu_eval(plan, f)
    err = _rel(q, _ref(f, "hard_sphere", 8))
    print(f"noisy {precision}: rel L2 {err:.3e}")
    assert err < TOL[precision]
    plan.close()


def test_conservation_projection_fp64(qc):
    f = wl.mixture_cells(2, 32, 8.0, 24, 3)
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    qd = torch.empty((24, 32, 32), dtype=torch.float64, device="cuda")
    plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"), qd)
    torch.cuda.synchronize()
    q = qd.cpu().numpy()
    mass = np.abs(q.sum(axis=(1, 2))) / np.abs(q).sum(axis=(1, 2))
    print(f"conserve: worst mass defect {mass.max():.3e}")
    assert mass.max() <= 1e-12
    mom = sp.moments(q, 2, 8.0)
    scale = sp.moments(np.abs(q), 2, 8.0)
    assert (np.abs(mom) <= 1e-12 * scale[:, [0, 0, 0, 3]] + 1e-14).all()
    ref = sp.project_conservative(_ref(f, "hard_sphere", 8), 2, 8.0)
    assert _rel(q, ref) < 1e-5
    plan.close()


@pytest.mark.parametrize("scheme", ["explicit", "imex"])
def test_step_matches_oracle(qc, scheme):
    f0 = wl.mixture_cells(2, 32, 8.0, 9, 8)
    plan = qc.Plan(2, 32, 8.0, "maxwell", 8, precision="fx16")
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((9,), -1, dtype=torch.int32, device="cuda")
    dt, eps = 0.05, 0.5
    plan.step(f, dt, eps, scheme, status)
    torch.cuda.synchronize()
    f32 = f0.astype(np.float32).astype(np.float64)
    q = _ref(f0, "maxwell", 8)
    if scheme == "explicit":
        want = stepping.explicit_euler(f32, q, dt, eps)
    else:
        want = stepping.imex_euler_penalized(f32, q, dt, eps, 2, 8.0)
    got = f.cpu().double().numpy()
    assert np.abs(got - want).max() <= 2e-6 * np.abs(want).max()
    assert (status.cpu().numpy() == 0).all()
    plan.close()


def test_step_flags_nonfinite_cell_only(qc):
    f0 = wl.mixture_cells(2, 32, 8.0, 6, 8)
    f0[3, 5, 7] = np.inf
    plan = qc.Plan(2, 32, 8.0, "maxwell", 8, precision="fx16")
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((6,), -1, dtype=torch.int32, device="cuda")
    plan.step(f, 0.01, 1.0, "explicit", status)
    torch.cuda.synchronize()
    st = status.cpu().numpy()
    assert st[3] == 1 and (np.delete(st, 3) == 0).all()
    assert np.isfinite(f.cpu().numpy()[[0, 1, 2, 4, 5]]).all()
    plan.close()


def test_full_workload_sampled_cells(qc):
    """4096-cell hard-sphere workload in the benchmark's launch shape; 96 sampled
    cells checked against the oracle. (Without the projection Q is stored in
    FP32 and its discrete mass is only as small as the parity error allows.)"""
    f = wl.config_inputs("hs2d_32")
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    q = _gpu_eval(plan, f)
    idx = np.random.default_rng(0).choice(len(f), 96, replace=False)
    ref = _ref(f[idx], "hard_sphere", 8)
    err = _rel(q[idx], ref)
    print(f"4096 cells: sampled rel L2 {err:.3e}")
    assert err < 1e-5 and _cell_rel(q[idx], ref) < 5e-5
    mass = np.abs(q.sum(axis=(1, 2))) / np.abs(q).sum(axis=(1, 2))
    assert mass.max() < 1e-3
    plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
def test_config3_full_batch_sampled_cells(qc, precision):
    """The 20000-cell 64x64 noisy workload (config 3) in one launch with the
    stored autotuner shape the benchmark times, FP64 projection: 32 cells spread
    over the batch against the oracle (batch and per-cell bounds of the
    precision), and the discrete mass of every cell."""
    f = wl.config_inputs("hs2d_64_noisy")
    plan = qc.Plan(2, 64, 10.0, "hard_sphere", 16, precision=precision, conserve=True)
    plan.load_tuning()
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    idx = np.linspace(0, len(f) - 1, 32).astype(int)
    got = q[idx].cpu().numpy()
    ref = sp.project_conservative(_ref(f[idx], "hard_sphere", 16, N=64, L=10.0), 2, 10.0)
    err, cerr = _rel(got, ref), _cell_rel(got, ref)
    print(f"config 3, 20000 cells, {precision}: 32 sampled cells rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < TOL[precision] and cerr < 5 * TOL[precision]
    qa = q.cpu().numpy()
    mass = np.abs(qa.sum(axis=(1, 2))) / np.abs(qa).sum(axis=(1, 2))
    assert mass.max() <= 1e-12
    plan.close()


def test_edge_cases(qc):
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    empty = torch.empty((0, 32, 32), dtype=torch.float32, device="cuda")
    plan.eval(empty)
    zero = torch.zeros((3, 32, 32), dtype=torch.float32, device="cuda")
    qz = plan.eval(zero)
    torch.cuda.synchronize()
    assert (qz.cpu().numpy() == 0).all()
    one = wl.mixture_cells(2, 32, 8.0, 1, 2)
    assert _rel(_gpu_eval(plan, one), _ref(one, "hard_sphere", 8)) < 1e-5
    # tiny and huge magnitudes: Q is quadratic, the scaling must be exact
    for s in (1e-12, 1e12):
        q = _gpu_eval(plan, one * s)
        assert _rel(q, _ref(one, "hard_sphere", 8) * s * s) < 1e-5
    plan.close()


@pytest.mark.parametrize("N,L,M", [(16, 8.0, 8), (32, 8.0, 8), (64, 10.0, 16)])
@pytest.mark.parametrize("e2", [-120, 120])
def test_fx16_extreme_magnitudes(qc, N, L, M, e2):
    """Near-vacuum (max |f| ~ 2^-121, the tails FP32 subnormal) and near-overflow
    (max |f| ~ 2^119) cells: the per-cell power-of-two scales of the mixed path
    must stay finite and exact, so Q (FP64 output, ~2^(2 e2)) keeps the relative
    accuracy of ordinary inputs."""
    f = (wl.mixture_cells(2, N, L, 3, 77).astype(np.float32) * np.float32(2.0 ** e2)).astype(np.float32)
    f64 = f.astype(np.float64)
    plan = qc.Plan(2, N, L, "hard_sphere", M, precision="fx16", conserve=True)
    q = plan.eval(torch.tensor(f, device="cuda"))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=M)
    ref = sp.project_conservative(sp.q_fast(f64, s), 2, L)
    assert np.isfinite(qn).all()
    err = _rel(qn, ref)
    print(f"N={N} scale 2^{e2}: rel L2 {err:.3e}")
    assert err < 1e-5
    plan.close()


def test_grid_stride_and_determinism(qc):
    """More cells than the grid holds (each wave loops), results bitwise repeatable
    and independent of the batch a cell is in."""
    plan = qc.Plan(2, 32, 8.0, "maxwell", 8, precision="fx16")
    cells = 256 * 8 * 4 + 3
    f = wl.mixture_cells(2, 32, 8.0, cells, 4)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    q1 = plan.eval(ft)
    q2 = plan.eval(ft)
    torch.cuda.synchronize()
    assert torch.equal(q1, q2)
    sub = plan.eval(ft[cells - 5:].contiguous())
    torch.cuda.synchronize()
    assert torch.equal(sub, q1[cells - 5:])
    idx = np.array([0, 1, cells // 2, cells - 1])
    assert _rel(q1.cpu().double().numpy()[idx], _ref(f[idx], "maxwell", 8)) < 1e-5
    plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
@pytest.mark.parametrize("kernel,M,L", [("maxwell", 16, 8.0), ("hard_sphere", 8, 8.0), ("hard_sphere", 8, 6.0)])
def test_parity_n16(qc, precision, kernel, M, L):
    f = wl.mixture_cells(2, 16, L, 21, 17)
    plan = qc.Plan(2, 16, L, kernel, M, precision=precision)
    q = _gpu_eval(plan, f)
    ref = _ref(f, kernel, M, N=16, L=L)
    err = _rel(q, ref)
    print(f"N=16 {precision} {kernel} M={M} L={L}: rel L2 {err:.3e}")
    assert err < TOL[precision]
    plan.close()


def test_n16_conserve_and_step(qc):
    f = wl.mixture_cells(2, 16, 8.0, 10, 3)
    plan = qc.Plan(2, 16, 8.0, "hard_sphere", 8, precision="fx16", conserve=True)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    assert (np.abs(qn.sum(axis=(1, 2))) / np.abs(qn).sum(axis=(1, 2))).max() <= 1e-12
    assert _rel(qn, sp.project_conservative(_ref(f, "hard_sphere", 8, N=16), 2, 8.0)) < 1e-5
    plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
def test_bkw_config1_on_gpu(qc, precision):
    """Config 1: BKW datum on [-8,8]^2, N = 16, Maxwell, M = 16, 100 explicit Euler
    steps of dt = 0.01 with qcoll_step; the GPU trajectory follows the FP64 oracle's
    and its error against the closed form at t = 1 matches the oracle's."""
    from oracle.bkw import bkw_grid, error_norms
    N, L = 16, 8.0
    f0 = bkw_grid(N, L, 0.0)[None]
    plan = qc.Plan(2, N, L, "maxwell", 16, precision=precision)
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    for _ in range(100):
        plan.step(f, 0.01, 1.0, "explicit")
    torch.cuda.synchronize()
    s = sp.Setup(d=2, N=N, L=L, kernel="maxwell", M=16)
    bank = sp.filter_bank(s)
    g = f0.astype(np.float64)
    for _ in range(100):
        g = g + 0.01 * sp.q_fast(g, s, bank)
    got = f.cpu().double().numpy()
    exact = bkw_grid(N, L, 1.0)[None]
    e_gpu, e_ora = error_norms(got, exact), error_norms(g, exact)
    print(f"BKW {precision}: GPU L1/L2/Linf {e_gpu}, oracle {e_ora}, traj diff {_rel(got, g):.2e}")
    assert _rel(got, g) < (2e-6 if precision == "fx16" else 2e-5)
    assert abs(e_gpu[0] - e_ora[0]) < 1e-3 * e_ora[0]
    plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
@pytest.mark.parametrize("N,L,kernel,M", [(8, 4.0, "maxwell", 8), (12, 5.0, "hard_sphere", 8),
                                          (24, 8.0, "hard_sphere", 8), (24, 8.0, "maxwell", 16),
                                          (28, 7.0, "hard_sphere", 12)])
def test_parity_padded_grids(qc, precision, N, L, kernel, M):
    """Grids smaller than the kernel tile (zero-padded DFT operands and filters)."""
    f = wl.mixture_cells(2, N, L, 13, 29)
    plan = qc.Plan(2, N, L, kernel, M, precision=precision)
    q = _gpu_eval(plan, f)
    ref = _ref(f, kernel, M, N=N, L=L)
    err = _rel(q, ref)
    print(f"N={N} {precision} {kernel} M={M}: rel L2 {err:.3e}")
    assert err < TOL[precision]
    plan.close()


def test_gpu_matches_real_space_brute_force(qc):
    """The GPU operator equals the Carleman integrals evaluated in real space on
    the trigonometric interpolant (oracle O3), with no Fourier multiplier formula."""
    from oracle.brute import q_brute
    N, L = 8, 4.0
    f = wl.mixture_cells(2, N, L, 2, 31)
    for kernel, K in [("maxwell", None), ("hard_sphere", 32)]:
        plan = qc.Plan(2, N, L, kernel, 8, K_r=K or 0, precision="fx16")
        q = _gpu_eval(plan, f)
        s = sp.Setup(d=2, N=N, L=L, kernel=kernel, M=8, K_r=K)
        for c in range(2):
            qb = q_brute(f[c].astype(np.float32).astype(np.float64), s).reshape(N, N)
            assert _rel(q[c], qb) < 1e-5
        plan.close()


@pytest.mark.parametrize("precision", ["fx16", "fp32"])
@pytest.mark.parametrize("N,L,kernel,M", [(64, 10.0, "hard_sphere", 16), (64, 10.0, "maxwell", 8),
                                          (48, 8.0, "hard_sphere", 8), (40, 8.0, "maxwell", 8),
                                          (34, 8.0, "hard_sphere", 8)])
def test_parity_tile64(qc, N, L, kernel, M, precision):
    """Grids of 34..64 points: radix-2 parity split over four wavefronts, the
    32-point DFT-GEMMs in FX16 or plain FP32."""
    f = wl.mixture_cells(2, N, L, 6, 41)
    plan = qc.Plan(2, N, L, kernel, M, precision=precision)
    q = _gpu_eval(plan, f)
    ref = _ref(f, kernel, M, N=N, L=L)
    err, cerr = _rel(q, ref), _cell_rel(q, ref)
    print(f"N={N} {precision} {kernel} M={M}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < TOL[precision] and cerr < 5 * TOL[precision]
    plan.close()


def test_tile64_fp32_noisy_conserve_step_and_stages(qc):
    """The plain FP32 path on the config-3 shape (64x64 on [-10,10]^2, hard
    spheres, M = 16, 1% noise): parity at the FP32 bound, FP64 projection, the
    single-stage and the multi-stage updates against the oracle."""
    f = wl.noisy_mixture_cells(2, 64, 10.0, 7, 1002, 0.01)
    ref = _ref(f, "hard_sphere", 16, N=64, L=10.0)
    plan = qc.Plan(2, 64, 10.0, "hard_sphere", 16, precision="fp32", conserve=True)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    err = _rel(qn, sp.project_conservative(ref, 2, 10.0))
    mass = (np.abs(qn.sum(axis=(1, 2))) / np.abs(qn).sum(axis=(1, 2))).max()
    print(f"N=64 fp32 noisy conserve: rel L2 {err:.3e}, mass {mass:.2e}")
    assert err < TOL["fp32"] and mass < 1e-12
    plan.close()
    plan = qc.Plan(2, 64, 10.0, "hard_sphere", 16, precision="fp32")
    f32 = f.astype(np.float32).astype(np.float64)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan.step(ft, 0.02, 1.0, "imex")
    torch.cuda.synchronize()
    want = stepping.imex_euler_penalized(f32, ref, 0.02, 1.0, 2, 10.0)
    assert np.abs(ft.cpu().double().numpy() - want).max() <= 2e-5 * np.abs(want).max()
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    plan.step_rk(ft, 0.02, 1.0, "ars222")
    torch.cuda.synchronize()
    s = sp.Setup(d=2, N=64, L=10.0, kernel="hard_sphere", M=16)
    bank = sp.filter_bank(s)
    want = stepping.imex_rk_penalized(f32, lambda g: sp.q_fast(g, s, bank), 0.02, 1.0, 2, 10.0, "ars222")
    assert np.abs(ft.cpu().double().numpy() - want).max() <= 2e-5 * np.abs(want).max()
    plan.close()


def test_tile64_noisy_conserve_and_step(qc):
    """Config-3 shape (64x64 on [-10,10]^2, hard spheres, M = 16, 1% noise): parity,
    FP64 projection, stage update."""
    f = wl.noisy_mixture_cells(2, 64, 10.0, 5, 1002, 0.01)
    plan = qc.Plan(2, 64, 10.0, "hard_sphere", 16, precision="fx16", conserve=True)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    qn = q.cpu().numpy()
    ref = sp.project_conservative(_ref(f, "hard_sphere", 16, N=64, L=10.0), 2, 10.0)
    err = _rel(qn, ref)
    mass = (np.abs(qn.sum(axis=(1, 2))) / np.abs(qn).sum(axis=(1, 2))).max()
    print(f"N=64 noisy conserve: rel L2 {err:.3e}, mass {mass:.2e}")
    assert err < 1e-5 and mass < 1e-12
    plan.close()
    plan = qc.Plan(2, 64, 10.0, "hard_sphere", 16, precision="fx16")
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    st = torch.full((5,), -1, dtype=torch.int32, device="cuda")
    plan.step(ft, 0.02, 1.0, "imex", st)
    torch.cuda.synchronize()
    f32 = f.astype(np.float32).astype(np.float64)
    want = stepping.imex_euler_penalized(f32, _ref(f, "hard_sphere", 16, N=64, L=10.0), 0.02, 1.0, 2, 10.0)
    assert np.abs(ft.cpu().double().numpy() - want).max() <= 2e-6 * np.abs(want).max()
    assert (st.cpu().numpy() == 0).all()
    plan.close()


@pytest.mark.parametrize("scheme", ["ars222", "bpr343"])
@pytest.mark.parametrize("N,precision", [(32, "fx16"), (16, "fx16"), (24, "fp32"), (48, "fx16")])
def test_step_rk_matches_oracle(qc, scheme, N, precision):
    """Multi-stage penalised IMEX step (one launch per stage) against the oracle's
    stage recursion with the FP64 operator; three steps in a row."""
    cells, L, dt, eps = 7, 8.0, 0.05, 0.5
    f0 = wl.mixture_cells(2, N, L, cells, 31 + N)
    plan = qc.Plan(2, N, L, "hard_sphere", 8, precision=precision)
    f = torch.tensor(f0, dtype=torch.float32, device="cuda")
    status = torch.full((cells,), -1, dtype=torch.int32, device="cuda")
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=8)
    bank = sp.filter_bank(s)
    want = f0.astype(np.float32).astype(np.float64)
    for _ in range(3):
        plan.step_rk(f, dt, eps, scheme, status)
        want = stepping.imex_rk_penalized(want, lambda F: sp.q_fast(F, s, bank), dt, eps, 2, L, scheme)
    torch.cuda.synchronize()
    got = f.cpu().double().numpy()
    err = np.abs(got - want).max() / np.abs(want).max()
    print(f"step_rk {scheme} N={N} {precision}: max rel {err:.3e}")
    assert err <= (3e-6 if precision == "fx16" else 3e-5)
    assert (status.cpu().numpy() == 0).all()
    plan.close()


def test_step_rk_argument_checks(qc):
    plan = qc.Plan(2, 32, 8.0, "maxwell", 8, precision="fx16")
    f = torch.tensor(wl.mixture_cells(2, 32, 8.0, 4, 1), dtype=torch.float32, device="cuda")
    need = qc.LIB.qcoll_step_rk_work_bytes(plan._h, qc.IMEX_BPR343, 4)
    assert need == 7 * 4 * 32 * 32 * 4 + 8 + 4 * 4 * 8   # 2S-3 FP32 slots, alignment, 4 FP64 moments per cell
    small = torch.empty(need // 4 - 1, dtype=torch.float32, device="cuda")
    with pytest.raises(qc.QcollError):
        plan.step_rk(f, 0.01, 1.0, "bpr343", work=small)
    with pytest.raises(qc.QcollError):
        plan.step_rk(f, -0.01, 1.0, "ars222")
    plan.close()


@pytest.mark.parametrize("scheme", ["ars222", "bpr343"])
def test_step_rk_work_buffer_4_byte_aligned(qc, scheme):
    """The stage work buffer needs only float alignment: the FP64 moments of f^n
    that stage 2 keeps for the later stages go to the next 8-byte boundary (the
    size query includes the slack). A buffer one float past an aligned address
    gives the same steps bitwise."""
    cells, N = 5, 32
    f0 = torch.tensor(wl.mixture_cells(2, N, 8.0, cells, 77), dtype=torch.float32, device="cuda")
    plan = qc.Plan(2, N, 8.0, "hard_sphere", 8, precision="fx16")
    need = int(qc.LIB.qcoll_step_rk_work_bytes(plan._h, qc._RK_SCHEMES[scheme], cells))
    big = torch.empty(need // 4 + 1, dtype=torch.float32, device="cuda")
    odd = big[1:]
    assert odd.data_ptr() % 8 == 4 and odd.numel() * 4 == need
    fa, fb = f0.clone(), f0.clone()
    for _ in range(2):
        plan.step_rk(fa, 0.05, 0.5, scheme)
        plan.step_rk(fb, 0.05, 0.5, scheme, work=odd)
    torch.cuda.synchronize()
    assert torch.equal(fa, fb)
    plan.close()


@pytest.mark.parametrize("conserve", [False, True])
def test_tile64_output_not_16_byte_aligned(qc, conserve):
    """The tile-64 kernels write Q through LDS as whole rows, with 16-byte
    stores when Q is 16-byte aligned (the kernel variant the host picks) and
    element stores otherwise: an output aligned only to its elements (8 bytes
    for double Q, 4 for float) gives the same results as an aligned one."""
    N, cells = 48, 5
    f = torch.tensor(wl.mixture_cells(2, N, 8.0, cells, 61), dtype=torch.float32, device="cuda")
    plan = qc.Plan(2, N, 8.0, "hard_sphere", 8, precision="fx16", conserve=conserve)
    dt = torch.float64 if conserve else torch.float32
    ref = plan.eval(f)
    buf = torch.full((cells * N * N + 1,), float("nan"), dtype=dt, device="cuda")
    q = buf[1:].view(cells, N, N)
    plan.eval(f, q)
    torch.cuda.synchronize()
    assert q.data_ptr() % 16 != 0
    assert torch.equal(q, ref)
    plan.close()
