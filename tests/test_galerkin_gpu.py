"""GPU parity of the dealiased (Galerkin) variant (section 3.3, eqs. (VAR) and
(ode) summed without wrap-around) against the oracle's 3/2-rule evaluation:
the interpolation onto the 3N/2 grid, the collision kernel of that grid with
the filters restricted to the active N-grid modes, and the restriction back,
all through qcoll_eval_galerkin.

Tolerances: those of the collocation path (mixed FX16 1e-5, plain FP32 2e-4
relative L2 over the batch, 5x per cell); the projection leaves mass, momentum
and energy at FP64 rounding.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import galerkin as og
from oracle import spectral as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"fx16": 1e-5, "fp32": 2e-4}


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import qcoll
    return qcoll


def _ref(f64, N, L, kernel, M, conserve=False):
    s = sp.Setup(d=2, N=N, L=L, kernel=kernel, M=M)
    q = og.q_galerkin(f64.astype(np.float32).astype(np.float64), s)
    return sp.project_conservative(q, 2, L) if conserve else q


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _cell_rel(a, b):
    n = a.shape[0]
    return (np.linalg.norm((a - b).reshape(n, -1), axis=1) / np.linalg.norm(b.reshape(n, -1), axis=1)).max()


# fine grids: 24 and 48 (tile 32 / tile 64 in FX16), 30 (FP32 tile 32), 60, 12
@pytest.mark.parametrize("N,L,kernel,M,precision,cells", [(16, 8.0, "hard_sphere", 8, "fx16", 7),
                                                          (32, 8.0, "hard_sphere", 8, "fx16", 5),
                                                          (20, 8.0, "maxwell", 8, "fp32", 6),
                                                          (40, 8.0, "maxwell", 16, "fx16", 3),
                                                          (8, 4.0, "hard_sphere", 8, "fp32", 9)])
def test_galerkin_parity(qc, N, L, kernel, M, precision, cells):
    f = wl.mixture_cells(2, N, L, cells, 500 + N)
    plan = qc.Plan(2, N, L, kernel, M, precision=precision, galerkin=True)
    q = plan.eval_galerkin(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    got = q.cpu().double().numpy()
    ref = _ref(f, N, L, kernel, M)
    err, cerr = _rel(got, ref), _cell_rel(got, ref)
    print(f"galerkin N={N} {precision} {kernel}: rel L2 {err:.3e}, worst cell {cerr:.3e}")
    assert err < TOL[precision] and cerr < 5 * TOL[precision]
    plan.close()


@pytest.mark.parametrize("N,precision", [(16, "fx16"), (32, "fx16"), (20, "fp32")])
def test_galerkin_conservation(qc, N, precision):
    cells, L = 4, 8.0
    f = wl.mixture_cells(2, N, L, cells, 600 + N)
    plan = qc.Plan(2, N, L, "hard_sphere", 8, precision=precision, conserve=True, galerkin=True)
    q = plan.eval_galerkin(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert q.dtype == torch.float64
    got = q.cpu().numpy()
    mom = sp.moments(got, 2, L)
    scale = sp.moments(np.abs(got), 2, L)
    worst = (np.abs(mom) / scale[:, [0, 0, 0, 3]]).max()
    print(f"galerkin N={N} conserve: worst |moment| / scale {worst:.3e}")
    assert (np.abs(mom) <= 1e-12 * scale[:, [0, 0, 0, 3]] + 1e-14).all()
    ref = _ref(f, N, L, "hard_sphere", 8, conserve=True)
    assert _rel(got, ref) < TOL[precision]
    plan.close()


def test_galerkin_many_cells_sampled(qc):
    """More cells than the interpolation/restriction grids hold (4096
    workgroups, grid-stride loop): sampled cells against the oracle, and the
    whole batch against a second call with a caller-owned work buffer."""
    N, L, cells = 16, 8.0, 4103
    f = wl.mixture_cells(2, N, L, cells, 77)
    plan = qc.Plan(2, N, L, "hard_sphere", 8, precision="fx16", galerkin=True)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    q = plan.eval_galerkin(ft)
    work = torch.empty(plan.galerkin_work_bytes(cells), dtype=torch.uint8, device="cuda")
    q2 = plan.eval_galerkin(ft, work=work)
    torch.cuda.synchronize()
    assert torch.equal(q, q2)
    idx = np.array([0, 2047, 4096, 4102])
    got = q[idx].cpu().double().numpy()
    ref = _ref(f[idx], N, L, "hard_sphere", 8)
    err = _rel(got, ref)
    print(f"galerkin 4103 cells: sampled rel L2 {err:.3e}")
    assert err < TOL["fx16"]
    plan.close()


def test_galerkin_rejects_other_calls_and_small_work(qc):
    plan = qc.Plan(2, 16, 8.0, "hard_sphere", 8, precision="fx16", galerkin=True)
    f = torch.tensor(wl.mixture_cells(2, 16, 8.0, 3, 5), dtype=torch.float32, device="cuda")
    with pytest.raises(qc.QcollError):
        plan.eval(f)
    with pytest.raises(qc.QcollError):
        plan.step(f, 0.01)
    small = torch.empty(plan.galerkin_work_bytes(3) - 1, dtype=torch.uint8, device="cuda")
    with pytest.raises(qc.QcollError):
        plan.eval_galerkin(f, work=small)
    empty = torch.empty((0, 16, 16), dtype=torch.float32, device="cuda")
    assert plan.eval_galerkin(empty).shape == (0, 16, 16)
    plan.close()
