"""GPU parity of the classical spectral method (FP64 direct O(N^4) sum, section
3.3) and of the variable-hard-sphere plans, through the C ABI, against the FP64
oracle.

Tolerances: the classical kernel is FP64 throughout (DFTs as N-point sums,
the double sum over n^2 mode pairs): relative L2 1e-11 against the oracle; the
projection leaves the moments at 1e-12 of their scale. VHS plans run the fast
kernels, whose tolerances are those of the collocation tests (mixed FX16 1e-5,
FP32 2e-4). With its plan's own separable modes the classical kernel computes
the fast operator in FP64, which serves as a full-batch reference for the
fast FX16 kernel.
"""

import numpy as np
import pytest

import workloads as wl
from oracle import classical as cl
from oracle import spectral as sp

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def qc():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2103_14890_amd import qcoll
    return qcoll


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("N,L,kernel,gamma,cells", [(16, 8.0, "maxwell", 1.0, 5), (12, 6.0, "hard_sphere", 1.0, 9),
                                                    (8, 4.0, "vhs", 0.5, 6), (16, 8.0, "vhs", -0.5, 3)])
def test_classical_parity(qc, N, L, kernel, gamma, cells):
    f = wl.mixture_cells(2, N, L, cells, 700 + N)
    plan = qc.Plan(2, N, L, kernel, 8, gamma=gamma, classical=True)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    s = sp.Setup(d=2, N=N, L=L, kernel=kernel, gamma=gamma, M=8)
    ref = cl.q_classical(f.astype(np.float32).astype(np.float64), s)
    got = q.cpu().double().numpy()
    err = _rel(got, ref)
    print(f"classical {kernel} g={gamma} N={N}: rel L2 {err:.3e}")
    # Q is stored as float32 without the projection: the bound is its rounding
    assert err < 1e-7
    plan.close()


@pytest.mark.parametrize("kernel", ["maxwell", "hard_sphere"])
def test_classical_conserve_fp64(qc, kernel):
    N, L, cells = 16, 8.0, 4
    f = wl.mixture_cells(2, N, L, cells, 31)
    plan = qc.Plan(2, N, L, kernel, 8, classical=True, conserve=True)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    assert q.dtype == torch.float64
    got = q.cpu().numpy()
    s = sp.Setup(d=2, N=N, L=L, kernel=kernel, M=8)
    ref = sp.project_conservative(cl.q_classical(f.astype(np.float32).astype(np.float64), s), 2, L)
    err = _rel(got, ref)
    mom = sp.moments(got, 2, L)
    scale = sp.moments(np.abs(got), 2, L)
    print(f"classical {kernel} conserve: rel L2 {err:.3e}")
    assert err < 1e-11
    assert (np.abs(mom) <= 1e-12 * scale[:, [0, 0, 0, 3]] + 1e-14).all()
    plan.close()


def test_separable_classical_is_a_full_batch_reference_for_the_fast_kernel(qc):
    """1024 cells on a 24^2 grid (hard spheres, M = 8): the FP64 direct sum with
    the fast plan's own modes against the oracle on sampled cells, then the FX16
    fast kernel against it on every cell."""
    N, L, cells = 24, 8.0, 1024
    f = wl.mixture_cells(2, N, L, cells, 77)
    ft = torch.tensor(f, dtype=torch.float32, device="cuda")
    ref_plan = qc.Plan(2, N, L, "hard_sphere", 8, classical=True, separable_modes=True, conserve=True)
    fast = qc.Plan(2, N, L, "hard_sphere", 8, precision="fx16", conserve=True)
    qr, qf = ref_plan.eval(ft), fast.eval(ft)
    torch.cuda.synchronize()
    qr, qf = qr.cpu().numpy(), qf.cpu().numpy()
    idx = np.array([0, 500, 1023])
    s = sp.Setup(d=2, N=N, L=L, kernel="hard_sphere", M=8)
    want = sp.project_conservative(sp.q_fast(f[idx].astype(np.float32).astype(np.float64), s), 2, L)
    e_ref = _rel(qr[idx], want)
    e_fast = _rel(qf, qr)
    # per cell, relative to the larger of the cell's norm and kappa |f|^2 (kappa
    # the median of |Q| / |f|^2 over the batch): the FX16 rounding scales with
    # the gain and loss terms, quadratic in f, not with their difference, which
    # is small for cells close to equilibrium
    dn = np.linalg.norm((qf - qr).reshape(cells, -1), axis=1)
    qn = np.linalg.norm(qr.reshape(cells, -1), axis=1)
    f2 = np.linalg.norm(f.reshape(cells, -1), axis=1) ** 2
    scale = np.maximum(qn, np.median(qn / f2) * f2)
    cell = (dn / scale).max()
    print(f"separable classical vs oracle {e_ref:.3e}; fast FX16 vs it over 1024 cells {e_fast:.3e}, "
          f"worst cell {cell:.3e} (against the cell's own norm {(dn / qn).max():.3e})")
    assert e_ref < 1e-11
    assert e_fast < 1e-5 and cell < 5e-5
    ref_plan.close()
    fast.close()


@pytest.mark.parametrize("gamma,precision,N", [(0.5, "fx16", 32), (-0.5, "fx16", 16), (0.0, "fp32", 24)])
def test_vhs_fast_parity(qc, gamma, precision, N):
    f = wl.mixture_cells(2, N, 8.0, 6, 900 + N)
    plan = qc.Plan(2, N, 8.0, "vhs", 8, gamma=gamma, precision=precision)
    q = plan.eval(torch.tensor(f, dtype=torch.float32, device="cuda"))
    torch.cuda.synchronize()
    s = sp.Setup(d=2, N=N, L=8.0, kernel="vhs", gamma=gamma, M=8)
    ref = sp.q_fast(f.astype(np.float32).astype(np.float64), s)
    err = _rel(q.cpu().double().numpy(), ref)
    print(f"vhs gamma={gamma} {precision} N={N}: rel L2 {err:.3e}")
    assert err < (1e-5 if precision == "fx16" else 2e-4)
    plan.close()
