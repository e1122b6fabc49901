"""GPU test of qcoll_step_rk_noalloc (the multi-stage IMEX step whose work
buffer is the library's fixed device array, for callers that cannot
allocate): through the C ABI, two calls in a row, the second on a smaller
input, each bitwise equal to qcoll_step_rk with a caller-owned work buffer;
the size limit; and no allocation by the call."""

import ctypes

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


def _noalloc(qc, plan, f, scheme, status):
    return qc.LIB.qcoll_step_rk_noalloc(plan._h, ctypes.c_void_p(f.data_ptr()), f.shape[0], 0.02, 0.7,
                                        qc._RK_SCHEMES[scheme], ctypes.c_void_p(status.data_ptr()),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


@pytest.mark.parametrize("d,N,L,M,precision,scheme,cells", [
    (2, 32, 8.0, 8, "fx16", "bpr343", (600, 37)),
    (2, 64, 10.0, 16, "fx16", "ars222", (120, 9)),
    (2, 24, 8.0, 8, "fp32", "ars222", (300, 5)),
    (3, 16, 8.0, 8, "fx16", "ars222", (40, 3)),
])
def test_noalloc_matches_step_rk_twice(qc, d, N, L, M, precision, scheme, cells):
    plan = qc.Plan(d, N, L, "hard_sphere", M, precision=precision)
    for k, n in enumerate(cells):   # two calls in a row, the second smaller
        f0 = wl.mixture_cells(d, N, L, n, 500 + 7 * k + N)
        a = torch.tensor(f0, dtype=torch.float32, device="cuda")
        b = a.clone()
        sa = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        sb = sa.clone()
        work = torch.empty(int(qc.LIB.qcoll_step_rk_work_bytes(plan._h, qc._RK_SCHEMES[scheme], n)) // 4,
                           dtype=torch.float32, device="cuda")
        plan.step_rk(b, 0.02, 0.7, scheme, sb, work=work)
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        assert _noalloc(qc, plan, a, scheme, sa) == qc.OK
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() == before
        assert torch.equal(a, b), (d, N, n)
        assert torch.equal(sa, sb) and (sa.cpu().numpy() == 0).all()
        assert not torch.equal(a, torch.tensor(f0, dtype=torch.float32, device="cuda"))
    plan.close()


def test_noalloc_size_limit_and_arguments(qc):
    plan = qc.Plan(2, 32, 8.0, "hard_sphere", 8, precision="fx16")
    f = torch.zeros((4, 32, 32), dtype=torch.float32, device="cuda")
    st = torch.zeros(4, dtype=torch.int32, device="cuda")
    limit = qc.NOALLOC_SCRATCH_BYTES // (7 * 1024 * 4)          # BPR(3,4,3): seven stage slots
    too_many = limit + 1
    rc = qc.LIB.qcoll_step_rk_noalloc(plan._h, ctypes.c_void_p(f.data_ptr()), too_many, 0.01, 1.0,
                                      qc.IMEX_BPR343, None, None)
    assert rc == qc.ETOOLARGE and qc.strerror(rc) != "unknown error"
    assert qc.LIB.qcoll_step_rk_noalloc(plan._h, None, 4, 0.01, 1.0, qc.IMEX_ARS222, None, None) == qc.EINVAL
    assert qc.LIB.qcoll_step_rk_noalloc(plan._h, ctypes.c_void_p(f.data_ptr()), 4, 0.01, 1.0, 9, None,
                                        None) == qc.EINVAL
    assert qc.LIB.qcoll_step_rk_noalloc(plan._h, ctypes.c_void_p(f.data_ptr()), 0, 0.01, 1.0, qc.IMEX_ARS222,
                                        None, None) == qc.OK
    del st
    plan.close()
