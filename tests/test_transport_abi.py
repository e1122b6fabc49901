"""CPU tests of the transport plan's host tables (built by the C++ plan from the
mesh arrays alone) against the oracle: central stencils (exact), geometry, the
least-squares operator of the optimal polynomial, the face averages of the
Taylor basis; and the argument checks of the C ABI."""

import ctypes

import numpy as np
import pytest

from oracle import transport as tr
from paper_2103_14890_amd import qcoll as qc
from workloads import mesh as wm


@pytest.fixture(scope="module")
def mesh():
    return wm.periodic_dual_mesh(12, seed=7)


@pytest.mark.parametrize("deg", [1, 2])
def test_host_tables_match_oracle(mesh, deg):
    P = qc.TransportPlan(mesh, deg, 16, 10.0, host_only=True)
    T = tr.Transport(mesh, deg)
    tg, wg = tr.gauss01(deg + 1)
    for i in range(mesh.n):
        st = P.table(0, i)
        ns = len(st) // 3
        assert ns == T.ne - 1
        got = [(int(st[s]), (st[ns + s], st[2 * ns + s])) for s in range(ns)]
        assert got == [(c, (float(a), float(b))) for c, (a, b) in T.central_stencil(i)]
        g, G = P.table(1, i), T.geom(i)
        assert abs(g[0] - G.area) <= 1e-14 * G.area
        assert np.abs(g[1:3] - G.xb).max() <= 1e-14 and abs(g[3] - G.h) <= 1e-14
        pinv = np.linalg.pinv(T.cell_tables(i)["A"])
        assert np.abs(P.table(2, i).reshape(T.K, -1) - pinv).max() <= 1e-10 * np.abs(pinv).max()
        poly = T.polygon(i)
        nv = len(poly)
        phi = np.stack([sum(w * T.basis_at(i, poly[a] + t * (poly[(a + 1) % nv] - poly[a])) for t, w in zip(tg, wg))
                        for a in range(nv)])
        assert np.abs(P.table(3, i).reshape(nv, T.K) - phi).max() <= 1e-12
    P.close()


def test_argument_checks(mesh):
    cp, vt, nb, sh, tw, gn = (np.ascontiguousarray(a, dtype=t) for a, t in (
        (mesh.cell_ptr, np.int64), (mesh.verts, np.float64), (mesh.nbr, np.int64),
        (mesh.shift, np.float64), (mesh.twin, np.int64), (mesh.gen, np.float64)))
    P64, PD = ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)

    def plan(cp=cp, nb=nb, tw=tw, sh=sh, deg=2, N=16, L=10.0, flags=qc.HOST_ONLY):
        h = ctypes.c_void_p()
        rc = qc.LIB.qcoll_transport_plan(ctypes.byref(h), len(gn), cp.ctypes.data_as(P64), vt.ctypes.data_as(PD),
                                         nb.ctypes.data_as(P64), sh.ctypes.data_as(PD), tw.ctypes.data_as(P64),
                                         gn.ctypes.data_as(PD), deg, N, L, flags)
        if rc == 0:
            qc.LIB.qcoll_transport_destroy(h)
        return rc
    assert plan() == 0
    for kw in (dict(deg=3), dict(deg=0), dict(N=1), dict(N=65), dict(L=0.0), dict(L=float("nan")),
               dict(flags=0x1 | qc.HOST_ONLY)):
        assert plan(**kw) == qc.EINVAL, kw
    bad = tw.copy()
    bad[[0, 1]] = bad[[1, 0]]
    assert plan(tw=bad) == qc.EINVAL                       # twin faces must pair up
    bad = nb.copy()
    bad[3] = len(gn)
    assert plan(nb=bad) == qc.EINVAL                       # neighbour out of range
    bad = sh.copy()
    bad[0, 0] += 0.5
    assert plan(sh=bad) == qc.EINVAL                       # image offsets are integers
    assert qc.LIB.qcoll_transport_plan(None, len(gn), cp.ctypes.data_as(P64), vt.ctypes.data_as(PD),
                                       nb.ctypes.data_as(P64), sh.ctypes.data_as(PD), tw.ctypes.data_as(P64),
                                       gn.ctypes.data_as(PD), 2, 16, 10.0, qc.HOST_ONLY) == qc.EINVAL
    P = qc.TransportPlan(mesh, 2, 16, 10.0, host_only=True)
    assert P.work_bytes() == len(nb) * 256 * 4
    assert qc.LIB.qcoll_transport_rhs(P._h, None, None, None, 0, None) == qc.EUNSUPPORTED
    assert qc.LIB.qcoll_transport_table(P._h, 9, 0, (ctypes.c_double * 4)(), 4) == qc.EINVAL
    assert qc.LIB.qcoll_transport_table(P._h, 1, mesh.n, (ctypes.c_double * 4)(), 4) == qc.EINVAL
    P.close()


def test_full_size_plan_builds():
    """The explosion_16k mesh (16384 polygons) plans on the host in seconds."""
    c = wm.TRANSPORT_CONFIGS["explosion_16k"]
    mesh, N, L = wm.periodic_dual_mesh(c["nx"], seed=c["seed"]), c["N"], c["L"]
    P = qc.TransportPlan(mesh, 2, N, L, host_only=True)
    assert P.work_bytes() == len(mesh.nbr) * N * N * 4
    P.close()
