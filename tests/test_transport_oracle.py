"""Pins of the transport oracle (CWENO reconstruction + Rusanov fluxes on the
centroid-dual polygonal mesh, section 2.2) against facts that do not come from
the oracle itself: the mesh tiles the periodic square, exact polygon moments
against an independent fan quadrature, exact reproduction of polynomial data,
free-stream preservation, discrete conservation, the non-oscillatory behaviour
of the nonlinear weights at a jump, and the observed order of accuracy on a
smooth periodic profile against the exact flux divergence."""

import numpy as np
import pytest

from oracle import transport as tr
from workloads import mesh as wm


def _fan_rule(n=8):
    """Collapsed Gauss rule on the reference triangle (0,0), (1,0), (0,1)."""
    t, w = np.polynomial.legendre.leggauss(n)
    t, w = 0.5 * (t + 1), 0.5 * w
    u, v = np.meshgrid(t, t, indexing="ij")
    wu, wv = np.meshgrid(w, w, indexing="ij")
    return (u * (1 - v)).ravel(), v.ravel(), (wu * wv * (1 - v)).ravel()


FAN = _fan_rule(8)


def fan_integral(P, fun):
    """Integral and area of a star-shaped polygon by triangles from its vertex mean."""
    c = P.mean(0)
    tot = area = 0.0
    for a in range(len(P)):
        p0, p1 = P[a], P[(a + 1) % len(P)]
        J = (p0[0] - c[0]) * (p1[1] - c[1]) - (p1[0] - c[0]) * (p0[1] - c[1])
        X = c[0] + FAN[0] * (p0[0] - c[0]) + FAN[1] * (p1[0] - c[0])
        Y = c[1] + FAN[0] * (p0[1] - c[1]) + FAN[1] * (p1[1] - c[1])
        tot += J * np.sum(FAN[2] * fun(X, Y))
        area += J * FAN[2].sum()
    return tot, area


@pytest.fixture(scope="module")
def mesh12():
    return wm.periodic_dual_mesh(12, seed=3)


def test_mesh_tiles_periodic_square(mesh12):
    m = mesh12
    T = tr.Transport(m, 1)
    areas = np.array([T.geom(i).area for i in range(m.n)])
    shoelace = []
    for i in range(m.n):
        P = T.polygon(i)
        Q = np.roll(P, -1, axis=0)
        shoelace.append(0.5 * np.sum(P[:, 0] * Q[:, 1] - Q[:, 0] * P[:, 1]))
    assert (areas > 0).all()
    assert abs(areas.sum() - 1.0) < 1e-13
    assert np.abs(areas - np.array(shoelace)).max() < 1e-15
    # every face appears twice with opposite orientation and opposite image offset
    assert (m.twin[m.twin] == np.arange(len(m.twin))).all()
    assert np.array_equal(m.shift[m.twin], -m.shift)


def test_polygon_moments_exact(mesh12):
    rng = np.random.default_rng(4)
    T = tr.Transport(mesh12, 2)
    for i in rng.choice(mesh12.n, 5, replace=False):
        P = T.polygon(int(i)) * 3.0 - 0.7
        for p in range(5):
            for q in range(5 - p):
                ref, _ = fan_integral(P, lambda x, y: x ** p * y ** q)
                assert abs(tr.polygon_moment(P, p, q) - ref) <= 1e-13 * max(1.0, abs(ref))


def _poly_data(T, deg, rng):
    """A random polynomial of total degree deg and its exact cell averages over
    shifted polygons (by the fan quadrature, independent of the oracle)."""
    coef = rng.normal(size=(deg + 1, deg + 1))
    fun = lambda x, y: sum(coef[p, q] * x ** p * y ** q for p in range(deg + 1) for q in range(deg + 1 - p))

    def values(j, s):
        tot, area = fan_integral(T.polygon(j, s), fun)
        return np.array([tot / area])
    return fun, values


@pytest.mark.parametrize("deg", [1, 2])
def test_reconstruction_reproduces_polynomials(mesh12, deg):
    rng = np.random.default_rng(10 + deg)
    T = tr.Transport(mesh12, deg)
    for i in rng.choice(mesh12.n, 6, replace=False):
        i = int(i)
        P = T.polygon(i)
        pts = P.mean(0) + 0.5 * (P - P.mean(0))[rng.integers(0, len(P), 4)] * rng.uniform(0.2, 1.0, (4, 1))
        # degree-deg data is reproduced by the optimal polynomial (linear weights)
        fun, values = _poly_data(T, deg, rng)
        c = T.reconstruct(i, None, values=values, linear_weights=True)
        got = values(i, (0.0, 0.0))[0] + T.basis_at(i, pts) @ c[:, 0]
        assert np.abs(got - fun(pts[:, 0], pts[:, 1])).max() < 1e-10
        # linear data: every candidate polynomial is exact, so any weights reproduce it
        fun1, values1 = _poly_data(T, 1, rng)
        c = T.reconstruct(i, None, values=values1)
        got = values1(i, (0.0, 0.0))[0] + T.basis_at(i, pts) @ c[:, 0]
        assert np.abs(got - fun1(pts[:, 0], pts[:, 1])).max() < 1e-10


def test_nonlinear_weights_damp_oscillations_at_a_jump(mesh12):
    """Data with a jump across a line through a cell: the CWENO weights leave a
    much smaller overshoot at the cell's faces than the linear weights."""
    T = tr.Transport(mesh12, 2)
    m = mesh12
    worst_lin = worst_nl = 0.0
    for i in range(0, m.n, 7):
        x0 = m.gen[i]

        def values(j, s, x0=x0):
            return np.array([1.0 if m.gen[j, 0] + s[0] > x0[0] + 0.02 else 0.0])
        P = T.polygon(i)
        fi = values(i, (0.0, 0.0))[0]
        for lin in (True, False):
            c = T.reconstruct(i, None, values=values, linear_weights=lin)
            u = fi + T.basis_at(i, P) @ c[:, 0]
            over = max(u.max() - 1.0, -u.min(), 0.0)
            if lin:
                worst_lin = max(worst_lin, over)
            else:
                worst_nl = max(worst_nl, over)
    assert worst_lin > 0.05
    assert worst_nl < 0.2 * worst_lin


@pytest.mark.parametrize("deg", [1, 2])
def test_free_stream_and_conservation(mesh12, deg):
    T = tr.Transport(mesh12, deg)
    vel = tr.velocity_pairs(4, 3.0)
    R = T.residual(np.full((mesh12.n, len(vel)), 0.7), vel)
    assert np.abs(R).max() < 1e-12
    f = np.random.default_rng(5).uniform(0.2, 1.0, size=(mesh12.n, len(vel)))
    R = T.residual(f, vel)
    area = np.array([T.geom(i).area for i in range(mesh12.n)])
    tot = (area[:, None] * R).sum(0)
    assert np.abs(tot).max() < 1e-12 * np.abs(area[:, None] * R).sum(0).max()


def _smooth_case(nx, deg):
    m = wm.periodic_dual_mesh(nx, seed=5)
    T = tr.Transport(m, deg)
    fun = lambda x, y: 1 + 0.3 * np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y)
    vel = np.array([[1.0, 0.4]])
    tg, wg = np.polynomial.legendre.leggauss(10)
    tg, wg = 0.5 * (tg + 1), 0.5 * wg
    fb, Rex = np.zeros((m.n, 1)), np.zeros((m.n, 1))
    for i in range(m.n):
        P = T.polygon(i)
        tot, area = fan_integral(P, fun)
        fb[i, 0] = tot / area
        acc = 0.0
        for k in range(len(P)):
            e = P[(k + 1) % len(P)] - P[k]
            ln = np.hypot(*e)
            x = P[k][None] + tg[:, None] * e[None]
            acc += ln * np.sum(wg * fun(x[:, 0], x[:, 1])) * (vel[0] @ np.array([e[1], -e[0]]) / ln)
        Rex[i, 0] = -acc / area
    return np.abs(T.residual(fb, vel) - Rex).mean()


@pytest.mark.parametrize("deg,min_order", [(1, 0.8), (2, 1.8)])
def test_order_of_accuracy(deg, min_order):
    """L1 error of the flux divergence against the exact one on two meshes."""
    e1, e2 = _smooth_case(12, deg), _smooth_case(24, deg)
    order = np.log2(e1 / e2)
    print(f"deg {deg}: L1 errors {e1:.3e} {e2:.3e}, order {order:.2f}")
    assert order >= min_order
