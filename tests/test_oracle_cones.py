"""Pins of the oracle's cone projections against what the mathematics fixes:
closed forms, Moreau's decomposition, idempotence, and brute-force
minimisation on small inputs (cones of Sec. II)."""
import math

import numpy as np
import pytest
import scipy.optimize

from oracle import cones as C


def rng(i=0):
    return np.random.default_rng(12345 + i)


# ----------------------------------------------------------------- SOC

def test_soc_closed_form_cases():
    # inside: unchanged
    v = np.array([0.3, -0.4, 1.0])
    assert np.array_equal(C.proj_soc(v), v)
    # polar: zero
    v = np.array([0.3, -0.4, -1.0])
    assert np.array_equal(C.proj_soc(v), np.zeros(3))
    # outside: ((|x| + t)/2) (x/|x|, 1); here |x| = 5, t = 1 -> 3 * (0.6, 0.8, 1)
    v = np.array([3.0, 4.0, 1.0])
    np.testing.assert_allclose(C.proj_soc(v), [1.8, 2.4, 3.0], rtol=0, atol=1e-15)
    # t is the LAST coordinate: swapping it changes the answer
    assert not np.allclose(C.proj_soc(np.array([1.0, 3.0, 4.0])), [1.8, 2.4, 3.0])


@pytest.mark.parametrize("k", [1, 2, 3, 7, 20])
def test_soc_moreau_idempotent(k):
    r = rng(k)
    for _ in range(200):
        v = r.standard_normal(k) * r.choice([0.1, 1, 10])
        p = C.proj_soc(v)
        q = C.proj_soc(-v)                     # SOC is self-dual: Pi_{K°}(v) = -Pi_K(-v)
        np.testing.assert_allclose(p - q, v, atol=1e-13 * (1 + np.abs(v).max()))
        assert abs(p @ q) <= 1e-12 * (1 + v @ v)
        np.testing.assert_allclose(C.proj_soc(p), p, atol=1e-14 * (1 + np.abs(v).max()))
        if k > 1:
            assert np.linalg.norm(p[:-1]) <= p[-1] + 1e-13


def test_soc_brute_force():
    r = rng(99)
    for _ in range(20):
        v = r.standard_normal(4) * 2
        cons = {"type": "ineq", "fun": lambda p: p[-1] - np.sqrt(p[:-1] @ p[:-1] + 1e-300)}
        best = None
        for start in [np.zeros(4) + [0, 0, 0, 1.0], np.abs(v), C.proj_soc(v) + 0.1]:
            res = scipy.optimize.minimize(lambda p: 0.5 * np.sum((p - v) ** 2), start,
                                          constraints=[cons], method="SLSQP",
                                          options=dict(ftol=1e-14, maxiter=500))
            if best is None or res.fun < best.fun:
                best = res
        np.testing.assert_allclose(C.proj_soc(v), best.x, atol=2e-5)


# ----------------------------------------------------------------- PSD

def test_smat_matches_paper_layout():
    # k = 3: x = (x1..x6), mat(x) = (1/sqrt2) [[sqrt2 x1, x2, x3], [x2, sqrt2 x4, x5], [x3, x5, sqrt2 x6]]
    x = np.arange(1.0, 7.0)
    s2 = math.sqrt(2.0)
    M = np.array([[s2 * 1, 2, 3], [2, s2 * 4, 5], [3, 5, s2 * 6]]) / s2
    np.testing.assert_allclose(C.smat(x, 3), M, atol=1e-15)
    np.testing.assert_allclose(C.svec(M), x, atol=1e-14)


def test_svec_is_isometry():
    r = rng(1)
    for k in [1, 2, 5, 9]:
        X = r.standard_normal((k, k)); X = X + X.T
        Y = r.standard_normal((k, k)); Y = Y + Y.T
        assert abs(C.svec(X) @ C.svec(Y) - np.trace(X @ Y)) < 1e-12 * (1 + np.abs(X).sum() * np.abs(Y).sum())


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_psd_moreau_and_membership(k):
    r = rng(k + 10)
    for _ in range(50):
        X = r.standard_normal((k, k)); X = X + X.T
        x = C.svec(X)
        p = C.proj_psd(x, k)
        q = C.proj_psd(-x, k)
        np.testing.assert_allclose(p - q, x, atol=1e-12 * (1 + np.abs(x).max()))
        assert abs(p @ q) < 1e-11 * (1 + x @ x)
        assert np.linalg.eigvalsh(C.smat(p, k)).min() >= -1e-12 * (1 + np.abs(x).max())
        np.testing.assert_allclose(C.proj_psd(p, k), p, atol=1e-12 * (1 + np.abs(x).max()))


def test_psd_brute_force_2x2():
    r = rng(3)
    for _ in range(10):
        x = r.standard_normal(3) * 2
        # minimise over PSD matrices written as L L^T, L lower triangular
        def f(l):
            L = np.array([[l[0], 0.0], [l[1], l[2]]])
            return np.sum((C.svec(L @ L.T) - x) ** 2)
        best = min((scipy.optimize.minimize(f, s0, method="BFGS", options=dict(gtol=1e-12))
                    for s0 in [np.array([1.0, 0.0, 1.0]), np.array([0.1, 0.5, -0.3]), r.standard_normal(3)]),
                   key=lambda res: res.fun)
        L = np.array([[best.x[0], 0.0], [best.x[1], best.x[2]]])
        np.testing.assert_allclose(C.proj_psd(x, 2), C.svec(L @ L.T), atol=1e-5)


# ----------------------------------------------------------------- exponential cone

def _exp_points(n, seed):
    r = rng(seed)
    pts = []
    for i in range(n):
        kind = i % 5
        v = r.standard_normal(3) * r.choice([0.1, 1.0, 5.0])
        if kind == 1:       # near the boundary
            s = abs(r.standard_normal()) + 0.1
            rho = r.standard_normal()
            v = np.array([s * math.exp(rho), s, s * rho]) + 1e-3 * r.standard_normal(3)
        elif kind == 2:     # x2 <= 0, x3 <= 0
            v = np.array([r.standard_normal(), -abs(r.standard_normal()), -abs(r.standard_normal())])
        pts.append(v)
    return pts


def _dual_violation(y):
    """max(0, -min <y, x>) over unit generators x of K_e: the rays
    (e^rho, 1, rho) and the face generators (1, 0, 0), (0, 0, -1).  This is the
    definition of the dual cone (Sec. II) checked directly, which stays well
    conditioned where the closed-form membership test of K_e* is not."""
    def f(rho):
        a = np.array([math.exp(rho), 1.0, rho])
        return y @ a / np.linalg.norm(a)
    grid = np.linspace(-60, 40, 4001)
    vals = np.array([f(g) for g in grid])
    i = int(np.argmin(vals))
    res = scipy.optimize.minimize_scalar(f, bounds=(grid[max(i - 1, 0)], grid[min(i + 1, 4000)]),
                                         method="bounded", options=dict(xatol=1e-12))
    worst = min(vals.min(), res.fun, y[0], -y[2])
    return max(0.0, -worst)


def _check_exp_kkt(v, p, tol=1e-9):
    scale = 1.0 + np.abs(v).max()
    assert C.in_exp(p, tol), (v, p)
    assert _dual_violation(p - v) <= tol * scale, (v, p)
    assert abs(p @ (p - v)) <= tol * scale * scale, (v, p)


def test_exp_cases_and_kkt():
    seen = set()
    for v in _exp_points(1000, 7):
        p = C.proj_exp(v)
        _check_exp_kkt(v, p)
        np.testing.assert_allclose(C.proj_exp(p), p, atol=1e-10 * (1 + np.abs(v).max()))
        t0, s0, r0 = v
        if C.in_exp(v):
            seen.add("in")
        elif C.in_exp_dual(-v):
            seen.add("polar")
        elif r0 <= 0 and s0 <= 0:
            seen.add("face")
        else:
            seen.add("root")
    assert seen == {"in", "polar", "face", "root"}


def test_exp_constructed_boundary_points():
    # v = p + beta * n with p = s (e^rho, 1, rho) on the boundary and n the outward
    # normal (-1, e^rho (1 - rho), e^rho): the projection is p.
    r = rng(5)
    for _ in range(200):
        s = math.exp(r.uniform(-2, 2))
        rho = r.uniform(-3, 3)
        beta = math.exp(r.uniform(-3, 1))
        p = s * np.array([math.exp(rho), 1.0, rho])
        nrm = np.array([-1.0, math.exp(rho) * (1 - rho), math.exp(rho)])
        v = p + beta * nrm
        np.testing.assert_allclose(C.proj_exp(v), p, rtol=1e-10, atol=1e-10 * np.abs(v).max())


def _brute_exp(v):
    # distance to the boundary rays s (e^rho, 1, rho), s >= 0, on a dense rho grid
    # refined by bounded scalar minimisation, plus the face and the apex.
    def dist2(rho):
        a = np.array([math.exp(rho), 1.0, rho])
        s = max(v @ a, 0.0) / (a @ a)
        return np.sum((s * a - v) ** 2), s * a
    grid = np.linspace(-40, 40, 16001)
    vals = [dist2(g)[0] for g in grid]
    i = int(np.argmin(vals))
    lo, hi = grid[max(i - 1, 0)], grid[min(i + 1, len(grid) - 1)]
    res = scipy.optimize.minimize_scalar(lambda g: dist2(g)[0], bounds=(lo, hi), method="bounded",
                                         options=dict(xatol=1e-12))
    cands = [dist2(res.x)[1], np.array([max(v[0], 0), 0, min(v[2], 0)]), np.zeros(3)]
    if C.in_exp(v):
        cands.append(v.copy())
    return min(cands, key=lambda p: np.sum((p - v) ** 2))


def test_exp_brute_force():
    for v in _exp_points(120, 11):
        p = C.proj_exp(v)
        q = _brute_exp(v)
        d_or = np.linalg.norm(p - v)
        d_bf = np.linalg.norm(q - v)
        assert d_or <= d_bf + 1e-9 * (1 + np.linalg.norm(v))
        np.testing.assert_allclose(p, q, atol=1e-4 * (1 + np.linalg.norm(v)))


def test_exp_dual_projection_moreau():
    for v in _exp_points(300, 13):
        pd = C.proj_exp_dual(v)
        assert _dual_violation(pd) <= 1e-9 * (1 + np.abs(v).max())
        assert C.in_exp(pd - v, 1e-9)
        assert abs(pd @ (pd - v)) <= 1e-9 * (1 + v @ v)


def test_dual_cone_dispatch_layout():
    from paper_1903_06477_amd.generators import Cone
    cone = Cone(z=2, l=3, q=[3, 4], s=[2], ep=2)
    r = rng(21)
    y = r.standard_normal(cone.rows())
    p = C.proj_dual_cone(y, cone)
    np.testing.assert_array_equal(p[:2], y[:2])                       # zero cone: dual is free
    np.testing.assert_array_equal(p[2:5], np.maximum(y[2:5], 0))
    np.testing.assert_allclose(p[5:8], C.proj_soc(y[5:8]))
    np.testing.assert_allclose(p[8:12], C.proj_soc(y[8:12]))
    np.testing.assert_allclose(p[12:15], C.proj_psd(y[12:15], 2))
    np.testing.assert_allclose(p[15:18], C.proj_exp_dual(y[15:18]))
    np.testing.assert_allclose(p[18:21], C.proj_exp_dual(y[18:21]))
