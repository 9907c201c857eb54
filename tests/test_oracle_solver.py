"""Pins of the oracle's linear step, T-oracle, directions and Algorithm 1
against identities, textbook routines, brute force and closed-form optima."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import cones as C
from oracle.linsys import DirectLinSys, Q_dense
from oracle import superscs as S
from paper_1903_06477_amd import generators as G

HERE = os.path.dirname(os.path.abspath(__file__))


def _prob_from_json(d):
    A = sp.csr_matrix(np.array(d["A"], dtype=float))
    cone = G.Cone(**d["cone"])
    return G.Problem(A=A, b=np.array(d["b"], float), c=np.array(d["c"], float), cone=cone)


# ------------------------------------------------------------ HSDE matrix, linear step

@pytest.mark.parametrize("m,n", [(12, 5), (5, 12), (30, 30)])
def test_Q_skew_and_orthogonal(m, n):
    r = np.random.default_rng(m * 100 + n)
    A = r.standard_normal((m, n))
    Q = Q_dense(A, r.standard_normal(m), r.standard_normal(n))
    np.testing.assert_array_equal(Q + Q.T, 0)
    for _ in range(10):
        u = r.standard_normal(m + n + 1)
        assert abs(u @ Q @ u) <= 1e-12 * (u @ u) * np.abs(Q).max()


@pytest.mark.parametrize("m,n,density", [(40, 15, 0.3), (15, 40, 0.3), (300, 100, 0.1), (120, 120, 0.05)])
def test_linear_step_against_dense_solve(m, n, density):
    r = G.rng_for(99, m + n)
    A = G.sprandn(m, n, density, r)
    b = r.standard_normal(m)
    c = r.standard_normal(n)
    lin = DirectLinSys(A, b, c)
    assert lin.delta >= 1.0
    IQ = np.eye(m + n + 1) + Q_dense(A, b, c)
    for _ in range(5):
        rhs = r.standard_normal(m + n + 1)
        x = lin.L(rhs)
        np.testing.assert_allclose(x, np.linalg.solve(IQ, rhs), rtol=1e-11, atol=1e-12)
        assert np.linalg.norm(IQ @ x - rhs) <= 1e-13 * np.linalg.norm(rhs) * np.linalg.norm(IQ, 2)


def test_linear_step_sparse_factor_path():
    r = G.rng_for(98, 0)
    A = G.sprandn(400, 300, 0.004, r)
    b = r.standard_normal(400)
    c = r.standard_normal(300)
    lin_s = DirectLinSys(A, b, c, dense_limit=0)
    assert lin_s.kind == "sparse"
    IQ = np.eye(701) + Q_dense(A, b, c)
    rhs = r.standard_normal(701)
    np.testing.assert_allclose(lin_s.L(rhs), np.linalg.solve(IQ, rhs), rtol=1e-10, atol=1e-11)


# ------------------------------------------------------------ T and R

def _lin_and_cone(seed=0):
    p = G.small_socp(seed)
    return p, DirectLinSys(p.A, p.b, p.c)


def T_op(lin, cone, u):
    ut, ub, Ru = S.residual(lin, cone, u)
    return u - Ru


def test_T_firmly_nonexpansive_and_homogeneous():
    p, lin = _lin_and_cone(1)
    r = np.random.default_rng(5)
    N = p.n + p.m + 1
    for _ in range(20):
        u, v = r.standard_normal(N), r.standard_normal(N)
        Tu, Tv = T_op(lin, p.cone, u), T_op(lin, p.cone, v)
        dT = Tu - Tv
        assert dT @ dT <= dT @ (u - v) + 1e-10 * (1 + (u - v) @ (u - v))
        np.testing.assert_allclose(T_op(lin, p.cone, 2 * u), 2 * Tu, rtol=1e-12, atol=1e-12)


def test_planted_fixed_point():
    p, lin = _lin_and_cone(2)
    u_star = np.concatenate([p.x_star, p.y_star + p.s_star, [1.0]])
    ut, ub, Ru = S.residual(lin, p.cone, u_star)
    assert np.linalg.norm(Ru) <= 1e-12 * np.linalg.norm(u_star)
    res = S.solve(p, S.Settings(eps=1e-9), u0=u_star, lin=lin)
    assert res.status == S.SOLVED and res.iters == 0
    np.testing.assert_allclose(res.x, p.x_star, atol=1e-9)


# ------------------------------------------------------------ directions

def test_restarted_broyden_matches_dense_sherman_morrison():
    # Product form of Algorithm 2 against the dense inverse update of Sec. IV-D-1:
    # H+ = H + (z - H xi~)(z^T H) / <H xi~, z>,  xi~ = (1 - theta) B z + theta xi.
    r = np.random.default_rng(8)
    N, mem, thb = 12, 4, 0.3
    rb = S.RestartedBroyden(mem, thb)
    H = np.eye(N)
    for it in range(9):
        z = r.standard_normal(N)
        xi = r.standard_normal(N) if it % 3 else 0.05 * r.standard_normal(N)   # small xi: Powell damping on
        res = r.standard_normal(N)
        if it and len(rb.Z) == 0:
            H = np.eye(N)
        B = np.linalg.inv(H)
        gamma = (H @ xi) @ z / (z @ z)
        theta = 1.0 if abs(gamma) >= thb else (1 - (1 if gamma >= 0 else -1) * thb) / (1 - gamma)
        xit = (1 - theta) * (B @ z) + theta * xi
        Hx = H @ xit
        H_new = H + np.outer(z - Hx, z @ H) / (Hx @ z)
        np.testing.assert_allclose(H_new @ xit, z, rtol=1e-9, atol=1e-9)         # secant condition
        assert abs(Hx @ z) >= thb * (z @ z) * (1 - 1e-9) or theta == 1.0           # Powell safeguard
        restart = len(rb.Z) == mem
        d = rb.direction(res, z, xi)
        np.testing.assert_allclose(d, -H_new @ res, rtol=1e-9, atol=1e-9)
        H = H_new
        if restart:
            # buffers now hold only the current factor (I + zt z^T)
            zt = rb.Zt[0]
            H = np.eye(N) + np.outer(zt, rb.Z[0])


def test_anderson_matches_lstsq():
    r = np.random.default_rng(9)
    N = 40
    aa = S.Anderson(5, reg=0.0)
    for _ in range(7):
        aa.push(r.standard_normal(N), r.standard_normal(N))
    res = r.standard_normal(N)
    t = aa.coefficients(res)
    Xi = np.stack(aa.Xi, axis=1)
    np.testing.assert_allclose(t, np.linalg.lstsq(Xi, res, rcond=None)[0], rtol=1e-9)
    Z = np.stack(aa.Z, axis=1)
    np.testing.assert_allclose(aa.direction(res), -res - (Z - Xi) @ t, rtol=1e-9)
    assert len(aa.Z) == 5                               # FIFO memory of the last pairs


# ------------------------------------------------------------ Algorithm 1 special cases

def test_zero_direction_is_plain_drs():
    # d = 0 and c0 = 0: every step is K2 at alpha = 1 with w = u, i.e. u+ = u - R u = T u.
    p, lin = _lin_and_cone(3)
    st = S.Settings(direction="zero", c0=0.0, lam=1.0, max_iters=25, eps=1e-14)
    res = S.solve(p, st, lin=lin)
    u = np.zeros(p.n + p.m + 1); u[-1] = 1.0
    for _ in range(25):
        ut = lin.L(u)
        u = u + C.proj_C(2 * ut - u, p.n, p.cone) - ut              # equation (drs)
    np.testing.assert_allclose(res.u, u, rtol=1e-12, atol=1e-13)
    assert res.counts["k2"] == 25


def rotation_instance(theta):
    """n = m = 1, A = [theta], b = c = 0, zero cone: (I + Q) acts on (x, y) as
    the complex scalar 1 - i theta (derivation in tests/golden/alg1_safeguards.json)."""
    return G.Problem(A=sp.csr_matrix(np.array([[theta]])), b=np.zeros(1), c=np.zeros(1), cone=G.Cone(z=1))


def test_alg1_safeguards_golden():
    """Step kinds, backtracks, ||R u||, eta and r_safe of the first seven
    iterations against the hand-derived closed forms: pins the K0 reset of eta,
    the r_safe update with q to the power nu, the K1/K2 tests, backtracking
    and the step at the backtracking cap (Algorithm 1)."""
    d = json.load(open(os.path.join(HERE, "golden", "alg1_safeguards.json")))
    for case in d["cases"]:
        st = S.Settings(direction="none", eps=1e-12, max_iters=len(case["kind"]), **case["settings"])
        res = S.solve(rotation_instance(case["theta"]), st, u0=np.array([1.0, 0.0, 1.0]))
        h = res.history
        assert res.status == S.MAX_ITERS and len(h) == len(case["kind"]), case["name"]
        assert [r["kind"] for r in h] == case["kind"], case["name"]
        assert [r["ls"] for r in h] == case["ls"], case["name"]
        for key in ("res", "eta", "r_safe"):
            np.testing.assert_allclose([r[key] for r in h], case[key], rtol=1e-12, err_msg=case["name"] + " " + key)


class _PowerIgnoringFloat(float):
    """A float whose powers are itself: q ** nu == q for every nu."""

    def __pow__(self, other):
        return float(self)


def test_alg1_safeguards_golden_detects_planted_mistakes():
    """The golden trace catches the misreadings it is meant to catch.  Planted
    in the oracle: q instead of q^nu in the r_safe update (the recorded r_safe
    then differs at nu = 0 and from nu = 3 on).  Checked on the fixture itself: with eta kept
    at eta0 instead of reset after a K0 step, the K0 test would already pass at
    nu = 3, where the derived trace takes a K1 step."""
    d = json.load(open(os.path.join(HERE, "golden", "alg1_safeguards.json")))
    case = d["cases"][0]
    kw = dict(case["settings"])
    kw["q"] = _PowerIgnoringFloat(kw["q"])
    st = S.Settings(direction="none", eps=1e-12, max_iters=len(case["kind"]), **kw)
    h = S.solve(rotation_instance(case["theta"]), st, u0=np.array([1.0, 0.0, 1.0])).history
    got = np.array([r["r_safe"] for r in h])
    assert np.allclose(got[1:3], case["r_safe"][1:3], rtol=1e-12)     # q^1 = q
    assert not np.isclose(got[0], case["r_safe"][0], rtol=1e-6)         # q^0 = 1
    assert not np.allclose(got[3:], case["r_safe"][3:], rtol=1e-6)
    assert case["kind"][3] == "K1" and case["res"][3] <= case["settings"]["c0"] * case["res"][0]


# ------------------------------------------------------------ whole solves

def test_closed_form_golden():
    d = json.load(open(os.path.join(HERE, "golden", "closed_form.json")))
    for key, v in d.items():
        if key.startswith("_"):
            continue
        p = _prob_from_json(v)
        for direction, mem in [("aa", 5), ("rb", 10)]:
            res = S.solve(p, S.Settings(eps=1e-9, direction=direction, mem=mem, max_iters=20000))
            assert res.status == S.SOLVED, (key, direction)
            np.testing.assert_allclose(res.x, v["x"], atol=1e-6)
            assert abs(res.info["pobj"] - v["pobj"]) <= 1e-7 * (1 + abs(v["pobj"]))
            if key != "eq_box":        # unique duals
                np.testing.assert_allclose(res.y, v["y"], atol=1e-6)


def _vertex_enumeration(p):
    A = p.A.toarray()
    m, n = A.shape
    best = math.inf
    for S_ in itertools.combinations(range(m), n):
        As = A[list(S_)]
        if abs(np.linalg.det(As)) < 1e-10:
            continue
        x = np.linalg.solve(As, p.b[list(S_)])
        if np.all(A @ x <= p.b + 1e-9):
            best = min(best, p.c @ x)
    return best


@pytest.mark.parametrize("seed", range(6))
def test_tiny_lp_vertex_enumeration(seed):
    p = G.tiny_lp(seed, n=3 + seed % 2, mg=5 + seed % 3)
    ref = _vertex_enumeration(p)
    res = S.solve(p, S.Settings(eps=1e-9, direction="aa", mem=5, max_iters=50000))
    assert res.status == S.SOLVED
    assert abs(res.info["pobj"] - ref) <= 1e-6 * (1 + abs(ref))


def _kkt_errors(p, x, y, s):
    from oracle.cones import proj_dual_cone
    A = p.A
    pr = np.linalg.norm(A @ x + s - p.b) / (1 + np.linalg.norm(p.b))
    dr = np.linalg.norm(A.T @ y + p.c) / (1 + np.linalg.norm(p.c))
    ydist = np.linalg.norm(y - proj_dual_cone(y, p.cone))
    # s in K: for cones without exp blocks K = K* up to the zero block (K = {0} there)
    return pr, dr, ydist


def test_config1_lp_planted():
    p = G.config1_lp()
    for st in [S.Settings(direction="rb", mem=10), S.Settings(direction="aa", mem=5)]:
        res = S.solve(p, st)
        assert res.status == S.SOLVED
        pstar = p.c @ p.x_star
        assert abs(res.info["pobj"] - pstar) <= 1e-5 * (1 + abs(pstar))
        pr, dr, ydist = _kkt_errors(p, res.x, res.y, res.s)
        assert pr <= 1e-6 and dr <= 1e-6 and ydist <= 1e-9
        assert np.all(res.s >= -1e-9)
        # x* unique: the active rows of the planted point have full column rank
        act = p.s_star < 1e-12
        assert np.linalg.matrix_rank(p.A.toarray()[act]) == p.n
        assert np.linalg.norm(res.x - p.x_star) <= 1e-3 * np.linalg.norm(p.x_star)


def test_small_socp_planted():
    p = G.small_socp(0)
    res = S.solve(p, S.Settings(direction="aa", mem=10, max_iters=5000))
    assert res.status == S.SOLVED
    pstar = p.c @ p.x_star
    assert abs(res.info["pobj"] - pstar) <= 1e-5 * (1 + abs(pstar))
    # s in K (zero rows are 0, R+ rows >= 0, SOC blocks inside)
    o = p.cone.z
    assert np.abs(res.s[:o]).max() <= 1e-6 * (1 + np.linalg.norm(p.b))
    assert res.s[o:o + p.cone.l].min() >= -1e-9
    o += p.cone.l
    for k in p.cone.q:
        blk = res.s[o:o + k]
        assert np.linalg.norm(blk[:-1]) <= blk[-1] + 1e-8
        o += k


@pytest.mark.parametrize("seed", range(3))
def test_infeasible_certificate(seed):
    p = G.infeasible_lp(seed)
    res = S.solve(p, S.Settings(eps=1e-7))
    assert res.status == S.INFEASIBLE
    y = res.y
    assert abs(p.b @ y + 1) <= 1e-10
    assert np.linalg.norm(p.A.T @ y) <= 1e-6 * np.linalg.norm(y) * np.linalg.norm(p.b) * 10
    assert y.min() >= -1e-12


@pytest.mark.parametrize("seed", range(3))
def test_unbounded_certificate(seed):
    p = G.unbounded_lp(seed)
    res = S.solve(p, S.Settings(eps=1e-7))
    assert res.status == S.UNBOUNDED
    x, s = res.x, res.s
    assert abs(p.c @ x + 1) <= 1e-10
    assert np.linalg.norm(p.A @ x + s) <= 1e-6 * np.linalg.norm(x) * np.linalg.norm(p.c) * 10
    assert s.min() >= -1e-12


def _planted_kkt_lp(seed, m=9, n=4):
    """LP min c'x, Ax + s = b, s >= 0 with a planted KKT point: y* and s*
    nonnegative with disjoint supports, b = A x* + s*, c = -A'y*; then the
    primal and dual residuals vanish and c'x* + b'y* = y*'s* = 0."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x = rng.standard_normal(n)
    y = np.zeros(m)
    s = np.zeros(m)
    act = rng.permutation(m)[: m // 2]
    y[act] = rng.uniform(0.5, 2.0, act.size)
    rest = np.setdiff1d(np.arange(m), act)
    s[rest] = rng.uniform(0.5, 2.0, rest.size)
    return DirectLinSys(A, A @ x + s, -A.T @ y), x, y, s


def _hsde_points(x, y, s, tau, ut_y):
    """(u, u~, u-bar) whose termination read-out is (x, y, s) scaled by tau:
    u-bar = (tau x, tau y, tau) and the slack tau s = y-bar - 2 u~_y + u_y
    (Sec. IV-C), for any choice of u~_y."""
    n, m = x.size, y.size
    ub = np.concatenate([tau * x, tau * y, [tau]])
    ut = np.concatenate([np.zeros(n), ut_y, [tau]])
    u = np.concatenate([np.zeros(n), tau * s - tau * y + 2.0 * ut_y, [tau]])
    return u, ut, ub


@pytest.mark.parametrize("tau", [1.0, 0.37, 12.5])
def test_termination_reads_out_planted_kkt_point(tau):
    """At a planted KKT point pr = dr = gap = 0 (up to rounding) for any
    tau > 0 (the read-out divides by tau), the status is SOLVED and
    (x, y, s) = (chi, psi, sigma) / tau."""
    lin, x, y, s = _planted_kkt_lp(3)
    ut_y = np.random.default_rng(4).standard_normal(y.size)
    u, ut, ub = _hsde_points(x, y, s, tau, ut_y)
    st, info, (xo, yo, so) = S.termination(lin, u, ut, ub, 1e-9)
    assert st == S.SOLVED
    assert max(info["pr"], info["dr"], info["gap"]) <= 1e-13
    np.testing.assert_allclose(xo, x, rtol=0, atol=1e-13)
    np.testing.assert_allclose(yo, y, rtol=0, atol=1e-13)
    np.testing.assert_allclose(so, s, rtol=0, atol=1e-13)
    assert info["pobj"] == pytest.approx(lin.c @ x, abs=1e-12)
    assert info["dobj"] == pytest.approx(-lin.b @ y, abs=1e-12)


def test_termination_residuals_of_known_perturbations():
    """Moving x* by delta along coordinate j leaves dr at 0 and makes
    pr = |delta| ||A e_j|| / (1 + ||b||) and the gap |delta c_j| over
    1 + |c'x| + |b'y|; moving y* by delta along an inactive row i makes
    dr = |delta| ||A' e_i|| / (1 + ||c||).  Neither reaches eps = 1e-6 here,
    so the status is 0 (continue)."""
    lin, x, y, s = _planted_kkt_lp(5)
    A = lin.A.toarray()
    b, c = lin.b, lin.c
    delta, j = 0.25, 2
    xp = x.copy(); xp[j] += delta
    st, info, _ = S.termination(lin, *_hsde_points(xp, y, s, 2.0, np.zeros(y.size)), 1e-6)
    assert st == 0
    assert info["pr"] == pytest.approx(abs(delta) * np.linalg.norm(A[:, j]) / (1 + np.linalg.norm(b)), rel=1e-12)
    assert info["dr"] <= 1e-14
    cx, by = c @ xp, b @ y
    assert info["gap"] == pytest.approx(abs(delta * c[j]) / (1 + abs(cx) + abs(by)), rel=1e-10)
    i = int(np.flatnonzero(y == 0)[0])
    yp = y.copy(); yp[i] += delta
    st, info, _ = S.termination(lin, *_hsde_points(x, yp, s, 1.0, np.zeros(y.size)), 1e-6)
    assert st == 0
    assert info["dr"] == pytest.approx(abs(delta) * np.linalg.norm(A[i]) / (1 + np.linalg.norm(c)), rel=1e-12)
    assert info["pr"] <= 1e-14


def test_termination_certificates_at_tau_zero():
    """tau = 0: a psi with A'psi = 0, psi >= 0 and b'psi < 0 is a certificate
    of primal infeasibility (ic = 0), returned as y = psi / (-b'psi); a chi
    with A chi + sigma = 0, sigma >= 0 and c'chi < 0 certifies unboundedness
    (uc = 0), returned as (x, s) = (chi, sigma) / (-c'chi)."""
    rng = np.random.default_rng(7)
    # infeasible: rows 0 and 1 are a'x + s0 = 1 and -a'x + s1 = -2 (sum: s0 + s1 = -1)
    a = rng.standard_normal(3)
    A = np.vstack([a, -a, rng.standard_normal((2, 3))])
    b = np.array([1.0, -2.0, 1.0, 1.0])
    lin = DirectLinSys(A, b, rng.standard_normal(3))
    psi = np.array([3.0, 3.0, 0.0, 0.0])
    ub = np.concatenate([np.zeros(3), psi, [0.0]])
    z = np.zeros(7)
    st, info, (xo, yo, so) = S.termination(lin, z, z, ub, 1e-8)
    assert st == S.INFEASIBLE
    assert info["ic"] <= 1e-15
    np.testing.assert_allclose(yo, psi / 3.0, rtol=0, atol=1e-15)
    assert lin.b @ yo == pytest.approx(-1.0, abs=1e-15)
    assert np.isnan(xo).all() and np.isnan(so).all()
    # unbounded: min -x0 with x0 free of every row: A chi = 0 for chi = e0
    A = np.hstack([np.zeros((4, 1)), rng.standard_normal((4, 2))])
    lin = DirectLinSys(A, rng.uniform(1, 2, 4), np.array([-2.0, 0.5, 0.5]))
    chi = np.array([1.5, 0.0, 0.0])
    ub = np.concatenate([chi, np.zeros(4), [0.0]])
    st, info, (xo, yo, so) = S.termination(lin, z, z, ub, 1e-8)
    assert st == S.UNBOUNDED
    assert info["uc"] <= 1e-15
    np.testing.assert_allclose(xo, chi / 3.0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(so, np.zeros(4), rtol=0, atol=1e-15)
    assert np.isnan(yo).all()


def _lasso_fista(Ad, bd, mu, iters=200000, tol=1e-13):
    A = Ad.toarray()
    L = np.linalg.norm(A, 2) ** 2
    x = np.zeros(A.shape[1]); yk = x.copy(); t = 1.0
    for _ in range(iters):
        g = A.T @ (A @ yk - bd)
        xn = yk - g / L
        xn = np.sign(xn) * np.maximum(np.abs(xn) - mu / L, 0)
        tn = (1 + math.sqrt(1 + 4 * t * t)) / 2
        yk = xn + ((t - 1) / tn) * (xn - x)
        if np.linalg.norm(xn - x) <= tol * (1 + np.linalg.norm(x)):
            x = xn
            break
        x, t = xn, tn
    return x, 0.5 * np.sum((A @ x - bd) ** 2) + mu * np.abs(x).sum()


@pytest.mark.parametrize("i", [0, 1])
def test_lasso_socp_matches_fista(i):
    p = G.config4_instance(i)
    Ad, bd, mu = p.meta["Ad"], p.meta["bd"], p.meta["mu"]
    _, fref = _lasso_fista(Ad, bd, mu)
    res = S.solve(p, S.Settings(eps=1e-8, direction="aa", mem=5, max_iters=20000))
    assert res.status == S.SOLVED
    n = p.meta["n_data"]
    x = res.x[:n]
    f = 0.5 * np.sum((Ad @ x - bd) ** 2) + mu * np.abs(x).sum()
    assert abs(f - fref) <= 1e-6 * (1 + abs(fref))
    assert abs(res.info["pobj"] - fref) <= 1e-6 * (1 + abs(fref))


def test_status_limits():
    p = G.config1_lp()
    res = S.solve(p, S.Settings(max_iters=1))
    assert res.status == S.MAX_ITERS
    res = S.solve(p, S.Settings(max_time=0.0))
    assert res.status == S.TIME_LIMIT
    bad = G.config1_lp()
    bad.b = bad.b.copy(); bad.b[0] = np.nan
    res = S.solve(bad, S.Settings(max_iters=5))
    assert res.status == S.NUMERICAL


# ------------------------------------------------------------ SCS's splitting

def test_scs_splitting_is_conjugate_to_drs():
    """DRS on N_C + Q and on Q + N_C are conjugate through the reflection
    R_L = 2 (I + Q)^{-1} - I (an isometry, Q being skew): with z0 = R_L u0, the
    relaxed iterates satisfy z^k = R_L u^k for every k, where u^k follows
    equation (drs) with relaxation (written out here step by step)."""
    p, lin = _lin_and_cone(4)
    lam = 1.3
    u = np.zeros(p.n + p.m + 1); u[-1] = 1.0
    u[:p.n] = np.random.default_rng(1).standard_normal(p.n) * 0.1
    z0 = 2.0 * lin.L(u) - u
    for k in (1, 7, 30):
        res = S.solve_scs(p, S.Settings(lam=lam, max_iters=k, eps=1e-14), z0=z0, lin=lin)
        uk = u.copy()
        for _ in range(k):
            ut = lin.L(uk)
            Tu = uk + C.proj_C(2 * ut - uk, p.n, p.cone) - ut          # equation (drs)
            uk = (1 - lam) * uk + lam * Tu                               # relaxed
        np.testing.assert_allclose(res.u, 2.0 * lin.L(uk) - uk, rtol=1e-10, atol=1e-12)


def test_scs_splitting_planted_fixed_point():
    """z* = u* - Q u* with u* = (x*, y*, 1) the planted optimum is a fixed
    point of SCS's splitting: R z* = 0 and the read-out returns (x*, y*, s*)."""
    p = G.config1_lp()
    lin = DirectLinSys(p.A, p.b, p.c)
    ustar = np.concatenate([p.x_star, p.y_star, [1.0]])
    zstar = ustar - Q_dense(p.A, p.b, p.c) @ ustar
    res = S.solve_scs(p, S.Settings(eps=1e-9), z0=zstar, lin=lin)
    assert res.status == S.SOLVED and res.iters == 0
    assert res.info["res_fp"] <= 1e-12 * np.linalg.norm(zstar)
    np.testing.assert_allclose(res.x, p.x_star, atol=1e-10)
    np.testing.assert_allclose(res.s, p.s_star, atol=1e-10)


@pytest.mark.parametrize("maker", ["lp", "socp"])
def test_scs_splitting_solves_planted_problems(maker):
    p = G.config1_lp() if maker == "lp" else G.small_socp(2)
    res = S.solve_scs(p, S.Settings(eps=1e-8, lam=1.5, max_iters=50000))
    assert res.status == S.SOLVED
    pstar = float(p.c @ p.x_star)
    assert abs(res.info["pobj"] - pstar) <= 1e-6 * (1 + abs(pstar))


@pytest.mark.parametrize("seed", [0, 1])
def test_scs_splitting_certificates(seed):
    r1 = S.solve_scs(G.infeasible_lp(seed), S.Settings(eps=1e-7, max_iters=50000))
    assert r1.status == S.INFEASIBLE
    r2 = S.solve_scs(G.unbounded_lp(seed), S.Settings(eps=1e-7, max_iters=50000))
    assert r2.status == S.UNBOUNDED


# ------------------------------------------------------------ Anderson by an updated QR

def test_anderson_qr_updates_keep_a_qr_factorisation():
    """After more pushes than the memory holds (drops by Givens rotations),
    Q stays orthonormal, Q R reproduces the stored Xi, R is upper triangular,
    and t equals numpy's least-squares solution."""
    r = np.random.default_rng(21)
    N = 40
    aa = S.AndersonQR(5)
    for _ in range(12):
        aa.push(r.standard_normal(N), r.standard_normal(N))
    Xi = np.stack(aa.Xi, axis=1)
    assert Xi.shape[1] == 5
    np.testing.assert_allclose(aa.Q.T @ aa.Q, np.eye(5), atol=1e-13)
    np.testing.assert_allclose(aa.Q @ aa.R, Xi, atol=1e-12 * np.abs(Xi).max())
    assert np.all(np.tril(aa.R, -1) == 0.0)
    res = r.standard_normal(N)
    np.testing.assert_allclose(aa.coefficients(res), np.linalg.lstsq(Xi, res, rcond=None)[0], rtol=1e-10)
    Z = np.stack(aa.Z, axis=1)
    t = aa.coefficients(res)
    np.testing.assert_allclose(aa.direction(res), -res - (Z - Xi) @ t, rtol=1e-12)


def test_anderson_qr_robust_where_normal_equations_lose_accuracy():
    """Xi with condition number ~1e7: the normal equations' t (cond ~1e14)
    loses most digits, the QR solution keeps the least-squares one."""
    r = np.random.default_rng(22)
    N, k = 60, 4
    U, _ = np.linalg.qr(r.standard_normal((N, k)))
    V, _ = np.linalg.qr(r.standard_normal((k, k)))
    Xi = U @ np.diag([1.0, 1e-2, 1e-5, 1e-7]) @ V.T
    qr, ne = S.AndersonQR(k), S.Anderson(k, reg=0.0)
    for j in range(k):
        z = r.standard_normal(N)
        qr.push(z, Xi[:, j])
        ne.push(z, Xi[:, j])
    res = Xi @ r.standard_normal(k) + 1e-3 * r.standard_normal(N)
    ref = np.linalg.lstsq(Xi, res, rcond=None)[0]
    e_qr = np.linalg.norm(qr.coefficients(res) - ref) / np.linalg.norm(ref)
    t_ne = ne.coefficients(res)
    e_ne = np.inf if t_ne is None else np.linalg.norm(t_ne - ref) / np.linalg.norm(ref)
    assert e_qr <= 1e-6
    assert e_ne > 100 * e_qr


def test_anderson_qr_solves_like_the_normal_equations():
    """Same problems, same answers: the QR form tracks the Gram form's
    trajectory closely at first (different rounding only) and both solve."""
    p = G.small_socp(2)
    lin = DirectLinSys(p.A, p.b, p.c)
    a = S.solve(p, S.Settings(direction="aa", mem=5, eps=1e-8), lin=lin)
    b = S.solve(p, S.Settings(direction="aa_qr", mem=5, eps=1e-8), lin=lin)
    assert a.status == b.status == S.SOLVED
    ra = np.array([h["res"] for h in a.history[:20]])
    rb = np.array([h["res"] for h in b.history[:20]])
    np.testing.assert_allclose(rb, ra, rtol=1e-7)
    assert abs(a.info["pobj"] - b.info["pobj"]) <= 1e-6 * (1 + abs(a.info["pobj"]))
