"""Pins of the oracle on the mixed PSD / exponential-cone instance (sparse PCA
blocks plus l1-regularised logistic regression), against what the two
subproblems fix independently of any cone programming:

* logistic part: the oracle's (w, beta) evaluated in the original objective
  sum_i log(1 + exp(-y_i (a_i^T w + beta))) + lam ||w||_1 is no better than
  the optimum found by L-BFGS-B on the smooth split form (w = w+ - w-,
  w+- >= 0), and within 1e-4 of it;
* sparse PCA blocks: each Z_b is PSD with unit trace (to the tolerance), and
  its value <S_b, Z_b> - lam ||Z_b||_1 is at least that of the best point a
  random-restart local search over Z = V V^T / ||V||_F^2 finds;
* the two parts are independent, so the cone program's optimal value is the
  sum of the two subproblem optima.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import superscs as S
from oracle.cones import smat
from paper_1903_06477_amd import generators as G


@pytest.fixture(scope="module")
def solved():
    p = G.small_sdp_exp(0)
    r = S.solve(p, S.Settings(direction="aa", mem=5, max_iters=20000))
    assert r.status == S.SOLVED
    return p, r


def _logistic(F, y, lam, w, beta):
    z = -y * (F @ w + beta)
    return float(np.sum(np.logaddexp(0.0, z)) + lam * np.sum(np.abs(w)))


def _logistic_opt(F, y, lam):
    p = F.shape[1]
    Fd = F.toarray()

    def f(v):
        wp, wm, beta = v[:p], v[p:2 * p], v[2 * p]
        w = wp - wm
        z = -y * (Fd @ w + beta)
        val = np.sum(np.logaddexp(0.0, z)) + lam * np.sum(wp + wm)
        sig = 1.0 / (1.0 + np.exp(-z))                  # d/dz log(1 + e^z)
        gz = -y * sig
        gw = Fd.T @ gz
        return val, np.concatenate([gw + lam, -gw + lam, [gz.sum()]])

    bounds = [(0, None)] * (2 * p) + [(None, None)]
    res = minimize(f, np.zeros(2 * p + 1), jac=True, method="L-BFGS-B", bounds=bounds,
                   options=dict(ftol=1e-15, gtol=1e-12, maxiter=20000))
    return res.fun


def test_logistic_part_matches_lbfgs(solved):
    p, r = solved
    o = p.meta["offsets"]
    F, y, lam = p.meta["F"], p.meta["labels"], p.meta["lam_log"]
    q, pf = F.shape
    w = r.x[o["w"]:o["w"] + pf]
    beta = r.x[o["beta"]]
    f_or = _logistic(F, y, lam, w, beta)
    f_star = _logistic_opt(F, y, lam)
    assert f_or >= f_star - 1e-7
    assert f_or - f_star <= 1e-4 * (1 + abs(f_star))
    # the epigraph variables carry the same value
    t = r.x[o["t"]:o["t"] + q]
    rr = r.x[o["r"]:o["r"] + pf]
    assert abs(t.sum() + lam * rr.sum() - f_or) <= 1e-4 * (1 + abs(f_or))


def _spca_value(S_, Z, lam):
    return float(np.sum(S_ * Z) - lam * np.sum(np.abs(Z)))


def test_spca_blocks_feasible_and_not_beaten(solved):
    p, r = solved
    lam = p.meta["lam_sdp"]
    orders = p.meta["orders"]
    o = p.meta["offsets"]
    off = o["Z"]
    rng = np.random.default_rng(11)
    for k in orders:
        D = k * (k + 1) // 2
        zs = r.x[off:off + D]
        cs = -p.c[off:off + D]                 # svec(S)
        Z, S_ = smat(zs, k), smat(cs, k)
        assert abs(np.trace(Z) - 1.0) <= 1e-5
        assert np.linalg.eigvalsh(Z).min() >= -1e-5
        val = _spca_value(S_, Z, lam)

        def negval(v):
            V = v.reshape(k, k)
            Zv = V @ V.T / max(np.sum(V * V), 1e-300)
            return -_spca_value(S_, Zv, lam)

        best = max(np.diag(S_) - lam)                   # Z = e_i e_i^T
        for _ in range(8):
            res = minimize(negval, rng.standard_normal(k * k), method="Powell",
                           options=dict(xtol=1e-10, ftol=1e-12, maxiter=20000))
            best = max(best, -res.fun)
        assert val >= best - 1e-4 * (1 + abs(best))
        off += D


def test_objective_is_sum_of_subproblem_optima(solved):
    p, r = solved
    F, y, lam = p.meta["F"], p.meta["labels"], p.meta["lam_log"]
    f_star = _logistic_opt(F, y, lam)
    o = p.meta["offsets"]
    off, spca = o["Z"], 0.0
    for k in p.meta["orders"]:
        D = k * (k + 1) // 2
        spca += _spca_value(smat(-p.c[off:off + D], k), smat(r.x[off:off + D], k), p.meta["lam_sdp"])
        off += D
    # pobj = <c, x> = -(sum of SPCA values) + logistic optimum (to the tolerance)
    assert abs(r.info["pobj"] - (f_star - spca)) <= 1e-4 * (1 + abs(r.info["pobj"]))
    assert math.isfinite(r.info["dobj"])


# ------------------------------------------------------------ benchmark families of Sec. V-B / V-D

def _svec_to_mat(v, d):
    import math
    M = np.zeros((d, d))
    jj, ii = np.triu_indices(d)
    sc = np.where(ii == jj, 1.0, 1.0 / math.sqrt(2.0))
    M[ii, jj] = v * sc
    M[jj, ii] = v * sc
    return M


def test_sdp_pca_family_instance_closed_form():
    """lam = 0: max tr(S Z) over tr Z = 1, Z PSD is the largest eigenvalue of
    S (closed form); lam > 0: the optimum lies between the value of the top
    eigenvector's rank-one Z and lam_max(S), and the returned Z is feasible."""
    from oracle import superscs as S
    p = G.sdp_pca_instance(6, 0.0, 1)
    r = S.solve(p, S.Settings(eps=1e-9, max_iters=50000))
    lmax = np.linalg.eigvalsh(p.meta["S"]).max()
    assert r.status == S.SOLVED and abs(-r.info["pobj"] - lmax) <= 1e-7 * (1 + lmax)
    d, lam = 8, 0.5
    p = G.sdp_pca_instance(d, lam, 2)
    r = S.solve(p, S.Settings(eps=1e-9, max_iters=50000))
    Smat = p.meta["S"]
    w, V = np.linalg.eigh(Smat)
    v = V[:, -1]
    lower = v @ Smat @ v - lam * np.abs(np.outer(v, v)).sum()
    val = -r.info["pobj"]
    assert r.status == S.SOLVED and lower - 1e-7 <= val <= w[-1] + 1e-7
    D = d * (d + 1) // 2
    Z = _svec_to_mat(r.x[:D], d)
    assert abs(np.trace(Z) - 1) <= 1e-7 and np.linalg.eigvalsh(Z).min() >= -1e-7
    assert abs((np.trace(Smat @ Z) - lam * np.abs(Z).sum()) - val) <= 1e-6


def test_logreg_family_instance_matches_smooth_minimiser():
    """The cone program's optimum equals the minimum of the l1-regularised
    logistic loss found by L-BFGS-B on the split form w = w+ - w-."""
    import scipy.optimize as so
    from oracle import superscs as S
    p = G.logreg_instance(10, 20, 1.0, 3)
    r = S.solve(p, S.Settings(eps=1e-9, max_iters=50000))
    F, y, lam = p.meta["F"].toarray(), p.meta["labels"], p.meta["lam"]
    k = F.shape[1]

    def f(z):
        wp, wm, beta = z[:k], z[k:2 * k], z[-1]
        mrg = -y * (F @ (wp - wm) + beta)
        val = lam * (wp.sum() + wm.sum()) + np.logaddexp(0.0, mrg).sum()
        sgm = 1.0 / (1.0 + np.exp(-mrg))
        g_w = F.T @ (-y * sgm)
        return val, np.concatenate([lam + g_w, lam - g_w, [np.sum(-y * sgm)]])

    bounds = [(0, None)] * (2 * k) + [(None, None)]
    res = so.minimize(f, np.zeros(2 * k + 1), jac=True, method="L-BFGS-B", bounds=bounds,
                      options=dict(ftol=1e-15, gtol=1e-12, maxiter=10000))
    assert r.status == S.SOLVED
    assert abs(r.info["pobj"] - res.fun) <= 1e-6 * (1 + abs(res.fun))
