"""Euclidean projections onto the cones of Sec. II and their duals (FP64).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Cone definitions (Sec. II, "a few examples of convex cones"):
  zero cone {0}^n, its dual is R^n;
  nonnegative orthant R+^n (self-dual);
  second-order cone {(x, t) : ||x||_2 <= t}, t is the LAST coordinate (self-dual);
  PSD cone on R^{k(k+1)/2} through the paper's mat operator (self-dual);
  exponential cone cl{(x1, x2, x3) : x1 >= x2 exp(x3/x2), x2 > 0}, not self-dual.
Dual cone: Sec. II.  The projection of Sec. IV-A onto C = R^n x K* x R+ needs
projections onto K*, assembled block by block here.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.optimize


# ---------------------------------------------------------------- zero / R+ / SOC

def proj_zero_dual(v):
    """Dual of the zero cone is the whole space: identity."""
    return np.array(v, dtype=np.float64, copy=True)


def proj_nonneg(v):
    return np.maximum(np.asarray(v, dtype=np.float64), 0.0)


def proj_soc(v):
    """Second-order cone {(x, t): ||x|| <= t}, t last (Sec. II (iii))."""
    v = np.asarray(v, dtype=np.float64)
    x, t = v[:-1], v[-1]
    nx = float(np.linalg.norm(x))
    if nx <= t:
        return v.copy()
    if nx <= -t:
        return np.zeros_like(v)
    a = 0.5 * (nx + t)
    out = np.empty_like(v)
    out[:-1] = (a / nx) * x
    out[-1] = a
    return out


# ---------------------------------------------------------------- PSD

def smat(x, k):
    """The paper's mat: diagonal entries are taken as they are, off-diagonal
    entries are divided by sqrt(2); column-major lower triangle (Sec. II (ii))."""
    x = np.asarray(x, dtype=np.float64)
    assert x.size == k * (k + 1) // 2
    M = np.zeros((k, k))
    o = 0
    for j in range(k):
        for i in range(j, k):
            if i == j:
                M[i, j] = x[o]
            else:
                M[i, j] = x[o] / math.sqrt(2.0)
                M[j, i] = M[i, j]
            o += 1
    return M


def svec(M):
    """Inverse of smat."""
    k = M.shape[0]
    out = np.empty(k * (k + 1) // 2)
    o = 0
    for j in range(k):
        for i in range(j, k):
            out[o] = M[i, j] if i == j else math.sqrt(2.0) * M[i, j]
            o += 1
    return out


def psd_order(rows):
    k = int(round((math.sqrt(8 * rows + 1) - 1) / 2))
    assert k * (k + 1) // 2 == rows
    return k


def proj_psd(x, k=None):
    """Projection on the PSD cone: eigendecomposition, negative eigenvalues
    set to zero (Sec. II (ii), read as positive SEMIdefinite)."""
    x = np.asarray(x, dtype=np.float64)
    if k is None:
        k = psd_order(x.size)
    M = smat(x, k)
    lam, V = np.linalg.eigh(M)
    return svec((V * np.maximum(lam, 0.0)) @ V.T)


# ---------------------------------------------------------------- exponential cone

def in_exp(v, tol=0.0):
    t, s, r = v
    if s > 0:
        if r / s > 700.0:                    # s e^(r/s) beyond the FP64 range: not in K_e
            return False
        return t - s * math.exp(r / s) >= -tol * max(1.0, abs(t))
    return s >= -tol and t >= -tol and r <= tol


def in_exp_dual(y, tol=0.0):
    """K_e* = {y3 < 0, -y3 exp(y2/y3) <= e y1} U {y3 = 0, y1 >= 0, y2 >= 0}
    (derived from the definition of the dual cone in Sec. II)."""
    y1, y2, y3 = y
    if y3 < 0:
        if y2 / y3 > 700.0:                  # -y3 e^(y2/y3) beyond the FP64 range: not in K_e*
            return False
        return -y3 * math.exp(y2 / y3) - math.e * y1 <= tol * max(1.0, abs(y1))
    return y3 <= tol and y1 >= -tol and y2 >= -tol


def _exp_root_fn(t0, s0, r0):
    # At the projection p = s (e^rho, 1, rho) (boundary ray with ratio
    # rho = x3/x2) and v0 - p is a nonnegative multiple of the outward normal
    # (-1, e^rho (1 - rho), e^rho).  Eliminating the two multipliers leaves one
    # equation in rho (Friberg 2021, "Projection onto the exponential cone: a
    # univariate root-finding problem"), restated here in this ordering:
    #   h(rho) = ((rho-1) r0 + s0) e^rho - (r0 - rho s0) e^-rho - (rho^2 - rho + 1) t0.
    # It is evaluated times e^-|rho|, which keeps its sign and cannot overflow.
    def h(rho):
        q = rho * (rho - 1.0) + 1.0
        if rho >= 0:
            return ((rho - 1.0) * r0 + s0) - (r0 - rho * s0) * math.exp(-2.0 * rho) \
                - q * t0 * math.exp(-rho)
        return ((rho - 1.0) * r0 + s0) * math.exp(2.0 * rho) - (r0 - rho * s0) \
            - q * t0 * math.exp(rho)
    return h


def proj_exp(v):
    """Euclidean projection onto K_e (Sec. II (v)) by case analysis plus a
    one-dimensional root solve for the boundary case."""
    v = np.asarray(v, dtype=np.float64)
    t0, s0, r0 = float(v[0]), float(v[1]), float(v[2])
    # case 1: already in the cone (points within rounding of the boundary count)
    if in_exp((t0, s0, r0)):
        return v.copy()
    if s0 > 0:
        g = s0 * math.exp(r0 / s0) if r0 / s0 < 700 else math.inf
        if t0 - g >= -4.0 * np.finfo(float).eps * max(abs(t0), g):
            return v.copy()
    # case 2: in the polar cone -K_e*, projection is 0
    if in_exp_dual((-t0, -s0, -r0)):
        return np.zeros(3)
    # case 3: x2 <= 0 and x3 <= 0: nearest point of the face {x2 = 0, x1 >= 0, x3 <= 0}
    if r0 <= 0 and s0 <= 0:
        return np.array([max(t0, 0.0), 0.0, r0])
    # case 4: boundary point with x2 > 0 and a strictly positive normal multiplier;
    # both multipliers positive confine rho to an interval (h < 0 left, > 0 right)
    if s0 > 0 and r0 > 0:
        lo, hi = 1.0 - s0 / r0, r0 / s0
    elif s0 > 0:
        lo, hi = -math.inf, r0 / s0
    else:
        lo, hi = 1.0 - s0 / r0, math.inf
    h = _exp_root_fn(t0, s0, r0)
    if math.isinf(lo):
        step = 1.0
        lo = hi - step
        while h(lo) > 0 and step < 1e12:
            step *= 2.0
            lo = hi - step
    if math.isinf(hi):
        step = 1.0
        hi = lo + step
        while h(hi) < 0 and step < 1e12:
            step *= 2.0
            hi = lo + step
    a, b = lo, hi
    if h(a) > 0 or h(b) < 0:
        # fall back to a scan: the sign change must lie inside the open interval
        grid = np.linspace(a, b, 20001)[1:-1]
        vals = np.array([h(g) for g in grid])
        idx = np.nonzero(np.diff(np.sign(vals)) != 0)[0]
        if idx.size:
            a, b = grid[idx[0]], grid[idx[0] + 1]
        else:                      # root within rounding of an end of the interval
            a = b = a if abs(h(a)) < abs(h(b)) else b
    if a == b:
        rho = a
    else:
        rho = scipy.optimize.brentq(h, a, b, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
    # Two equivalent ways to recover the point from rho: the primal one,
    # p = s (e^rho, 1, rho) with s = (s0 + (rho - 1) r0) / (rho^2 - rho + 1), and
    # the dual one, p = v0 - beta n with beta e^rho = (r0 - rho s0) / (rho^2 - rho + 1).
    # Take the one whose forward rounding error is smaller (the other loses
    # digits to cancellation near an end of the interval).
    qq = rho * rho - rho + 1.0
    num_p = s0 + (rho - 1.0) * r0
    num_d = r0 - rho * s0
    eps = np.finfo(float).eps
    na = math.sqrt(1.0 + rho * rho + (math.exp(2.0 * rho) if rho < 350 else math.inf))
    err_p = eps * (abs(s0) + abs((rho - 1.0) * r0)) / qq * na
    nn_scaled = math.sqrt((math.exp(-2.0 * rho) if rho > -350 else math.inf)
                          + 1.0 + (1.0 - rho) ** 2)          # e^-rho * ||n||
    err_d = eps * (abs(r0) + abs(rho * s0)) / qq * nn_scaled + eps * float(np.abs(v).max())
    if err_p <= err_d:
        sc = num_p / qq
        x1 = math.exp(math.log(sc) + rho) if sc > 0 else 0.0
        pt = np.array([x1, sc, sc * rho])
    else:
        bexp = num_d / qq                              # beta e^rho
        beta = bexp * math.exp(-rho)
        pt = v - np.array([-beta, bexp * (1.0 - rho), bexp])
    cand = [pt,
            np.array([max(t0, 0.0), 0.0, min(r0, 0.0)]),
            np.zeros(3)]
    best = min(cand, key=lambda p: float(np.linalg.norm(p - v)))
    return best


def proj_exp_dual(v):
    """Moreau: v = Pi_{K*}(v) + Pi_{-K}(v) and Pi_{-K}(v) = -Pi_K(-v)."""
    v = np.asarray(v, dtype=np.float64)
    return v + proj_exp(-v)


# ---------------------------------------------------------------- whole cones

def proj_dual_cone(y, cone):
    """Projection on K* block by block, rows ordered zero | R+ | SOC | PSD | exp."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    o = 0
    out[o:o + cone.z] = proj_zero_dual(y[o:o + cone.z])
    o += cone.z
    out[o:o + cone.l] = proj_nonneg(y[o:o + cone.l])
    o += cone.l
    for k in cone.q:
        out[o:o + k] = proj_soc(y[o:o + k])
        o += k
    for k in cone.s:
        r = k * (k + 1) // 2
        out[o:o + r] = proj_psd(y[o:o + r], k)
        o += r
    for _ in range(cone.ep):
        out[o:o + 3] = proj_exp_dual(y[o:o + 3])
        o += 3
    assert o == y.size
    return out


def proj_C(w, n, cone):
    """Pi_C for C = R^n x K* x R+ (Sec. III-A, definition of C)."""
    w = np.asarray(w, dtype=np.float64)
    out = np.empty_like(w)
    out[:n] = w[:n]
    out[n:-1] = proj_dual_cone(w[n:-1], cone)
    out[-1] = max(w[-1], 0.0)
    return out
