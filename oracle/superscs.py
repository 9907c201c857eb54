"""SuperSCS, Algorithm 1 of the paper, in plain FP64 NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sources in the paper:
  * DRS on Q + N_C, equation (drs), Sec. IV-A; T and R = I - T, Sec. IV-A/B.
  * SuperMann steps K0/K1/K2 with backtracking, Algorithm 1, Sec. IV-B.
  * Linearity trick for the line search (w~ = u~ + alpha d~), Sec. IV-B.
  * Termination (pr, dr, gap, ic, uc), Sec. IV-C.
  * Restarted Broyden directions, Sec. IV-D-1 and Algorithm 2.
  * Anderson's acceleration, Sec. IV-D-2.
  * SCS's splitting (DRS on N_C + Q), Sec. IV-A: solve_scs.
Readings of silent or garbled points (each named where it is used):
  R1 cold start u0 = (0, 0, 1).           R2 w = u + d in a K0 step.
  R3 backtracking capped at ls_max, then the KM step u - lambda R u.
  R4 q^nu is q to the power of the iteration counter.
  R5 the (z, xi) pair used at iteration nu comes from iteration nu-1's last
     trial point w; none at nu = 0; no push when z = 0.
  R6 Algorithm 2's denominator <s^i, H xi~^i> read as <z^i, H xi~^i>.
  R7 Algorithm 2's restart: clear the buffers, then store the current pair.
  R8 Anderson: FIFO memory of the last mem pairs; t from the regularised
     normal equations (Xi^T Xi + mu I) t = Xi^T R u with
     mu = 1e-12 tr(Xi^T Xi) / k; a non-finite t gives d = -R u.
  R9 ic and uc divided by -<b, y> and -<c, x> so both are nonnegative.
  R10 returned triplet is the barred one; certificates normalised to
      <b, y> = -1 and <c, x> = -1.  R11 Euclidean norms throughout.
  R12 precedence: SOLVED, then INFEASIBLE, then UNBOUNDED.
  R27 SCS's splitting (solve_scs): the candidate's s is psi-bar - z_psi.
  R17 c0, c1, q, sigma, lambda are inputs of Algorithm 1 without values in the
      paper except c0 = 0.1 for restarted Broyden (Sec. IV-D-1); defaults
      c0 0.99 (0.1 for RB), c1 0.9999, q 0.999, sigma 0.01, lambda 1.5.
"""
from __future__ import annotations

import dataclasses
import math
import time
from typing import List, Optional

import numpy as np

from .cones import proj_C
from .linsys import DirectLinSys

SOLVED, INFEASIBLE, UNBOUNDED, MAX_ITERS, TIME_LIMIT, NUMERICAL = 1, 2, 3, 4, 5, 6
STATUS_NAMES = {1: "solved", 2: "infeasible", 3: "unbounded", 4: "max_iters",
                5: "time_limit", 6: "numerical"}


@dataclasses.dataclass
class Settings:
    eps: float = 1e-6
    direction: str = "aa"          # "rb" (Algorithm 2), "aa" (Anderson, normal equations), "aa_qr"
                                   # (Anderson, updated QR), "none" (d = -Ru), "zero" (d = 0)
    mem: int = 5
    c0: Optional[float] = None     # default 0.1 for RB (Sec. IV-D-1), 0.99 for AA
    c1: float = 0.9999             # c1, q, lam: reading R17 (the paper leaves them open); with
    q: float = 0.999               # c1 = q = 0.99 and lam = 1 Anderson stalls in K2 steps and
    sigma: float = 0.01            # restarted Broyden in backtracking-cap steps on some SOCPs
    lam: float = 1.5
    thetabar: float = 0.1
    ls_max: int = 10
    max_iters: int = 10000
    max_time: float = math.inf
    aa_reg: float = 1e-12

    def c0_value(self) -> float:
        if self.c0 is not None:
            return self.c0
        return 0.1 if self.direction == "rb" else 0.99


# ----------------------------------------------------------------------------
# Directions
# ----------------------------------------------------------------------------

class RestartedBroyden:
    """Algorithm 2 (modified restarted Broyden), products of rank-one factors:
    H = (I + zt_m z_m^T) ... (I + zt_1 z_1^T), H_0 = I."""

    def __init__(self, mem: int, thetabar: float):
        self.mem = mem
        self.thetabar = thetabar
        self.Z: List[np.ndarray] = []
        self.Zt: List[np.ndarray] = []

    def apply(self, v):
        v = v.copy()
        for zi, zti in zip(self.Z, self.Zt):
            v = v + float(zi @ v) * zti
        return v

    def direction(self, r, z=None, xi=None):
        if z is None:
            return -self.apply(r)
        d = -r.copy()
        zt = xi.copy()
        for zi, zti in zip(self.Z, self.Zt):
            zt = zt + float(zi @ zt) * zti
            d = d + float(zi @ d) * zti
        gamma = float(zt @ z) / float(z @ z)
        if abs(gamma) >= self.thetabar:
            theta = 1.0
        else:
            sgn = 1.0 if gamma >= 0 else -1.0          # sgn(0) = 1
            theta = (1.0 - sgn * self.thetabar) / (1.0 - gamma)
        zt = (1.0 - theta) * z + theta * zt               # H xi~
        zt = (z - zt) / float(z @ zt)                     # new auxiliary vector (R6)
        d = d + float(z @ d) * zt
        if len(self.Z) == self.mem:                       # restart (R7)
            self.Z, self.Zt = [z.copy()], [zt]
        else:
            self.Z.append(z.copy())
            self.Zt.append(zt)
        return d


class Anderson:
    """Anderson's acceleration (Sec. IV-D-2): d = -Ru - (Z - Xi) t with t the
    least-squares solution of Xi t = Ru (normal equations, reading R8)."""

    def __init__(self, mem: int, reg: float = 1e-12):
        self.mem = mem
        self.reg = reg
        self.Z: List[np.ndarray] = []
        self.Xi: List[np.ndarray] = []

    def push(self, z, xi):
        self.Z.append(z.copy())
        self.Xi.append(xi.copy())
        if len(self.Z) > self.mem:
            self.Z.pop(0)
            self.Xi.pop(0)

    def coefficients(self, r):
        Xi = np.stack(self.Xi, axis=1)
        G = Xi.T @ Xi
        k = G.shape[0]
        mu = self.reg * float(np.trace(G)) / k
        with np.errstate(all="ignore"):
            try:
                t = np.linalg.solve(G + mu * np.eye(k), Xi.T @ r)
            except np.linalg.LinAlgError:
                return None
        if not np.all(np.isfinite(t)):
            return None
        return t

    def direction(self, r):
        if not self.Z:
            return -r.copy()
        t = self.coefficients(r)
        if t is None:
            return -r.copy()
        Z = np.stack(self.Z, axis=1)
        Xi = np.stack(self.Xi, axis=1)
        return -r - (Z - Xi) @ t


class AndersonQR:
    """Anderson's acceleration with t from a QR factorisation of Xi that is
    updated at every iteration (Sec. IV-D-2, the paper's alternative to the
    normal equations): Xi = Q R with orthonormal Q (N x k) and upper
    triangular R, columns oldest first.  A new pair appends a column by
    classical Gram-Schmidt with one re-orthogonalisation; when the memory is
    full the oldest column is dropped first and R's Hessenberg remainder is
    restored to triangular form by Givens rotations, applied to Q's columns
    alike.  t = R^{-1} Q^T R u; a non-finite t or a zero diagonal gives
    d = -R u."""

    def __init__(self, mem: int):
        self.mem = mem
        self.Z: List[np.ndarray] = []
        self.Xi: List[np.ndarray] = []
        self.Q = None                 # N x k
        self.R = None                 # k x k

    def _drop_oldest(self):
        self.Z.pop(0)
        self.Xi.pop(0)
        H = self.R[:, 1:].copy()      # k x (k-1), upper Hessenberg
        Q = self.Q.copy()
        k = H.shape[0]
        for i in range(k - 1):
            a, b = H[i, i], H[i + 1, i]
            r = math.hypot(a, b)
            c, s = (1.0, 0.0) if r == 0.0 else (a / r, b / r)
            Hi, Hj = H[i, :].copy(), H[i + 1, :].copy()
            H[i, :], H[i + 1, :] = c * Hi + s * Hj, -s * Hi + c * Hj
            H[i + 1, i] = 0.0                   # annihilated by construction
            Qi, Qj = Q[:, i].copy(), Q[:, i + 1].copy()
            Q[:, i], Q[:, i + 1] = c * Qi + s * Qj, -s * Qi + c * Qj
        self.R = H[:k - 1, :]
        self.Q = Q[:, :k - 1]

    def push(self, z, xi):
        if len(self.Z) == self.mem:
            self._drop_oldest()
        self.Z.append(z.copy())
        self.Xi.append(xi.copy())
        if self.Q is None or self.Q.shape[1] == 0:
            r = float(np.linalg.norm(xi))
            if not (r > 0.0):                   # a zero xi: not stored
                self.Z.pop()
                self.Xi.pop()
                return
            self.Q = (xi / r).reshape(-1, 1)
            self.R = np.array([[r]])
            return
        c1 = self.Q.T @ xi
        q = xi - self.Q @ c1
        c2 = self.Q.T @ q                       # re-orthogonalisation
        q = q - self.Q @ c2
        r = float(np.linalg.norm(q))
        if not (r > 1e-14 * float(np.linalg.norm(xi))):   # xi in the span of the memory: not stored
            self.Z.pop()
            self.Xi.pop()
            return
        k = self.R.shape[0]
        R = np.zeros((k + 1, k + 1))
        R[:k, :k] = self.R
        R[:k, k] = c1 + c2
        R[k, k] = r
        self.R = R
        self.Q = np.concatenate([self.Q, (q / r).reshape(-1, 1)], axis=1)

    def coefficients(self, r):
        with np.errstate(all="ignore"):
            rhs = self.Q.T @ r
            k = rhs.size
            t = np.zeros(k)
            for i in range(k - 1, -1, -1):             # back substitution
                t[i] = (rhs[i] - self.R[i, i + 1:] @ t[i + 1:]) / self.R[i, i]
        if not np.all(np.isfinite(t)):
            return None
        return t

    def direction(self, r):
        if not self.Z:
            return -r.copy()
        t = self.coefficients(r)
        if t is None:
            return -r.copy()
        Z = np.stack(self.Z, axis=1)
        Xi = np.stack(self.Xi, axis=1)
        return -r - (Z - Xi) @ t


# ----------------------------------------------------------------------------
# T-oracle and termination
# ----------------------------------------------------------------------------

def residual(lin: DirectLinSys, cone, u):
    """(u~, u-bar, R u) with u~ = (I+Q)^{-1} u, u-bar = Pi_C(2u~ - u) and
    R u = u~ - u-bar (equation (drs) and R = I - T, Sec. IV-A/B)."""
    ut = lin.L(u)
    ub = proj_C(2.0 * ut - u, lin.n, cone)
    return ut, ub, ut - ub


def termination(lin: DirectLinSys, u, ut, ub, eps):
    """Sec. IV-C.  Returns (status or 0, info dict, (x, y, s))."""
    n, m = lin.n, lin.m
    A, b, c = lin.A, lin.b, lin.c
    chi, psi, tau = ub[:n], ub[n:n + m], ub[-1]
    sig = psi - 2.0 * ut[n:n + m] + u[n:n + m]
    Ax_s = A @ chi + sig
    Aty = lin.At @ psi
    cx = float(c @ chi)
    by = float(b @ psi)
    nb = float(np.linalg.norm(b))
    nc = float(np.linalg.norm(c))
    info = dict(pr=math.inf, dr=math.inf, gap=math.inf, ic=math.inf, uc=math.inf,
                pobj=math.nan, dobj=math.nan, tau=float(tau))
    if tau > 0:
        info["pr"] = float(np.linalg.norm(Ax_s - b * tau)) / tau / (1.0 + nb)
        info["dr"] = float(np.linalg.norm(Aty + c * tau)) / tau / (1.0 + nc)
        info["gap"] = abs(cx + by) / tau / (1.0 + abs(cx) / tau + abs(by) / tau)
        info["pobj"] = cx / tau
        info["dobj"] = -by / tau
    if by < 0:
        info["ic"] = nb * float(np.linalg.norm(Aty)) / (-by)
    if cx < 0:
        info["uc"] = nc * float(np.linalg.norm(Ax_s)) / (-cx)
    if tau > 0 and info["pr"] <= eps and info["dr"] <= eps and info["gap"] <= eps:
        return SOLVED, info, (chi / tau, psi / tau, sig / tau)
    if info["ic"] < eps:
        nanx = np.full(n, np.nan)
        return INFEASIBLE, info, (nanx, psi / (-by), np.full(m, np.nan))
    if info["uc"] < eps:
        return UNBOUNDED, info, (chi / (-cx), np.full(m, np.nan), sig / (-cx))
    if tau > 0:
        return 0, info, (chi / tau, psi / tau, sig / tau)
    return 0, info, (np.full(n, np.nan), np.full(m, np.nan), np.full(m, np.nan))


# ----------------------------------------------------------------------------
# Algorithm 1
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Result:
    status: int
    x: np.ndarray
    y: np.ndarray
    s: np.ndarray
    iters: int
    info: dict
    history: list
    counts: dict
    u: np.ndarray
    setup_s: float = 0.0
    solve_s: float = 0.0

    @property
    def status_name(self):
        return STATUS_NAMES.get(self.status, "?")


def solve(prob, settings: Settings = Settings(), u0=None, lin: DirectLinSys = None,
          record: bool = True) -> Result:
    """Algorithm 1 with the directions of Sec. IV-D."""
    t_setup = time.perf_counter()
    A, b, c, cone = prob.A, prob.b, prob.c, prob.cone
    m, n = A.shape
    assert cone.rows() == m, "cone sizes must add up to the number of rows"
    if lin is None:
        lin = DirectLinSys(A, b, c)
    setup_s = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    st = settings
    c0 = st.c0_value()
    u = np.zeros(n + m + 1)
    u[-1] = 1.0                                            # R1
    if u0 is not None:
        u = np.asarray(u0, dtype=np.float64).copy()
    rb = RestartedBroyden(st.mem, st.thetabar) if st.direction == "rb" else None
    aa = (Anderson(st.mem, st.aa_reg) if st.direction == "aa"
          else AndersonQR(st.mem) if st.direction == "aa_qr" else None)
    counts = dict(k0=0, k1=0, k2=0, km=0, backtracks=0)
    history = []
    eta0 = eta = r_safe = None
    pend = None            # (z, Rw or None [= next R u], Ru_prev)
    status, info, xys = 0, {}, None
    nu = 0
    for nu in range(st.max_iters + 1):
        ut, ub, Ru = residual(lin, cone, u)                 # fresh solve every iteration
        nRu = float(np.linalg.norm(Ru))
        if nu == 0:
            eta0 = eta = r_safe = nRu
        status, info, xys = termination(lin, u, ut, ub, st.eps)
        info["res_fp"] = nRu
        if not math.isfinite(nRu):
            status = NUMERICAL
        if status:
            break
        if nu == st.max_iters:
            status = MAX_ITERS
            break
        if time.perf_counter() - t0 > st.max_time:
            status = TIME_LIMIT
            break
        # memory push of the previous pair (R5), then the direction
        z = xi = None
        if pend is not None:
            zp, Rwp, Rup = pend
            if float(np.linalg.norm(zp)) > 0:
                z = zp
                xi = (Ru if Rwp is None else Rwp) - Rup
        if rb is not None:
            d = rb.direction(Ru, z, xi)
        elif aa is not None:
            if z is not None:
                aa.push(z, xi)
            d = aa.direction(Ru)
        elif st.direction == "zero":
            d = np.zeros_like(Ru)
        else:
            d = -Ru
        rec = dict(nu=nu, res=nRu, pr=info["pr"], dr=info["dr"], gap=info["gap"],
                   d_ratio=float(np.linalg.norm(d)) / nRu if nRu > 0 else 0.0)
        if nRu <= c0 * eta:                                  # K0
            u_new = u + d
            eta = nRu
            pend = (d.copy(), None, Ru)                      # R2: w = u + d
            counts["k0"] += 1
            rec.update(kind="K0", ls=0)
        else:
            dt = lin.L(d)                                    # second linear solve
            alpha = 1.0
            done = False
            for k in range(st.ls_max):
                w = u + alpha * d
                wt = ut + alpha * dt                         # linearity of (I+Q)^{-1}
                Rw = wt - proj_C(2.0 * wt - w, n, cone)
                nRw = float(np.linalg.norm(Rw))
                rho = float(Rw @ (u - (w - Rw)))             # <Rw, u - Tw>
                if nRu <= r_safe and nRw <= st.c1 * nRu:     # K1
                    u_new = w
                    r_safe = nRw + st.q ** nu * eta0         # R4
                    counts["k1"] += 1
                    rec.update(kind="K1", ls=k)
                    done = True
                elif rho >= st.sigma * nRu * nRw:            # K2
                    u_new = u - st.lam * (rho / (nRw * nRw)) * Rw
                    counts["k2"] += 1
                    rec.update(kind="K2", ls=k)
                    done = True
                if done:
                    pend = (w - u, Rw, Ru)
                    break
                alpha *= 0.5
                counts["backtracks"] += 1
            if not done:                                     # R3
                u_new = u - st.lam * Ru
                pend = (np.zeros_like(u), Ru, Ru)
                counts["km"] += 1
                rec.update(kind="KM", ls=st.ls_max)
        if record:
            rec.update(eta=eta, r_safe=r_safe)               # safeguards after the step
            history.append(rec)
        u = u_new
    x, y, s = xys
    return Result(status=status, x=x, y=y, s=s, iters=nu, info=info, history=history,
                  counts=counts, u=u, setup_s=setup_s, solve_s=time.perf_counter() - t0)


# ----------------------------------------------------------------------------
# SCS's splitting
# ----------------------------------------------------------------------------

def solve_scs(prob, settings: Settings = Settings(), z0=None, lin: DirectLinSys = None,
              record: bool = True) -> Result:
    """SCS as the paper describes it (Sec. IV-A, "SCS and DRS"): Douglas-
    Rachford splitting on N_C + Q, the reverse order of (drs), relaxed by
    lambda (equation (km-updates) applied to that splitting's operator):
        u-bar = Pi_C(z),   u~ = (I + Q)^{-1}(2 u-bar - z),
        R z = u-bar - u~,  z+ = z - lambda R z.
    No SuperMann steps.  Termination (Sec. IV-C) on the candidate u-bar =
    (chi, psi, tau)-bar with sigma-bar = psi-bar - z_psi: at a fixed point
    u~ = u-bar, so (I + Q) u-bar = 2 u-bar - z and u-bar - z = Q u-bar, whose
    psi part is b tau - A chi (reading R27).  Cold start z0 = (0, 0, 1)."""
    t_setup = time.perf_counter()
    A, cone = prob.A, prob.cone
    m, n = A.shape
    assert cone.rows() == m, "cone sizes must add up to the number of rows"
    if lin is None:
        lin = DirectLinSys(A, prob.b, prob.c)
    setup_s = time.perf_counter() - t_setup
    t0 = time.perf_counter()
    st = settings
    z = np.zeros(n + m + 1)
    z[-1] = 1.0
    if z0 is not None:
        z = np.asarray(z0, dtype=np.float64).copy()
    history = []
    status, info, xys = 0, {}, None
    nu = 0
    for nu in range(st.max_iters + 1):
        ub = proj_C(z, n, cone)
        ut = lin.L(2.0 * ub - z)
        Rz = ub - ut
        nRz = float(np.linalg.norm(Rz))
        # termination with sigma-bar = psi-bar - z_psi: the paper's read-out
        # psi-bar - 2 psi~ + psi evaluated with psi~ = psi = z_psi
        status, info, xys = termination(lin, z, z, ub, st.eps)
        info["res_fp"] = nRz
        if not math.isfinite(nRz):
            status = NUMERICAL
        if status:
            break
        if nu == st.max_iters:
            status = MAX_ITERS
            break
        if time.perf_counter() - t0 > st.max_time:
            status = TIME_LIMIT
            break
        if record:
            history.append(dict(nu=nu, res=nRz, pr=info["pr"], dr=info["dr"], gap=info["gap"], kind="K2", ls=0))
        z = z - st.lam * Rz
    x, y, s = xys
    return Result(status=status, x=x, y=y, s=s, iters=nu, info=info, history=history,
                  counts=dict(k0=0, k1=0, k2=nu, km=0, backtracks=0), u=z, setup_s=setup_s,
                  solve_s=time.perf_counter() - t0)
