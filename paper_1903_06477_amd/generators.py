"""Seeded synthetic conic programs shaped like the paper's workloads.

This module builds problem data only: matrices, vectors and cone layouts for
the standard form of Sec. III, problem (P): minimise <c, x> subject to
b - A x = s, s in K.  It contains none of the solver's arithmetic (no linear
steps, projections, directions or termination tests), so both the GPU
library and the CPU oracle may consume its output.

Cone layout of s and y (rows of A, b): zero | R+ | SOC ... | PSD ... | exp ...
  * SOC blocks are (x, t) with t LAST (Sec. II, second-order cone).
  * PSD blocks are the column-major lower triangle with off-diagonal entries
    scaled by sqrt(2), the inverse of the paper's mat operator (Sec. II).
  * exp blocks are (x1, x2, x3) with x1 >= x2 exp(x3 / x2) (Sec. II).

Random streams: numpy PCG64 seeded with 1_000_000 * config + instance.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np
import scipy.sparse as sp


def rng_for(config: int, instance: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1_000_000 * config + instance))


@dataclasses.dataclass
class Cone:
    z: int = 0                       # zero-cone rows (equalities)
    l: int = 0                       # nonnegative-orthant rows
    q: List[int] = dataclasses.field(default_factory=list)   # SOC sizes
    s: List[int] = dataclasses.field(default_factory=list)   # PSD orders
    ep: int = 0                      # number of exponential cones

    def rows(self) -> int:
        return (self.z + self.l + sum(self.q)
                + sum(k * (k + 1) // 2 for k in self.s) + 3 * self.ep)

    def as_dict(self) -> Dict:
        return dict(z=self.z, l=self.l, q=list(self.q), s=list(self.s), ep=self.ep)


@dataclasses.dataclass
class Problem:
    A: sp.csr_matrix                 # m x n, float64, sorted indices
    b: np.ndarray                    # m
    c: np.ndarray                    # n
    cone: Cone
    name: str = ""
    x_star: Optional[np.ndarray] = None   # planted primal solution, if any
    y_star: Optional[np.ndarray] = None
    s_star: Optional[np.ndarray] = None
    meta: Dict = dataclasses.field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.A.shape[0]

    @property
    def n(self) -> int:
        return self.A.shape[1]


def _csr(A) -> sp.csr_matrix:
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sum_duplicates()
    A.sort_indices()
    A.indptr = A.indptr.astype(np.int32)
    A.indices = A.indices.astype(np.int32)
    return A


def sprandn(m: int, n: int, density: float, rng: np.random.Generator) -> sp.csr_matrix:
    """m x n sparse matrix with the given density and N(0,1) nonzeros."""
    A = sp.random(m, n, density=density, format="csr", random_state=rng,
                  data_rvs=rng.standard_normal)
    return _csr(A)


# ---------------------------------------------------------------------------
# Planted primal-dual optima (configs 1 and 2)
# ---------------------------------------------------------------------------

def _planted_soc_pair(k: int, rng: np.random.Generator):
    """A complementary pair (s, y) on one second-order cone of size k (t last)."""
    case = rng.integers(0, 3)
    v = rng.standard_normal(k - 1)
    nv = np.linalg.norm(v)
    s = np.zeros(k)
    y = np.zeros(k)
    if case == 0:            # s interior, y = 0
        s[:-1] = v
        s[-1] = nv + abs(rng.standard_normal())
    elif case == 1:          # s = 0, y interior
        y[:-1] = v
        y[-1] = nv + abs(rng.standard_normal())
    else:                    # both on the boundary, opposite rays
        e = v / nv if nv > 0 else np.eye(k - 1)[0]
        a = abs(rng.standard_normal())
        beta = abs(rng.standard_normal())
        s[:-1] = a * e
        s[-1] = a
        y[:-1] = -beta * e
        y[-1] = beta
    return s, y


def planted(A: sp.csr_matrix, cone: Cone, rng: np.random.Generator, name: str = "") -> Problem:
    """Feasible (P)/(D) pair with a known optimum (x*, y*, s*): complementary
    s* in K, y* in K* on every block, b = A x* + s*, c = -A^T y*."""
    m, n = A.shape
    assert cone.rows() == m
    assert not cone.s and cone.ep == 0, "planted construction covers zero/R+/SOC"
    x = rng.standard_normal(n)
    s = np.zeros(m)
    y = np.zeros(m)
    o = 0
    y[o:o + cone.z] = rng.standard_normal(cone.z)
    o += cone.z
    perm = rng.permutation(cone.l)
    half = cone.l // 2
    blk_s = np.zeros(cone.l)
    blk_y = np.zeros(cone.l)
    blk_s[perm[:half]] = np.abs(rng.standard_normal(half))
    blk_y[perm[half:]] = np.abs(rng.standard_normal(cone.l - half))
    s[o:o + cone.l] = blk_s
    y[o:o + cone.l] = blk_y
    o += cone.l
    for k in cone.q:
        s[o:o + k], y[o:o + k] = _planted_soc_pair(k, rng)
        o += k
    b = A @ x + s
    c = -(A.T @ y)
    return Problem(A=A, b=b, c=c, cone=cone, name=name, x_star=x, y_star=y, s_star=s)


def config1_lp(instance: int = 0) -> Problem:
    """Random feasible LP in conic form: m=300, n=100, 10% density, K = R+^300."""
    rng = rng_for(1, instance)
    A = sprandn(300, 100, 0.10, rng)
    return planted(A, Cone(l=300), rng, name="lp_300x100")


def soc_sizes(rem: int, rng: np.random.Generator, lo: int = 3, hi: int = 50) -> List[int]:
    sizes = []
    while rem > hi:
        k = int(rng.integers(lo, min(hi, rem - lo) + 1))
        sizes.append(k)
        rem -= k
    if rem > 0:
        sizes.append(rem)
    return sizes


def config2_socp(instance: int = 0, n: int = 20000, m: int = 50000, density: float = 1e-3,
                 nz: int = 1000, nl: int = 20000) -> Problem:
    """Sparse SOCP: zero 1000 + R+ 20000 + SOC sizes U{3..50} filling the rest."""
    rng = rng_for(2, instance)
    A = sprandn(m, n, density, rng)
    cone = Cone(z=nz, l=nl, q=soc_sizes(m - nz - nl, rng))
    return planted(A, cone, rng, name=f"socp_{m}x{n}")


def small_socp(seed: int, n: int = 60, m: int = 150, density: float = 0.08,
               nz: int = 10, nl: int = 60) -> Problem:
    """Config-2 recipe at a size the oracle solves in well under a second."""
    rng = rng_for(20, seed)
    A = sprandn(m, n, density, rng)
    cone = Cone(z=nz, l=nl, q=soc_sizes(m - nz - nl, rng, 3, 12))
    return planted(A, cone, rng, name=f"socp_small_{seed}")


# ---------------------------------------------------------------------------
# Tiny LPs for vertex enumeration, certificates
# ---------------------------------------------------------------------------

def tiny_lp(seed: int, n: int = 3, mg: int = 5, box: float = 2.0) -> Problem:
    """min c^T x s.t. G x <= h, -box <= x <= box; conic rows [G; I; -I]."""
    rng = rng_for(30, seed)
    G = rng.standard_normal((mg, n))
    xf = rng.uniform(-0.5, 0.5, n)
    h = G @ xf + np.abs(rng.standard_normal(mg)) * 0.5
    A = np.vstack([G, np.eye(n), -np.eye(n)])
    b = np.concatenate([h, box * np.ones(n), box * np.ones(n)])
    c = rng.standard_normal(n)
    return Problem(A=_csr(A), b=b, c=c, cone=Cone(l=mg + 2 * n), name=f"tiny_lp_{seed}")


def infeasible_lp(seed: int, n: int = 20, m: int = 50, density: float = 0.3) -> Problem:
    """Primal-infeasible LP with certificate y0 >= 0, A^T y0 = 0, <b, y0> = -1."""
    rng = rng_for(31, seed)
    A = sprandn(m, n, density, rng).toarray()
    y0 = np.abs(rng.standard_normal(m))
    A = A - np.outer(y0, y0 @ A) / (y0 @ y0)
    b = rng.standard_normal(m)
    b = b - ((b @ y0 + 1.0) / (y0 @ y0)) * y0
    c = rng.standard_normal(n)
    return Problem(A=_csr(A), b=b, c=c, cone=Cone(l=m), name=f"infeasible_{seed}",
                   meta=dict(y_cert=y0))


def unbounded_lp(seed: int, n: int = 20, m: int = 50, density: float = 0.3) -> Problem:
    """Dual-infeasible (unbounded) LP with ray x0: -A x0 = s0 in K, <c, x0> = -1."""
    rng = rng_for(32, seed)
    A = sprandn(m, n, density, rng).toarray()
    x0 = rng.standard_normal(n)
    s0 = np.abs(rng.standard_normal(m))
    A = A - np.outer(A @ x0 + s0, x0) / (x0 @ x0)
    c = rng.standard_normal(n)
    c = c - ((c @ x0 + 1.0) / (x0 @ x0)) * x0
    xf = rng.standard_normal(n)
    sf = np.abs(rng.standard_normal(m))
    b = A @ xf + sf
    return Problem(A=_csr(A), b=b, c=c, cone=Cone(l=m), name=f"unbounded_{seed}",
                   meta=dict(x_cert=x0))


# ---------------------------------------------------------------------------
# LASSO as an SOCP (Sec. V-C shape; configs 4 and 5)
# ---------------------------------------------------------------------------

def lasso_socp(Ad: sp.csr_matrix, bd: np.ndarray, mu: float, name: str = "") -> Problem:
    """min 1/2 ||Ad x - bd||^2 + mu ||x||_1 as a cone program in z = (x, r, t).

    min mu 1^T r + t/2 s.t. r - x >= 0, r + x >= 0 (R+ 2n) and
    (Ad x - bd, (t-1)/2, (t+1)/2) in SOC of size md + 2 (t last), which
    encodes ||Ad x - bd||^2 <= t."""
    md, n = Ad.shape
    I = sp.identity(n, format="csr")
    Z = sp.csr_matrix((n, 1))
    top = sp.hstack([I, -I, Z])                        # s = r - x
    mid = sp.hstack([-I, -I, Z])                       # s = r + x
    soc = sp.hstack([-Ad, sp.csr_matrix((md, n)), sp.csr_matrix((md, 1))])
    tail = sp.csr_matrix(np.array([[0.0] * (2 * n) + [-0.5], [0.0] * (2 * n) + [-0.5]]))
    A = _csr(sp.vstack([top, mid, soc, tail]))
    b = np.concatenate([np.zeros(2 * n), -bd, [-0.5, 0.5]])
    c = np.concatenate([np.zeros(n), mu * np.ones(n), [0.5]])
    return Problem(A=A, b=b, c=c, cone=Cone(l=2 * n, q=[md + 2]), name=name,
                   meta=dict(Ad=Ad, bd=bd, mu=mu, n_data=n, m_data=md))


def lasso_data(rng: np.random.Generator, md: int, n: int, density: float,
               A: Optional[sp.csr_matrix] = None):
    if A is None:
        A = sprandn(md, n, density, rng)
    x0 = np.zeros(n)
    k = max(1, int(round(0.1 * n)))
    idx = rng.choice(n, size=k, replace=False)
    x0[idx] = rng.standard_normal(k)
    b = A @ x0 + 0.05 * rng.standard_normal(md)
    mu = 0.1 * float(np.max(np.abs(A.T @ b)))
    return A, b, mu


def config4_instance(i: int) -> Problem:
    """One instance of the batched LASSO family: n ~ U{20..400}, m ~ U{ceil(n/2)..2n}."""
    rng = rng_for(4, i)
    n = int(rng.integers(20, 401))
    md = int(rng.integers(math.ceil(n / 2), 2 * n + 1))
    A, b, mu = lasso_data(rng, md, n, 0.05)
    return lasso_socp(A, b, mu, name=f"lasso4_{i}")


def config5_shared_A() -> sp.csr_matrix:
    return sprandn(2000, 1000, 0.02, rng_for(5, 10**6 - 1))


def config5_instance(i: int, A: sp.csr_matrix) -> Problem:
    """Instance i of the shared-A LASSO family (only bd and mu vary)."""
    rng = rng_for(5, i)
    A, b, mu = lasso_data(rng, A.shape[0], A.shape[1], 0.0, A=A)
    return lasso_socp(A, b, mu, name=f"lasso5_{i}")


def config5_family(indices, A: sp.csr_matrix) -> List[Problem]:
    """Instances of the shared-A LASSO family with one conic matrix object
    shared by all of them (the same data as config5_instance(i, A), built
    without re-assembling the conic matrix per instance)."""
    base = lasso_socp(A, np.zeros(A.shape[0]), 1.0)
    md, n = A.shape
    out = []
    for i in indices:
        rng = rng_for(5, int(i))
        _, bd, mu = lasso_data(rng, md, n, 0.0, A=A)
        b = np.concatenate([np.zeros(2 * n), -bd, [-0.5, 0.5]])
        c = np.concatenate([np.zeros(n), mu * np.ones(n), [0.5]])
        out.append(Problem(A=base.A, b=b, c=c, cone=base.cone, name=f"lasso5_{int(i)}",
                           meta=dict(Ad=A, bd=bd, mu=mu, n_data=n, m_data=md)))
    return out


def spmv_scaled(m: int = 5_000_000, n: int = 20_000, per_row: int = 20, seed: int = 0) -> Problem:
    """The SOCP workload's matrix shape scaled in its rows to exceed the
    on-package cache: m x n with per_row N(0,1) nonzeros in every row (the
    SOCP has 20 per row on average), columns distinct and sorted (sorted
    uniform draws spread by their rank), K = R+^m, b = c = 0.  For
    measuring the CG's products; not a solve workload."""
    rng = rng_for(7, seed)
    cols = np.sort(rng.integers(0, n - per_row + 1, size=(m, per_row), dtype=np.int32), axis=1)
    cols += np.arange(per_row, dtype=np.int32)[None, :]
    vals = rng.standard_normal(m * per_row)
    indptr = np.arange(0, m * per_row + 1, per_row, dtype=np.int64)
    A = sp.csr_matrix((vals, cols.reshape(-1), indptr.astype(np.int32)), shape=(m, n))
    A.has_sorted_indices = True
    return Problem(A=A, b=np.zeros(m), c=np.zeros(n), cone=Cone(l=m), name=f"spmv_{m}x{n}")


def spmv_ragged(m: int, n: int, max_per_row: int, seed: int = 0) -> Problem:
    """An m x n operator whose row lengths are uniform on 0..max_per_row
    (empty rows included), columns distinct and sorted within each row,
    values N(0,1); K = R+^m, b = c = 0.  For the SpMV's ragged-row cases; not
    a solve workload."""
    rng = rng_for(8, seed)
    lens = rng.integers(0, max_per_row + 1, size=m)
    indptr = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(lens, out=indptr[1:])
    nnz = int(indptr[-1])
    row = np.repeat(np.arange(m), lens)
    draw = rng.integers(0, n - np.repeat(lens, lens) + 1)
    order = np.lexsort((draw, row))                # sorted within each row
    pos = np.arange(nnz) - indptr[row]             # place within the row
    cols = (draw[order] + pos).astype(np.int32)    # strictly increasing in a row
    vals = rng.standard_normal(nnz)
    A = sp.csr_matrix((vals, cols, indptr.astype(np.int32)), shape=(m, n))
    A.has_sorted_indices = True
    return Problem(A=A, b=np.zeros(m), c=np.zeros(n), cone=Cone(l=m), name=f"spmv_ragged_{m}x{n}")


def lasso_dm_instance(n: int, kappa: float, mu: float, seed: int = 0) -> Problem:
    """One problem of the LASSO benchmark family of Sec. V-C: A in R^{m x n}
    with m = ceil(n/5) and condition number kappa (A = U diag(s) V^T, U, V
    with orthonormal columns drawn from Gaussian matrices, s geometric from 1
    down to 1/kappa), b = A x0 + 0.05 N(0,1) with 10%-sparse x0, weight mu
    (the paper's n in {631, 1000, 1585, 2512}, kappa in {10, 215, 4600, 1e5},
    mu in {0.01, 0.1, 1}).  The paper does not publish its generator; this one
    fixes the stated sizes, conditioning and weights, with a dense A."""
    rng = rng_for(6, seed)
    md = int(math.ceil(n / 5))
    U, _ = np.linalg.qr(rng.standard_normal((md, md)))
    V, _ = np.linalg.qr(rng.standard_normal((n, md)))
    s = np.geomspace(1.0, 1.0 / kappa, md)
    Ad = (U * s[None, :]) @ V.T
    x0 = np.zeros(n)
    k = max(1, int(round(0.1 * n)))
    idx = rng.choice(n, size=k, replace=False)
    x0[idx] = rng.standard_normal(k)
    b = Ad @ x0 + 0.05 * rng.standard_normal(md)
    return lasso_socp(sp.csr_matrix(Ad), b, mu, name=f"lasso_dm_n{n}_k{kappa:g}_mu{mu:g}_{seed}")


def lasso_dm_family(seeds: int = 1) -> List[Problem]:
    """The 48 (n, kappa, mu) combinations of the family, `seeds` problems each."""
    return [lasso_dm_instance(n, kap, mu, 1000 * i + s)
            for i, (n, kap, mu) in enumerate((n, kap, mu) for n in (631, 1000, 1585, 2512)
                                             for kap in (10.0, 215.0, 4600.0, 1e5) for mu in (0.01, 0.1, 1.0))
            for s in range(seeds)]


# ---------------------------------------------------------------------------
# mixed SDP / exponential-cone instance: sparse PCA blocks plus an
# l1-regularised logistic regression, one block-diagonal problem

def _svec_pairs(k: int):
    """(i, j) of the column-major lower-triangle packing, i >= j, and the
    scale of each entry (1 on the diagonal, sqrt(2) off it)."""
    jj, ii = np.triu_indices(k)          # ordered by j, then i >= j
    scale = np.where(ii == jj, 1.0, math.sqrt(2.0))
    return ii, jj, scale


def config3_sdp_exp(instance: int = 0, nblk: int = 64, k: int = 64, kbig: int = 256, q: int = 5000,
                    p: int = 1000, density: float = 0.01, lam_sdp: float = 2.0) -> Problem:
    """Sparse PCA:  max <S_b, Z_b> - lam ||Z_b||_1, tr Z_b = 1, Z_b PSD for
    nblk blocks of order k and one of order kbig (S = (G + G^T) / 2, G with
    N(0, 1) entries), written with T_b >= |Z_b| entrywise; plus logistic
    regression  min sum_i log(1 + exp(-y_i (a_i^T w + beta))) + lam_log ||w||_1
    over q samples of p features (F at `density`, N(0, 1); labels +-1;
    lam_log = 0.1 * ||F^T y||_inf / 2), each loss term through two exponential
    cones: t_i >= log(exp(0) + exp(z_i)) iff u1 + u2 <= 1, (u1, 1, -t_i) and
    (u2, 1, z_i - t_i) in K_exp.

    Variables: [svec Z (all blocks) | svec T | w | beta | r | t | u1 | u2].
    Rows: zero (one trace row per block) | R+ (T - Z, T + Z, 1 - u1 - u2,
    r - w, r + w) | PSD (svec Z per block) | exp (two cones per sample)."""
    rng = rng_for(3, instance)
    orders = [k] * nblk + ([kbig] if kbig > 0 else [])
    D = [o * (o + 1) // 2 for o in orders]
    Dt = int(sum(D))
    offs = np.concatenate([[0], np.cumsum(D)]).astype(np.int64)
    # data
    cZ = np.zeros(Dt)
    wT = np.zeros(Dt)
    diag_pos = []
    for b, o in enumerate(orders):
        Gm = rng.standard_normal((o, o))
        S = 0.5 * (Gm + Gm.T)
        ii, jj, sc = _svec_pairs(o)
        cZ[offs[b]:offs[b + 1]] = -(S[ii, jj] * sc)
        wT[offs[b]:offs[b + 1]] = np.where(ii == jj, 1.0, math.sqrt(2.0))
        diag_pos.append(offs[b] + np.nonzero(ii == jj)[0])
    F = sprandn(q, p, density, rng)
    y = np.where(rng.random(q) < 0.5, -1.0, 1.0)
    lam_log = 0.1 * 0.5 * float(np.max(np.abs(F.T @ y)))
    # variable offsets
    oZ, oT = 0, Dt
    ow = 2 * Dt
    obeta = ow + p
    orr = obeta + 1
    ot = orr + p
    ou1 = ot + q
    ou2 = ou1 + q
    n = ou2 + q
    c = np.zeros(n)
    c[oZ:oZ + Dt] = cZ
    c[oT:oT + Dt] = lam_sdp * wT
    c[orr:orr + p] = lam_log
    c[ot:ot + q] = 1.0
    rows, cols, vals, bvec = [], [], [], []
    r0 = 0

    def add(rr, cc, vv):
        rows.append(np.asarray(rr, np.int64))
        cols.append(np.asarray(cc, np.int64))
        vals.append(np.asarray(vv, np.float64))

    # zero: tr Z_b = 1  (s = 1 - tr Z_b)
    for b in range(len(orders)):
        add(np.full(len(diag_pos[b]), r0 + b), oZ + diag_pos[b], np.ones(len(diag_pos[b])))
    bvec.append(np.ones(len(orders)))
    r0 += len(orders)
    nz = len(orders)
    # R+: T - Z >= 0, T + Z >= 0
    e = np.arange(Dt)
    add(r0 + e, oT + e, -np.ones(Dt)); add(r0 + e, oZ + e, np.ones(Dt)); r0 += Dt
    add(r0 + e, oT + e, -np.ones(Dt)); add(r0 + e, oZ + e, -np.ones(Dt)); r0 += Dt
    bvec.append(np.zeros(2 * Dt))
    # R+: 1 - u1 - u2 >= 0
    eq = np.arange(q)
    add(r0 + eq, ou1 + eq, np.ones(q)); add(r0 + eq, ou2 + eq, np.ones(q)); r0 += q
    bvec.append(np.ones(q))
    # R+: r - w >= 0, r + w >= 0
    ep_ = np.arange(p)
    add(r0 + ep_, orr + ep_, -np.ones(p)); add(r0 + ep_, ow + ep_, np.ones(p)); r0 += p
    add(r0 + ep_, orr + ep_, -np.ones(p)); add(r0 + ep_, ow + ep_, -np.ones(p)); r0 += p
    bvec.append(np.zeros(2 * p))
    nl = 2 * Dt + q + 2 * p
    # PSD: s = svec Z_b
    add(r0 + e, oZ + e, -np.ones(Dt)); r0 += Dt
    bvec.append(np.zeros(Dt))
    # exp: per sample (u1, 1, -t) and (u2, 1, -y_i (a_i^T w + beta) - t)
    eb = np.zeros(6 * q)
    base = r0 + 6 * eq
    add(base, ou1 + eq, -np.ones(q))                 # s = u1
    eb[6 * eq + 1] = 1.0                               # s = 1
    add(base + 2, ot + eq, np.ones(q))                 # s = -t
    add(base + 3, ou2 + eq, -np.ones(q))               # s = u2
    eb[6 * eq + 4] = 1.0
    Fc = F.tocoo()
    add(base[Fc.row] + 5, ow + Fc.col, y[Fc.row] * Fc.data)   # s = -y (a^T w + beta) - t
    add(base + 5, np.full(q, obeta), y)
    add(base + 5, ot + eq, np.ones(q))
    bvec.append(eb)
    r0 += 6 * q
    m = r0
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
    cone = Cone(z=nz, l=nl, s=orders, ep=2 * q)
    return Problem(A=_csr(A), b=np.concatenate(bvec), c=c, cone=cone, name=f"sdp_exp_{m}x{n}",
                   meta=dict(F=F, labels=y, lam_log=lam_log, lam_sdp=lam_sdp, orders=orders,
                             offsets=dict(Z=oZ, T=oT, w=ow, beta=obeta, r=orr, t=ot, u1=ou1, u2=ou2)))


def small_sdp_exp(seed: int = 0) -> Problem:
    """The mixed SDP / exp instance at a size the oracle solves in seconds."""
    return config3_sdp_exp(instance=1000 + seed, nblk=2, k=4, kbig=7, q=30, p=6, density=0.3)


# ---------------------------------------------------------------------------
# Benchmark families of Sec. V-B (l1-regularised sparse PCA SDP) and Sec. V-D
# (l1-regularised logistic regression), one problem per call

def sdp_pca_instance(d: int, lam: float, seed: int = 0) -> Problem:
    """max tr(S Z) - lam ||Z||_1 s.t. tr Z = 1, Z PSD (problem (rpca), Sec.
    V-B) with S = (G + G^T) / 2, G of N(0,1) entries, as a cone program in
    (svec Z, svec T): min -<svec S, svec Z> + lam <w, svec T> with rows
    tr Z = 1 (zero), T - Z >= 0 and T + Z >= 0 (R+), svec Z in the PSD cone
    (w = 1 on the diagonal, sqrt 2 off it, so <w, svec T> = sum |Z_ij| at the
    optimum).  The paper does not publish its generator; this one takes the
    stated sizes d and weights lam."""
    rng = rng_for(8, seed)
    Gm = rng.standard_normal((d, d))
    S = 0.5 * (Gm + Gm.T)
    ii, jj, sc = _svec_pairs(d)
    D = d * (d + 1) // 2
    c = np.concatenate([-(S[ii, jj] * sc), lam * np.where(ii == jj, 1.0, math.sqrt(2.0))])
    diag = np.nonzero(ii == jj)[0]
    e = np.arange(D)
    rows = [np.zeros(d, np.int64), 1 + e, 1 + e, 1 + D + e, 1 + D + e, 1 + 2 * D + e]
    cols = [diag, D + e, e, D + e, e, e]
    vals = [np.ones(d), -np.ones(D), np.ones(D), -np.ones(D), -np.ones(D), -np.ones(D)]
    m = 1 + 3 * D
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, 2 * D))
    b = np.concatenate([[1.0], np.zeros(3 * D)])
    return Problem(A=_csr(A), b=b, c=c, cone=Cone(z=1, l=2 * D, s=[d]), name=f"sdp_pca_d{d}_lam{lam:g}_{seed}",
                   meta=dict(S=S, lam=lam))


def sdp_pca_dm_family(seeds: int = 1) -> List[Problem]:
    """The sparse-PCA family of Sec. V-B: d in {50, 120, 140, 180}, lam in
    {0.1, 2, 5}, `seeds` problems per combination."""
    return [sdp_pca_instance(d, lam, 100 * i + s)
            for i, (d, lam) in enumerate((d, lam) for d in (50, 120, 140, 180) for lam in (0.1, 2.0, 5.0))
            for s in range(seeds)]


def logreg_instance(p: int, q: int, lam: float, seed: int = 0, density: float = 1.0) -> Problem:
    """min lam ||w||_1 + sum_i log(1 + exp(-y_i (a_i^T w + beta))) (problem
    (logreg) of Sec. V-D, read with labels y_i in {-1, 1} and intercept beta)
    over q samples a_i in R^p with N(0,1) entries (at `density`), labels
    +-1.  Each loss term through two exponential cones: t_i >=
    log(1 + exp(z_i)) iff u1 + u2 <= 1, (u1, 1, -t_i) and (u2, 1, z_i - t_i) in
    K_exp, with z_i = -y_i (a_i^T w + beta); |w| <= r by 2p R+ rows.
    Variables [w | beta | r | t | u1 | u2]."""
    rng = rng_for(9, seed)
    F = sprandn(q, p, density, rng) if density < 1.0 else sp.csr_matrix(rng.standard_normal((q, p)))
    y = np.where(rng.random(q) < 0.5, -1.0, 1.0)
    ow, obeta = 0, p
    orr = obeta + 1
    ot = orr + p
    ou1 = ot + q
    ou2 = ou1 + q
    n = ou2 + q
    c = np.zeros(n)
    c[orr:orr + p] = lam
    c[ot:ot + q] = 1.0
    rows, cols, vals, bvec = [], [], [], []

    def add(rr, cc, vv):
        rows.append(np.asarray(rr, np.int64))
        cols.append(np.asarray(cc, np.int64))
        vals.append(np.asarray(vv, np.float64))

    r0 = 0
    eq = np.arange(q)
    add(r0 + eq, ou1 + eq, np.ones(q)); add(r0 + eq, ou2 + eq, np.ones(q)); r0 += q    # 1 - u1 - u2 >= 0
    bvec.append(np.ones(q))
    ep_ = np.arange(p)
    add(r0 + ep_, orr + ep_, -np.ones(p)); add(r0 + ep_, ow + ep_, np.ones(p)); r0 += p      # r - w >= 0
    add(r0 + ep_, orr + ep_, -np.ones(p)); add(r0 + ep_, ow + ep_, -np.ones(p)); r0 += p     # r + w >= 0
    bvec.append(np.zeros(2 * p))
    nl = q + 2 * p
    eb = np.zeros(6 * q)
    base = r0 + 6 * eq
    add(base, ou1 + eq, -np.ones(q))
    eb[6 * eq + 1] = 1.0
    add(base + 2, ot + eq, np.ones(q))
    add(base + 3, ou2 + eq, -np.ones(q))
    eb[6 * eq + 4] = 1.0
    Fc = F.tocoo()
    add(base[Fc.row] + 5, ow + Fc.col, y[Fc.row] * Fc.data)
    add(base + 5, np.full(q, obeta), y)
    add(base + 5, ot + eq, np.ones(q))
    bvec.append(eb)
    m = r0 + 6 * q
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
    return Problem(A=_csr(A), b=np.concatenate(bvec), c=c, cone=Cone(l=nl, ep=2 * q),
                   name=f"logreg_p{p}_q{q}_lam{lam:g}_{seed}", meta=dict(F=F, labels=y, lam=lam, p=p, q=q))


def logreg_dm_family(seeds: int = 1) -> List[Problem]:
    """The logistic-regression family of Sec. V-D: p in {80, 100}, q in {50,
    100, 120}, lam in {10, 20, 50}, `seeds` problems per combination."""
    return [logreg_instance(p, q, lam, 100 * i + s)
            for i, (p, q, lam) in enumerate((p, q, lam) for p in (80, 100) for q in (50, 100, 120)
                                            for lam in (10.0, 20.0, 50.0))
            for s in range(seeds)]
