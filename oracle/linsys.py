"""Direct solve of the DRS linear step (I + Q)^{-1} r, FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. IV-A, equation (drs), first line: u~ = (I + Q)^{-1} u, where Q is the
skew-symmetric HSDE matrix of Sec. III-A,
    Q = [[0, A^T, c], [-A, 0, b], [-c^T, -b^T, 0]].
The paper states the system may be solved directly by a sparse LDL
factorisation.  Here the factorisation is of the SPD normal matrix that the
block elimination below leaves (I + A^T A when m >= n, else I + A A^T):
Cholesky (dense) or unpivoted symmetric LU (sparse) -- both are LDL^T with
the pivots in D.

Block elimination.  Write I + Q = [[M, h], [-h^T, 1]] with h = (c, b) and
M = [[I, A^T], [-A, I]].  Then
  M^{-1}(rx, ry): (I + A^T A) px = rx - A^T ry, py = ry + A px,
  g = M^{-1} h, delta = 1 + h^T g  (delta >= 1, since M^{-1} has a positive
  definite symmetric part),
  L(r) = (p - t g, t) with p = M^{-1}(rx, ry) and t = (r_tau + h^T p) / delta.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla


class DirectLinSys:
    def __init__(self, A, b, c, dense_limit: int = 25000):
        A = sp.csr_matrix(A, dtype=np.float64)
        self.A = A
        self.At = sp.csr_matrix(A.T)
        self.b = np.asarray(b, dtype=np.float64)
        self.c = np.asarray(c, dtype=np.float64)
        m, n = A.shape
        self.m, self.n = m, n
        self.normal = "AtA" if m >= n else "AAt"
        k = n if self.normal == "AtA" else m
        K = (self.At @ A) if self.normal == "AtA" else (A @ self.At)
        K = K + sp.identity(k, format="csr")
        density = K.nnz / float(k * k)
        if k <= dense_limit and (density > 0.02 or k <= 4000):
            self.kind = "dense"
            self._fac = scipy.linalg.cho_factor(K.toarray(), lower=True, check_finite=False)
            self._solve = lambda v: scipy.linalg.cho_solve(self._fac, v, check_finite=False)
        else:
            self.kind = "sparse"
            self._lu = spla.splu(sp.csc_matrix(K), permc_spec="MMD_AT_PLUS_A",
                                 diag_pivot_thresh=0.0, options=dict(SymmetricMode=True))
            self._solve = self._lu.solve
        h = np.concatenate([self.c, self.b])
        self.h = h
        gx, gy = self.solve_M(self.c, self.b)
        self.g = np.concatenate([gx, gy])
        self.delta = 1.0 + float(h @ self.g)

    def solve_M(self, rx, ry):
        """(px, py) = M^{-1}(rx, ry)."""
        if self.normal == "AtA":
            px = self._solve(rx - self.At @ ry)
            py = ry + self.A @ px
        else:
            py = self._solve(ry + self.A @ rx)
            px = rx - self.At @ py
        return px, py

    def L(self, r):
        """(I + Q)^{-1} r for r in R^{n+m+1}."""
        r = np.asarray(r, dtype=np.float64)
        n, m = self.n, self.m
        px, py = self.solve_M(r[:n], r[n:n + m])
        p = np.concatenate([px, py])
        t = (r[-1] + float(self.h @ p)) / self.delta
        return np.concatenate([p - t * self.g, [t]])


def Q_dense(A, b, c):
    """The HSDE matrix Q of Sec. III-A as a dense array (small sizes, tests)."""
    A = np.asarray(A.toarray() if sp.issparse(A) else A, dtype=np.float64)
    m, n = A.shape
    N = n + m + 1
    Q = np.zeros((N, N))
    Q[:n, n:n + m] = A.T
    Q[:n, -1] = c
    Q[n:n + m, :n] = -A
    Q[n:n + m, -1] = b
    Q[-1, :n] = -c
    Q[-1, n:n + m] = -b
    return Q
