"""The direct linear step (I + A^T A factored by a dense Cholesky on the device,
its inverse formed from the factor, one dense product per step) against the
oracle's direct solve (Sec. IV-A).

Parity: (I + Q)^{-1} r within 1e-12 relative (both sides direct; I + A^T A is
well conditioned on these instances, so the bar is a small multiple of the
factorisation's rounding), on orders below, at and across the factor's block
size of 64, with ragged last blocks, and on the 2000 x 1000 shared operator of
the learned-warm-start family (16 blocks); whole solves with the same
trajectory checks and KKT bars as the CG path, and no CG iterations reported.
"""
import numpy as np
import pytest

from paper_1903_06477_amd import generators as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sscs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_06477_amd import sscs as S
    S.lib()
    return S


def _lin(prob):
    import oracle
    return oracle.DirectLinSys(prob.A, prob.b, prob.c)


def _random_lp(m, n, density, seed):
    r = G.rng_for(43, seed)
    return G.Problem(A=G.sprandn(m, n, density, r), b=r.standard_normal(m), c=r.standard_normal(n),
                     cone=G.Cone(l=m))


@pytest.mark.parametrize("m,n,density", [(30, 1, 0.5), (90, 40, 0.1), (200, 64, 0.05), (300, 65, 0.05),
                                         (500, 150, 0.03), (900, 333, 0.01)])
def test_direct_linear_step_matches_oracle(sscs, m, n, density):
    prob = _random_lp(m, n, density, n)
    lin = _lin(prob)
    rr = np.random.default_rng(n)
    print(f"direct linear step, m {m} n {n} ({(n + 63) // 64} blocks)", flush=True)
    with sscs.Solver(prob, sscs.Settings(linsys="direct")) as s:
        for _ in range(3):
            rhs = rr.standard_normal(prob.n + prob.m + 1)
            ref = lin.L(rhs)
            got = s.linear_step(rhs)
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_direct_linear_step_shared_operator_of_the_learned_family(sscs):
    """The 2000 x 1000 operator at 2% density (16 blocks of the factor)."""
    A = G.config5_shared_A()
    r = G.rng_for(44, 0)
    prob = G.Problem(A=A, b=r.standard_normal(A.shape[0]), c=r.standard_normal(A.shape[1]),
                     cone=G.Cone(l=A.shape[0]))
    lin = _lin(prob)
    print("direct linear step, 2000 x 1000 shared operator", flush=True)
    with sscs.Solver(prob, sscs.Settings(linsys="direct")) as s:
        for k in range(2):
            rhs = np.random.default_rng(k).standard_normal(prob.n + prob.m + 1)
            ref = lin.L(rhs)
            got = s.linear_step(rhs)
            assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


def test_direct_solves_match_oracle(sscs):
    """Whole solves on the direct step: the LP workload (restarted Broyden) and
    a small SOCP (Anderson); ||R u|| trajectory equal to the oracle's (both
    direct) for the first iterations, KKT recomputed on the host, objective."""
    import test_gpu_parity as T
    _, S = T._oracle()
    prob = G.config1_lp()
    info, ref, ncmp = T._compare_solve(sscs, prob, S.Settings(direction="rb", mem=10),
                                       sscs.Settings(direction="rb", mem=10, linsys="direct", record_trace=True))
    assert info["cg_iters"] == 0
    print(f"LP: iters gpu {info['iters']} oracle {ref.iters}, trajectory equal for {ncmp} iterations")
    prob = G.small_socp(2)
    info, ref, ncmp = T._compare_solve(sscs, prob, S.Settings(direction="aa", mem=5),
                                       sscs.Settings(direction="aa", mem=5, linsys="direct", record_trace=True))
    assert info["cg_iters"] == 0
    print(f"SOCP: iters gpu {info['iters']} oracle {ref.iters}, trajectory equal for {ncmp} iterations")


def test_direct_rejections(sscs):
    """Batches and instances past the size limit are refused with a reason."""
    prob = G.config1_lp()
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.BatchSolver([prob, prob], sscs.Settings(linsys="direct"))
    big = _random_lp(10, 4097, 0.01, 1)
    with pytest.raises(sscs.SSCSError, match="unsupported"):
        sscs.Solver(big, sscs.Settings(linsys="direct"))
