"""GPU tests of the mixed-precision arm (FP32 operator inside CG, FP64
residuals and refinement) and of the one-workgroup solve kernel, against the
CPU oracle through the C ABI.

Bars: the mixed linear step equals the oracle's direct FP64 solve to 1e-9
relative at CG tolerance 1e-13 (each refinement round recomputes the residual
in FP64, so the FP32 operator's 2^-24 relative rounding only slows the
convergence of the rounds); end-to-end solves meet pr, dr, gap <= eps
recomputed on the CPU in FP64 from the returned (x, y, s), with the objective
within 1e-6 relative of the oracle's (both sides solved to eps 1e-8, since two
solutions that each just meet 1e-6 can differ in objective by ~1e-5)."""
import os

import numpy as np
import pytest

from paper_1903_06477_amd import generators as G

pytestmark = pytest.mark.gpu

EPS_OBJ = 1e-8


@pytest.fixture(scope="module")
def sscs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_06477_amd import sscs as S
    S.lib()
    return S


def _kkt(prob, x, y, s):
    nb, nc = np.linalg.norm(prob.b), np.linalg.norm(prob.c)
    pr = np.linalg.norm(prob.A @ x + s - prob.b) / (1 + nb)
    dr = np.linalg.norm(prob.A.T @ y + prob.c) / (1 + nc)
    cx, by = prob.c @ x, prob.b @ y
    return pr, dr, abs(cx + by) / (1 + abs(cx) + abs(by))


def _mixed_cones(seed=0):
    r = G.rng_for(40, seed)
    cone = G.Cone(z=5, l=12, q=[1, 3, 7, 20, 70], s=[1, 3, 6], ep=4)
    m = cone.rows()
    return G.Problem(A=G.sprandn(m, 40, 0.2, r), b=r.standard_normal(m), c=r.standard_normal(40), cone=cone)


@pytest.mark.parametrize("maker", ["lp", "socp", "cones", "tall", "wide"])
def test_mixed_linear_step_matches_oracle(sscs, maker):
    import oracle
    r = G.rng_for(41, 1)
    prob = {"lp": G.config1_lp, "socp": lambda: G.small_socp(2), "cones": _mixed_cones,
            "tall": lambda: G.Problem(A=G.sprandn(500, 70, 0.05, r), b=r.standard_normal(500),
                                      c=r.standard_normal(70), cone=G.Cone(l=500)),
            "wide": lambda: G.Problem(A=G.sprandn(60, 200, 0.1, r), b=r.standard_normal(60),
                                      c=r.standard_normal(200), cone=G.Cone(l=60))}[maker]()
    print(f"mixed linear step {maker} n={prob.n} m={prob.m}", flush=True)
    lin = oracle.DirectLinSys(prob.A, prob.b, prob.c)
    rr = np.random.default_rng(6)
    with sscs.Solver(prob, sscs.Settings(cg_tol=1e-13, cg_max=5000, precision="mixed")) as s:
        for _ in range(3):
            rhs = rr.standard_normal(prob.n + prob.m + 1)
            ref = lin.L(rhs)
            got = s.linear_step(rhs)
            assert np.linalg.norm(got - ref) <= 1e-9 * np.linalg.norm(ref)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("grid", ["auto", "1"])
def test_end_to_end_precision_and_kernel(sscs, precision, grid):
    """config-1 LP (restarted Broyden) and a small SOCP (Anderson), on the grid
    kernel and on the one-workgroup kernel (grid forced to 1)."""
    from oracle import superscs as S
    cases = [(G.config1_lp(), "rb", 10), (G.small_socp(2), "aa", 5)]
    wg = 1 if grid == "1" else 0
    for prob, d, mem in cases:
        print(f"solve {prob.name or 'socp'} {precision} grid={grid}", flush=True)
        ref = S.solve(prob, S.Settings(direction=d, mem=mem, eps=EPS_OBJ))
        with sscs.Solver(prob, sscs.Settings(direction=d, mem=mem, eps=EPS_OBJ, cg_tol=1e-12, cg_max=5000,
                                             precision=precision, workgroups=wg)) as s:
            x, y, sv, info = s.solve()
        assert info["status"] == sscs.SOLVED == ref.status
        assert max(_kkt(prob, x, y, sv)) <= EPS_OBJ * 1.0001
        assert abs(info["pobj"] - ref.info["pobj"]) <= 1e-6 * (1 + abs(ref.info["pobj"]))


@pytest.mark.skip(reason="the batched engine's mixed-precision form ran without finishing on the GPU in an "
                         "early test whose code is no longer in the tree; its cause has not been shown (a CPU "
                         "emulation of the current refinement rounds on these six instances ends every linear "
                         "step within 129 CG passes and 4 rounds and solves each instance), so the form stays "
                         "switched off (sscs_batch_create returns SSCS_E_UNSUPPORTED for it)")
def test_mixed_batch_lasso(sscs):
    from oracle import superscs as S
    probs = [G.config4_instance(i) for i in range(6)]
    st = sscs.Settings(direction="aa", mem=5, eps=EPS_OBJ, cg_tol=1e-12, cg_max=2000, precision="mixed",
                       max_time=20.0)
    bs = sscs.BatchSolver(probs, st)
    x, y, sv, infos = bs.solve()
    parts = bs.split(x, y, sv)
    for i, p in enumerate(probs):
        ref = S.solve(p, S.Settings(direction="aa", mem=5, eps=EPS_OBJ))
        assert infos[i]["status"] == sscs.SOLVED
        assert max(_kkt(p, *parts[i])) <= EPS_OBJ * 1.0001
        assert abs(infos[i]["pobj"] - ref.info["pobj"]) <= 1e-6 * (1 + abs(ref.info["pobj"]))
    bs.close()
