"""GPU checks at the full workload sizes, in the launch configuration bench.py
times.  Where the oracle cannot finish a whole solve in seconds, properties
that hold at any size are checked on the GPU's outputs, recomputed on the host
in FP64:

* the sparse SOCP (n = 20000, m = 50000): solved, pr/dr/gap <= 1e-6 from the
  returned (x, y, s), y in K* and s in K to 1e-6, objective within 1e-4 of the
  planted optimum <c, x*>;
* 4096 batched LASSO instances: every one solved with pr/dr/gap <= 1e-6;
* the PSD / exponential-cone instance (m = 535113): the projection onto K* of
  the whole row space equals the oracle's, block by block (1e-10), and the
  product by A equals scipy's (1e-13)."""
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


def _kkt(prob, x, y, s):
    nb, nc = np.linalg.norm(prob.b), np.linalg.norm(prob.c)
    pr = np.linalg.norm(prob.A @ x + s - prob.b) / (1 + nb)
    dr = np.linalg.norm(prob.A.T @ y + prob.c) / (1 + nc)
    cx, by = prob.c @ x, prob.b @ y
    return pr, dr, abs(cx + by) / (1 + abs(cx) + abs(by))


def test_socp_20000x50000_solves_to_tolerance(sscs):
    import bench
    from oracle.cones import proj_dual_cone
    prob = G.config2_socp()
    st = bench.bench_settings(sscs, 20000)
    st.data_on_device = False
    print("SOCP 20000 x 50000, bench settings", flush=True)
    with sscs.Solver(prob, st) as s:
        x, y, sv, info = s.solve()
    assert info["status"] == sscs.SOLVED
    assert max(_kkt(prob, x, y, sv)) <= 1e-6 * 1.0001
    assert np.linalg.norm(y - proj_dual_cone(y, prob.cone)) <= 1e-6 * (1 + np.linalg.norm(y))
    z = prob.cone.z
    s_nz = sv.copy()
    s_nz[:z] = 0.0
    assert np.linalg.norm(sv[:z]) <= 1e-5 * (1 + np.linalg.norm(prob.b))
    assert np.linalg.norm(s_nz - proj_dual_cone(s_nz, prob.cone)) <= 1e-6 * (1 + np.linalg.norm(sv))
    pstar = prob.c @ prob.x_star
    assert abs(prob.c @ x - pstar) <= 1e-4 * (1 + abs(pstar))


def test_lasso_batch_4096_all_solved(sscs):
    import bench
    probs = [G.config4_instance(i) for i in range(4096)]
    st = bench.bench_settings(sscs, 20000)
    st.data_on_device = False
    print("4096 LASSO instances", flush=True)
    bs = sscs.BatchSolver(probs, st)
    x, y, sv, infos = bs.solve()
    parts = bs.split(x, y, sv)
    worst = 0.0
    for i, p in enumerate(probs):
        assert infos[i]["status"] == sscs.SOLVED, i
        worst = max(worst, max(_kkt(p, *parts[i])))
    bs.close()
    print(f"worst host-recomputed residual {worst:.3e}")
    assert worst <= 1e-6 * 1.0001


def test_sdp_exp_full_projection_and_spmv(sscs):
    from oracle.cones import proj_dual_cone
    prob = G.config3_sdp_exp()
    r = np.random.default_rng(33)
    print(f"PSD/exp instance m={prob.m} n={prob.n}", flush=True)
    with sscs.Solver(prob, sscs.Settings(cg_tol=1e-10)) as s:
        xv = r.standard_normal(prob.n)
        got = s.spmv(xv)
        ref = prob.A @ xv
        assert np.max(np.abs(got - ref)) <= 1e-13 * (1 + np.max(np.abs(ref)))
        for step in range(2):
            yv = r.standard_normal(prob.m) if step == 0 else yv + 1e-4 * r.standard_normal(prob.m)
            got = s.project_dual_cone(yv)
            ref = proj_dual_cone(yv, prob.cone)
            np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10 * (1 + np.abs(yv).max()))


def _g31(got, ref, u):
    """Relative fixed-point-residual difference at the same input u."""
    return np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-3 * np.linalg.norm(u))


def _parity_at_probes(sscs, prob, probes, label):
    """G31 <= 1e-9 (fixed-point residual at the same input) and the linear
    step within 1e-10 of the oracle's direct solve, on the launch
    configuration the library picks for the instance (the one bench.py times)."""
    import time
    import oracle
    from oracle import superscs as S
    t0 = time.perf_counter()
    lin = oracle.DirectLinSys(prob.A, prob.b, prob.c)
    print(f"{label}: oracle factor ({lin.kind}) {time.perf_counter() - t0:.1f}s", flush=True)
    rr = np.random.default_rng(11)
    with sscs.Solver(prob, sscs.Settings(cg_tol=1e-14, cg_max=5000)) as s:
        for name, u in probes:
            _, _, Ru_ref = S.residual(lin, prob.cone, u)
            _, Ru = s.residual(u)
            e = _g31(Ru, Ru_ref, u)
            print(f"{label} probe {name}: ||Ru|| {np.linalg.norm(Ru_ref):.3e}, G31 {e:.2e}", flush=True)
            assert e <= 1e-9, name
        for k in range(2):
            rhs = rr.standard_normal(prob.n + prob.m + 1)
            ref = lin.L(rhs)
            got = s.linear_step(rhs)
            e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
            print(f"{label} linear step {k}: rel {e:.2e}", flush=True)
            assert e <= 1e-10


def test_socp_20000x50000_parity_at_probe_points(sscs):
    """Sparse SOCP at full size on the operator-in-LDS grid: the cold start,
    a random point, an oracle iterate and a point near the planted fixed point
    (u* = (x*, y* + s*, 1) plus 1e-3 noise)."""
    from oracle import superscs as S
    prob = G.config2_socp()
    N = prob.n + prob.m + 1
    rr = np.random.default_rng(12)
    cold = np.zeros(N); cold[-1] = 1.0
    ustar = np.concatenate([prob.x_star, prob.y_star + prob.s_star, [1.0]])
    it = S.solve(prob, S.Settings(direction="aa", mem=5, max_iters=8), record=False).u
    probes = [("cold", cold), ("random", rr.standard_normal(N)), ("oracle iterate 8", it),
              ("near u*", ustar + 1e-3 * rr.standard_normal(N))]
    _parity_at_probes(sscs, prob, probes, "SOCP 20000x50000")


def test_sdp_exp_parity_at_probe_points(sscs):
    """PSD/exp instance at full size (m = 535113): its order-256 block takes
    the whole-grid block-Jacobi path.  Cold start, a random point and an
    oracle iterate."""
    from oracle import superscs as S
    prob = G.config3_sdp_exp()
    N = prob.n + prob.m + 1
    rr = np.random.default_rng(13)
    cold = np.zeros(N); cold[-1] = 1.0
    it = S.solve(prob, S.Settings(direction="aa", mem=5, max_iters=6), record=False).u
    probes = [("cold", cold), ("random", rr.standard_normal(N)), ("oracle iterate 6", it)]
    _parity_at_probes(sscs, prob, probes, "PSD/exp 349033x535113")


def test_sdp_exp_full_solve_meets_tolerance(sscs):
    """A complete solve of the PSD/exp instance with the benchmark's settings:
    solved, pr/dr/gap <= 1e-6 recomputed on the host from the returned
    (x, y, s), y in K* and s in K (zero rows of s at 0) to 1e-6."""
    import bench
    from oracle.cones import proj_dual_cone, proj_C
    prob = G.config3_sdp_exp()
    st = bench.bench_settings(sscs, 20000)
    st.data_on_device = False
    print("PSD/exp full solve, bench settings", flush=True)
    with sscs.Solver(prob, st) as s:
        x, y, sv, info = s.solve()
    print(f"status {info['status_name']} iters {info['iters']} time {info['solve_s']:.1f}s", flush=True)
    assert info["status"] == sscs.SOLVED
    assert max(_kkt(prob, x, y, sv)) <= 1e-6 * 1.0001
    assert np.linalg.norm(y - proj_dual_cone(y, prob.cone)) <= 1e-6 * (1 + np.linalg.norm(y))
    z = prob.cone.z
    assert np.linalg.norm(sv[:z]) <= 1e-5 * (1 + np.linalg.norm(prob.b))
    # s in K: K is self-dual on R+, SOC and PSD; the exp cone is not, so s is
    # checked there through Moreau (s = Pi_K(s))
    from oracle.cones import proj_exp
    e0 = prob.m - 3 * prob.cone.ep
    s_nz = sv.copy(); s_nz[:z] = 0.0
    s_head = s_nz[:e0]
    cone_head = G.Cone(z=prob.cone.z, l=prob.cone.l, q=prob.cone.q, s=prob.cone.s, ep=0)
    assert np.linalg.norm(s_head - proj_dual_cone(s_head, cone_head)) <= 1e-6 * (1 + np.linalg.norm(sv))
    se = sv[e0:].reshape(-1, 3)
    d = max(np.linalg.norm(v - proj_exp(v)) for v in se)
    assert d <= 1e-6 * (1 + np.linalg.norm(sv))


@pytest.mark.parametrize("m,n,per_row", [(2_000_000, 2000, 10), (5_000_000, 20_000, 20)])
def test_spmv_column_panel_form(sscs, m, n, per_row):
    """The stand-alone SpMV on operators large enough for its column-panel
    form (x panels staged in LDS; A^T of these shapes has 98 and 245 panels
    whose partial sums are added in order), against scipy in FP64: every
    entry within the summation bound 1e-13 of the row's |v| |x| sum."""
    p = G.spmv_scaled(m=m, n=n, per_row=per_row)
    r = np.random.default_rng(m + n)
    print(f"column-panel SpMV {m} x {n}, {p.A.nnz} nonzeros", flush=True)
    with sscs.Solver(p, sscs.Settings(cg_tol=1e-10, cg_max=50)) as s:
        x = r.standard_normal(n)
        got = s.spmv(x)
        ref = p.A @ x
        bound = abs(p.A) @ np.abs(x)
        assert np.all(np.abs(got - ref) <= 1e-13 * bound + 1e-300)
        t = r.standard_normal(m)
        got_t = s.spmv(t, transpose=True)
        ref_t = p.A.T @ t
        bound_t = abs(p.A).T @ np.abs(t)
        assert np.all(np.abs(got_t - ref_t) <= 1e-13 * bound_t + 1e-300)


@pytest.mark.parametrize("m,n,max_per_row", [(1_000_000, 20_000, 40), (4_000_000, 4000, 8)])
def test_spmv_column_panel_ragged_rows(sscs, m, n, max_per_row):
    """The column-panel SpMV on rows of 0..max_per_row entries (empty rows,
    rows shorter and longer than one batch of four lanes' entries): the first
    shape takes the batched row walk on A (one panel) and on A^T (49 panels,
    binomial row lengths per panel), the second the one-step walk with two
    lanes per row on A.  Same bound as the fixed-length case."""
    p = G.spmv_ragged(m, n, max_per_row, seed=m % 97)
    r = np.random.default_rng(m + n + 1)
    print(f"column-panel SpMV, ragged rows, {m} x {n}, {p.A.nnz} nonzeros", flush=True)
    with sscs.Solver(p, sscs.Settings(cg_tol=1e-10, cg_max=50)) as s:
        x = r.standard_normal(n)
        got = s.spmv(x)
        ref = p.A @ x
        bound = abs(p.A) @ np.abs(x)
        assert np.all(np.abs(got - ref) <= 1e-13 * bound + 1e-300)
        empty = np.diff(p.A.indptr) == 0
        assert empty.any() and np.all(got[empty] == 0.0)
        t = r.standard_normal(m)
        got_t = s.spmv(t, transpose=True)
        ref_t = p.A.T @ t
        bound_t = abs(p.A).T @ np.abs(t)
        assert np.all(np.abs(got_t - ref_t) <= 1e-13 * bound_t + 1e-300)
        # the panels' partial sums are added in panel order whatever the
        # launch order: a repeated product is the same bit for bit
        assert np.array_equal(s.spmv(x), got)
        assert np.array_equal(s.spmv(t, transpose=True), got_t)
