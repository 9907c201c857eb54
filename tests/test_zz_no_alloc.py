"""The allocation-free entry point sscs_solve_noalloc against the batched
engine it shares its kernels with (sscs_batch_create + sscs_batch_solve on a
batch of one), through the C ABI: two calls in a row, the second on a smaller
instance (the static scratch keeps the first call's contents), a third back
on a larger one.  Bar: same status and iteration count, x, y, s equal to the
batched result (the same kernels on the same data: bitwise, with 1e-12
relative as the stated floor), and pr, dr, gap <= eps recomputed on the host
in FP64."""
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


def _close(a, b):
    return np.linalg.norm(a - b) <= 1e-12 * max(np.linalg.norm(b), 1e-300)


def test_noalloc_matches_batched_engine(sscs):
    st = sscs.Settings(direction="aa", mem=5, eps=1e-8, cg_tol=1e-12, cg_max=2000, max_iters=20000)
    cases = [("LASSO config-4 instance 0", G.config4_instance(0)), ("LP 300x100", G.config1_lp()),
             ("PSD/exp small", G.small_sdp_exp(0)), ("LASSO config-4 instance 3", G.config4_instance(3))]
    for name, prob in cases:
        print(f"noalloc vs batch of one: {name} n={prob.n} m={prob.m} nnz={prob.A.nnz}", flush=True)
        x, y, s, info = sscs.solve_noalloc(prob, st)
        bs = sscs.BatchSolver([prob], st)
        xb, yb, sb, ib = bs.solve()
        bs.close()
        ib = ib[0]
        bitwise = np.array_equal(x, xb) and np.array_equal(y, yb) and np.array_equal(s, sb)
        print(f"  status {info['status_name']} iters {info['iters']} (batch {ib['iters']}), bitwise {bitwise}",
              flush=True)
        assert info["status"] == ib["status"] == sscs.SOLVED
        assert info["iters"] == ib["iters"]
        assert _close(x, xb) and _close(y, yb) and _close(s, sb)
        assert max(_kkt(prob, x, y, s)) <= st.eps * 1.0001


def test_noalloc_device_buffers_and_warm_start(sscs):
    """data_on_device: u0 and the outputs are device tensors; a warm start at
    the planted optimum stops at iteration 0."""
    import torch
    prob = G.small_socp(3)
    st = sscs.Settings(eps=1e-9, cg_tol=1e-14, data_on_device=True)
    u_star = np.concatenate([prob.x_star, prob.y_star + prob.s_star, [1.0]])
    dev = torch.device("cuda:0")
    out = (torch.empty(prob.n, dtype=torch.float64, device=dev), torch.empty(prob.m, dtype=torch.float64, device=dev),
           torch.empty(prob.m, dtype=torch.float64, device=dev))
    u0 = torch.from_numpy(u_star).to(dev)
    x, y, s, info = sscs.solve_noalloc(prob, st, u0=u0, out=out)
    assert info["status"] == sscs.SOLVED and info["iters"] == 0
    np.testing.assert_allclose(x.cpu().numpy(), prob.x_star, atol=1e-8)
