"""GPU tests of the warm-start network kernels, through the C ABI.

Bars: the matrix-core product equals the FP64 product of the BF16-rounded
operands to FP32 accumulation error (|C - C_ref| <= 2^-20 K max|a||b| + 1e-6,
element by element).  Forward outputs, loss and every gradient are compared
with the FP64 reference network twice: (i) with the reference's BF16 operand
model (every product operand rounded to BF16 as the kernels do), where only
FP32 accumulation and the FP32 -> BF16 double rounding of intermediates
differ: relative Frobenius error <= 1e-3 per layer and max entry error <=
2e-3 of the layer's largest entry; (ii) with exact FP64 arithmetic:
cosine >= 0.999 and relative Frobenius error <= 2e-2 per tensor, except where
BF16 operands alone already cost more.  The bound used there is derived, not
chosen: by the triangle inequality ||g - e|| <= ||g - q|| + ||q - e|| for the
GPU gradient g, the BF16 operand model q and the exact e, with ||g - q|| <=
1e-3 ||q|| from bar (i), so rel(g, e) <= rel(q, e) + 2e-3.  rel(q, e) is the
cost of BF16 operands in exact arithmetic; it exceeds 2e-2 only for the first
layer's weight gradient of the two larger networks (3.1e-2 and 3.4e-2), where
ReLU masks of the backward pass flip at pre-activations that BF16 rounding
moves across zero (110 of 131072 entries in the first hidden layer of the
2000-512-512-10005 network: sqrt(110/131072) = 2.9% of the error signal).
u0 assembly is exact in FP64 of the FP32 inputs; a few Adam steps on a fixed
batch lower the loss; a small learned warm start reaches the solver's
tolerance, checked on the host in FP64."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1903_06477_amd import mlp
    from paper_1903_06477_amd import sscs
    sscs.lib()
    return mlp


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()


@pytest.mark.parametrize("shape", [(1, 1, 1), (37, 70, 45), (200, 130, 300), (64, 64, 32), (129, 257, 2000)])
def test_gemm_nt_matches_bf16_product(M, shape):
    from oracle.mlp import bf16_round
    m, n, k = shape
    r = np.random.default_rng(m * 7 + n * 3 + k)
    A = r.standard_normal((m, k)).astype(np.float32)
    B = r.standard_normal((n, k)).astype(np.float32)
    print(f"gemm_nt M={m} N={n} K={k}", flush=True)
    C = M.gemm_nt(_dev(A), _dev(B)).cpu().numpy().astype(np.float64)
    Ar, Br = bf16_round(A), bf16_round(B)
    ref = Ar @ Br.T
    bound = 2.0 ** -20 * k * np.abs(Ar).max() * np.abs(Br).max() + 1e-6
    assert np.max(np.abs(C - ref)) <= bound


def _rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


def _cos(a, b):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-300))


def _close_model(a, b):
    return _rel(a, b) <= 1e-3 and np.max(np.abs(a - b)) <= 2e-3 * np.max(np.abs(b))


def _close_exact(a, b, model):
    """GPU value a against the exact FP64 value b, given the BF16 operand
    model's value: cosine >= 0.999, relative error <= 2e-2 or, where the
    model itself is further from b, <= rel(model, b) + 2e-3."""
    bar = max(2e-2, _rel(model, b) + 2e-3)
    return _rel(a, b) <= bar and _cos(a, b) >= 0.999


@pytest.mark.parametrize("widths,batch", [([20, 33, 17, 9], 50), ([300, 128, 96, 700], 130),
                                          ([2000, 512, 512, 10005], 256)])
def test_forward_and_gradients_match_oracle(M, widths, batch):
    from oracle import mlp as ref
    print(f"mlp widths={widths} batch={batch}", flush=True)
    r = np.random.default_rng(len(widths) * 11 + batch)
    net = M.MLP(widths, max_batch=batch + 5, seed=3)
    Ws = [(r.standard_normal((widths[i + 1], widths[i])) * np.sqrt(2.0 / widths[i])).astype(np.float32)
          for i in range(len(widths) - 1)]
    bs = [(r.standard_normal(widths[i + 1]) * 0.1).astype(np.float32) for i in range(len(widths) - 1)]
    net.set_params(Ws, bs)
    W2, b2 = net.get_params()
    for a, b in zip(Ws + bs, W2 + b2):
        assert np.array_equal(a, b)
    X = r.standard_normal((batch, widths[0])).astype(np.float32)
    T = r.standard_normal((batch, widths[-1])).astype(np.float32)
    Y = net.forward(_dev(X)).cpu().numpy()
    Yq, _ = ref.forward(Ws, bs, X, q=ref.bf16_round)
    Ye, _ = ref.forward(Ws, bs, X)
    assert _close_model(Y, Yq) and _close_exact(Y, Ye, Yq)
    L, dWs, dbs = net.gradients(_dev(X), _dev(T))
    Lq, dWq, dbq = ref.loss_and_grads(Ws, bs, X, T, q=ref.bf16_round)
    Le, dWe, dbe = ref.loss_and_grads(Ws, bs, X, T)
    assert abs(L - Lq) <= 1e-4 * Lq and abs(L - Le) <= 1e-2 * Le
    for l in range(len(Ws)):
        print(f"layer {l}: dW rel vs model {_rel(dWs[l], dWq[l]):.2e}, vs exact {_rel(dWs[l], dWe[l]):.2e} "
              f"(model vs exact {_rel(dWq[l], dWe[l]):.2e}), cos vs exact {_cos(dWs[l], dWe[l]):.6f}; "
              f"db rel vs exact {_rel(dbs[l], dbe[l]):.2e}", flush=True)
        assert _close_model(dWs[l], dWq[l]) and _close_exact(dWs[l], dWe[l], dWq[l]), l
        assert _close_model(dbs[l], dbq[l]) and _close_exact(dbs[l], dbe[l], dbq[l]), l
    net.close()


def test_adam_steps_lower_the_loss(M):
    r = np.random.default_rng(5)
    widths = [40, 64, 64, 10]
    net = M.MLP(widths, max_batch=256, seed=1)
    X = r.standard_normal((256, 40)).astype(np.float32)
    T = np.tanh(X[:, :10] * 0.7 + 0.3 * X[:, 10:20] ** 2).astype(np.float32)
    Xd, Td = _dev(X), _dev(T)
    losses = [net.train_step(Xd, Td, 3e-3) for _ in range(150)]
    assert all(np.isfinite(losses))
    assert losses[-1] < 0.2 * losses[0]
    net.close()


def test_create_is_deterministic_and_rejects_bad_batches(M):
    from paper_1903_06477_amd import sscs as S
    a, b = M.MLP([10, 20, 3], 8, seed=9), M.MLP([10, 20, 3], 8, seed=9)
    c = M.MLP([10, 20, 3], 8, seed=10)
    Wa, _ = a.get_params()
    Wb, _ = b.get_params()
    Wc, _ = c.get_params()
    assert all(np.array_equal(x, y) for x, y in zip(Wa, Wb))
    assert not np.array_equal(Wa[0], Wc[0])
    lim = np.sqrt(1.0 / 10)
    assert np.abs(Wa[0]).max() <= lim and np.abs(Wa[0]).max() > 0.5 * lim
    X = _dev(np.zeros((9, 10)))
    with pytest.raises(S.SSCSError):
        a.forward(X)
    for n in (a, b, c):
        n.close()


def test_assemble_u0_exact(M):
    r = np.random.default_rng(2)
    count, n, m = 5, 7, 11
    P = r.standard_normal((count, n + 2 * m)).astype(np.float32)
    u0 = M.assemble_u0(_dev(P), n, m).cpu().numpy()
    Pd = P.astype(np.float64)
    ref = np.concatenate([Pd[:, :n], Pd[:, n:n + m] + Pd[:, n + m:], np.ones((count, 1))], axis=1)
    assert np.array_equal(u0, ref)


def test_small_learned_warm_start_solves(M):
    """End to end on the LASSO family: solves for training data, a few epochs
    of training, predictions assembled into u0, warm batched solve; every
    warm-solved instance meets the tolerance recomputed on the host, and the
    warm start takes fewer iterations than the cold start on the held-out
    instances.  Against the warm start built from the training targets' mean
    the result is printed, not asserted: at this training size the network
    does not beat it (the full-size comparison is a benchmark leg)."""
    from paper_1903_06477_amd import warmstart as W
    res = W.experiment(ntrain=192, ntest=32, epochs=30, log=lambda s: print(s, flush=True))
    print(f"iterations: cold {res['iters_cold_mean']:.0f}, network warm {res['iters_warm_mean']:.0f}, "
          f"training-mean warm {res['iters_mean_start']:.0f}", flush=True)
    assert res["cold_solved"] == 1.0
    assert res["loss_last"] < res["loss_first"]
    assert res["iters_warm_mean"] < res["iters_cold_mean"]
    # every test instance ends solved: by its warm start, or by the cold fallback
    assert res["final_solved"] == 1.0
    assert res["warm_worst_residual"] <= 1e-6 * 1.0001
