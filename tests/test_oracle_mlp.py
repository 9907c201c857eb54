"""Pins of the FP64 reference network: gradients against central finite
differences, and a loss that falls under plain gradient descent."""
import numpy as np

from oracle import mlp


def _net(widths, seed=0):
    r = np.random.default_rng(seed)
    Ws = [r.standard_normal((widths[i + 1], widths[i])) * np.sqrt(2.0 / widths[i]) for i in range(len(widths) - 1)]
    bs = [r.standard_normal(widths[i + 1]) * 0.1 for i in range(len(widths) - 1)]
    return Ws, bs


def test_gradients_match_finite_differences():
    widths = [5, 7, 6, 4]
    Ws, bs = _net(widths)
    r = np.random.default_rng(1)
    X = r.standard_normal((9, 5))
    T = r.standard_normal((9, 4))
    L, dWs, dbs = mlp.loss_and_grads(Ws, bs, X, T)
    h = 1e-6
    for l in range(len(Ws)):
        for idx in [(0, 0), (widths[l + 1] - 1, widths[l] - 1), (1, 2 % widths[l])]:
            Wp = [w.copy() for w in Ws]; Wp[l][idx] += h
            Wm = [w.copy() for w in Ws]; Wm[l][idx] -= h
            fd = (mlp.loss_and_grads(Wp, bs, X, T)[0] - mlp.loss_and_grads(Wm, bs, X, T)[0]) / (2 * h)
            assert abs(fd - dWs[l][idx]) <= 1e-7 * (1 + abs(fd))
        for j in [0, widths[l + 1] - 1]:
            bp = [b.copy() for b in bs]; bp[l][j] += h
            bm = [b.copy() for b in bs]; bm[l][j] -= h
            fd = (mlp.loss_and_grads(Ws, bp, X, T)[0] - mlp.loss_and_grads(Ws, bm, X, T)[0]) / (2 * h)
            assert abs(fd - dbs[l][j]) <= 1e-7 * (1 + abs(fd))


def test_gradient_descent_reduces_loss():
    widths = [6, 16, 3]
    Ws, bs = _net(widths, 2)
    r = np.random.default_rng(3)
    X = r.standard_normal((64, 6))
    T = np.tanh(X[:, :3] * 0.5)
    L0 = mlp.loss_and_grads(Ws, bs, X, T)[0]
    for _ in range(200):
        L, dWs, dbs = mlp.loss_and_grads(Ws, bs, X, T)
        Ws = [W - 0.05 * g for W, g in zip(Ws, dWs)]
        bs = [b - 0.05 * g for b, g in zip(bs, dbs)]
    assert L < 0.5 * L0


def test_bf16_rounding():
    vals = np.array([1.0, 1.00390625, 1.005859375, -2.5, 3.0e38], dtype=np.float32)
    out = mlp.bf16_round(vals)
    assert out[0] == 1.0
    assert out[1] == 1.0                       # tie 1 + 2^-8 rounds to even (1.0)
    assert out[2] == 1.0078125                 # above the tie rounds up
    assert out[3] == -2.5


def test_operand_model_is_exact_on_representable_data():
    """Small integers are BF16-exact and so are all products of this
    network (|values| < 256, power-of-two loss scale): the BF16 operand model
    then equals exact arithmetic bit for bit."""
    r = np.random.default_rng(4)
    widths = [6, 5, 4, 4]
    Ws = [r.integers(-1, 2, size=(widths[i + 1], widths[i])).astype(float) for i in range(3)]
    bs = [r.integers(-1, 2, size=widths[i + 1]).astype(float) for i in range(3)]
    X = r.integers(-2, 3, size=(4, 6)).astype(float)
    T = r.integers(-2, 3, size=(4, 4)).astype(float) * 0.5
    e = mlp.loss_and_grads(Ws, bs, X, T)
    q = mlp.loss_and_grads(Ws, bs, X, T, q=mlp.bf16_round)
    assert e[0] == q[0]
    for a, b in zip(e[1] + e[2], q[1] + q[2]):
        assert np.array_equal(a, b)


def test_operand_model_stays_near_exact():
    """BF16 operands (unit roundoff 2^-9) move the gradients of a random
    network by a few units of that roundoff, and the loss by less."""
    widths = [30, 40, 20, 10]
    Ws, bs = _net(widths, 6)
    r = np.random.default_rng(7)
    X = r.standard_normal((64, 30))
    T = r.standard_normal((64, 10))
    Le, dWe, dbe = mlp.loss_and_grads(Ws, bs, X, T)
    Lq, dWq, dbq = mlp.loss_and_grads(Ws, bs, X, T, q=mlp.bf16_round)
    assert abs(Lq - Le) <= 2 ** -8 * Le
    for a, b in zip(dWq + dbq, dWe + dbe):
        assert 0 < np.linalg.norm(a - b) <= 0.05 * np.linalg.norm(b)
