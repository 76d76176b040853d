"""Pins of the FP64 network oracle: backward pass against central finite
differences, and the masked softmax against its definition."""
import numpy as np

from oracle import mlp


def _problem(seed=0, rows=7, d_in=6, width=5, k=4):
    rng = np.random.default_rng(seed)
    p = mlp.init(d_in, width, k, seed=seed)
    p["b1"] = rng.normal(size=width) * 0.1
    p["b2"] = rng.normal(size=width) * 0.1
    p["b3"] = rng.normal(size=k) * 0.1
    X = rng.normal(size=(rows, d_in))
    T = rng.random((rows, k))
    T[:, -1] = -1.0                         # last slot invalid everywhere
    T[0, 1] = -1.0
    for r in range(rows):
        v = T[r] >= 0
        T[r, v] /= T[r, v].sum()
    w = rng.random(rows) + 0.5
    return p, X, T, w


def test_backward_matches_finite_differences():
    p, X, T, w = _problem()
    loss, g, _ = mlp.loss_and_grad(p, X, T, w)
    eps = 1e-6
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        num = np.zeros_like(p[name])
        it = np.nditer(p[name], flags=["multi_index"])
        for _ in it:
            i = it.multi_index
            old = p[name][i]
            p[name][i] = old + eps
            lp, _, _ = mlp.loss_and_grad(p, X, T, w)
            p[name][i] = old - eps
            lm, _, _ = mlp.loss_and_grad(p, X, T, w)
            p[name][i] = old
            num[i] = (lp - lm) / (2 * eps)
        assert np.allclose(g[name], num, rtol=1e-5, atol=1e-7), name


def test_masked_softmax_and_loss_definition():
    p, X, T, w = _problem(seed=1)
    loss, _, P = mlp.loss_and_grad(p, X, T, w)
    Z, _ = mlp.forward(p, X)
    ref = 0.0
    for r in range(X.shape[0]):
        v = T[r] >= 0
        z = Z[r][v]
        q = np.exp(z - z.max()) / np.exp(z - z.max()).sum()
        assert np.allclose(P[r][v], q) and np.all(P[r][~v] == 0)
        ref += w[r] * -(T[r][v] * np.log(q)).sum()
    assert abs(loss - ref) < 1e-12 * max(1.0, abs(ref))


def test_adam_first_steps_closed_form():
    """Adam's bias correction makes the first step lr * g / (|g| + eps) for
    every weight whatever beta1, beta2 (m1 / (1 - b1) = g, v1 / (1 - b2) =
    g^2), and a second step with the same gradient moves by the same amount;
    weight decay adds wd * w to the gradient."""
    rng = np.random.default_rng(3)
    w = rng.standard_normal(50)
    g = rng.standard_normal(50)
    z = np.zeros(50)
    lr, eps = 1e-2, 1e-8
    for b1, b2 in ((0.9, 0.999), (0.5, 0.9)):
        w1, m1, v1 = mlp.adam_step(w, g, z, z, 1, lr=lr, b1=b1, b2=b2, eps=eps)
        assert np.allclose(w1, w - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
        w2, _, _ = mlp.adam_step(w1, g, m1, v1, 2, lr=lr, b1=b1, b2=b2, eps=eps)
        assert np.allclose(w2, w1 - lr * g / (np.abs(g) + eps), rtol=0, atol=1e-14)
    wd = 0.3
    w1, _, _ = mlp.adam_step(w, g, z, z, 1, lr=lr, eps=eps, wd=wd)
    ge = g + wd * w
    assert np.allclose(w1, w - lr * ge / (np.abs(ge) + eps), rtol=0, atol=1e-15)
