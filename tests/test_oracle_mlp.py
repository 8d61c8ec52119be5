"""Pins of the CPU network oracle: its backward pass against central finite
differences of its loss, on a random subset of weights and biases."""
import numpy as np

from oracle import mlp


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(0)
    sizes = [5, 7, 6, 4]
    params = mlp.init_params(sizes, seed=1)
    params = [(W, b + 0.1 * rng.standard_normal(b.shape)) for W, b in params]
    X = rng.standard_normal((9, 5))
    T = rng.standard_normal((9, 4))
    loss, grads = mlp.loss_and_grads(params, X, T)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for _ in range(6):
            i, j = rng.integers(W.shape[0]), rng.integers(W.shape[1])
            Wp = W.copy(); Wp[i, j] += h
            Wm = W.copy(); Wm[i, j] -= h
            lp = mlp.loss_and_grads(params[:li] + [(Wp, b)] + params[li + 1:], X, T)[0]
            lm = mlp.loss_and_grads(params[:li] + [(Wm, b)] + params[li + 1:], X, T)[0]
            assert abs((lp - lm) / (2 * h) - grads[li][0][i, j]) <= 1e-7
        j = rng.integers(b.shape[0])
        bp = b.copy(); bp[j] += h
        bm = b.copy(); bm[j] -= h
        lp = mlp.loss_and_grads(params[:li] + [(W, bp)] + params[li + 1:], X, T)[0]
        lm = mlp.loss_and_grads(params[:li] + [(W, bm)] + params[li + 1:], X, T)[0]
        assert abs((lp - lm) / (2 * h) - grads[li][1][j]) <= 1e-7


def test_loss_is_half_mean_squared_error():
    params = [(np.eye(3), np.zeros(3))]
    X = np.array([[1.0, 2.0, 3.0], [0.0, 0.0, 0.0]])
    T = np.zeros((2, 3))
    loss, _ = mlp.loss_and_grads(params, X, T)
    assert np.isclose(loss, 0.5 * 14.0 / 2)
