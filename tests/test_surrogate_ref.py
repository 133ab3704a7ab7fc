"""The FP64 reference surrogate (the judge of the GPU training kernels) checked
against central finite differences of its own loss."""
import numpy as np
import pytest

from castgen import configs
from oracle import surrogate_ref as S


def small_case(seed=0, layers=3, width=8):
    p = configs.hex_cube(n=3, noise_amp=0.0, dirichlet_x0=None)
    N = p["xyz"].shape[0]
    ptr, col = S.graph_mean_operator(p["conn"], N)
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (N, S.N_FEAT))
    t = rng.normal(0, 1, N)
    params = S.init_params(width, layers, seed)
    for k in params:                         # non-zero biases exercise every term
        params[k] = params[k] + rng.normal(0, 0.1, params[k].shape)
    return params, X, t, ptr, col, layers


def test_mean_operator_and_transpose():
    params, X, t, ptr, col, layers = small_case()
    N = ptr.size - 1
    assert np.all(np.diff(ptr) == np.diff(ptr))
    deg = np.diff(ptr)
    assert deg.min() == 7 and deg.max() == 26           # corner and interior nodes of a 3^3 hex grid
    h = np.random.default_rng(1).normal(size=(N, 4))
    g = np.random.default_rng(2).normal(size=(N, 4))
    # <A h, g> = <h, A^T g>
    assert np.sum(S.apply_mean(ptr, col, h) * g) == pytest.approx(np.sum(h * S.apply_mean_T(ptr, col, g)), rel=1e-13)
    ones = np.ones((N, 1))
    assert np.allclose(S.apply_mean(ptr, col, ones), 1.0)


@pytest.mark.parametrize("layers", [1, 3])
def test_gradients_match_central_differences(layers):
    params, X, t, ptr, col, layers = small_case(layers=layers)
    loss, g, _ = S.loss_and_grad(params, X, t, ptr, col, layers)
    rng = np.random.default_rng(3)
    eps = 1e-6
    for name, val in params.items():
        idx = [tuple(rng.integers(0, s) for s in val.shape) for _ in range(4)]
        for ix in idx:
            old = val[ix]
            val[ix] = old + eps
            lp, _, _ = S.loss_and_grad(params, X, t, ptr, col, layers)
            val[ix] = old - eps
            lm, _, _ = S.loss_and_grad(params, X, t, ptr, col, layers)
            val[ix] = old
            fd = (lp - lm) / (2 * eps)
            assert g[name][ix] == pytest.approx(fd, rel=1e-5, abs=1e-9), (name, ix)
