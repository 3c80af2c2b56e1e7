"""Pins of the FP64 surrogate-network reference: finite differences of the loss,
pooling and im2col against direct loops (CPU only)."""
import numpy as np

from oracle import cnn
from synth.surrogate import init_params


def test_param_count():
    assert cnn.n_params() == 662235


def test_conv_matches_direct_loops():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(2, 3, 5, 4))
    W = rng.normal(size=(4, 3, 3, 3))
    b = rng.normal(size=4)
    y, _ = cnn.conv_forward(x, W, b)
    ref = np.zeros((2, 4, 5, 4))
    for n in range(2):
        for o in range(4):
            for i in range(5):
                for j in range(4):
                    s = b[o]
                    for c in range(3):
                        for ky in range(3):
                            for kx in range(3):
                                yy, xx = i + ky - 1, j + kx - 1
                                if 0 <= yy < 5 and 0 <= xx < 4:
                                    s += W[o, c, ky, kx] * x[n, c, yy, xx]
                    ref[n, o, i, j] = s
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_pool_backward_routes_to_first_max():
    x = np.array([[[[1.0, 3.0, 2.0, 2.0], [3.0, 0.0, 2.0, 1.0]]]])
    y = cnn.pool_forward(x)
    assert y.tolist() == [[[[3.0, 2.0]]]]
    d = cnn.pool_backward(np.array([[[[5.0, 7.0]]]]), x)
    assert d.tolist() == [[[[0.0, 5.0, 7.0, 0.0], [0.0, 0.0, 0.0, 0.0]]]]


def test_loss_gradient_finite_differences():
    rng = np.random.default_rng(1)
    p = init_params(3)
    x = rng.normal(size=(2, 5, 32, 32))
    t = rng.normal(size=(2, 27))
    loss, g = cnn.loss_and_grad(p, x, t)
    # a sample of coordinates in every layer
    offs = np.cumsum([0] + [int(np.prod(s)) for s in cnn.param_shapes()])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += list(rng.integers(a, b, size=4))
    for i in idx:
        h = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (cnn.loss_and_grad(pp, x, t)[0] - cnn.loss_and_grad(pm, x, t)[0]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.max(np.abs(g))), (i, fd, g[i])
