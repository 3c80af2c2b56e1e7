"""Seeded inputs for the surrogate initialiser network: initial weights and
minibatch orders (random numbers the training draws are inputs).

Parameter blob order (float32 on the device): for each convolution (5->32,
32->64, 64->64, 64->128; 3x3) the weights [out][in][3][3] then the bias [out];
then the 2048->256 and 256->27 dense layers, weights [out][in] then bias.
"""
import numpy as np

SHAPES = []
for _ci, _co in ((5, 32), (32, 64), (64, 64), (64, 128)):
    SHAPES += [(_co, _ci, 3, 3), (_co,)]
for _fi, _fo in ((2048, 256), (256, 27)):
    SHAPES += [(_fo, _fi), (_fo,)]
N_PARAMS = int(sum(np.prod(s) for s in SHAPES))


def init_params(seed):
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; flat float64."""
    rng = np.random.default_rng(seed)
    out = []
    for s in SHAPES:
        if len(s) == 1:
            out.append(np.zeros(s))
        else:
            fan_in = int(np.prod(s[1:]))
            out.append(rng.normal(0.0, np.sqrt(2.0 / fan_in), s))
    return np.concatenate([a.ravel() for a in out])


def epoch_orders(n, epochs, seed):
    """One random permutation of range(n) per epoch, int32 (epochs, n)."""
    rng = np.random.default_rng(seed)
    return np.stack([rng.permutation(n) for _ in range(epochs)]).astype(np.int32)
