"""Random pixel subsamples for the pixel-subsampled ELBO estimator: which 8-row blocks of
each patch image are kept.  Only the random draws live here (seeded); the estimator itself
is computed by the oracle and by the GPU path from these masks."""
import numpy as np

BLOCK_ROWS = 8


def block_masks(img_h, p, seed):
    """Keep each 8-row block of every image independently with probability p.

    Returns (keep, off): keep is uint8 over all blocks of all images (image-major), off[i] the
    index of image i's first block (int64, length n_images + 1)."""
    h = np.asarray(img_h, dtype=np.int64)
    nb = (h + BLOCK_ROWS - 1) // BLOCK_ROWS
    off = np.concatenate([[0], np.cumsum(nb)]).astype(np.int64)
    rng = np.random.default_rng(seed)
    keep = (rng.random(int(off[-1])) < p).astype(np.uint8)
    return keep, off
