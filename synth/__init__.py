"""Seeded synthetic inputs for the Celeste ELBO / Newton hot path.

This package is the ONLY code shared by the FP64 oracle and the HIP product
path.  It draws catalogs, PSFs, sky levels and Poisson pixels by sampling the
generative model (section III-A; the paper generates its test data the same
way) and holds none of the variational arithmetic: no ELBO, no expectations,
no derivatives, no Kullback-Leibler terms.  Pixels are made by shooting
photons (Poisson count per band, positions drawn from the PSF and the galaxy
prototype mixtures, binned into unit pixels) on top of Poisson sky.
"""
from . import subsample  # noqa: F401
from .generate import (  # noqa: F401
    PRIOR, load_profiles, SynthBatch, SynthField, make_config, make_field, CONFIG_SEED_BASE, N_PARAMS,
)
