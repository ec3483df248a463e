"""Seeded synthetic inputs (Gaussian mixtures) used by both the oracle checks and the GPU library."""
from .mixture import (MixtureSpec, WORKLOADS, gen_mixture, gen_queries, sample_rows)  # noqa: F401
