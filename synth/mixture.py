"""Seeded synthetic Gaussian-mixture inputs shared by the tests, the oracle checks and the benchmark.

This module only *draws data*; it contains none of the assignment arithmetic.  Both the CPU
oracle and the GPU library are fed from here, so a workload is fully described by
(recipe, seed).

Recipe (the same for every workload):

* ``SeedSequence(seed).spawn(4)`` gives four independent streams:
  [0] component means, [1] component labels, [2] noise / per-component scales,
  [3] sampling (queries, subsamples, k-means++ draws are *not* taken from here).
* mixture weights are uniform over the ``M`` components;
* means ``mu_m ~ N(0, I_d)``;
* a point is ``x = mu_z + sigma_z * eps`` with ``eps ~ N(0, I_d)``;
* ``sigma`` is either a scalar (isotropic) or, for "loguniform", a per-component,
  per-dimension draw from log-uniform[lo, hi];
* ``norm`` is ``"unit"`` (rows L2-normalised), ``"none"``, or ``"lognormal"``
  (direction normalised, then scaled by a norm drawn from lognormal(0, s)).
* with ``groups = G > 0`` the component means cluster: ``mu_m = nu_(m mod G) + spread * mu'_m``
  with group means ``nu_g ~ N(0, I_d)`` from a stream spawned off [0] and ``mu'_m`` the draw
  above (``groups = 0`` leaves the means exactly as before).

Rows are produced in chunks of ``CHUNK`` rows, each chunk from its own spawned child
stream, so any row range can be regenerated without generating the rows before it.
"""
from __future__ import annotations

import dataclasses
import numpy as np

CHUNK = 1 << 20


@dataclasses.dataclass(frozen=True)
class MixtureSpec:
    n: int
    d: int
    components: int
    sigma: object = 0.3            # float (isotropic) or ("loguniform", lo, hi)
    norm: object = "unit"          # "unit" | "none" | ("lognormal", s)
    seed: int = 0
    groups: int = 0                # > 0: component means cluster around this many group means
    group_spread: float = 1.0


def _streams(seed: int):
    return np.random.SeedSequence(seed).spawn(4)


def _component_params(spec: MixtureSpec):
    ss = _streams(spec.seed)
    rng_mu = np.random.Generator(np.random.PCG64(ss[0]))
    mu = rng_mu.standard_normal((spec.components, spec.d))
    if spec.groups > 0:
        rng_nu = np.random.Generator(np.random.PCG64(ss[0].spawn(1)[0]))
        nu = rng_nu.standard_normal((spec.groups, spec.d))
        mu = nu[np.arange(spec.components) % spec.groups] + spec.group_spread * mu
    rng_sig = np.random.Generator(np.random.PCG64(ss[2].spawn(1)[0]))
    if isinstance(spec.sigma, tuple) and spec.sigma[0] == "loguniform":
        lo, hi = float(spec.sigma[1]), float(spec.sigma[2])
        sig = np.exp(rng_sig.uniform(np.log(lo), np.log(hi), size=(spec.components, spec.d)))
    else:
        sig = np.full((spec.components, 1), float(spec.sigma))
    return mu, sig


def _rows(spec: MixtureSpec, mu, sig, lo: int, hi: int, total: int, stream_tag: int) -> np.ndarray:
    """Rows [lo, hi) of a ``total``-row stream selected by ``stream_tag`` (0 = data, 1 = queries).

    Every chunk is always drawn whole, so a row's value does not depend on the range asked for."""
    ss = _streams(spec.seed)
    out = np.empty((hi - lo, spec.d), dtype=np.float32)
    first_chunk, last_chunk = lo // CHUNK, (hi - 1) // CHUNK
    lab_root = ss[1].spawn(2)[stream_tag]
    noise_root = ss[2].spawn(3)[1 + stream_tag]
    nchunks = last_chunk + 1
    lab_children = lab_root.spawn(nchunks)
    noise_children = noise_root.spawn(nchunks)
    for c in range(first_chunk, last_chunk + 1):
        c_lo, c_hi = c * CHUNK, (c + 1) * CHUNK
        rows_in_chunk = min(c_hi, total) - c_lo
        rl = np.random.Generator(np.random.PCG64(lab_children[c]))
        rn = np.random.Generator(np.random.PCG64(noise_children[c]))
        z = rl.integers(0, spec.components, size=rows_in_chunk)
        eps = rn.standard_normal((rows_in_chunk, spec.d))
        block = mu[z] + sig[z] * eps
        if spec.norm == "unit":
            block /= np.linalg.norm(block, axis=1, keepdims=True)
        elif isinstance(spec.norm, tuple) and spec.norm[0] == "lognormal":
            block /= np.linalg.norm(block, axis=1, keepdims=True)
            block *= rn.lognormal(0.0, float(spec.norm[1]), size=(rows_in_chunk, 1))
        s_lo, s_hi = max(lo, c_lo), min(hi, c_lo + rows_in_chunk)
        out[s_lo - lo:s_hi - lo] = block[s_lo - c_lo:s_hi - c_lo]
    return out


def gen_mixture(spec: MixtureSpec, lo: int = 0, hi: int | None = None) -> np.ndarray:
    """Data rows [lo, hi) as a C-contiguous float32 array of shape (hi-lo, d)."""
    hi = spec.n if hi is None else hi
    mu, sig = _component_params(spec)
    return _rows(spec, mu, sig, lo, hi, spec.n, 0)


def gen_queries(spec: MixtureSpec, nq: int) -> np.ndarray:
    """``nq`` query rows from the same mixture, drawn from a stream separate from the data."""
    mu, sig = _component_params(spec)
    return _rows(spec, mu, sig, 0, nq, nq, 1)


def sample_rows(spec: MixtureSpec, count: int, population: int | None = None) -> np.ndarray:
    """A sorted uniform subsample (without replacement) of row ids, from the sampling stream."""
    population = spec.n if population is None else population
    rng = np.random.Generator(np.random.PCG64(_streams(spec.seed)[3]))
    return np.sort(rng.choice(population, size=min(count, population), replace=False))


# The workloads, by what they are.
LOGU = ("loguniform", 0.05, 0.5)
WORKLOADS = {
    "mix64_n20k_d64": dict(spec=MixtureSpec(20_000, 64, 64, 0.3, "unit", 0), K=256, iters=10,
                           lambdas=(1.0,)),
    "mix4096_n1m_d128": dict(spec=MixtureSpec(1_000_000, 128, 4096, LOGU, "unit", 0), K=2000,
                             iters=15, lambdas=(0.0, 0.5, 1.0, 1.5), queries=10_000,
                             check_rows=20_000, cpu_rows=100_000),
    "mix4096g64_n1m_d128": dict(spec=MixtureSpec(1_000_000, 128, 4096, LOGU, "unit", 0, groups=64),
                                K=2000, iters=15, lambdas=(1.0,), queries=10_000,
                                check_rows=20_000, cpu_rows=100_000),
    "mix16384_n10m_d96": dict(spec=MixtureSpec(10_000_000, 96, 16384, LOGU, "unit", 0), K=40_000,
                              iters=10, lambdas=(1.0,), seed_subsample=1_000_000,
                              check_rows=100_000, cpu_rows=10_000),
    "mix8192_n2m_d768_lognorm": dict(spec=MixtureSpec(2_000_000, 768, 8192, LOGU,
                                                      ("lognormal", 0.5), 0),
                                     K=10_000, iters=10, lambdas=(0.5, 1.0, 1.5),
                                     seed_subsample=500_000, check_rows=20_000, cpu_rows=5_000),
}
