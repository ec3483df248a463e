"""Further spilled assignments on the GPU (soar_spill_further, Section 3.5.1) against the oracle:
every row's next assignment equals the oracle's, or is a near-tie of it, and the reported loss is
the exact loss at that index."""
import numpy as np
import pytest

import oracle as O
from synth import MixtureSpec, WORKLOADS, gen_mixture, sample_rows

pytestmark = pytest.mark.gpu


def _soar():
    import paper_2404_00774_amd as soar
    return soar


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _ti(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).cuda()


def _run(X, C, P, lam):
    nxt, loss, st = _soar().spill_further(_t(X), _t(C), _ti(P), lam, stats=True)
    return nxt.cpu().numpy(), loss.cpu().numpy(), st


def _check(X, C, lam, P, res):
    j = O.verify_further(X, C, lam, P, res[0], res[1])
    bad = np.flatnonzero(~j["ok"])
    assert bad.size == 0, (bad[:5], res[0][bad[:5]], j["j_star"][bad[:5]], j["regret"][bad[:5]])
    assert j["loss_ok"].all()
    return j


def _random_priors(rng, n, K, m):
    P = np.empty((n, m), np.int64)
    for i in range(n):
        P[i] = rng.choice(K, m, replace=False)
    return P


@pytest.mark.parametrize("n,d,K", [
    (1, 16, 4), (63, 5, 9), (257, 64, 300), (300, 96, 1000), (129, 128, 257),
    # rows above 128 dimensions: chunks of 64 (ragged last chunk, several tiles, one tile)
    (200, 200, 130), (70, 768, 66), (65, 1024, 5), (129, 129, 70),
    # more centroids than the full scan keeps in LDS
    (300, 32, 9000)])
@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("lam", [0.0, 1.0])
def test_edge_shapes(n, d, K, m, lam):
    print(f"further n={n} d={d} K={K} m={m} lam={lam}", flush=True)
    rng = np.random.default_rng(n * 7 + d * 13 + K + m)
    X = rng.standard_normal((n, d)).astype(np.float32)
    C = (rng.standard_normal((K, d)) * 0.7).astype(np.float32)
    A, _ = O.assign_multi(X, C, lam, m)
    _check(X, C, lam, A, _run(X, C, A, lam))


@pytest.mark.parametrize("m", [1, 2, 3])
def test_random_earlier_assignments(m):
    """The loss is defined for any distinct earlier assignments, not only nearest ones."""
    rng = np.random.default_rng(40 + m)
    n, d, K = 3000, 48, 500
    X = gen_mixture(MixtureSpec(n, d, 64, 0.3, "unit", m))
    C = X[rng.choice(n, K, replace=False)] * 0.9
    P = _random_priors(rng, n, K, m)
    for lam in (0.5, 1.5):
        print(f"random priors m={m} lam={lam}", flush=True)
        _check(X, C, lam, P, _run(X, C, P, lam))


def test_one_earlier_assignment_is_the_spill():
    soar = _soar()
    X = gen_mixture(MixtureSpec(20_000, 64, 64, 0.3, "unit", 9))
    C = X[np.random.default_rng(3).choice(len(X), 400, replace=False)].copy()
    for lam in (0.5, 1.0):
        p, s, _, ls = soar.assign(_t(X), _t(C), lam, spill_form="direct")
        nxt, loss = soar.spill_further(_t(X), _t(C), p.reshape(-1, 1), lam)
        assert np.array_equal(nxt.cpu().numpy(), s.cpu().numpy())
        np.testing.assert_allclose(loss.cpu().numpy(), ls.cpu().numpy(), rtol=2e-6, atol=0)


def test_integer_ties_duplicates_and_zero_residuals():
    """Integer data: every loss is exact in the FP64 decision, so the lowest-index arg-min is the
    only answer; duplicate centroids tie exactly and rows on an earlier centroid have r = 0."""
    rng = np.random.default_rng(6)
    n, d, K = 2000, 4, 40
    C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
    C[17] = C[1]
    C[33] = C[5]
    X = rng.integers(-2, 3, size=(n, d)).astype(np.float32)
    for m in (1, 2, 3):
        A, _ = O.assign_multi(X, C, 1.0, m)
        X2 = X.copy()
        X2[:60] = C[A[:60, m - 1]]               # r = 0 for the last earlier assignment
        A2, _ = O.assign_multi(X2, C, 1.0, m)
        for lam in (0.0, 1.0, 1.5):
            print(f"ties m={m} lam={lam}", flush=True)
            res = _run(X2, C, A2, lam)
            j = _check(X2, C, lam, A2, res)
            assert np.array_equal(res[0], j["j_star"])


def test_chain_of_four_assignments_matches_oracle_steps():
    """assign_multi(M = 4) on the GPU against the oracle's own chain (n = 20,000, d = 64,
    K = 256, a Lloyd-trained codebook): each step is checked on the rows whose earlier
    assignments equal the oracle's, and those are nearly all rows (a near-tie may send a row's
    chain elsewhere, which the step checks allow)."""
    soar = _soar()
    w = WORKLOADS["mix64_n20k_d64"]
    X = gen_mixture(w["spec"])
    C, _, _ = O.train_codebook(X, w["K"], 3, seed=0)
    C = C.astype(np.float32)
    for lam in (0.5, 1.0):
        A, V = soar.assign_multi(_t(X), _t(C), lam, 4)
        A, V = A.cpu().numpy(), V.cpu().numpy()
        W, _ = O.assign_multi(X, C, lam, 4)
        assert (np.sort(A, axis=1)[:, 1:] != np.sort(A, axis=1)[:, :-1]).all()
        for k in (2, 3):
            same = (A[:, :k] == W[:, :k]).all(axis=1)
            print(f"chain lam={lam} step {k}: {int(same.sum())} rows share the oracle's priors",
                  flush=True)
            assert same.mean() > 0.99
            rows = np.flatnonzero(same)
            _check(X[rows], C, lam, W[rows, :k], (A[rows, k], V[rows, k]))


def test_validation_and_errors():
    soar = _soar()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((10, 8)).astype(np.float32)
    C = rng.standard_normal((5, 8)).astype(np.float32)
    good = np.tile(np.array([[0, 1]]), (10, 1))
    nxt, _ = soar.spill_further(_t(X), _t(C), _ti(good), 1.0)
    assert ((nxt.cpu().numpy() >= 2) & (nxt.cpu().numpy() < 5)).all()
    for bad in (np.tile(np.array([[0, 5]]), (10, 1)), np.tile(np.array([[2, 2]]), (10, 1)),
                np.tile(np.array([[-1, 2]]), (10, 1))):
        with pytest.raises(soar.SoarError) as e:
            soar.spill_further(_t(X), _t(C), _ti(bad), 1.0)
        assert e.value.status == -1
    with pytest.raises(soar.SoarError):
        soar.spill_further(_t(X), _t(C[:2]), _ti(good), 1.0)          # K must exceed m
    with pytest.raises(soar.SoarError):
        soar.spill_further(_t(X), _t(C), _ti(np.zeros((10, 4))), 1.0)   # m <= 3
    with pytest.raises(soar.SoarError):
        soar.spill_further(_t(X), _t(C), _ti(good), -1.0)
    Xn = X.copy()
    Xn[3, 2] = np.nan
    with pytest.raises(soar.SoarError) as e:
        soar.spill_further(_t(Xn), _t(C), _ti(good), 1.0)
    assert e.value.status == -5


def test_full_size_sampled():
    """n = 1,000,000, d = 128, K = 2000 (the workload the benchmark times this on): the third
    assignment given two distinct earlier assignments per row (seeded; the loss is defined for
    any), the oracle checks 5000 sampled rows."""
    soar = _soar()
    w = WORKLOADS["mix4096_n1m_d128"]
    spec = w["spec"]
    X = gen_mixture(spec)
    C = X[sample_rows(spec, w["K"])]
    rng = np.random.default_rng(12)
    a0 = rng.integers(0, w["K"], len(X))
    a1 = (a0 + rng.integers(1, w["K"], len(X))) % w["K"]
    Pn = np.stack([a0, a1], axis=1)
    nxt, loss, st = soar.spill_further(_t(X), _t(C), _ti(Pn), 1.0, stats=True)
    print("further full size", st, flush=True)
    idx = np.sort(rng.choice(len(X), 5000, replace=False))
    _check(X[idx], C, 1.0, Pn[idx], (nxt.cpu().numpy()[idx], loss.cpu().numpy()[idx]))
    assert st["rows_full_scan"] < 0.02 * len(X)
