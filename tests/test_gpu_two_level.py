"""Two-level VQ probing on the GPU (soar_search_two_level; App. A.4.1, the partition centres
quantized again) against the oracle's search_two_level: the upper probe, the partitions listed
under it and their top t are the same decisions on both sides (FP64 sums in dimension order),
so the probed lists and the results agree; with every upper centroid probed the search is
soar_search's."""
import numpy as np
import pytest

import oracle as O
from synth import MixtureSpec, gen_mixture, gen_queries

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


def _compare(got, want, Qn, Xn):
    """ids equal wherever the oracle's scores are not tied within 1e-12 (relative); scores at the
    GPU's ids equal their exact values; searched counts equal."""
    gi, gs, gn = (a.cpu().numpy() for a in got)
    wi, ws, wn = want
    assert np.array_equal(gn, wn)
    assert np.array_equal(gi < 0, wi < 0)
    ok = gi >= 0
    exact = np.einsum("ij,ikj->ik", Qn.astype(np.float64),
                      Xn[np.where(ok, gi, 0)].astype(np.float64))
    assert np.allclose(gs[ok], exact[ok], rtol=1e-12, atol=1e-12)
    diff = (gi != wi) & ok
    if diff.any():
        assert np.allclose(gs[diff], ws[diff], rtol=1e-12, atol=1e-12), (gi[diff], wi[diff])


def _index(X, C, U, A):
    soar = _soar()
    ua, _ = O.primary_plain(C, U)
    off, ids = soar.build_lists(_ti(A[0]), _ti(A[1]) if len(A) > 1 else None, len(C))
    uoff, uids = soar.build_lists(_ti(ua), None, len(U))
    return ua, off, ids, uoff, uids


@pytest.fixture(scope="module")
def small():
    spec = MixtureSpec(20_000, 64, 64, 0.3, "unit", 31)
    X = gen_mixture(spec)
    Q = gen_queries(spec, 200)
    C, _, _ = O.train_codebook(X, 200, 3, seed=5)
    C = C.astype(np.float32)
    U, _, _ = O.train_codebook(C, 16, 5, seed=6)
    U = U.astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)
    return X, Q, C, U, [p, s]


@pytest.mark.parametrize("t2,t", [(1, 1), (2, 5), (4, 10), (3, 300), (16, 10), (16, 256),
                                  (16, 257)])
def test_matches_oracle(small, t2, t):
    X, Q, C, U, A = small
    ua, off, ids, uoff, uids = _index(X, C, U, A)
    print(f"two-level t2={t2} t={t}", flush=True)
    got = _soar().search_two_level(_t(Q), _t(U), uoff, uids, t2, _t(C), _t(X), off, ids, t, 10)
    _compare(got, O.search_two_level(Q, X, C, U, ua, A, t2, t, 10), Q, X)


def test_full_upper_probe_is_flat_search(small):
    X, Q, C, U, A = small
    soar = _soar()
    ua, off, ids, uoff, uids = _index(X, C, U, A)
    for t in (1, 8, 256, 300):
        got = soar.search_two_level(_t(Q), _t(U), uoff, uids, len(U), _t(C), _t(X), off, ids, t,
                                    10)
        flat = soar.search(_t(Q), _t(C), _t(X), off, ids, t, 10)
        for g, f in zip(got, flat):
            assert np.array_equal(g.cpu().numpy(), f.cpu().numpy())


@pytest.mark.parametrize("K,K2", [(60, 7), (5000, 64)])
def test_integer_ties(K, K2):
    """Integer centroids, upper centroids and queries: upper and lower scores tie exactly and
    often; K = 5000 is beyond what the top-t selection stages in LDS."""
    rng = np.random.default_rng(K + K2)
    n, d = 4000, 6
    C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
    U = rng.integers(-1, 2, size=(K2, d)).astype(np.float32)
    X = (C[rng.integers(0, K, n)] + rng.standard_normal((n, d)) * 0.3).astype(np.float32)
    Q = rng.integers(-2, 3, size=(25, d)).astype(np.float32)
    a0 = rng.integers(0, K, n)
    a1 = (a0 + rng.integers(1, K, n)) % K
    ua, off, ids, uoff, uids = _index(X, C, U, [a0, a1])
    for t2, t in ((1, 3), (2, 40), (5, 300), (K2, 17)):
        print(f"two-level ties K={K} t2={t2} t={t}", flush=True)
        got = _soar().search_two_level(_t(Q), _t(U), uoff, uids, t2, _t(C), _t(X), off, ids, t, 10)
        _compare(got, O.search_two_level(Q, X, C, U, ua, [a0, a1], t2, t, 10), Q, X)


def test_validation(small):
    X, Q, C, U, A = small
    soar = _soar()
    ua, off, ids, uoff, uids = _index(X, C, U, A)
    with pytest.raises(soar.SoarError):
        soar.search_two_level(_t(Q), _t(U), uoff, uids, 2, _t(C), _t(X), off, ids, 4, 17)
    with pytest.raises(soar.SoarError):
        soar.search_two_level(_t(Q), _t(U), uoff, uids, 0, _t(C), _t(X), off, ids, 4, 10)
    rng = np.random.default_rng(3)
    Xb = rng.standard_normal((40, 1040)).astype(np.float32)
    Cb, Ub = Xb[:4].copy(), Xb[:2].copy()
    offb, idsb = soar.build_lists(_ti(np.arange(40) % 4), None, 4)
    uoffb, uidsb = soar.build_lists(_ti(np.array([0, 1, 0, 1])), None, 2)
    with pytest.raises(soar.SoarError) as e:
        soar.search_two_level(_t(Xb[:3]), _t(Ub), uoffb, uidsb, 1, _t(Cb), _t(Xb), offb, idsb, 2,
                              5)
    assert e.value.status == -4
