"""Search over lists with PQ-coded copies on the GPU (soar_lists_codes, soar_search_pq; Section 2.2
search with the Section 3.5 index layout) against the oracle's search_pq.  Every estimate and
exact score is the same FP64 arithmetic in the same order on both sides, so ids, scores and the
counts of estimated copies must be equal, not merely close."""
import numpy as np
import pytest

import oracle as O
from synth import MixtureSpec, WORKLOADS, gen_mixture, gen_queries

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


def _tu8(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint8)).cuda()


def _index(X, C, A, codes):
    """The GPU lists of assignments A (list of arrays) with their copies' packed codes."""
    soar = _soar()
    off, ids = soar.build_lists(_ti(A[0]), _ti(A[1]) if len(A) > 1 else None, len(C))
    lc, mx = soar.list_codes(off, ids, _ti(np.stack(A, axis=1)), _tu8(O.pq_pack(codes)))
    return off, ids, lc, mx


def _run(X, C, A, codes, P, Q, t, R, k):
    soar = _soar()
    off, ids, lc, mx = _index(X, C, A, codes)
    gi, gs, gn = soar.search_pq(_t(Q), _t(C), _t(X), off, ids, lc, _t(P), None, t, R, k)
    return gi.cpu().numpy(), gs.cpu().numpy(), gn.cpu().numpy()


def _check(got, want):
    gi, gs, gn = got
    wi, ws, wn = want
    assert np.array_equal(gn, wn)
    assert np.array_equal(gi, wi), np.argwhere(gi != wi)[:5]
    assert np.array_equal(gs, ws)


@pytest.fixture(scope="module")
def small():
    spec = MixtureSpec(20_000, 64, 64, 0.3, "unit", 21)
    X = gen_mixture(spec)
    Q = gen_queries(spec, 200)
    C, _, _ = O.train_codebook(X, 200, 3, seed=4)
    C = C.astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)
    rng = np.random.default_rng(9)
    P = (rng.standard_normal((32, 16, 2)) * 0.15).astype(np.float32)
    codes = O.soar_pq_codes(X, C, P, [p, s])
    return X, Q, C, [p, s], codes, P


def test_list_codes_follow_the_lists(small):
    X, Q, C, A, codes, P = small
    off, ids, lc, mx = _index(X, C, A, codes)
    off, ids, lc = off.cpu().numpy(), ids.cpu().numpy(), lc.cpu().numpy()
    packed = O.pq_pack(codes)
    assert mx == int(np.diff(off).max())
    for p in range(len(C)):
        for pos in range(off[p], off[p + 1]):
            i = ids[pos]
            j = 0 if A[0][i] == p else 1
            assert A[j][i] == p
            assert np.array_equal(lc[pos], packed[i, j])


@pytest.mark.parametrize("t,R,k", [(1, 10, 10), (3, 40, 10), (8, 100, 16), (40, 200, 5),
                                   (500, 64, 10), (2, 1, 1)])
@pytest.mark.parametrize("spilled", [False, True])
def test_matches_oracle(small, t, R, k, spilled):
    X, Q, C, A, codes, P = small
    A2 = A if spilled else A[:1]
    c2 = codes if spilled else codes[:, :1]
    print(f"search_pq t={t} R={R} k={k} spilled={spilled}", flush=True)
    _check(_run(X, C, A2, c2, P, Q, t, R, k), O.search_pq(Q, X, C, A2, c2, P, t, R, k))


def test_large_rerank_equals_exact_search(small):
    """R at least the points reached: the same answer as the exact search (soar_search)."""
    X, Q, C, A, codes, P = small
    soar = _soar()
    off, ids, lc, mx = _index(X, C, A, codes)
    for t in (1, 4):
        gi, gs, gn = soar.search_pq(_t(Q), _t(C), _t(X), off, ids, lc, _t(P), None, t, 4096, 10)
        ei, es, en = soar.search(_t(Q), _t(C), _t(X), off, ids, t, 10)
        assert int(en.max()) <= 4096
        assert np.array_equal(gi.cpu().numpy(), ei.cpu().numpy())
        assert np.array_equal(gs.cpu().numpy(), es.cpu().numpy())
        assert np.array_equal(gn.cpu().numpy(), en.cpu().numpy())


@pytest.mark.parametrize("d,s", [(36, 2), (40, 2), (48, 1), (64, 4), (128, 8), (32, 16)])
def test_shapes_ties_and_empty_lists(d, s):
    """Code widths with and without whole 4-byte words; integer data (estimates and scores tie
    often and exactly); partitions that list nothing; queries reaching fewer than k points."""
    rng = np.random.default_rng(d + s)
    n, K = 400, 60
    X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
    a0 = rng.integers(0, K // 2, n)                      # the upper half lists nothing
    a1 = (a0 + rng.integers(1, K // 2, n)) % (K // 2)
    P = rng.integers(-2, 3, size=(d // s, 16, s)).astype(np.float32)
    Q = rng.integers(-2, 3, size=(30, d)).astype(np.float32)
    codes = O.soar_pq_codes(X, C, P, [a0, a1])
    for t, R, k in ((1, 16, 16), (2, 5, 4), (7, 30, 10), (K + 5, 50, 16)):
        print(f"shapes d={d} s={s} t={t} R={R} k={k}", flush=True)
        _check(_run(X, C, [a0, a1], codes, P, Q, t, R, k),
               O.search_pq(Q, X, C, [a0, a1], codes, P, t, R, k))


def test_validation(small):
    X, Q, C, A, codes, P = small
    soar = _soar()
    off, ids, lc, mx = _index(X, C, A, codes)
    Qg, Cg, Xg, Pg = _t(Q), _t(C), _t(X), _t(P)
    bound = soar.lists_probe_bound(off, 2)
    lens = np.sort(np.diff(off.cpu().numpy()))[::-1]
    assert bound == int(lens[:2].sum()) and soar.lists_probe_bound(off, 1) == mx
    with pytest.raises(soar.SoarError) as e:
        soar.search_pq(Qg, Cg, Xg, off, ids, lc, Pg, bound, 2, 5, 10)        # R < k
    assert e.value.status == -1
    with pytest.raises(soar.SoarError) as e:
        soar.search_pq(Qg, Cg, Xg, off, ids, lc, Pg, bound - 1, 2, 20, 10)   # two longer lists
    assert e.value.status == -1
    import torch
    raw = torch.empty(lc.numel() + 4, dtype=torch.uint8, device=lc.device)
    mis = raw[1:1 + lc.numel()].view(lc.shape)
    mis.copy_(lc)
    with pytest.raises(soar.SoarError) as e:
        soar.search_pq(Qg, Cg, Xg, off, ids, mis, Pg, bound, 2, 20, 10)    # not 4-byte aligned
    assert e.value.status == -1
    bad_assign = _ti(np.stack([(A[0] + 1) % len(C), A[1]], axis=1))
    with pytest.raises(soar.SoarError) as e:
        soar.list_codes(off, ids, bad_assign, _tu8(O.pq_pack(codes)))
    assert e.value.status == -1
    rng = np.random.default_rng(2)
    Xb = rng.standard_normal((50, 1040)).astype(np.float32)
    Cb = Xb[:4].copy()
    Pb = rng.standard_normal((520, 16, 2)).astype(np.float32)
    offb, idsb = soar.build_lists(_ti(np.arange(50) % 4), None, 4)
    lcb = torch.zeros((50, 260), dtype=torch.uint8, device=offb.device)
    with pytest.raises(soar.SoarError) as e:
        soar.search_pq(_t(Xb[:3]), _t(Cb), _t(Xb), offb, idsb, lcb, _t(Pb), 13, 1, 10, 5)
    assert e.value.status == -4


def test_full_size_sampled():
    """n = 1,000,000, d = 128, K = 2000 (the search workload's sizes, list lengths about 1000):
    seeded assignments and codes (the search is defined for any lists and codes), all 10,000
    queries searched on the GPU, 40 of them checked against the oracle."""
    soar = _soar()
    w = WORKLOADS["mix4096_n1m_d128"]
    spec = w["spec"]
    X = gen_mixture(spec)
    Q = gen_queries(spec, w["queries"])
    rng = np.random.default_rng(77)
    n, d, K = spec.n, spec.d, w["K"]
    C = X[rng.choice(n, K, replace=False)] * np.float32(0.9)
    a0 = rng.integers(0, K, n)
    a1 = (a0 + rng.integers(1, K, n)) % K
    P = (rng.standard_normal((d // 2, 16, 2)) * 0.1).astype(np.float32)
    codes = rng.integers(0, 16, size=(n, 2, d // 2))
    off, ids, lc, mx = _index(X, C, [a0, a1], codes)
    gi, gs, gn = soar.search_pq(_t(Q), _t(C), _t(X), off, ids, lc, _t(P), None, 8, 100, 10)
    gi, gs, gn = gi.cpu().numpy(), gs.cpu().numpy(), gn.cpu().numpy()
    sample = np.sort(np.random.default_rng(5).choice(len(Q), 40, replace=False))
    want = O.search_pq(Q[sample], X, C, [a0, a1], codes, P, 8, 100, 10)
    _check((gi[sample], gs[sample], gn[sample]), want)
    print("full size: copies estimated per query", float(gn.mean()), flush=True)
