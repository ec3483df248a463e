"""GPU query-side probing (inverted lists, MIPS over the codebook, exact re-rank, one count per
spilled point) against the oracle's search() on the same assignments."""
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


def _compare(got, want, Qn, Xn):
    """ids equal wherever the oracle's scores are not tied within 1e-12 (relative); scores at the
    GPU's ids equal their exact values; searched counts equal."""
    gi, gs, gn = (a.cpu().numpy() for a in got)
    wi, ws, wn = want
    assert np.array_equal(gn, wn)
    assert np.array_equal(gi < 0, wi < 0)
    ok = gi >= 0
    exact = np.einsum("ij,ikj->ik", Qn.astype(np.float64), Xn[np.where(ok, gi, 0)].astype(np.float64))
    assert np.allclose(gs[ok], exact[ok], rtol=1e-12, atol=1e-12)
    diff = (gi != wi) & ok
    if diff.any():
        # a different id only where the oracle's ranking has a near-tie at that place
        assert np.allclose(gs[diff], ws[diff], rtol=1e-12, atol=1e-12), (gi[diff], wi[diff])


@pytest.fixture(scope="module")
def setup():
    spec = MixtureSpec(20_000, 64, 64, 0.3, "unit", 17)
    X = gen_mixture(spec)
    Q = gen_queries(spec, 300)
    C, _, _ = O.train_codebook(X, 200, 3, seed=2)
    C = C.astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)       # the lists' assignments come from the oracle too
    import torch
    return (X, Q, C, torch.from_numpy(p.astype(np.int32)).cuda(),
            torch.from_numpy(s.astype(np.int32)).cuda())


def test_lists_are_the_assignments(setup):
    X, Q, C, p, s = setup
    soar = _soar()
    off, ids = soar.build_lists(p, s, len(C))
    off, ids = off.cpu().numpy(), ids.cpu().numpy()
    want = O.partition_lists([p.cpu().numpy(), s.cpu().numpy()], len(C))
    assert off[0] == 0 and off[-1] == 2 * len(X)
    for j in range(len(C)):
        assert np.array_equal(np.sort(ids[off[j]:off[j + 1]]), np.sort(want[j]))


@pytest.mark.parametrize("t", [1, 3, 16, 200, 500])
@pytest.mark.parametrize("spilled", [False, True])
def test_search_matches_oracle(setup, t, spilled):
    X, Q, C, p, s = setup
    soar = _soar()
    off, ids = soar.build_lists(p, s if spilled else None, len(C))
    got = soar.search(_t(Q), _t(C), _t(X), off, ids, t, 10)
    assign = [p.cpu().numpy()] + ([s.cpu().numpy()] if spilled else [])
    want = O.search(Q, X, C, assign, t, 10)
    print(f"t={t} spilled={spilled}: searched {float(want[2].mean()):.0f}", flush=True)
    _compare(got, want, Q, X)


def test_search_ties_and_short_lists():
    """Duplicate centroids tie in the probe (the lower index goes first), a query that reaches
    fewer than k points gets -1 places, and k = 16."""
    rng = np.random.default_rng(4)
    X = rng.standard_normal((90, 8)).astype(np.float32)
    C = rng.standard_normal((12, 8)).astype(np.float32)
    C[7] = C[3]                                   # exact tie in every query's probe
    Q = rng.standard_normal((40, 8)).astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)
    soar = _soar()
    import torch
    pg = torch.from_numpy(p.astype(np.int32)).cuda()
    sg = torch.from_numpy(s.astype(np.int32)).cuda()
    off, ids = soar.build_lists(pg, sg, len(C))
    for t in (1, 2, 5):
        got = soar.search(_t(Q), _t(C), _t(X), off, ids, t, 16)
        _compare(got, O.search(Q, X, C, [p, s], t, 16), Q, X)
    with pytest.raises(soar.SoarError):
        soar.search(_t(Q), _t(C), _t(X), off, ids, 2, 17)


@pytest.mark.parametrize("K", [300, 5000])
def test_probe_selection_ties_and_depths(K):
    """The probe keeps a query's t best partitions in the order of a stable descending sort:
    integer centroids and queries make many exact score ties across the t-th place, on both
    sides of the depth where the selection hands over to the full sort (t = 256), and with more
    centroids than the selection stages in LDS (K = 5000)."""
    rng = np.random.default_rng(K)
    n, d = 6000, 8
    C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
    X = (C[rng.integers(0, K, n)] + rng.standard_normal((n, d)) * 0.3).astype(np.float32)
    Q = rng.integers(-2, 3, size=(30, d)).astype(np.float32)
    a0 = rng.integers(0, K, n)
    a1 = (a0 + rng.integers(1, K, n)) % K
    soar = _soar()
    import torch
    off, ids = soar.build_lists(torch.from_numpy(a0.astype(np.int32)).cuda(),
                                torch.from_numpy(a1.astype(np.int32)).cuda(), K)
    for t in (1, 3, 64, 255, 256, 257, 400):
        print(f"probe selection K={K} t={t}", flush=True)
        got = soar.search(_t(Q), _t(C), _t(X), off, ids, t, 10)
        _compare(got, O.search(Q, X, C, [a0, a1], t, 10), Q, X)
