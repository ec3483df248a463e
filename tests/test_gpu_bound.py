"""The spill bound of the BF16/FP8 forms against the FP64 oracle.

A row whose spill the bound confines to the topk centroids nearest its primary centroid skips the
spill sweep and has those centroids re-scored exactly, so its spill must be exact by the
acceptance rule (conditional on the GPU's primary); its candidates must be the oracle's nearest
centroids of that primary.  The other rows go through the sweep as before.  The inputs here are
small, so the tests ask for the table (SOAR_BOUND_ALWAYS) unless they test the library's own
decision; the benchmark-size tests in test_gpu_lowp.py run that decision.
"""
import numpy as np
import pytest

import oracle as O
from synth import MixtureSpec, gen_mixture

pytestmark = pytest.mark.gpu


def _soar():
    import paper_2404_00774_amd as soar
    return soar


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _run(X, C, lam, prec, topk=0, bound="always"):
    import torch
    soar = _soar()
    n, d = X.shape
    K = len(C)
    ws = torch.empty(soar.assign_workspace_size(n, d, K, lam, prec, topk), dtype=torch.uint8,
                     device="cuda")
    p, s, dp, ls, st = soar.assign(_t(X), _t(C), lam, precision=prec, topk=topk, stats=True,
                                   workspace=ws, bound=bound)
    cp, cs, key = soar.assign_candidates(ws, n, d, K, lam, prec, topk, bound_key=True)
    return (p.cpu().numpy(), s.cpu().numpy(), dp.cpu().numpy(), ls.cpu().numpy(), st,
            cs.cpu().numpy(), key.cpu().numpy())


@pytest.fixture(scope="module")
def clustered():
    # about 2.4 centroids per mixture component and 100 rows per partition, as in the benchmark's
    # n=10M, d=96, K=40,000 workload (16,384 components), scaled down
    X = gen_mixture(MixtureSpec(60000, 96, 250, ("loguniform", 0.05, 0.5), "unit", 3))
    C, _, _ = O.train_codebook(X, 600, 4, seed=0)
    return X, C.astype(np.float32)


@pytest.mark.parametrize("prec,lam", [("bf16", 1.0), ("bf16", 0.5), ("fp8", 1.0), ("bf16", 1.5)])
def test_bounded_rows_are_exact(clustered, prec, lam):
    X, C = clustered
    n, K = len(X), len(C)
    p, s, dp, ls, st, cs, key = _run(X, C, lam, prec)
    bounded = key < 0
    print(prec, lam, "rows bounded", st["rows_bounded"], "of", n, flush=True)
    assert st["rows_bounded"] == int(bounded.sum())
    assert st["rows_bounded"] > 0.4 * n
    assert np.all(p >= 0) and np.all(key[~bounded] == p[~bounded])
    j = O.verify(X, C, lam, p, s, dp, ls)
    assert j["pdist_ok"].all() and j["sloss_ok"].all()
    # bounded rows: exact spill by the acceptance rule, conditional on the GPU's primary
    bad = np.flatnonzero(bounded & ~j["spill_ok"])
    assert bad.size == 0, (bad[:10], s[bad[:10]], j["s_star"][bad[:10]])
    # ... with the oracle's nearest centroids of the primary as candidates (where the oracle's
    # M-th and (M+1)-th distances are apart by more than the FP32 ranking's resolution)
    M = cs.shape[1]
    nb, beyond = O.centroid_neighbours(C, M)
    C64 = C.astype(np.float64)
    rows = np.flatnonzero(bounded)
    for i in rows[:: max(1, len(rows) // 4000)]:
        q = p[i]
        dm = np.sqrt(((C64[q] - C64[nb[q, M - 1]]) ** 2).sum())
        if beyond[q] - dm > 1e-4 * beyond[q]:
            assert set(cs[i]) == set(nb[q]), (i, q, cs[i], nb[q])
    # the whole call stays within the low-precision form's bar
    assert float(j["spill_regret"].mean()) <= 1e-3 and float(j["primary_regret"].mean()) <= 1e-3


def test_bound_matches_the_sweep(clustered):
    # with and without the bound the answers agree wherever both are exact by the rule
    X, C = clustered
    a = _run(X, C, 1.0, "bf16")
    b = _run(X, C, 1.0, "bf16", bound=False)
    assert b[4]["rows_bounded"] == 0 and a[4]["rows_bounded"] > 0
    assert np.array_equal(a[0], b[0])               # the primary does not depend on the bound
    ja = O.verify(X, C, 1.0, a[0], a[1], a[2], a[3])
    jb = O.verify(X, C, 1.0, b[0], b[1], b[2], b[3])
    both = ja["spill_ok"] & jb["spill_ok"]
    gap = np.abs(ja["spill_regret"][both] - jb["spill_regret"][both])
    assert gap.max() <= 1e-6
    # the bound never loses a row the sweep had right
    assert int((~ja["spill_ok"]).sum()) <= int((~jb["spill_ok"]).sum())


def test_short_codebook_every_row_bounded():
    # K - 1 < topk: every other centroid is a candidate of every row, so every spill is exact
    X = gen_mixture(MixtureSpec(4000, 32, 8, 0.3, "unit", 1))
    C = X[np.random.default_rng(0).choice(4000, 5, replace=False)].astype(np.float32)
    p, s, dp, ls, st, cs, key = _run(X, C, 1.0, "bf16")
    assert st["rows_bounded"] == 4000 and np.all(key == -1)
    j = O.verify(X, C, 1.0, p, s, dp, ls)
    assert j["spill_ok"].all() and j["sloss_ok"].all()


@pytest.mark.parametrize("topk", [12, 4])
def test_bound_follows_topk(clustered, topk):
    # the bound serves topk <= 8 only; a smaller topk keeps fewer neighbours and bounds fewer rows
    X, C = clustered
    p, s, dp, ls, st, cs, key = _run(X, C, 1.0, "bf16", topk=topk)
    if topk > 8:
        assert st["rows_bounded"] == 0
    else:
        assert 0 < st["rows_bounded"] < len(X)
        j = O.verify(X, C, 1.0, p, s, dp, ls)
        assert np.all(j["spill_ok"][key < 0])


def test_auto_mode_skips_small_calls(clustered):
    # below 2^40 n K d the library does not build the table on its own
    X, C = clustered
    p, s, dp, ls, st, cs, key = _run(X, C, 1.0, "bf16", bound="auto")
    assert st["rows_bounded"] == 0
    j = O.verify(X, C, 1.0, p, s, dp, ls)
    assert j["pdist_ok"].all() and j["sloss_ok"].all()


def test_conflicting_bound_flags_rejected(clustered):
    import paper_2404_00774_amd as soar
    X, C = clustered
    with pytest.raises(soar.SoarError):
        soar.assign(_t(X[:1000]), _t(C), 1.0, precision="bf16", bound="always",
                    flags=soar.NO_BOUND)
