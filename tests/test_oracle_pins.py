"""Pins of the CPU oracle to what the paper and the mathematics fix (no GPU needed).

Each test checks the oracle against something other than itself: a value or statement the paper
makes about its worked example, a closed form, exact rational brute force, a library routine, or
an invariant.  A dropped term, a wrong sign, a wrong index or a transposed operand in the oracle
fails at least one of them.
"""
import itertools
import math
import os
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy import special, stats

import oracle as O
from oracle.philox import philox4x32_10, philox_index, philox_uniform24


# ------------------------------------------------------------------------------------------------
# Philox4x32-10: known-answer vectors published with the generator (Random123 distribution).
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("ctr,key,want", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, want):
    assert philox4x32_10(ctr, key) == want


def test_philox_draw_ranges():
    us = [philox_uniform24(7, m) for m in range(2000)]
    assert all(0.0 <= u < 1.0 for u in us)
    assert abs(np.mean(us) - 0.5) < 0.03
    idx = [philox_index(7, m, 13) for m in range(2000)]
    assert set(idx) == set(range(13))


# ------------------------------------------------------------------------------------------------
# W1: Figure 3 (Section 3.3), coordinates as drawn in the paper.
# ------------------------------------------------------------------------------------------------
def _fig3(golden_dir):
    pts = {}
    with open(os.path.join(golden_dir, "fig3_coordinates.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, a, b = line.split()
                pts[name] = (float(a), float(b))
    x = np.array([pts["x"]], dtype=np.float32)
    C = np.array([pts["C1"], pts["C2"], pts["C3"]], dtype=np.float32)
    return x, C


def test_fig3_primary_and_naive_spill(golden_dir):
    x, C = _fig3(golden_dir)
    p, _ = O.primary_plain(x, C)
    assert p[0] == 0                       # the text: pi(x) = 1
    s, _ = O.spill_plain(x, C, 0.0, p)     # lambda = 0 is plain second-nearest (Cor. 3.1.1)
    assert s[0] == 1                       # the text: the naive spill picks C2
    d = np.sum((x.astype(np.float64) - C) ** 2, axis=1)
    assert d[2] > d[1]                     # the text: C3 is farther from x than C2


def test_fig3_collinear_centroid_is_penalised_fully(golden_dir):
    """C2 is collinear with C1 and x, so r' = (1 + eps) r and the projection term is all of
    ||r'||^2: L(C2) = (1 + lambda) ||r'||^2 for every lambda (up to the figure's rounding)."""
    x, C = _fig3(golden_dir)
    r = x[0].astype(np.float64) - C[0]
    rp = x[0].astype(np.float64) - C[1]
    eps = np.linalg.norm(rp) / np.linalg.norm(r) - 1.0
    assert 0.3 < eps < 0.5
    assert np.allclose(rp, (1 + eps) * r, atol=2e-3)
    for lam in (0.0, 0.5, 1.0, 2.0):
        L = O.soar_losses(x[0], C, lam, 0)
        assert L[1] == pytest.approx((1 + lam) * np.dot(rp, rp), rel=1e-5)


def test_fig3_soar_moves_spill_to_c3(golden_dir):
    """The text: pi'(x) = 3 would have been the better spill; SOAR reaches it once lambda is large
    enough, and keeps the naive choice for small lambda."""
    x, C = _fig3(golden_dir)
    picks = {lam: int(O.spill_plain(x, C, lam, np.array([0]))[0][0])
             for lam in (0.0, 0.5, 1.0, 1.5, 2.0, 4.0)}
    assert picks[0.0] == 1 and picks[0.5] == 1
    assert picks[2.0] == 2 and picks[4.0] == 2
    lams = sorted(picks)
    switched = [picks[a] != picks[b] for a, b in zip(lams, lams[1:])]
    assert sum(switched) == 1              # one crossover, never back


# ------------------------------------------------------------------------------------------------
# W2: Corollary 3.1.2 (orthogonal residual unpenalised) and a parallel residual (fully penalised).
# ------------------------------------------------------------------------------------------------
def test_orthogonal_and_parallel_residuals():
    x = np.zeros((1, 2), dtype=np.float32)
    C = np.array([[1.0, 0.0], [0.0, 1.25], [-1.125, 0.0]], dtype=np.float32)
    # r = (-1, 0); r'_1 = (0, -1.25) is orthogonal, r'_2 = (1.125, 0) is parallel to r
    for lam in (0.0, 0.1, 0.5, 1.0, 3.0):
        L = O.soar_losses(x[0], C, lam, 0)
        assert L[1] == 1.5625                        # ||r'||^2, no penalty (Cor. 3.1.2)
        assert L[2] == pytest.approx(1.265625 * (1 + lam), rel=1e-15)   # proj_r r' = r'
        s = O.spill_plain(x, C, lam, np.array([0]))[0][0]
        assert s == (2 if 1.265625 * (1 + lam) < 1.5625 else 1)


# ------------------------------------------------------------------------------------------------
# W3: Corollary 3.1.1 -- lambda = 0 is Euclidean assignment: the spill is the second-nearest.
# ------------------------------------------------------------------------------------------------
def test_lambda_zero_is_second_nearest():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((500, 12)).astype(np.float32)
    C = rng.standard_normal((40, 12)).astype(np.float32)
    D = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    order = np.argsort(D, axis=1, kind="stable")
    p, dp = O.primary_plain(X, C)
    s, ls = O.spill_plain(X, C, 0.0)
    assert np.array_equal(p, order[:, 0])
    assert np.array_equal(s, order[:, 1])
    assert np.allclose(ls, np.take_along_axis(D, order[:, 1:2], 1)[:, 0], rtol=1e-13)


# ------------------------------------------------------------------------------------------------
# W4: exact rational brute force on tiny integer inputs (ties, r = 0, duplicate centroids).
# The projection is formed as a vector, (<r, r'>/<r, r>) r, and then squared -- a different route
# to ||proj_r r'||^2 than the oracle's closed form.
# ------------------------------------------------------------------------------------------------
def _brute(X, C, lam):
    K = len(C)
    out = []
    for x in X:
        d = [sum((Fr(a) - Fr(b)) ** 2 for a, b in zip(x, c)) for c in C]
        p = min(range(K), key=lambda j: (d[j], j))
        r = [Fr(a) - Fr(b) for a, b in zip(x, C[p])]
        rr = sum(v * v for v in r)
        losses = []
        for c in C:
            rp = [Fr(a) - Fr(b) for a, b in zip(x, c)]
            if rr == 0:
                proj_sq = Fr(0)
            else:
                coef = sum(u * v for u, v in zip(r, rp)) / rr
                proj_sq = sum((coef * u) ** 2 for u in r)
            losses.append(sum(v * v for v in rp) + lam * proj_sq)
        s = min((j for j in range(K) if j != p), key=lambda j: (losses[j], j))
        out.append((p, d[p], s, losses))
    return out


@pytest.mark.parametrize("lam", [Fr(0), Fr(1, 2), Fr(1), Fr(3, 2), Fr(3)])
def test_bruteforce_exact_rationals(lam):
    rng = np.random.default_rng(11)
    ties_seen = 0
    for trial in range(150):
        n, K, d = rng.integers(1, 7), rng.integers(2, 6), rng.integers(1, 4)
        X = rng.integers(-2, 3, size=(n, d))
        C = rng.integers(-2, 3, size=(K, d))
        if trial % 5 == 0:
            C[-1] = C[0]                               # duplicate centroid
        if trial % 7 == 0:
            X[0] = C[rng.integers(0, K)]               # r = 0
        ref = _brute(X.tolist(), C.tolist(), lam)
        p, dp = O.primary_plain(X.astype(np.float32), C.astype(np.float32))
        s, ls = O.spill_plain(X.astype(np.float32), C.astype(np.float32), float(lam), p)
        for i, (bp, bd, bs, bl) in enumerate(ref):
            assert p[i] == bp                          # integer distances: FP64 exact
            assert dp[i] == float(bd)
            best = bl[bs]
            assert bl[int(s[i])] == best and s[i] != p[i]
            if sorted(bl[j] for j in range(K) if j != bp)[:2].count(best) > 1:
                ties_seen += 1
            if lam == 0:
                assert s[i] == bs                      # exact: lowest index among equals
            assert ls[i] == pytest.approx(float(best), rel=1e-14, abs=1e-14)
    assert ties_seen > 0


# ------------------------------------------------------------------------------------------------
# W5: Theorem 3.1 by Monte Carlo of Eq. 2 with w(t) = |t|^lambda and q uniform on the sphere.
# The constant of proportionality follows from the moments of one coordinate of a uniform
# point on S^{d-1}: E|t|^a = Gamma(d/2) Gamma((a+1)/2) / (sqrt(pi) Gamma((a+d)/2)).
# ------------------------------------------------------------------------------------------------
def _abs_moment(a, d):
    return math.exp(special.gammaln(d / 2) + special.gammaln((a + 1) / 2)
                    - 0.5 * math.log(math.pi) - special.gammaln((a + d) / 2))


@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5])
def test_theorem_3_1_monte_carlo(lam):
    d = 8
    rng = np.random.default_rng(5)
    r = rng.standard_normal(d)
    rps = [rng.standard_normal(d), 0.3 * r + 0.1 * rng.standard_normal(d),
           np.cross(np.r_[1.0, 0, 0], np.r_[0, 1.0, 0]).tolist() + [0.0] * (d - 3)]
    rps = [np.asarray(v, dtype=np.float64) for v in rps]
    acc = np.zeros(len(rps))
    total = 0
    for _ in range(8):
        q = rng.standard_normal((250_000, d))
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        w = np.abs(q @ r / np.linalg.norm(r)) ** lam
        for k, rp in enumerate(rps):
            acc[k] += np.sum(w * (q @ rp) ** 2)
        total += q.shape[0]
    mc = acc / total
    kappa = (_abs_moment(lam, d) - _abs_moment(lam + 2, d)) / (d - 1)
    # the oracle's loss for residual r (centroid -r of x = 0) and candidate residual r'
    C = np.vstack([-r] + [-rp for rp in rps])
    L = O.soar_losses(np.zeros(d), C, lam, 0)[1:]
    assert np.allclose(mc / L, kappa, rtol=0.012)
    # the parallel moment must equal (1 + lambda) kappa, i.e. lambda enters linearly
    assert _abs_moment(lam + 2, d) == pytest.approx((1 + lam) * kappa, rel=1e-12)


def test_lemma_3_2_correlation():
    d = 10
    rng = np.random.default_rng(9)
    r, rp = rng.standard_normal(d), rng.standard_normal(d)
    q = rng.standard_normal((400_000, d))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    rho = np.corrcoef(q @ r, q @ rp)[0, 1]
    C = np.vstack([-r, -rp])
    pen = O.soar_losses(np.zeros(d), C, 1.0, 0)[1] - O.soar_losses(np.zeros(d), C, 0.0, 0)[1]
    # ||proj_r r'|| = ||r'|| rho
    assert math.sqrt(pen) == pytest.approx(np.linalg.norm(rp) * abs(rho), rel=0.01)


# ------------------------------------------------------------------------------------------------
# Invariants V1-V6
# ------------------------------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rnd_case():
    rng = np.random.default_rng(21)
    X = rng.standard_normal((2000, 16)).astype(np.float32)
    X /= np.linalg.norm(X, axis=1, keepdims=True)
    C = (rng.standard_normal((64, 16)) * 0.3).astype(np.float32)
    return X, C


@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 1.5])
def test_v1_v2_v4_bounds(rnd_case, lam):
    X, C = rnd_case
    p, dp = O.primary_plain(X, C)
    s, ls = O.spill_plain(X, C, lam, p)
    D = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    d2 = np.partition(D, 1, axis=1)[:, 1]
    assert np.all(d2 <= ls * (1 + 1e-12))
    assert np.all(ls <= (1 + lam) * d2 * (1 + 1e-12))
    if lam == 0.0:
        assert np.allclose(ls, d2, rtol=1e-13)
    for i in range(0, 2000, 97):
        L = O.soar_losses(X[i], C, lam, p[i])
        assert L[p[i]] == pytest.approx((1 + lam) * dp[i], rel=1e-12)   # V2


def test_v3_invariances(rnd_case):
    X, C = rnd_case
    lam = 1.0
    p, _ = O.primary_plain(X, C)
    s, ls = O.spill_plain(X, C, lam, p)
    # scaling by 2 is exact: same indices, losses times 4 exactly
    p2, _ = O.primary_plain(2 * X, 2 * C)
    s2, ls2 = O.spill_plain(2 * X, 2 * C, lam, p2)
    assert np.array_equal(p, p2) and np.array_equal(s, s2) and np.array_equal(4 * ls, ls2)
    # permuting centroids permutes the answer
    perm = np.random.default_rng(1).permutation(C.shape[0])
    inv = np.argsort(perm)
    pp, _ = O.primary_plain(X, C[perm])
    sp, lsp = O.spill_plain(X, C[perm], lam, pp)
    assert np.array_equal(perm[pp], p) and np.array_equal(perm[sp], s)
    assert np.allclose(lsp, ls, rtol=1e-12)
    assert np.array_equal(inv[p], pp)
    # rotation and translation (float64 inputs to keep them exact enough)
    Q, _ = np.linalg.qr(np.random.default_rng(2).standard_normal((16, 16)))
    v = np.random.default_rng(4).standard_normal(16)
    for f in (lambda A: A.astype(np.float64) @ Q, lambda A: A.astype(np.float64) + v):
        pr, _ = O.primary_plain(f(X), f(C))
        sr, lsr = O.spill_plain(f(X), f(C), lam, pr)
        assert np.array_equal(pr, p) and np.array_equal(sr, s)
        assert np.allclose(lsr, ls, rtol=1e-9)


def test_v6_lambda_sweep_monotone(rnd_case):
    """Raising lambda can only raise ||r'||^2 and lower cos^2(r, r') (Figure 9's trend, exact per
    point for minimisers of f + lambda g)."""
    X, C = rnd_case
    X64, C64 = X.astype(np.float64), C.astype(np.float64)
    p, _ = O.primary_plain(X, C)
    R = X64 - C64[p]
    prev_sq, prev_cos = None, None
    for lam in (0.0, 0.25, 0.5, 1.0, 1.5, 2.0, 4.0):
        s, _ = O.spill_plain(X, C, lam, p)
        Rp = X64 - C64[s]
        sq = (Rp * Rp).sum(1)
        cos2 = (R * Rp).sum(1) ** 2 / ((R * R).sum(1) * sq)
        if prev_sq is not None:
            assert np.all(sq >= prev_sq - 1e-12)
            assert np.all(cos2 <= prev_cos + 1e-12)
        prev_sq, prev_cos = sq, cos2


def test_fast_equals_plain_bitwise(rnd_case):
    X, C = rnd_case
    for lam in (0.0, 1.0, 1.5):
        a = O.assign(X, C, lam, fast=False)
        b = O.assign(X, C, lam, fast=True)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_fast_equals_plain_small_config():
    """The fast mode against the plain one at the small parity workload's size (n = 20,000,
    d = 64, K = 256, a Lloyd-trained codebook), at every lambda the workload is run with."""
    from synth.mixture import WORKLOADS, gen_mixture
    w = WORKLOADS["mix64_n20k_d64"]
    X = gen_mixture(w["spec"])
    C, _, _ = O.train_codebook(X, w["K"], 3, seed=0)
    for lam in (0.0, 0.5, 1.0, 1.5):
        a = O.assign(X, C, lam, fast=False)
        b = O.assign(X, C, lam, fast=True)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)


def test_fast_screen_under_cancellation():
    """Rows and centroids near a common point far from the origin: the GEMM expansion loses about
    1e-4 to cancellation while the distances differ by about 1e-6, so the expansion alone misranks
    them.  The fast mode must still equal the plain one (its rounding margin keeps every row's
    true arg-min among the directly evaluated candidates); a margin short of the expansion's error
    would fail here."""
    rng = np.random.default_rng(77)
    n, d, K = 1500, 16, 50
    base = np.zeros(d)
    base[0] = 1.0e5
    C = base + 1e-3 * rng.standard_normal((K, d))
    X = base + 1e-3 * rng.standard_normal((n, d))
    # the expansion alone does misrank here
    Dh = (X * X).sum(1)[:, None] - 2.0 * X @ C.T + (C * C).sum(1)[None, :]
    Dd = ((X[:, None, :] - C[None, :, :]) ** 2).sum(-1)
    assert (Dh.argmin(1) != Dd.argmin(1)).mean() > 0.1
    for lam in (0.0, 1.0):
        a = O.assign(X, C, lam, fast=False)
        b = O.assign(X, C, lam, fast=True)
        for u, v in zip(a, b):
            assert np.array_equal(u, v)
    assert np.array_equal(O.assign(X, C, 0.0)[0], Dd.argmin(1))


# ------------------------------------------------------------------------------------------------
# Further spilled assignments (Section 3.5.1; the loss is the reading that adds one Theorem 3.1
# penalty per earlier residual).
# ------------------------------------------------------------------------------------------------
def test_further_lambda_zero_is_mth_nearest():
    """With lambda = 0 every penalty vanishes: the m-th assignment is the m-th nearest centroid
    (stable order, so ties go to the lower index)."""
    rng = np.random.default_rng(31)
    X = rng.integers(-3, 4, size=(400, 5)).astype(np.float32)
    C = rng.integers(-3, 4, size=(30, 5)).astype(np.float32)
    D = ((X[:, None, :].astype(np.float64) - C[None].astype(np.float64)) ** 2).sum(-1)
    order = np.argsort(D, axis=1, kind="stable")
    for fast in (False, True):
        A, V = O.assign_multi(X, C, 0.0, 4, fast=fast)
        assert np.array_equal(A, order[:, :4])
        assert np.array_equal(V, np.take_along_axis(D, order[:, :4], 1))


def test_further_with_one_prior_is_the_soar_spill():
    rng = np.random.default_rng(32)
    X = rng.standard_normal((500, 12)).astype(np.float32)
    C = rng.standard_normal((60, 12)).astype(np.float32)
    p, _ = O.primary_plain(X, C)
    for lam in (0.5, 1.0, 2.0):
        s, ls = O.spill_plain(X, C, lam, p)
        j, lj = O.spill_further_plain(X, C, lam, p[:, None])
        assert np.array_equal(s, j) and np.array_equal(ls, lj)


def test_further_orthogonal_priors_closed_form():
    """x = 0 with earlier residuals r_0 = (1, 0, 0) and r_1 = (0, 2, 0), orthogonal.  A candidate
    residual orthogonal to both is not penalised; one inside their span is penalised by all of
    its length (the two projections add up to ||r'||^2), so its loss is (1 + lambda) ||r'||^2."""
    x = np.zeros((1, 3), np.float32)
    C = np.array([[-1, 0, 0], [0, -2, 0], [0, 0, -1.5], [-0.75, -0.5, 0], [-1.25, 0, 0],
                  [-0.5, 0, -1.0]], np.float32)
    for lam in (0.0, 0.25, 1.0, 3.0):
        L = O.further_losses(x[0], C, lam, [0, 1])
        assert L[2] == 2.25
        assert L[3] == pytest.approx((1 + lam) * 13 / 16, rel=1e-15)
        assert L[4] == pytest.approx((1 + lam) * 1.5625, rel=1e-15)
        assert L[5] == pytest.approx(1.25 + lam * 0.25, rel=1e-15)     # only r_0 sees it
        j, lj = O.spill_further_plain(x, C, lam, np.array([[0, 1]]))
        want = min(range(2, 6), key=lambda k: (L[k], k))
        assert j[0] == want and lj[0] == L[want]


def _brute_further(x, C, lam, prior):
    """Exact rationals; each projection formed as the vector (<r_k, r'>/<r_k, r_k>) r_k and then
    squared."""
    res = [[Fr(a) - Fr(b) for a, b in zip(x, C[k])] for k in prior]
    rrs = [sum(v * v for v in r) for r in res]
    losses = []
    for c in C:
        rp = [Fr(a) - Fr(b) for a, b in zip(x, c)]
        total = sum(v * v for v in rp)
        for r, rr in zip(res, rrs):
            if rr != 0:
                coef = sum(u * v for u, v in zip(r, rp)) / rr
                total += lam * sum((coef * u) ** 2 for u in r)
        losses.append(total)
    j = min((k for k in range(len(C)) if k not in prior), key=lambda k: (losses[k], k))
    return j, losses[j]


@pytest.mark.parametrize("lam", [Fr(0), Fr(1, 2), Fr(1), Fr(5, 2)])
def test_further_bruteforce_exact_rationals(lam):
    rng = np.random.default_rng(33)
    for trial in range(120):
        m = int(rng.integers(1, 4))
        K, d = int(rng.integers(m + 1, m + 5)), int(rng.integers(1, 4))
        X = rng.integers(-2, 3, size=(3, d))
        C = rng.integers(-2, 3, size=(K, d))
        if trial % 4 == 0:
            C[-1] = C[0]                              # duplicate centroid
        P = np.stack([rng.permutation(K)[:m] for _ in range(3)])
        if trial % 5 == 0:
            X[0] = C[P[0, 0]]                         # an earlier residual of zero
        j, l = O.spill_further_plain(X.astype(np.float32), C.astype(np.float32), float(lam), P)
        for i in range(3):
            bj, bl = _brute_further(X[i], C, lam, list(P[i]))
            assert j[i] == bj, (trial, i)
            assert l[i] == pytest.approx(float(bl), rel=1e-14, abs=1e-14)


def test_further_symmetric_in_prior_order_and_fast_equals_plain():
    rng = np.random.default_rng(34)
    X = rng.standard_normal((800, 10)).astype(np.float32)
    C = rng.standard_normal((90, 10)).astype(np.float32)
    A, _ = O.assign_multi(X, C, 1.0, 3)
    P = A[:, :3]
    for lam in (0.5, 1.5):
        j0, l0 = O.spill_further_plain(X, C, lam, P)
        j1, l1 = O.spill_further_plain(X, C, lam, P[:, ::-1])
        assert np.array_equal(j0, j1) and np.allclose(l0, l1, rtol=1e-14, atol=0)
        jf, lf = O.spill_further_fast(X, C, lam, P)
        assert np.array_equal(j0, jf) and np.array_equal(l0, lf)
    with pytest.raises(ValueError):
        O.spill_further_plain(X[:2], C, 1.0, np.array([[1, 1], [2, 3]]))
    with pytest.raises(ValueError):
        O.spill_further_plain(X[:1], C[:2], 1.0, np.array([[0, 1]]))


# ------------------------------------------------------------------------------------------------
# PQ residual codes and the memory model (Section 3.5, implementation considerations).
# ------------------------------------------------------------------------------------------------
def test_pq_encode_bruteforce_exact():
    """Exact rational distances per subspace; ties go to the lowest codeword index."""
    rng = np.random.default_rng(41)
    for trial in range(60):
        M, h, s = int(rng.integers(1, 4)), int(rng.integers(2, 6)), int(rng.integers(1, 4))
        P = rng.integers(-2, 3, size=(M, h, s))
        if trial % 3 == 0:
            P[:, -1] = P[:, 0]                         # duplicate codewords: ties
        R = rng.integers(-3, 4, size=(7, M * s))
        codes = O.pq_encode(R.astype(np.float32), P.astype(np.float32))
        for i in range(7):
            for m in range(M):
                d2 = [sum((Fr(int(R[i, m * s + t])) - Fr(int(P[m, k, t]))) ** 2 for t in range(s))
                      for k in range(h)]
                want = min(range(h), key=lambda k: (d2[k], k))
                assert codes[i, m] == want, (trial, i, m)


def test_soar_pq_codes_encode_each_assignments_residual():
    """Each assignment's code is the code of x - c_a (integer data: exact), so a point's primary
    and spilled copies carry different codes of different residuals."""
    rng = np.random.default_rng(43)
    X = rng.integers(-4, 5, size=(40, 6)).astype(np.float32)
    C = rng.integers(-4, 5, size=(9, 6)).astype(np.float32)
    P = rng.integers(-3, 4, size=(3, 16, 2)).astype(np.float32)
    a0, a1 = rng.integers(0, 9, 40), rng.integers(0, 9, 40)
    codes = O.soar_pq_codes(X, C, P, [a0, a1])
    assert codes.shape == (40, 2, 3)
    for i in range(40):
        for j, a in enumerate((a0, a1)):
            r = X[i].astype(np.int64) - C[a[i]].astype(np.int64)
            for m in range(3):
                d2 = [int(((r[2 * m:2 * m + 2] - P[m, k].astype(np.int64)) ** 2).sum())
                      for k in range(16)]
                assert codes[i, j, m] == min(range(16), key=lambda k: (d2[k], k))


def test_pq_decode_encode_round_trip_and_optimality():
    rng = np.random.default_rng(42)
    M, h, s, n = 8, 16, 4, 300
    P = rng.standard_normal((M, h, s))
    codes = rng.integers(0, h, size=(n, M))
    Y = O.pq_decode(codes, P)
    assert Y.shape == (n, M * s)
    assert np.array_equal(O.pq_encode(Y, P), codes)      # a codeword encodes to itself
    R = rng.standard_normal((n, M * s))
    c = O.pq_encode(R, P)
    err = ((R - O.pq_decode(c, P)) ** 2).reshape(n, M, s).sum(-1)
    for k in range(h):                                   # no other codeword is closer
        other = ((R.reshape(n, M, s) - P[None, :, k, :]) ** 2).sum(-1)
        assert (err <= other + 1e-12).all()
    packed = O.pq_pack(c)
    assert packed.shape == (n, M // 2)
    assert np.array_equal(packed & 15, c[:, 0::2]) and np.array_equal(packed >> 4, c[:, 1::2])


def test_spill_memory_model():
    """The relative growth is (4 + d/(2s)) / (b d + 4 + d/(2s)); for large d it tends to
    1/(2s + 1) with int8 and 1/(8s + 1) with float32 copies (Section 3.5), and the float32 case
    with s = 2 gives the paper's 1/17 estimate for its Glove index."""
    for s_ in (1, 2, 4):
        assert O.spill_memory_overhead(10 ** 7, s_, 1) == pytest.approx(1 / (2 * s_ + 1), rel=1e-5)
        assert O.spill_memory_overhead(10 ** 7, s_, 4) == pytest.approx(1 / (8 * s_ + 1), rel=1e-5)
    assert O.spill_memory_overhead(10 ** 7, 2, 4) == pytest.approx(1 / 17, rel=1e-5)
    d, s_ = 128, 2
    extra = Fr(4) + Fr(d, 2 * s_)
    assert O.spill_memory_overhead(d, s_, 4) == pytest.approx(float(extra / (4 * d + extra)),
                                                              rel=1e-15)
    one = O.index_bytes(1000, d, s_, 1, 4)
    two = O.index_bytes(1000, d, s_, 2, 4)
    assert two - one == 1000 * float(extra)
    assert (two - one) / one == pytest.approx(O.spill_memory_overhead(d, s_, 4), rel=1e-15)


def test_input_validation():
    X = np.zeros((3, 2), np.float32)
    with pytest.raises(ValueError):
        O.spill_plain(X, np.zeros((1, 2), np.float32), 1.0)
    with pytest.raises(ValueError):
        O.spill_plain(X, np.zeros((2, 2), np.float32), -0.5)
    with pytest.raises(ValueError):
        O.spill_fast(X, np.zeros((2, 2), np.float32), float("nan"))


# ------------------------------------------------------------------------------------------------
# KMR (Eq. 1) and Rank (Section 2.1)
# ------------------------------------------------------------------------------------------------
def test_rank_and_kmr_bruteforce():
    rng = np.random.default_rng(13)
    Q = rng.integers(-2, 3, size=(6, 3)).astype(np.float64)
    X = rng.integers(-2, 3, size=(25, 3)).astype(np.float32)
    C = rng.integers(-2, 3, size=(5, 3)).astype(np.float32)
    ranks = O.partition_ranks(Q, C)
    for i, q in enumerate(Q):
        for j, c in enumerate(C):
            want = sum(1 for c2 in C if float(np.dot(q, c)) <= float(np.dot(q, c2)))
            assert ranks[i, j] == want
    k = 3
    gt = O.mips_topk(Q, X, k)
    for i, q in enumerate(Q):
        want = sorted(range(len(X)), key=lambda v: (-float(np.dot(q, X[v])), v))[:k]
        assert list(gt[i]) == want
    p, _ = O.primary_plain(X, C)
    s, _ = O.spill_plain(X, C, 1.0, p)
    ts = list(range(0, 6))
    kmr1, searched1 = O.kmr_curve(Q, X, C, [p], k, ts, gt)
    kmr2, searched2 = O.kmr_curve(Q, X, C, [p, s], k, ts, gt)
    for t, v in zip(ts, kmr1):
        want = np.mean([[ranks[i, p[vv]] <= t for vv in gt[i]] for i in range(len(Q))])
        assert v == pytest.approx(want)
    assert kmr1[0] == 0.0 and kmr1[-1] == 1.0 and np.all(np.diff(kmr1) >= 0)
    assert np.all(kmr2 >= kmr1)                        # V7
    assert searched2[-1] == 2 * len(X) and searched1[-1] == len(X)


# ------------------------------------------------------------------------------------------------
# Lloyd iterations and k-means++ seeding
# ------------------------------------------------------------------------------------------------
def test_lloyd_textbook_1d():
    X = np.array([[0.0], [1.0], [10.0], [11.0]], dtype=np.float32)
    C = np.array([[0.0], [1.0]])
    lab, _, C1, counts, _ = O.lloyd_step(X, C, fast=False)
    assert list(lab) == [0, 1, 1, 1] and list(counts) == [1, 3]
    assert C1[0, 0] == 0.0 and C1[1, 0] == pytest.approx(22 / 3, rel=1e-15)
    _, _, C2, _, _ = O.lloyd_step(X, C1, fast=False)
    assert list(C2[:, 0]) == [0.5, 10.5]


def test_lloyd_update_group_means_and_empty():
    rng = np.random.default_rng(2)
    X = rng.standard_normal((300, 5)).astype(np.float32)
    lab = rng.integers(0, 7, size=300)
    lab[lab == 3] = 4                                   # cluster 3 empty
    Cp = rng.standard_normal((7, 5))
    C, counts = O.lloyd_update(X, lab, Cp)
    for j in range(7):
        rows = [X[i].astype(np.float64) for i in range(300) if lab[i] == j]
        if rows:
            assert np.allclose(C[j], np.mean(rows, axis=0), rtol=1e-14, atol=1e-15)
        else:
            assert np.array_equal(C[j], Cp[j])
    assert counts[3] == 0
    # K = 1 gives the global mean
    C1, _ = O.lloyd_update(X, np.zeros(300, int), np.zeros((1, 5)))
    assert np.allclose(C1[0], X.astype(np.float64).mean(0), rtol=1e-13)


def test_lloyd_inertia_non_increasing():
    from synth import MixtureSpec, gen_mixture
    X = gen_mixture(MixtureSpec(3000, 8, 10, 0.3, "unit", 4))
    _, _, inertia = O.train_codebook(X, 16, 8, seed=3)
    assert all(b <= a * (1 + 1e-12) for a, b in zip(inertia, inertia[1:]))


def test_kmeanspp_frequencies_chi2():
    X = np.array([[0, 0], [1, 0], [0, 2], [3, 0], [0, -1]], dtype=np.float32)
    X64 = X.astype(np.float64)
    n, N = len(X), 6000
    first = np.zeros(n)
    pair = np.zeros((n, n))
    for seed in range(N):
        _, rows = O.kmeanspp(X, 2, seed)
        first[rows[0]] += 1
        pair[rows[0], rows[1]] += 1
    assert stats.chisquare(first).pvalue > 1e-3
    for f in range(n):
        D2 = ((X64 - X64[f]) ** 2).sum(1)
        prob = D2 / D2.sum()
        obs = pair[f]
        mask = prob > 0
        assert obs[~mask].sum() == 0                    # never re-pick a chosen row
        expct = prob[mask] * obs.sum()
        assert stats.chisquare(obs[mask], expct).pvalue > 1e-3


def test_dsq_sample_half_open_intervals():
    # rows own [prefix_{i-1}, prefix_i); zero-width rows (already chosen) are never drawn
    D2 = np.array([0.0, 1.0, 0.0, 1.0])
    assert O.dsq_sample(D2, 0.0) == 1
    assert O.dsq_sample(D2, 0.5) == 3          # target 1.0 sits on the boundary after row 1
    assert O.dsq_sample(D2, 0.5 - 2 ** -24) == 1
    assert O.dsq_sample(np.zeros(3), 0.3) == -1


def test_kmeanspp_distinct_and_degenerate():
    rng = np.random.default_rng(0)
    X = rng.standard_normal((200, 4)).astype(np.float32)
    _, rows = O.kmeanspp(X, 50, 123)
    assert len(set(rows.tolist())) == 50
    Xd = np.ones((6, 3), np.float32)                   # sum D^2 = 0 after the first pick
    _, rows = O.kmeanspp(Xd, 4, 5)
    rest = [i for i in range(6) if i != rows[0]][:3]
    assert list(rows[1:]) == rest


def test_verify_accepts_oracle_and_rejects_wrong(rnd_case):
    X, C = rnd_case
    p, dp, s, ls = O.assign(X, C, 1.0)
    j = O.verify(X, C, 1.0, p, s, dp, ls)
    assert j["all_ok"]
    bad = s.copy()
    bad[5] = p[5]                                      # the primary is never a valid spill
    bad[6] = (s[6] + 1) % C.shape[0] if (s[6] + 1) % C.shape[0] != p[6] else (s[6] + 2) % C.shape[0]
    j = O.verify(X, C, 1.0, p, bad, dp, ls)
    assert not j["spill_ok"][5] and not j["spill_ok"][6] and j["spill_ok"].sum() == len(X) - 2


def test_verify_with_reference_equals_plain_verify():
    """verify() with a precomputed reference gives the same judgement as without it, also for
    rows whose (perturbed) primary differs from the oracle's."""
    rng = np.random.default_rng(5)
    X = rng.standard_normal((400, 12)).astype(np.float32)
    C = rng.standard_normal((30, 12)).astype(np.float32)
    lam = 1.0
    ref = O.reference(X, C, lam)
    p = ref["p_star"].copy()
    s = ref["s_given_p_star"].copy()
    p[::7] = (p[::7] + 1) % len(C)          # wrong primaries on some rows
    s[::11] = (s[::11] + 3) % len(C)        # wrong spills on others
    s[s == p] = (s[s == p] + 1) % len(C)
    a = O.verify(X, C, lam, p, s)
    b = O.verify(X, C, lam, p, s, ref=ref)
    for k in ("primary_ok", "spill_ok", "primary_regret", "spill_regret", "s_star", "l_star"):
        assert np.array_equal(a[k], b[k]), k
    assert a["all_ok"] == b["all_ok"] and not a["all_ok"]


# ---- query-side probing (Section 2.2 search over the spilled lists) ----

def test_search_with_every_partition_is_brute_force_mips():
    """Probing all K partitions scores every point: the result is the exact MIPS top-k."""
    rng = np.random.default_rng(31)
    X = rng.standard_normal((400, 6)).astype(np.float32)
    C = rng.standard_normal((12, 6)).astype(np.float32)
    Q = rng.standard_normal((25, 6)).astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)
    ids, scores, searched = O.search(Q, X, C, [p, s], len(C), 10)
    assert np.array_equal(ids, O.mips_topk(Q, X, 10))
    assert np.all(searched == 2 * len(X))          # every point through both of its lists
    assert np.allclose(scores, np.take_along_axis(Q.astype(np.float64) @ X.T.astype(np.float64),
                                                  ids, axis=1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("t", [1, 2, 5])
def test_search_recall_is_kmr(t):
    """Every true neighbour in a probed list survives the exact re-rank, so the recall of the
    search at depth t is the KMR curve of Eq. 1 at t (a neighbour counts if either of its
    partitions ranks within t), and the points scored are the summed sizes of the probed lists:
    two routes, one through the lists, one through the ranks."""
    rng = np.random.default_rng(32 + t)
    X = rng.standard_normal((600, 8)).astype(np.float32)
    C = rng.standard_normal((30, 8)).astype(np.float32)
    Q = rng.standard_normal((40, 8)).astype(np.float32)
    p, _, s, _ = O.assign(X, C, 1.0)
    gt = O.mips_topk(Q, X, 10)
    for assign in ([p], [p, s]):
        ids, _, searched = O.search(Q, X, C, assign, t, 10)
        kmr, pts = O.kmr_curve(Q, X, C, assign, 10, [t], gt=gt)
        recall = np.mean([len(set(a) & set(b)) / 10 for a, b in zip(ids, gt)])
        assert abs(recall - kmr[0]) < 1e-12
        assert abs(searched.mean() - pts[0]) < 1e-9


def test_search_hand_example():
    """Two partitions on a line; the query probes only the better one, and the spilled copy of
    point 2 makes it reachable from there, listed once."""
    C = np.array([[1.0, 0.0], [-1.0, 0.0]], np.float32)
    X = np.array([[2.0, 0.0], [-2.0, 0.0], [0.1, 0.0], [-0.1, 0.0]], np.float32)
    primary = np.array([0, 1, 0, 1])
    spill = np.array([1, 0, 1, 0])
    Q = np.array([[1.0, 0.0]], np.float32)
    ids, scores, searched = O.search(Q, X, C, [primary], 1, 3)
    assert ids.tolist() == [[0, 2, -1]] and searched.tolist() == [2]
    ids, scores, searched = O.search(Q, X, C, [primary, spill], 1, 3)
    # partition 0 now lists 0, 2 (primary) and 1, 3 (spilled): the best three by <q, x>
    assert ids.tolist() == [[0, 2, 3]] and searched.tolist() == [4]
    assert scores.tolist() == [[2.0, np.float32(0.1).item(), np.float32(-0.1).item()]]


# ------------------------------------------------------------------------------------------------
# Search over PQ-coded lists (Section 2.2 search with the Section 3.5 index layout)
# ------------------------------------------------------------------------------------------------
def test_ordered_sums_exact_on_integers():
    """seq_dot, probe_partitions_seq and pq_lut against exact integer arithmetic; the ADC
    identity: the centre's score plus the LUT entries of a code is <q, c + decode(code)>."""
    rng = np.random.default_rng(61)
    A = rng.integers(-5, 6, size=(7, 10))
    B = rng.integers(-5, 6, size=(9, 10))
    S = O.seq_dot(A.astype(np.float32), B.astype(np.float32))
    for i in range(7):
        for j in range(9):
            assert S[i, j] == sum(int(A[i, u]) * int(B[j, u]) for u in range(10))
    parts, ps = O.probe_partitions_seq(A.astype(np.float32), B.astype(np.float32), 4)
    for i in range(7):
        want = sorted(range(9), key=lambda j: (-int(A[i] @ B[j]), j))[:4]
        assert parts[i].tolist() == want
        assert ps[i].tolist() == [float(A[i] @ B[j]) for j in want]
    P = rng.integers(-3, 4, size=(5, 16, 2))
    q = A[0]
    L = O.pq_lut(q.astype(np.float32), P.astype(np.float32))
    for m in range(5):
        for k in range(16):
            assert L[m, k] == int(q[2 * m:2 * m + 2] @ P[m, k])
    codes = rng.integers(0, 16, size=(30, 5))
    c = B[3]
    a = O.pq_scores(float(q @ c), L, codes)
    dec = O.pq_decode(codes, P.astype(np.float64))
    assert np.array_equal(a, (dec + c) @ q)


def _search_pq_brute(Q, X, C, A, codes, P, t, R, k):
    """Exact rationals on integer data, straight from the description."""
    out_i, out_s = [], []
    K, M = len(C), P.shape[0]
    s = P.shape[2]
    for q in Q:
        qf = [Fr(int(v)) for v in q]
        dot = lambda v: sum(a * Fr(int(b)) for a, b in zip(qf, v))
        probe = sorted(range(K), key=lambda j: (-dot(C[j]), j))[:t]
        best = {}
        for p in probe:
            for j, a in enumerate(A):
                for i in np.flatnonzero(np.asarray(a) == p).tolist():
                    r_hat = [int(P[m, codes[i, j, m], u]) for m in range(M) for u in range(s)]
                    v = dot(C[p]) + dot(r_hat)
                    best[i] = max(best.get(i, v), v)
        keep = sorted(best, key=lambda i: (-best[i], i))[:R]
        top = sorted(keep, key=lambda i: (-dot(X[i]), i))[:k]
        out_i.append(top + [-1] * (k - len(top)))
        out_s.append([float(dot(X[i])) for i in top] + [-np.inf] * (k - len(top)))
    return np.array(out_i), np.array(out_s)


def test_search_pq_brute_force():
    """Integer data (every FP64 sum exact, many ties): ids and scores equal an exact-rational
    evaluation of the description, for depths, re-rank sizes and one or two assignments; the
    copies scored are the summed sizes of the probed lists."""
    rng = np.random.default_rng(62)
    for trial in range(12):
        n, d, K, s = 60, 4, 6, 2
        X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
        C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
        P = rng.integers(-2, 3, size=(d // s, 16, s)).astype(np.float32)
        Q = rng.integers(-2, 3, size=(5, d)).astype(np.float32)
        a0 = rng.integers(0, K, n)
        a1 = (a0 + rng.integers(1, K, n)) % K
        A = [a0, a1] if trial % 3 else [a0]
        codes = O.soar_pq_codes(X, C, P, A)
        t, R, k = int(rng.integers(1, 4)), int(rng.integers(1, 12)), int(rng.integers(1, 6))
        ids, sc, scored = O.search_pq(Q, X, C, A, codes, P, t, R, k)
        wi, ws = _search_pq_brute(Q, X, C, A, codes, P, t, R, k)
        assert np.array_equal(ids, wi), trial
        assert np.array_equal(sc, ws), trial
        parts, _ = O.probe_partitions_seq(Q, C, t)
        assert scored.tolist() == [sum(int((a == p).sum()) for p in pr for a in A) for pr in parts]


def test_search_pq_large_rerank_is_exact_search():
    """With every reached point re-scored (R >= n) the codes only order the candidates, so the
    result is the exact search over the probed lists (integer data: exact)."""
    rng = np.random.default_rng(63)
    n, d, K = 300, 8, 20
    X = rng.integers(-4, 5, size=(n, d)).astype(np.float32)
    C = rng.integers(-3, 4, size=(K, d)).astype(np.float32)
    Q = rng.integers(-3, 4, size=(12, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(d // 2, 16, 2)).astype(np.float32)
    p, _, s_, _ = O.assign(X, C, 1.0)
    codes = O.soar_pq_codes(X, C, P, [p, s_])
    for t in (1, 3, K):
        ids, sc, scored = O.search_pq(Q, X, C, [p, s_], codes, P, t, n, 10)
        wi, ws, wn = O.search(Q, X, C, [p, s_], t, 10)
        assert np.array_equal(ids, wi) and np.array_equal(sc, ws) and np.array_equal(scored, wn)


def test_search_pq_spilled_copy_uses_its_own_code():
    """A point whose primary copy's code is poor and whose spilled copy's code is exact is taken
    into a re-rank of one point through its spilled copy: each copy keeps its own residual's
    code, and a point its best copy's estimate."""
    C = np.array([[1.0, 0.0], [0.0, 1.0]], np.float32)
    P = np.zeros((1, 16, 2), np.float32)
    P[0, 1] = [1.0, 0.0]                         # exact residual of point 0 from partition 1
    P[0, 2] = [-4.0, 0.0]
    X = np.array([[1.0, 1.0], [1.0, 0.5]], np.float32)
    A = [np.array([0, 0]), np.array([1, 1])]
    codes = np.zeros((2, 2, 1), np.int64)
    codes[0, 0, 0] = 2                           # point 0, primary copy: estimate 1 - 4 = -3
    codes[0, 1, 0] = 1                           # point 0, spilled copy: estimate 1 + 1 = 2
    codes[1, 0, 0] = 0                           # point 1, primary copy: estimate 1 + 0 = 1
    codes[1, 1, 0] = 2                           # point 1, spilled copy: estimate -3
    Q = np.array([[1.0, 1.0]], np.float32)
    ids, sc, scored = O.search_pq(Q, X, C, A, codes, P, 2, 2, 2)
    assert ids.tolist() == [[0, 1]] and sc.tolist() == [[2.0, 1.5]] and scored.tolist() == [4]
    ids, _, _ = O.search_pq(Q, X, C, A, codes, P, 2, 1, 2)
    assert ids.tolist() == [[0, -1]]
    ids, _, _ = O.search_pq(Q, X, C, A[:1], codes[:, :1], P, 2, 1, 2)
    assert ids.tolist() == [[1, -1]]             # without the spilled copies point 1 leads


# ------------------------------------------------------------------------------------------------
# Two-level VQ probing (App. A.4.1)
# ------------------------------------------------------------------------------------------------
def test_two_level_probe_brute_force_and_full_upper_probe():
    """Integer data, exact: the upper probe, the listed partitions and the top t by score then
    index follow the description; probing every upper centroid gives the flat probe; fewer listed
    partitions than t leave -1 places."""
    rng = np.random.default_rng(71)
    for trial in range(20):
        K, K2, d = int(rng.integers(3, 25)), int(rng.integers(1, 6)), int(rng.integers(1, 5))
        C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
        U = rng.integers(-2, 3, size=(K2, d)).astype(np.float32)
        ua = rng.integers(0, K2, K)
        Q = rng.integers(-2, 3, size=(6, d)).astype(np.float32)
        t2, t = int(rng.integers(1, K2 + 1)), int(rng.integers(1, K + 3))
        parts, sc = O.probe_two_level(Q, U, ua, C, t2, t)
        for i, q in enumerate(Q.astype(np.int64)):
            ups = sorted(range(K2), key=lambda u: (-int(q @ U[u]), u))[:t2]
            cand = [p for p in range(K) if ua[p] in ups]
            want = sorted(cand, key=lambda p: (-int(q @ C[p]), p))[:t]
            assert parts[i].tolist() == want + [-1] * (t - len(want)), trial
            assert sc[i, :len(want)].tolist() == [float(q @ C[p]) for p in want]
        flat, fsc = O.probe_partitions_seq(Q, C, min(t, K))
        parts, sc = O.probe_two_level(Q, U, ua, C, K2, min(t, K))
        assert np.array_equal(parts, flat) and np.array_equal(sc, fsc)


def test_two_level_search_full_upper_probe_is_flat_search_and_a_missed_partition():
    rng = np.random.default_rng(72)
    n, d, K, K2 = 400, 6, 30, 5
    X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    C = rng.integers(-2, 3, size=(K, d)).astype(np.float32)
    U = rng.integers(-2, 3, size=(K2, d)).astype(np.float32)
    ua = rng.integers(0, K2, K)
    Q = rng.integers(-2, 3, size=(10, d)).astype(np.float32)
    p, _, s_, _ = O.assign(X, C, 1.0)
    for t in (1, 4, K):
        got = O.search_two_level(Q, X, C, U, ua, [p, s_], K2, t, 8)
        want = O.search(Q, X, C, [p, s_], t, 8)
        for g, w in zip(got, want):
            assert np.array_equal(g, w)
    # the query's best partition sits under the second upper centroid, which is not probed
    C2 = np.array([[3.0, 0.0], [1.0, 0.0], [0.0, 1.0]], np.float32)
    U2 = np.array([[1.0, 0.0], [0.0, 1.0]], np.float32)
    ua2 = np.array([1, 0, 1])
    q = np.array([[1.0, 0.2]], np.float32)
    parts, _ = O.probe_two_level(q, U2, ua2, C2, 1, 2)
    assert parts.tolist() == [[1, -1]]
    parts, _ = O.probe_two_level(q, U2, ua2, C2, 2, 2)
    assert parts.tolist() == [[0, 1]]


# ------------------------------------------------------------------------------------------------
# Spill bound (Section 3.4's loss, Cauchy-Schwarz and the triangle inequality): the spill lies
# within ||r|| + sqrt((1 + lambda) ||x - c_j2||^2) of the primary centroid, so rows whose
# radius stays below the (M+1)-th nearest centroid have their spill among the M nearest.
# ------------------------------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [0.0, 0.5, 1.0, 4.0])
def test_spill_bound_confines_the_spill(lam):
    from synth import MixtureSpec, gen_mixture
    X = gen_mixture(MixtureSpec(3000, 16, 40, ("loguniform", 0.05, 0.5), "unit", 5))
    C, _, _ = O.train_codebook(X, 100, 3, seed=0)
    p, _ = O.primary_plain(X, C)
    s, _ = O.spill_plain(X, C, lam, p)
    C64 = C.astype(np.float64)
    for M in (1, 4, 8):
        mask, radius, nb, beyond = O.spill_bound_rows(X, C, lam, p, M)
        # the radius bounds the spill's distance from c_p on every row, decided or not
        reach = np.sqrt(((C64[p] - C64[s]) ** 2).sum(1))
        assert np.all(reach <= radius * (1 + 1e-12))
        # decided rows have their spill among the M nearest centroids of c_p
        assert all(s[i] in nb[p[i]] for i in np.flatnonzero(mask))
        if M == 8:
            assert mask.mean() > 0.3, mask.mean()   # the bound decides a good share of rows


def test_spill_bound_radius_is_tight_where_it_should_be():
    # x on the segment between c_0 and c_1 with c_1 the spill: the radius is reached exactly
    # when lambda = 0 (||c_0 - c_1|| = ||r|| + ||x - c_1||)
    X = np.array([[1.0, 0.0]], dtype=np.float32)
    C = np.array([[0.0, 0.0], [3.0, 0.0], [0.0, 9.0]], dtype=np.float32)
    mask, radius, nb, beyond = O.spill_bound_rows(X, C, 0.0, [0], 1)
    assert radius[0] == 3.0 and nb[0, 0] == 1 and beyond[0] == 9.0 and mask[0]
    mask, radius, _, _ = O.spill_bound_rows(X, C, 8.0, [0], 1)
    assert radius[0] == 1.0 + 6.0 and mask[0]
    mask, radius, _, _ = O.spill_bound_rows(X, C, 24.0, [0], 1)
    assert radius[0] == 11.0 and not mask[0]


def test_centroid_neighbours_order_ties_and_short_codebooks():
    C = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [3, 0]], dtype=np.float32)
    nb, beyond = O.centroid_neighbours(C, 2)
    # from c_0 three centroids are at distance 1: the two lowest indices are kept
    assert list(nb[0]) == [1, 2] and beyond[0] == 1.0
    assert list(nb[4]) == [1, 0] and beyond[4] == np.sqrt(10.0)
    nb, beyond = O.centroid_neighbours(C[:3], 4)
    assert list(nb[1]) == [0, 2, -1, -1] and np.isinf(beyond).all()
    # brute force on random centroids
    R = np.random.default_rng(3).standard_normal((30, 5)).astype(np.float32)
    nb, beyond = O.centroid_neighbours(R, 6)
    for q in range(30):
        dd = [(float(np.sqrt(((R[q].astype(float) - R[j]) ** 2).sum())), j) for j in range(30)
              if j != q]
        dd.sort()
        assert [j for _, j in dd[:6]] == list(nb[q]) and dd[6][0] == beyond[q]
