"""CPU FP64 oracle for SOAR spilled assignment and the Lloyd k-means that trains its codebook.

TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library imports, links or runs this file; only the
tests, the smoke check and the benchmark's CPU-baseline leg may use it.  It shares no code with
the HIP path.

Everything is computed in float64 from float32 inputs (promotion is exact), by direct
differences, in the order the paper states the method:

* primary assignment, Section 2.2: pi(x) = argmin_i ||x - C_i||^2;
* partitioning residual, Section 3.1: r = x - C_pi(x);
* SOAR spill, Section 3.4 (Eq. 2 evaluated by Theorem 3.1):
  pi'(x) = argmin_{j != pi(x)} ||x - C_j||^2 + lambda * ||proj_r (x - C_j)||^2, and
  ||proj_r r'||^2 = <r, r'>^2 / ||r||^2;
* indexing pipeline, Section 3.5: train VQ, primary, residual, spill;
* further spilled assignments, Section 3.5.1: each adds one Theorem 3.1 penalty per earlier
  residual (a reading: the paper gives no formula);
* PQ codes of each assignment's residual and the index memory model, Section 3.5;
* two-level VQ probing (App. A.4.1): the partition centres quantized again, a query's partitions
  taken from the lists of its best upper centroids;
* search over the lists with PQ-coded copies (Section 2.2 search, Section 3.5 layout): each
  probed copy scored from its own residual code, a point keeping its best copy, the best points
  re-scored exactly (a reading: the paper describes PQ as an intermediate scoring stage);
* KMR curve, Eq. 1 (Section 2.2.1), with Rank as in Section 2.1.

Readings where the paper is silent (each is listed with its reason in the design notes):

* arg-min ties go to the lowest index (paper silent);
* the primary is excluded *by index* (a duplicate centroid at another index stays eligible);
* ||r|| = 0 makes the projection term 0 (the formula is 0/0 there);
* Lloyd: an empty cluster keeps its previous centroid; the iteration count is exact;
* k-means++: first centre uniform over rows, then one row per round drawn with probability
  proportional to D^2; if sum D^2 = 0 the lowest-index row not yet chosen is taken.  Its random
  draws come from Philox4x32-10 (``oracle/philox.py``), the same published generator the GPU
  library implements on its own.

Two modes:
* ``*_plain``: the definition, all K distances/losses by direct differences (chunked);
* ``*_fast``: an FP64 GEMM expansion screens candidates with a rigorous rounding margin, and every
  surviving candidate is recomputed by the very same direct-difference routine, so the result is
  bit-identical to plain mode (checked in the tests).
"""
from __future__ import annotations

import numpy as np

from .philox import philox_uniform24, philox_index

_U64 = 2.0 ** -53
_CHUNK_BYTES = 128 << 20


def _f64(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _chunk_rows(K: int, d: int, planes: int = 2) -> int:
    return max(1, int(_CHUNK_BYTES // max(1, planes * K * d * 8)))


# ----------------------------------------------------------------------------------------------
# Direct-difference kernels (the definition).  Every loss the oracle reports comes from these two
# functions, in both modes, so the two modes agree to the last bit.
# ----------------------------------------------------------------------------------------------

def _sqdist(diff: np.ndarray) -> np.ndarray:
    """||x - c||^2 from diff = x - c over the last axis (Section 2.2)."""
    return (diff * diff).sum(axis=-1)


def _soar_loss(diff: np.ndarray, r: np.ndarray, rr: np.ndarray, lam: float) -> np.ndarray:
    """||r'||^2 + lam * <r, r'>^2 / ||r||^2 with r' = diff (Theorem 3.1; zero penalty if r = 0)."""
    sq = _sqdist(diff)
    proj = (diff * r).sum(axis=-1)
    safe = np.where(rr > 0.0, rr, 1.0)
    pen = np.where(rr > 0.0, lam * (proj * proj) / safe, 0.0)
    return sq + pen


# ----------------------------------------------------------------------------------------------
# Primary assignment (Section 2.2)
# ----------------------------------------------------------------------------------------------

def primary_plain(X, C):
    """pi_i = argmin_j ||x_i - c_j||^2 (lowest index on ties) and that distance, float64."""
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    pi = np.empty(n, dtype=np.int64)
    dist = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, d)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        D = _sqdist(X[lo:hi, None, :] - C[None, :, :])
        pi[lo:hi] = np.argmin(D, axis=1)
        dist[lo:hi] = D[np.arange(hi - lo), pi[lo:hi]]
    return pi, dist


def _pick_min(rows, cols, vals, n):
    """Per row, the smallest value, ties to the lowest column."""
    order = np.lexsort((cols, vals, rows))
    r_sorted = rows[order]
    first = np.ones(len(order), dtype=bool)
    first[1:] = r_sorted[1:] != r_sorted[:-1]
    sel = order[first]
    out_c = np.full(n, -1, dtype=np.int64)
    out_v = np.full(n, np.inf)
    out_c[rows[sel]] = cols[sel]
    out_v[rows[sel]] = vals[sel]
    return out_c, out_v


def _screen_bound(X, C, scale):
    """Rigorous bound on |expansion - exact| and |direct - exact| per row: scale*(d+8)*u*(|x|+cmax)^2."""
    d = X.shape[1]
    cmax = np.sqrt((C * C).sum(axis=1).max())
    xn = np.sqrt((X * X).sum(axis=1))
    return 4.0 * scale * (d + 8) * _U64 * (xn + cmax) ** 2


def primary_fast(X, C):
    """Same result as ``primary_plain``; an FP64 GEMM screens, direct differences decide."""
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    cc = (C * C).sum(axis=1)
    xx = (X * X).sum(axis=1)
    bound = _screen_bound(X, C, 1.0)
    pi = np.empty(n, dtype=np.int64)
    dist = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, 1, planes=2)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        Dh = xx[lo:hi, None] - 2.0 * (X[lo:hi] @ C.T) + cc[None, :]
        thr = Dh.min(axis=1) + 2.0 * bound[lo:hi]
        rows, cols = np.nonzero(Dh <= thr[:, None])
        vals = _sqdist(X[lo + rows] - C[cols])
        c, v = _pick_min(rows, cols, vals, hi - lo)
        pi[lo:hi], dist[lo:hi] = c, v
    return pi, dist


# ----------------------------------------------------------------------------------------------
# SOAR spilled assignment (Section 3.4, Eq. 2, Theorem 3.1)
# ----------------------------------------------------------------------------------------------

def _check_lambda(lam):
    lam = float(lam)
    if not np.isfinite(lam) or lam < 0.0:
        raise ValueError("lambda must be finite and >= 0")
    return lam


def soar_losses(x, C, lam, p):
    """All K losses of one row given its primary index p (the primary itself included)."""
    x, C = _f64(x), _f64(C)
    r = x - C[p]
    rr = _sqdist(r)
    return _soar_loss(x[None, :] - C, r[None, :], np.full(C.shape[0], rr), float(lam))


def spill_plain(X, C, lam, primary=None):
    """pi'_i = argmin_{j != pi_i} L_ij (lowest index on ties) and L at that index, float64.

    ``primary`` may be given (for example a GPU primary that was a legitimate near-tie); otherwise
    it is recomputed by ``primary_plain``."""
    lam = _check_lambda(lam)
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    if K < 2:
        raise ValueError("a spill needs at least two centroids")
    p = primary_plain(X, C)[0] if primary is None else np.asarray(primary, dtype=np.int64)
    sp = np.empty(n, dtype=np.int64)
    loss = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, d, planes=3)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        m = hi - lo
        R = X[lo:hi] - C[p[lo:hi]]
        rr = _sqdist(R)
        L = _soar_loss(X[lo:hi, None, :] - C[None, :, :], R[:, None, :], rr[:, None], lam)
        L[np.arange(m), p[lo:hi]] = np.inf
        sp[lo:hi] = np.argmin(L, axis=1)
        loss[lo:hi] = L[np.arange(m), sp[lo:hi]]
    return sp, loss


def spill_fast(X, C, lam, primary=None):
    """Same result as ``spill_plain``; FP64 GEMMs screen, the direct-difference loss decides."""
    lam = _check_lambda(lam)
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    if K < 2:
        raise ValueError("a spill needs at least two centroids")
    p = primary_fast(X, C)[0] if primary is None else np.asarray(primary, dtype=np.int64)
    cc = (C * C).sum(axis=1)
    xx = (X * X).sum(axis=1)
    bound = _screen_bound(X, C, 1.0 + 3.0 * lam)
    sp = np.empty(n, dtype=np.int64)
    loss = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, 1, planes=4)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        m = hi - lo
        Xb = X[lo:hi]
        R = Xb - C[p[lo:hi]]
        rr = _sqdist(R)
        a = (R * Xb).sum(axis=1)
        S = Xb @ C.T
        T = R @ C.T
        E = a[:, None] - T
        pen = np.where(rr[:, None] > 0, lam * E * E / np.where(rr > 0, rr, 1.0)[:, None], 0.0)
        Lh = xx[lo:hi, None] - 2.0 * S + cc[None, :] + pen
        Lh[np.arange(m), p[lo:hi]] = np.inf
        thr = Lh.min(axis=1) + 2.0 * bound[lo:hi]
        rows, cols = np.nonzero(Lh <= thr[:, None])
        vals = _soar_loss(Xb[rows] - C[cols], R[rows], rr[rows], lam)
        c, v = _pick_min(rows, cols, vals, m)
        sp[lo:hi], loss[lo:hi] = c, v
    return sp, loss


def assign(X, C, lam, fast=True):
    """The indexing pipeline's assignment step (Section 3.5): primary, residual, spill."""
    prim = primary_fast if fast else primary_plain
    spl = spill_fast if fast else spill_plain
    p, dp = prim(X, C)
    s, ls = spl(X, C, lam, primary=p)
    return p, dp, s, ls


# ----------------------------------------------------------------------------------------------
# Codebook training: k-means++ seeding and Lloyd iterations
# ----------------------------------------------------------------------------------------------

def dsq_sample(D2, u):
    """Inverse-CDF draw proportional to D^2: row i owns [prefix_{i-1}, prefix_i) of [0, sum D^2),
    so the pick is the smallest i with prefix_i > u * sum(D^2).  Returns -1 if sum(D^2) = 0."""
    pref = np.cumsum(np.asarray(D2, dtype=np.float64))
    S = pref[-1]
    if not S > 0.0:
        return -1
    return int(np.searchsorted(pref, u * S, side="right"))


def kmeanspp(X, K, seed):
    """k-means++ seeding.  Round 0 takes row philox_index(seed, 0, n); round m >= 1 draws
    u = philox_uniform24(seed, m) and takes the smallest row i with prefix_i(D^2) > u * sum(D^2),
    where D is the distance to the nearest centre chosen so far.  Returns (C float64 K x d, rows)."""
    X = _f64(X)
    n, d = X.shape
    if K < 1 or K > n:
        raise ValueError("need 1 <= K <= n")
    rows = np.empty(K, dtype=np.int64)
    chosen = np.zeros(n, dtype=bool)
    rows[0] = philox_index(seed, 0, n)
    chosen[rows[0]] = True
    D2 = _sqdist(X - X[rows[0]])
    for m in range(1, K):
        i = dsq_sample(D2, philox_uniform24(seed, m))
        if i < 0:
            i = int(np.flatnonzero(~chosen)[0])
        rows[m] = i
        chosen[i] = True
        D2 = np.minimum(D2, _sqdist(X - X[i]))
    return X[rows].copy(), rows


def lloyd_update(X, labels, C_prev):
    """c_j <- mean of the rows labelled j; an empty cluster keeps c_j from ``C_prev``."""
    X, C_prev = _f64(X), _f64(C_prev)
    K, d = C_prev.shape
    labels = np.asarray(labels, dtype=np.int64)
    counts = np.bincount(labels, minlength=K)
    sums = np.zeros((K, d))
    np.add.at(sums, labels, X)
    C = C_prev.copy()
    nz = counts > 0
    C[nz] = sums[nz] / counts[nz, None]
    return C, counts


def lloyd_step(X, C, fast=True):
    """One Lloyd iteration: assign against C (Section 2.2), then recentre."""
    prim = primary_fast if fast else primary_plain
    labels, dist = prim(X, C)
    C_next, counts = lloyd_update(X, labels, C)
    return labels, dist, C_next, counts, float(dist.sum())


def train_codebook(X, K, iters, seed, C_init=None, fast=True):
    """k-means++ (unless ``C_init``), then exactly ``iters`` Lloyd iterations.

    Returns (C, labels against the final C, inertia[iters + 1])."""
    C = kmeanspp(X, K, seed)[0] if C_init is None else _f64(C_init)
    inertia = []
    for _ in range(iters):
        _, _, C, _, e = lloyd_step(X, C, fast)
        inertia.append(e)
    prim = primary_fast if fast else primary_plain
    labels, dist = prim(X, C)
    inertia.append(float(dist.sum()))
    return C, labels, inertia


# ----------------------------------------------------------------------------------------------
# MIPS ground truth, Rank, KMR (Section 2.1, Eq. 1)
# ----------------------------------------------------------------------------------------------

def mips_topk(Q, X, k, chunk=64):
    """Exact MIPS top-k ids per query (ties to the lowest id), float64."""
    Q, X = _f64(Q), _f64(X)
    out = np.empty((Q.shape[0], k), dtype=np.int64)
    for lo in range(0, Q.shape[0], chunk):
        S = Q[lo:lo + chunk] @ X.T
        part = np.argpartition(-S, k, axis=1)[:, :k + 1] if X.shape[0] > k else \
            np.tile(np.arange(X.shape[0]), (S.shape[0], 1))
        for i in range(S.shape[0]):
            # candidates: everything scoring at least the (k)-th best value, ordered by (-s, id)
            kth = np.sort(S[i, part[i]])[::-1][min(k, part.shape[1]) - 1]
            cand = np.flatnonzero(S[i] >= kth)
            order = np.lexsort((cand, -S[i, cand]))
            out[lo + i] = cand[order[:k]]
    return out


def partition_ranks(Q, C):
    """Rank(q, C_j, C) = #{j'' : <q, C_j> <= <q, C_j''>} for every query and centroid (ties count
    against C_j, Section 2.1)."""
    Q, C = _f64(Q), _f64(C)
    S = Q @ C.T
    srt = np.sort(S, axis=1)
    K = C.shape[0]
    ranks = np.empty(S.shape, dtype=np.int64)
    for i in range(S.shape[0]):
        ranks[i] = K - np.searchsorted(srt[i], S[i], side="left")
    return ranks


def kmr_curve(Q, X, C, assignments, k, ts, gt=None):
    """Eq. 1 with a datapoint found at depth t if any of its partitions has Rank <= t.

    ``assignments`` is a list of int arrays (one per assignment: [pi] or [pi, pi']).
    Returns (kmr values at ``ts``, datapoints searched at ``ts``)."""
    gt = mips_topk(Q, X, k) if gt is None else gt
    ranks = partition_ranks(Q, C)
    K = C.shape[0]
    best = None
    for a in assignments:
        rk = np.take_along_axis(ranks, np.asarray(a, dtype=np.int64)[gt], axis=1)
        best = rk if best is None else np.minimum(best, rk)
    kmr = np.array([(best <= t).mean() for t in ts])
    sizes = np.zeros(K, dtype=np.int64)
    for a in assignments:
        sizes += np.bincount(np.asarray(a, dtype=np.int64), minlength=K)
    S = _f64(Q) @ _f64(C).T
    order = np.argsort(-S, axis=1, kind="stable")
    csz = np.cumsum(sizes[order], axis=1)
    searched = np.array([csz[:, min(t, K) - 1].mean() if t > 0 else 0.0 for t in ts])
    return kmr, searched


# ----------------------------------------------------------------------------------------------
# Acceptance rule for a GPU result
# ----------------------------------------------------------------------------------------------

def reference(X, C, lam, fast=True):
    """The oracle's answer for every row: primary and its distance, and the spill and its loss
    given that primary.  ``verify`` can reuse it for several GPU results on the same rows."""
    prim = primary_fast if fast else primary_plain
    spl = spill_fast if fast else spill_plain
    p_star, d_star = prim(X, C)
    s_star, l_star = spl(X, C, lam, primary=p_star)
    return dict(p_star=p_star, d_star=d_star, s_given_p_star=s_star, l_given_p_star=l_star)


def verify(X, C, lam, gpu_primary, gpu_spill, gpu_pdist=None, gpu_sloss=None, fast=True,
          band=1e-6, loss_tol=1e-5, ref=None):
    """Check a GPU assignment against the oracle.

    * primary: accepted if equal to the oracle's, or its exact distance is within ``band``
      (relative) of the best;
    * spill: checked with the oracle conditioned on the GPU primary; accepted if equal, or not the
      primary and its exact loss within ``band`` (relative) of the best;
    * reported distance / loss: within ``loss_tol`` (relative) of the exact value at the GPU's index.
    ``ref`` (from ``reference`` on the same rows, C and lambda) saves recomputing the oracle: the
    spill is then recomputed only for rows whose GPU primary differs from the oracle's.
    Returns a dict of per-row boolean arrays and regret statistics."""
    X, C = _f64(X), _f64(C)
    n = X.shape[0]
    gp = np.asarray(gpu_primary, dtype=np.int64)
    gs = np.asarray(gpu_spill, dtype=np.int64)
    K = C.shape[0]
    valid = (gp >= 0) & (gp < K) & (gs >= 0) & (gs < K)
    gp_c = np.clip(gp, 0, K - 1)
    gs_c = np.clip(gs, 0, K - 1)
    prim = primary_fast if fast else primary_plain
    spl = spill_fast if fast else spill_plain
    if ref is None:
        p_star, d_star = prim(X, C)
    else:
        p_star, d_star = ref["p_star"], ref["d_star"]
    d_gpu = _sqdist(X - C[gp_c])
    dscale = np.maximum(d_star, 1e-12)
    prim_ok = valid & ((gp == p_star) | (d_gpu - d_star <= band * dscale))
    if ref is None:
        s_star, l_star = spl(X, C, lam, primary=gp_c)
    else:
        s_star = ref["s_given_p_star"].copy()
        l_star = ref["l_given_p_star"].copy()
        diff = np.flatnonzero(gp_c != p_star)
        if diff.size:
            s_star[diff], l_star[diff] = spl(X[diff], C, lam, primary=gp_c[diff])
    R = X - C[gp_c]
    rr = _sqdist(R)
    l_gpu = _soar_loss(X - C[gs_c], R, rr, float(lam))
    tau = np.maximum(l_star, 1e-12)
    spill_ok = valid & ((gs == s_star) | ((gs != gp) & (l_gpu - l_star <= band * tau)))
    out = dict(primary_ok=prim_ok, spill_ok=spill_ok,
               primary_regret=(d_gpu - d_star) / dscale,
               spill_regret=(l_gpu - l_star) / tau,
               primary_mismatch=int((gp != p_star).sum()),
               spill_mismatch=int((gs != s_star).sum()),
               p_star=p_star, s_star=s_star, d_star=d_star, l_star=l_star)
    if gpu_pdist is not None:
        out["pdist_ok"] = np.abs(np.asarray(gpu_pdist, np.float64) - d_gpu) <= loss_tol * dscale
    if gpu_sloss is not None:
        out["sloss_ok"] = np.abs(np.asarray(gpu_sloss, np.float64) - l_gpu) <= loss_tol * tau
    out["all_ok"] = bool(prim_ok.all() and spill_ok.all()
                         and out.get("pdist_ok", np.ones(n, bool)).all()
                         and out.get("sloss_ok", np.ones(n, bool)).all())
    return out


# ----------------------------------------------------------------------------------------------
# Further spilled assignments (Section 3.5.1).  The paper states only that each later assignment
# weighs the score errors of all earlier ones.  Reading taken here: the m-th assignment adds one
# Theorem 3.1 penalty per earlier residual,
#     L_m(j) = ||x - c_j||^2 + lambda * sum_k <r_k, x - c_j>^2 / ||r_k||^2,  r_k = x - c_{pi_k},
# minimised over the centroids not assigned yet.  With one earlier assignment (the primary) this
# is the SOAR spill.
# ----------------------------------------------------------------------------------------------

def _prior_array(prior, n, K):
    P = np.asarray(prior, dtype=np.int64)
    if P.ndim == 1:
        P = P[:, None]
    if P.ndim != 2 or P.shape[0] != n or P.shape[1] < 1:
        raise ValueError("prior must be [n x m] with m >= 1")
    if P.shape[1] >= K:
        raise ValueError("need more centroids than earlier assignments")
    if ((P < 0) | (P >= K)).any():
        raise ValueError("prior indices out of range")
    srt = np.sort(P, axis=1)
    if (srt[:, 1:] == srt[:, :-1]).any():
        raise ValueError("a row's earlier assignments must be distinct")
    return P


def _further_loss(diff, R, rr, lam):
    """||r'||^2 + lam * sum_k <r_k, r'>^2 / ||r_k||^2 with r' = diff [..., d] and the earlier
    residuals R [..., m, d], rr [..., m] (terms with r_k = 0 dropped)."""
    sq = _sqdist(diff)
    pen = np.zeros_like(sq)
    for k in range(R.shape[-2]):
        proj = (diff * R[..., k, :]).sum(axis=-1)
        rk = rr[..., k]
        safe = np.where(rk > 0.0, rk, 1.0)
        pen = pen + np.where(rk > 0.0, lam * (proj * proj) / safe, 0.0)
    return sq + pen


def further_losses(x, C, lam, prior):
    """All K losses of one row given its earlier assignments (those included)."""
    x, C = _f64(x), _f64(C)
    P = np.asarray(prior, dtype=np.int64).reshape(-1)
    R = x[None, :] - C[P]
    rr = _sqdist(R)
    return _further_loss(x[None, :] - C, R[None], rr[None], float(lam))


def spill_further_plain(X, C, lam, prior):
    """Next assignment of every row given its earlier ones prior [n x m]: the arg-min of the
    further loss over the centroids not in the row's prior (lowest index on ties), and that loss,
    all K losses by direct differences."""
    lam = _check_lambda(lam)
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    P = _prior_array(prior, n, K)
    m = P.shape[1]
    out = np.empty(n, dtype=np.int64)
    loss = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, d, planes=2 + m)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        rows = np.arange(hi - lo)
        R = X[lo:hi, None, :] - C[P[lo:hi]]                      # [b, m, d]
        rr = _sqdist(R)
        L = _further_loss(X[lo:hi, None, :] - C[None, :, :], R[:, None, :, :], rr[:, None, :], lam)
        for k in range(m):
            L[rows, P[lo:hi, k]] = np.inf
        out[lo:hi] = np.argmin(L, axis=1)
        loss[lo:hi] = L[rows, out[lo:hi]]
    return out, loss


def spill_further_fast(X, C, lam, prior):
    """Same result as ``spill_further_plain``; FP64 GEMMs screen with a rounding margin that grows
    with the number of penalty terms, the direct-difference loss decides."""
    lam = _check_lambda(lam)
    X, C = _f64(X), _f64(C)
    n, d = X.shape
    K = C.shape[0]
    P = _prior_array(prior, n, K)
    m = P.shape[1]
    cc = (C * C).sum(axis=1)
    xx = (X * X).sum(axis=1)
    bound = _screen_bound(X, C, 1.0 + 3.0 * m * lam)
    out = np.empty(n, dtype=np.int64)
    loss = np.empty(n, dtype=np.float64)
    step = _chunk_rows(K, 1, planes=3 + m)
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        b = hi - lo
        rows = np.arange(b)
        Xb = X[lo:hi]
        R = Xb[:, None, :] - C[P[lo:hi]]                          # [b, m, d]
        rr = _sqdist(R)
        Lh = xx[lo:hi, None] - 2.0 * (Xb @ C.T) + cc[None, :]
        for k in range(m):
            a = (R[:, k, :] * Xb).sum(axis=1)
            E = a[:, None] - R[:, k, :] @ C.T
            rk = rr[:, k]
            Lh = Lh + np.where(rk[:, None] > 0, lam * E * E / np.where(rk > 0, rk, 1.0)[:, None],
                               0.0)
        for k in range(m):
            Lh[rows, P[lo:hi, k]] = np.inf
        thr = Lh.min(axis=1) + 2.0 * bound[lo:hi]
        r_, c_ = np.nonzero(Lh <= thr[:, None])
        vals = _further_loss(Xb[r_] - C[c_], R[r_], rr[r_], lam)
        c, v = _pick_min(r_, c_, vals, b)
        out[lo:hi], loss[lo:hi] = c, v
    return out, loss


def assign_multi(X, C, lam, M, fast=True):
    """M assignments per row: the primary (Section 2.2), then M - 1 further assignments, each
    given all earlier ones.  Returns ([n x M] indices, [n x M] distance / losses)."""
    if M < 1:
        raise ValueError("M >= 1")
    prim = primary_fast if fast else primary_plain
    nxt = spill_further_fast if fast else spill_further_plain
    p, dp = prim(X, C)
    A = [p]
    V = [dp]
    for _ in range(1, M):
        j, v = nxt(X, C, lam, np.stack(A, axis=1))
        A.append(j)
        V.append(v)
    return np.stack(A, axis=1), np.stack(V, axis=1)


def verify_further(X, C, lam, prior, gpu_next, gpu_loss=None, band=1e-6, loss_tol=1e-5,
                   fast=True):
    """Check a GPU further assignment given the same earlier ones: accepted if equal to the
    oracle's, or not among the earlier ones and its exact loss within ``band`` (relative) of the
    best; a reported loss must lie within ``loss_tol`` (relative) of the exact loss at the GPU's
    index."""
    X, C = _f64(X), _f64(C)
    n = X.shape[0]
    K = C.shape[0]
    P = _prior_array(prior, n, K)
    g = np.asarray(gpu_next, dtype=np.int64)
    valid = (g >= 0) & (g < K) & (g[:, None] != P).all(axis=1)
    gc = np.clip(g, 0, K - 1)
    nxt = spill_further_fast if fast else spill_further_plain
    j_star, l_star = nxt(X, C, lam, P)
    R = X[:, None, :] - C[P]
    l_gpu = _further_loss(X - C[gc], R, _sqdist(R), float(lam))
    tau = np.maximum(l_star, 1e-12)
    ok = valid & ((g == j_star) | (l_gpu - l_star <= band * tau))
    out = dict(ok=ok, regret=(l_gpu - l_star) / tau, mismatch=int((g != j_star).sum()),
               j_star=j_star, l_star=l_star)
    if gpu_loss is not None:
        out["loss_ok"] = np.abs(np.asarray(gpu_loss, np.float64) - l_gpu) <= loss_tol * tau
    out["all_ok"] = bool(ok.all() and out.get("loss_ok", np.ones(n, bool)).all())
    return out


# ----------------------------------------------------------------------------------------------
# Product-quantized residual codes and the index memory model (Section 3.5, implementation
# considerations).  Each assignment of a point stores the PQ code of its own residual x - c_a:
# with h = 16 centres per subspace of s dimensions a code takes d / (2 s) bytes, plus a 4-byte id
# in the list; the highest-bitrate copy of the point is stored once.  Spilling therefore adds
# 4 + d / (2 s) bytes per point.
# ----------------------------------------------------------------------------------------------

def pq_encode(R, P):
    """codes[i, m] = argmin_k ||R[i, m s:(m + 1) s] - P[m, k]||^2 (lowest index on ties), all in
    float64.  R [n x d], P [M x h x s] with d = M s."""
    R, P = _f64(R), _f64(P)
    n, d = R.shape
    M, h, s = P.shape
    if M * s != d:
        raise ValueError("P must cover d = M s dimensions")
    codes = np.empty((n, M), dtype=np.int64)
    step = max(1, int(_CHUNK_BYTES // max(1, 8 * M * h * s)))
    for lo in range(0, n, step):
        hi = min(n, lo + step)
        diff = R[lo:hi].reshape(hi - lo, M, 1, s) - P[None]
        codes[lo:hi] = np.argmin((diff * diff).sum(axis=-1), axis=2)
    return codes


def pq_decode(codes, P):
    """The reconstruction [n x d] of PQ codes [n x M] with codebook P [M x h x s]."""
    P = _f64(P)
    M, h, s = P.shape
    codes = np.asarray(codes, dtype=np.int64)
    return P[np.arange(M)[None, :], codes].reshape(codes.shape[0], M * s)


def soar_pq_codes(X, C, P, assignments):
    """PQ codes of every assignment's residual: [n x len(assignments) x M]."""
    X, C = _f64(X), _f64(C)
    return np.stack([pq_encode(X - C[np.asarray(a, dtype=np.int64)], P) for a in assignments],
                    axis=1)


def pq_pack(codes):
    """4-bit codes [.., M] (M even, values < 16) as bytes [.., M / 2]: subspace 2 j in the low
    nibble of byte j, 2 j + 1 in the high nibble."""
    c = np.asarray(codes, dtype=np.int64)
    if c.shape[-1] % 2 or (c < 0).any() or (c > 15).any():
        raise ValueError("4-bit codes of an even number of subspaces")
    return (c[..., 0::2] | (c[..., 1::2] << 4)).astype(np.uint8)


def index_bytes(n, d, s, assignments, highres_bytes_per_dim):
    """Bytes of a VQ-PQ index: per assignment a 4-byte id and a d / (2 s)-byte PQ code, per point
    one highest-bitrate copy of highres_bytes_per_dim bytes per dimension."""
    return n * (assignments * (4 + d / (2 * s)) + highres_bytes_per_dim * d)


def spill_memory_overhead(d, s, highres_bytes_per_dim):
    """Relative index growth from one assignment to two: (4 + d/(2s)) / (hd + 4 + d/(2s))."""
    extra = 4 + d / (2 * s)
    return extra / (highres_bytes_per_dim * d + extra)


# ----------------------------------------------------------------------------------------------
# Query-side probing (Section 2.2 search with the spilled lists of Section 3.5)
# ----------------------------------------------------------------------------------------------

def probe_partitions(Q, C, t):
    """Per query, the t partitions with the largest <q, c> (MIPS over the codebook), best first;
    equal scores go to the lower partition index.  float64."""
    Q, C = _f64(Q), _f64(C)
    S = Q @ C.T
    K = C.shape[0]
    t = min(int(t), K)
    out = np.empty((Q.shape[0], t), dtype=np.int64)
    cols = np.arange(K)
    for i in range(Q.shape[0]):
        out[i] = np.lexsort((cols, -S[i]))[:t]
    return out


def partition_lists(assignments, K):
    """The inverted lists: for every partition the ids assigned to it by any of the assignments,
    ascending (a point spilled into a second partition is listed in both)."""
    lists = []
    for j in range(K):
        ids = [np.flatnonzero(np.asarray(a) == j) for a in assignments]
        lists.append(np.concatenate(ids) if ids else np.empty(0, np.int64))
    return lists


def search(Q, X, C, assignments, t, k):
    """VQ search: probe the t best partitions of every query, take the union of their lists
    (a point listed twice through its spilled copy counts once), score every candidate exactly
    by <q, x> and return the k best, ties to the lowest id.

    Returns (ids int64 [nq, k], -1 where fewer than k candidates; scores float64 [nq, k], -inf
    there; searched int64 [nq]: the datapoints scored, i.e. the summed sizes of the probed
    lists, spilled copies included)."""
    Q, X, C = _f64(Q), _f64(X), _f64(C)
    K = C.shape[0]
    lists = partition_lists(assignments, K)
    parts = probe_partitions(Q, C, t)
    nq = Q.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    scores = np.full((nq, k), -np.inf)
    searched = np.zeros(nq, dtype=np.int64)
    for i in range(nq):
        members = [lists[p] for p in parts[i]]
        searched[i] = sum(len(m) for m in members)
        cand = np.unique(np.concatenate(members)) if members else np.empty(0, np.int64)
        if cand.size == 0:
            continue
        s = X[cand] @ Q[i]
        order = np.lexsort((cand, -s))[:k]
        ids[i, :order.size] = cand[order]
        scores[i, :order.size] = s[order]
    return ids, scores, searched


# ----------------------------------------------------------------------------------------------
# Search over the lists with PQ-coded copies (Section 2.2 search, Section 3.5 index layout): the
# probed partitions' copies are scored from their residual codes, the best points by that score
# are re-scored exactly.  Every sum here runs in FP64 in one stated order (dimension order, then
# subspace order), so each ranking decision is reproducible to the last bit.
# ----------------------------------------------------------------------------------------------

def seq_dot(A, B):
    """<a_i, b_j> for all rows of A [na x d] and B [nb x d]: FP64, summed in dimension order."""
    A, B = _f64(A), _f64(B)
    S = np.zeros((A.shape[0], B.shape[0]))
    for t in range(A.shape[1]):
        S += A[:, t, None] * B[None, :, t]
    return S


def probe_partitions_seq(Q, C, t):
    """probe_partitions with the scores summed in dimension order: (partitions [nq, t] best
    first, equal scores to the lower index; their scores [nq, t])."""
    S = seq_dot(Q, C)
    K = C.shape[0]
    t = min(int(t), K)
    cols = np.arange(K)
    parts = np.empty((S.shape[0], t), dtype=np.int64)
    for i in range(S.shape[0]):
        parts[i] = np.lexsort((cols, -S[i]))[:t]
    return parts, np.take_along_axis(S, parts, axis=1)


def pq_lut(q, P):
    """LUT[m, k] = <q_m, P[m, k]> for one query q [d] and PQ codebook P [M x h x s]: FP64, summed
    over the s dimensions of the subspace in order."""
    q, P = _f64(q), _f64(P)
    M, h, s = P.shape
    qm = q.reshape(M, s)
    L = np.zeros((M, h))
    for t in range(s):
        L += qm[:, t, None] * P[:, :, t]
    return L


def pq_scores(score_c, lut, codes):
    """Approximate <q, x> of copies coded by `codes` [n x M] in a partition whose centre scores
    score_c: score_c + LUT[0, code_0] + LUT[1, code_1] + ..., added in subspace order (FP64)."""
    codes = np.asarray(codes, dtype=np.int64)
    a = np.full(codes.shape[0], float(score_c))
    for m in range(codes.shape[1]):
        a = a + lut[m, codes[:, m]]
    return a


def search_pq(Q, X, C, assignments, codes, P, t, R, k):
    """VQ-PQ search with spilled copies.  Per query: the t best partitions (probe_partitions_seq);
    every copy listed there, i.e. a point i with assignments[j][i] = p, is scored approximately by
    pq_scores with the code codes[i, j] of its own residual x_i - c_p; a point reached through
    several probed copies keeps its largest approximate score; the R best points by that score
    (ties to the lower id) are scored exactly by <q, x> (FP64, dimension order) and the k best
    of them are returned (ties to the lower id).

    codes: [n x len(assignments) x M] unpacked 4-bit codes.  Returns (ids int64 [nq, k], -1
    where fewer than k points; scores float64 [nq, k], -inf there; scored int64 [nq]: copies
    scored from their codes, i.e. the summed sizes of the probed lists)."""
    Q, X, C = _f64(Q), _f64(X), _f64(C)
    codes = np.asarray(codes, dtype=np.int64)
    K = C.shape[0]
    A = [np.asarray(a, dtype=np.int64) for a in assignments]
    # members[p][j]: the points with assignments[j] == p, ascending (a stable sort per assignment)
    members = [[] for _ in range(K)]
    for a in A:
        order = np.argsort(a, kind="stable")
        bounds = np.searchsorted(a[order], np.arange(K + 1))
        for p in range(K):
            members[p].append(order[bounds[p]:bounds[p + 1]])
    parts, pscore = probe_partitions_seq(Q, C, t)
    nq = Q.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    scores = np.full((nq, k), -np.inf)
    scored = np.zeros(nq, dtype=np.int64)
    for i in range(nq):
        lut = pq_lut(Q[i], P)
        best = {}
        for r in range(parts.shape[1]):
            p = int(parts[i, r])
            for j, mem in enumerate(members[p]):
                if mem.size == 0:
                    continue
                scored[i] += mem.size
                a = pq_scores(pscore[i, r], lut, codes[mem, j])
                for v, s in zip(mem.tolist(), a.tolist()):
                    if v not in best or s > best[v]:
                        best[v] = s
        if not best:
            continue
        cand = np.fromiter(best.keys(), dtype=np.int64, count=len(best))
        approx = np.fromiter(best.values(), dtype=np.float64, count=len(best))
        keep = cand[np.lexsort((cand, -approx))[:R]]
        exact = seq_dot(X[keep], Q[i:i + 1])[:, 0]
        order = np.lexsort((keep, -exact))[:k]
        ids[i, :order.size] = keep[order]
        scores[i, :order.size] = exact[order]
    return ids, scores, scored


# ----------------------------------------------------------------------------------------------
# Two-level VQ (App. A.4.1: the partition centres are vector-quantized again): a query probes the
# upper centroids first and scores only the partitions listed under the best of them.
# ----------------------------------------------------------------------------------------------

def probe_two_level(Q, U, upper_assign, C, t2, t):
    """Per query: the t2 upper centroids with the largest <q, u> (seq_dot; equal scores to the
    lower index), the partitions p with upper_assign[p] among them, and of those the t with the
    largest <q, c_p> (seq_dot; equal scores to the lower partition index), best first.

    Returns (parts int64 [nq, t], -1 where fewer than t partitions were listed; their scores
    float64 [nq, t], -inf there)."""
    ua = np.asarray(upper_assign, dtype=np.int64)
    uparts, _ = probe_partitions_seq(Q, U, t2)
    S = seq_dot(Q, C)
    nq = S.shape[0]
    parts = np.full((nq, t), -1, dtype=np.int64)
    scores = np.full((nq, t), -np.inf)
    for i in range(nq):
        cand = np.flatnonzero(np.isin(ua, uparts[i]))
        if cand.size == 0:
            continue
        order = np.lexsort((cand, -S[i, cand]))[:t]
        parts[i, :order.size] = cand[order]
        scores[i, :order.size] = S[i, cand[order]]
    return parts, scores


def search_two_level(Q, X, C, U, upper_assign, assignments, t2, t, k):
    """search() with the partitions of probe_two_level: the union of the probed lists (a point
    listed twice counts once) scored exactly by <q, x> (FP64, dimension order), the k best returned
    (ties to the lower id).  Returns (ids [nq, k] with -1 padding, scores [nq, k] with -inf
    padding, searched [nq]: the summed sizes of the probed lists)."""
    Q, X = _f64(Q), _f64(X)
    K = np.asarray(C).shape[0]
    lists = partition_lists(assignments, K)
    parts, _ = probe_two_level(Q, U, upper_assign, C, t2, t)
    nq = Q.shape[0]
    ids = np.full((nq, k), -1, dtype=np.int64)
    scores = np.full((nq, k), -np.inf)
    searched = np.zeros(nq, dtype=np.int64)
    for i in range(nq):
        members = [lists[p] for p in parts[i] if p >= 0]
        searched[i] = sum(len(m) for m in members)
        cand = np.unique(np.concatenate(members)) if members else np.empty(0, np.int64)
        if cand.size == 0:
            continue
        s = seq_dot(X[cand], Q[i:i + 1])[:, 0]
        order = np.lexsort((cand, -s))[:k]
        ids[i, :order.size] = cand[order]
        scores[i, :order.size] = s[order]
    return ids, scores, searched


# ---- Spill bound (a consequence of Section 3.4's loss) ----
#
# For a row with primary p, residual r and any centroid j2 != p, the spill j* has
# ||x - c_j*||^2 <= L(j*) <= L(j2) <= (1 + lambda) ||x - c_j2||^2 (the penalty term of Theorem
# 3.1 lies between 0 and lambda ||x - c||^2 by Cauchy-Schwarz), hence, by the triangle
# inequality, ||c_p - c_j*|| <= ||r|| + sqrt((1 + lambda) ||x - c_j2||^2).  The library uses this
# to decide some rows' spill from a few centroids; these two functions state it plainly so that
# the tests can pin it and check the library's decisions.

def centroid_neighbours(C, M):
    """For every centroid p: the M other centroids nearest to c_p (float64 direct differences,
    ties to the lowest index; -1 where K - 1 < M) and the distance from c_p to the (M+1)-th
    nearest other centroid (inf when no other centroid is left out)."""
    C = _f64(C)
    K = C.shape[0]
    m = min(M, K - 1)
    nb = np.full((K, M), -1, dtype=np.int64)
    beyond = np.full(K, np.inf)
    idx = np.arange(K)
    for p in range(K):
        dist = np.sqrt(_sqdist(C - C[p]))
        dist[p] = np.inf
        order = np.lexsort((idx, dist))
        nb[p, :m] = order[:m]
        if K - 1 > M:
            beyond[p] = dist[order[M]]
    return nb, beyond


def spill_bound_rows(X, C, lam, primary, M):
    """Rows whose spill the bound confines to the M centroids nearest their primary centroid.

    j2 is taken as the nearest centroid other than the primary.  Returns (mask [n] bool,
    radius [n] = ||r|| + sqrt((1 + lam) ||x - c_j2||^2), neighbours [K, M] and the distance to
    the (M+1)-th nearest centroid [K] from ``centroid_neighbours``)."""
    lam = _check_lambda(lam)
    X, C = _f64(X), _f64(C)
    p = np.asarray(primary, dtype=np.int64)
    n = X.shape[0]
    nb, beyond = centroid_neighbours(C, M)
    radius = np.empty(n)
    for i in range(n):
        dist2 = _sqdist(X[i][None, :] - C)
        rn = np.sqrt(dist2[p[i]])
        dist2[p[i]] = np.inf
        radius[i] = rn + np.sqrt((1.0 + lam) * dist2.min())
    return radius < beyond[p], radius, nb, beyond
