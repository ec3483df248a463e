"""Serving index: continuous batching of insert requests, results identical alone and in a mix,
inverted lists equal to the assignments, admission by arena memory."""
import threading
import time

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


@pytest.fixture(scope="module")
def data():
    X = gen_mixture(MixtureSpec(30_000, 64, 32, 0.3, "unit", 7))
    C, _ = O.kmeanspp(X[:5000], 300, 1)
    return X, C.astype(np.float32)


@pytest.mark.parametrize("prec", ["bf16", "fp32", "fp8"])
def test_mixed_requests_match_standalone_assign(data, prec):
    soar = _soar()
    X, C = data
    lam = 1.0
    # serving steps run the direct spill form (their batches are small); the BF16 / FP8 forms
    # round differently in the grouped form, so the reference is the direct form too
    ref_p, ref_s, _, _ = soar.assign(_t(X), _t(C), lam, precision=prec, spill_form="direct")
    ref_p, ref_s = ref_p.cpu().numpy(), ref_s.cpu().numpy()
    ix = soar.SoarIndex(_t(C), lam, precision=prec, max_step_rows=1024, list_capacity=100_000)
    rng = np.random.default_rng(3)
    sizes = np.minimum(np.exp(rng.uniform(0, np.log(4097), 60)).astype(int), 4096)
    tickets, lo = [], 0
    for sz in sizes:
        sz = int(min(sz, len(X) - lo))
        if sz <= 0:
            break
        tickets.append((ix.insert(X[lo:lo + sz], lo), lo, sz))
        lo += sz
    print(f"{prec}: {len(tickets)} requests, {lo} rows", flush=True)
    for t, a, sz in tickets:
        p, s = ix.wait(t, timeout=60.0)
        assert np.array_equal(p, ref_p[a:a + sz]) and np.array_equal(s, ref_s[a:a + sz])
    # lists hold exactly the assignments of the inserted ids
    lists = {k: ix.list(k) for k in range(len(C))}
    got = sorted((int(i), k) for k, ids in lists.items() for i in ids)
    want = sorted([(i, int(ref_p[i])) for i in range(lo)] + [(i, int(ref_s[i])) for i in range(lo)])
    assert got == want
    ix.close()
    if prec == "fp32":
        j = O.verify(X[:lo], C, lam, ref_p[:lo], ref_s[:lo])
        assert j["primary_ok"].all() and j["spill_ok"].all()


def test_first_steps_right_after_create(data):
    """Requests inserted the moment an index exists, before its slot threads may have started
    waiting: every answer must be this request's own (a slot's waiter takes a step only after
    the step's events are recorded)."""
    soar = _soar()
    X, C = data
    ref_p, ref_s, _, _ = soar.assign(_t(X[:3000]), _t(C), 1.0, precision="bf16",
                                     spill_form="direct")
    ref_p, ref_s = ref_p.cpu().numpy(), ref_s.cpu().numpy()
    for trial in range(6):
        ix = soar.SoarIndex(_t(C), 1.0, precision="bf16", max_step_rows=512,
                            list_capacity=20_000)
        lo = 500 * trial
        ts = [ix.insert(X[lo:lo + 100], lo), ix.insert(X[lo + 100:lo + 500], lo + 100)]
        p1, s1 = ix.wait(ts[0], timeout=60.0)
        p2, s2 = ix.wait(ts[1], timeout=60.0)
        ix.close()
        assert np.array_equal(np.concatenate([p1, p2]), ref_p[lo:lo + 500]), trial
        assert np.array_equal(np.concatenate([s1, s2]), ref_s[lo:lo + 500]), trial


def test_alone_and_in_concurrent_mix(data):
    soar = _soar()
    X, C = data
    ix = soar.SoarIndex(_t(C), 1.0, precision="bf16", max_step_rows=512, list_capacity=200_000)
    A = X[:777]
    pa, sa = ix.wait(ix.insert(A, 0), timeout=60.0)
    # the same rows again, submitted from a second thread while others stream in
    out = {}

    def client():
        time.sleep(0.002)
        out["t"] = ix.insert(A, 100_000)

    th = threading.Thread(target=client)
    th.start()
    others = [ix.insert(X[1000 + 300 * k:1000 + 300 * (k + 1)], 1000 + 300 * k) for k in range(20)]
    th.join()
    pb, sb = ix.wait(out["t"], timeout=60.0)
    for t in others:
        ix.wait(t, timeout=60.0)
    assert np.array_equal(pa, pb) and np.array_equal(sa, sb)
    ix.close()


@pytest.mark.parametrize("prec", ["bf16", "fp8", "fp32"])
def test_split_codebook_steps(prec):
    """With K = 8192 every serving sweep runs as two codebook splits (one per 4096 centroids)
    whose candidates (BF16/FP8) or exact answers (FP32) are joined: the answers are the oracle's
    within the low-precision bound (FP32: exactly, and equal to the unsplit assignment),
    the same alone and in a mix of request sizes, and the lists hold exactly them.  (d = 128, the
    serving workload's width.)"""
    soar = _soar()
    X = gen_mixture(MixtureSpec(12_000, 128, 256, 0.3, "unit", 11))
    C = (X[np.random.default_rng(5).choice(len(X), 8192, replace=False)] * 0.97).astype(np.float32)
    ix = soar.SoarIndex(_t(C), 1.0, precision=prec, max_step_rows=1024, list_capacity=100_000)
    n, lo, tickets = 6000, 0, []
    for sz in (1, 37, 500, 1024, 2000, 2438):
        tickets.append((ix.insert(X[lo:lo + sz], lo), lo, sz))
        lo += sz
    p, s = np.empty(n, np.int32), np.empty(n, np.int32)
    for t, a, sz in tickets:
        p[a:a + sz], s[a:a + sz] = ix.wait(t, timeout=60.0)
    pa, sa = ix.wait(ix.insert(X[:500], 50_000), timeout=60.0)
    if not (np.array_equal(pa, p[:500]) and np.array_equal(sa, s[:500])):
        # which of the two answers the oracle accepts, and where they part
        ja = O.verify(X[:500], C, 1.0, pa, sa)
        jp = O.verify(X[:500], C, 1.0, p[:500], s[:500])
        bad = np.flatnonzero(pa != p[:500])
        print("repeat differs at", bad[:10], "count", bad.size, "repeat ok",
              float(ja["primary_ok"].mean()), "first ok", float(jp["primary_ok"].mean()),
              "stats", ix.stats(), flush=True)
    assert np.array_equal(pa, p[:500]) and np.array_equal(sa, s[:500])
    got = sorted((int(i), k) for k in range(len(C)) for i in ix.list(k) if i < n)
    want = sorted([(i, int(p[i])) for i in range(n)] + [(i, int(s[i])) for i in range(n)])
    assert got == want
    ix.close()
    j = O.verify(X[:n], C, 1.0, p, s)
    bound = 1e-3
    print(prec, "split serving: primary regret", float(j["primary_regret"].mean()),
          "spill regret", float(j["spill_regret"].mean()), flush=True)
    assert np.all(s != p) and np.all((p >= 0) & (p < len(C))) and np.all((s >= 0) & (s < len(C)))
    assert j["primary_regret"].mean() <= bound and j["spill_regret"].mean() <= bound
    if prec == "fp32":
        # exact: the joined splits give the unsplit answer
        assert j["primary_ok"].all() and j["spill_ok"].all()
        rp, rs, _, _ = _soar().assign(_t(X[:n]), _t(C), 1.0, spill_form="direct")
        assert np.array_equal(p, rp.cpu().numpy()) and np.array_equal(s, rs.cpu().numpy())


@pytest.mark.parametrize("prec", ["bf16", "fp8", "fp32"])
def test_serving_codebook_50k_eight_splits(prec):
    """The serving shape: K = 50,000 centroids at d = 128, so every sweep runs as 8 codebook
    splits.  Requests of mixed sizes, the oracle's judgement of every row within the
    low-precision bound (FP32: exact), identical answers for a repeated request, and exact
    lists."""
    soar = _soar()
    X = gen_mixture(MixtureSpec(56_000, 128, 2048, 0.3, "unit", 13))
    C = (X[:50_000] * 0.97).astype(np.float32)
    Y = X[50_000:]
    ix = soar.SoarIndex(_t(C), 1.0, precision=prec, max_step_rows=2048, list_capacity=50_000)
    n, lo, tickets = len(Y), 0, []
    for sz in (1, 15, 300, 2048, 1500, 2136):
        tickets.append((ix.insert(Y[lo:lo + sz], lo), lo, sz))
        lo += sz
    assert lo == n
    p, s = np.empty(n, np.int32), np.empty(n, np.int32)
    for t, a, sz in tickets:
        p[a:a + sz], s[a:a + sz] = ix.wait(t, timeout=120.0)
    pa, sa = ix.wait(ix.insert(Y[:300], 100_000), timeout=60.0)
    assert np.array_equal(pa, p[:300]) and np.array_equal(sa, s[:300])
    got = sorted((int(i), k) for k in np.unique(np.concatenate([p, s])) for i in ix.list(int(k))
                 if i < n)
    want = sorted([(i, int(p[i])) for i in range(n)] + [(i, int(s[i])) for i in range(n)])
    assert got == want
    ix.close()
    j = O.verify(Y, C, 1.0, p, s)
    print(prec, "K=50000 serving: primary regret", float(j["primary_regret"].mean()),
          "spill regret", float(j["spill_regret"].mean()), "index disagreement",
          float((p != j["p_star"]).mean()), flush=True)
    assert np.all(s != p) and np.all((p >= 0) & (p < len(C))) and np.all((s >= 0) & (s < len(C)))
    assert j["primary_regret"].mean() <= 1e-3 and j["spill_regret"].mean() <= 1e-3
    if prec == "fp32":
        assert j["primary_ok"].all() and j["spill_ok"].all()


def test_admission_waits_for_memory_and_rejects_too_large(data):
    soar = _soar()
    X, C = data
    # 500 list chunks of 64 ids: a step of 256 rows may need 8 + 300 chunks in the worst case, so
    # a second step has to wait for the first to finish, and later steps shrink to what fits
    ix = soar.SoarIndex(_t(C), 1.0, precision="bf16", max_step_rows=256, list_capacity=0)
    size0 = ix.arena.numel()                 # fixed part + 2 K spare chunks
    chunk = ix.CHUNK_BYTES
    ix.close()
    ix = soar.SoarIndex(_t(C), 1.0, precision="bf16", max_step_rows=256,
                        arena_bytes=size0 - 2 * len(C) * chunk + 500 * chunk)
    assert ix.stats()["chunks_total"] == 500
    tickets = [ix.insert(X[256 * k:256 * (k + 1)], 256 * k) for k in range(4)]
    got = {}
    for k, t in enumerate(tickets):
        got[k] = ix.wait(t, timeout=60.0)
        assert (got[k][0] >= 0).all() and (got[k][1] >= 0).all()
    with pytest.raises(soar.SoarError) as e:
        ix.insert(X[:25_000], 0)             # 50,000 ids can never fit 500 chunks of 64
    assert e.value.status == -2
    # the index keeps working after the rejection, and its lists hold exactly what was inserted
    p5, s5 = ix.wait(ix.insert(X[2000:2100], 2000), timeout=60.0)
    lists = sorted((int(i), k) for k in range(len(C)) for i in ix.list(k))
    want = sorted([(256 * k + i, int(got[k][0][i])) for k in range(4) for i in range(256)] +
                  [(256 * k + i, int(got[k][1][i])) for k in range(4) for i in range(256)] +
                  [(2000 + i, int(p5[i])) for i in range(100)] +
                  [(2000 + i, int(s5[i])) for i in range(100)])
    assert lists == want
    ix.close()


def test_long_lists_and_small_request_behind_a_large_one(data):
    """Lists are chains of chunks with no cap per partition: with K = 2 every point sits in both
    lists, so each list grows to 80,000 ids.  A 40-row request submitted right after a
    60,000-row request (many steps) joins the next step and finishes first, and the steps
    overlap on the device."""
    soar = _soar()
    X, C = data
    X = np.concatenate([X, X, X])[:80_000]
    C2 = C[:2].copy()
    ix = soar.SoarIndex(_t(C2), 1.0, precision="bf16", max_step_rows=2048, list_capacity=200_000)
    big = ix.insert(X[:60_000], 0)
    small = ix.insert(X[60_000:60_040], 60_000)
    ps, ss = ix.wait(small, timeout=60.0)
    with pytest.raises(soar.SoarError) as e:
        ix.wait(big, timeout=0.0)            # the large request is still being served
    assert e.value.status == -6
    pb, sb = ix.wait(big, timeout=120.0)
    rest = ix.insert(X[60_040:], 60_040)
    pr, sr = ix.wait(rest, timeout=120.0)
    st = ix.stats()
    print("stats", st, flush=True)
    assert st["max_steps_in_flight"] >= 2 and st["rows"] == 80_000
    ref_p, ref_s, _, _ = soar.assign(_t(X), _t(C2), 1.0, precision="bf16", spill_form="direct")
    ref_p, ref_s = ref_p.cpu().numpy(), ref_s.cpu().numpy()
    assert np.array_equal(np.concatenate([pb, ps, pr]), ref_p)
    assert np.array_equal(np.concatenate([sb, ss, sr]), ref_s)
    for k in range(2):
        ids = np.sort(ix.list(k))
        assert len(ids) == 80_000 and np.array_equal(ids, np.arange(80_000))
    ix.close()


def test_wait_timeout_and_destroy_with_queued_work(data):
    soar = _soar()
    X, C = data
    ix = soar.SoarIndex(_t(C), 1.0, precision="fp32", max_step_rows=1024, list_capacity=100_000)
    t = ix.insert(X[:20_000], 0)
    try:
        ix.wait(t, timeout=0.0)
    except soar.SoarError as e:
        assert e.status == -6                # still running: the ticket stays valid
        p, s = ix.wait(t, timeout=60.0)
        assert (p >= 0).all()
    for k in range(5):
        ix.insert(X[k * 100:(k + 1) * 100], k * 100)
    ix.close()                               # drains the queue and returns


def test_create_validation(data):
    soar = _soar()
    X, C = data
    with pytest.raises(soar.SoarError):
        soar.SoarIndex(_t(C[:1]), 1.0)
    with pytest.raises(soar.SoarError):
        soar.SoarIndex(_t(C), -1.0)
