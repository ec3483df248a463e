"""PQ codes of the residuals on the GPU (soar_pq_encode, Section 3.5) against the oracle: every
code is the nearest codeword of its residual piece (ties to the lowest index), packed two per
byte, for each of a point's assignments."""
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


def _unpack(packed):
    p = np.asarray(packed, dtype=np.int64)
    out = np.empty(p.shape[:-1] + (2 * p.shape[-1],), dtype=np.int64)
    out[..., 0::2] = p & 15
    out[..., 1::2] = p >> 4
    return out


def _check(X, C, P, A, got):
    """Codes equal the oracle's, or (a near-tie) have the same FP64 distance within 1e-12."""
    want = O.soar_pq_codes(X, C, P, [A[:, j] for j in range(A.shape[1])])
    g = _unpack(got)
    assert g.shape == want.shape
    diff = np.argwhere(g != want)
    Pd = P.astype(np.float64)
    M, h, s = P.shape
    for i, j, m in diff:
        r = X[i, m * s:(m + 1) * s].astype(np.float64) - C[A[i, j], m * s:(m + 1) * s]
        dg = ((r - Pd[m, g[i, j, m]]) ** 2).sum()
        dw = ((r - Pd[m, want[i, j, m]]) ** 2).sum()
        assert abs(dg - dw) <= 1e-12 * max(dw, 1e-30), (i, j, m, dg, dw)
    return diff.shape[0]


@pytest.mark.parametrize("d,s", [(128, 1), (128, 2), (128, 4), (96, 8), (64, 16), (2, 1),
                                 (768, 2), (1024, 4), (40, 2)])
def test_codes_match_oracle(d, s):
    rng = np.random.default_rng(d * 31 + s)
    n, K, m = 3000, 200, 2
    X = rng.standard_normal((n, d)).astype(np.float32)
    C = (rng.standard_normal((K, d)) * 0.8).astype(np.float32)
    P = (rng.standard_normal((d // s, 16, s)) * 0.5).astype(np.float32)
    A = np.stack([rng.integers(0, K, n), rng.integers(0, K, n)], axis=1)
    print(f"pq d={d} s={s}", flush=True)
    got = _soar().pq_encode(_t(X), _t(C), _ti(A), _t(P)).cpu().numpy()
    assert got.shape == (n, m, d // s // 2)
    assert _check(X, C, P, A, got) <= n * m * (d // s) // 10000


def test_integer_ties_are_exact():
    """Integer data: every distance is exact, so the lowest-index nearest codeword is the only
    answer, also where duplicated codewords tie."""
    rng = np.random.default_rng(7)
    n, d, s, K = 1000, 16, 2, 30
    X = rng.integers(-3, 4, size=(n, d)).astype(np.float32)
    C = rng.integers(-3, 4, size=(K, d)).astype(np.float32)
    P = rng.integers(-2, 3, size=(d // s, 16, s)).astype(np.float32)
    P[:, 9] = P[:, 2]
    A = np.stack([rng.integers(0, K, n) for _ in range(3)], axis=1)
    got = _soar().pq_encode(_t(X), _t(C), _ti(A), _t(P)).cpu().numpy()
    want = O.soar_pq_codes(X, C, P, [A[:, j] for j in range(3)])
    assert np.array_equal(_unpack(got), want)
    assert np.array_equal(got, O.pq_pack(want))


def test_validation():
    soar = _soar()
    rng = np.random.default_rng(1)
    X = rng.standard_normal((10, 8)).astype(np.float32)
    C = rng.standard_normal((5, 8)).astype(np.float32)
    P = rng.standard_normal((4, 16, 2)).astype(np.float32)
    with pytest.raises(soar.SoarError) as e:
        soar.pq_encode(_t(X), _t(C), _ti(np.full((10, 1), 5)), _t(P))
    assert e.value.status == -1
    with pytest.raises(ValueError):
        soar.pq_encode(_t(X), _t(C), _ti(np.zeros((10, 1))), _t(P[:3]))
    Xb = rng.standard_normal((4, 1040)).astype(np.float32)
    Cb = rng.standard_normal((3, 1040)).astype(np.float32)
    Pb = rng.standard_normal((520, 16, 2)).astype(np.float32)
    with pytest.raises(soar.SoarError) as e:
        soar.pq_encode(_t(Xb), _t(Cb), _ti(np.zeros((4, 1))), _t(Pb))
    assert e.value.status == -4


def test_trained_codebook_on_the_workload_sampled():
    """n = 1,000,000, d = 128, K = 2000: a PQ codebook (s = 2) trained by the oracle (k-means per
    subspace) on the primary residuals of a 20,000-row sample, two distinct seeded assignments
    per row (codes are defined for any), the codes of every row on the GPU, and the oracle on
    5000 sampled rows."""
    soar = _soar()
    w = WORKLOADS["mix4096_n1m_d128"]
    spec = w["spec"]
    X = gen_mixture(spec)
    K = w["K"]
    C = X[sample_rows(spec, K)]
    rng = np.random.default_rng(5)
    sub = np.sort(rng.choice(len(X), 20_000, replace=False))
    p_sub, _ = O.primary_fast(X[sub], C)
    R = X[sub].astype(np.float64) - C[p_sub]
    P = np.stack([O.train_codebook(R[:, 2 * m:2 * m + 2], 16, 5, seed=m)[0]
                  for m in range(X.shape[1] // 2)]).astype(np.float32)
    a0 = rng.integers(0, K, len(X))
    a1 = (a0 + rng.integers(1, K, len(X))) % K
    A = np.stack([a0, a1], axis=1)
    codes = soar.pq_encode(_t(X), _t(C), _ti(A), _t(P)).cpu().numpy()
    idx = np.sort(rng.choice(len(X), 5000, replace=False))
    assert _check(X[idx], C, P, A[idx], codes[idx]) <= 5
