"""soar_assign_noalloc (the allocation-free variant of soar_assign, whose workspace is a fixed
device array) against soar_assign, through the C ABI: two calls in a row, the second smaller,
must give the same outputs bit for bit (the same kernels run on both workspaces)."""
import ctypes

import numpy as np
import pytest

from synth import MixtureSpec, gen_mixture

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _noalloc(soar, X, C, lam, prec):
    import torch
    n, d = X.shape
    K = C.shape[0]
    out = [torch.full((n,), -9, dtype=torch.int32, device="cuda") for _ in range(2)] + \
          [torch.full((n,), -9.0, dtype=torch.float32, device="cuda") for _ in range(2)]
    o = soar._opts(lam, prec, 0, 0.0, 0)
    st = soar._lib.soar_assign_noalloc(soar._ptr(X), n, d, soar._ptr(C), K, ctypes.byref(o),
                                       *[soar._ptr(t) for t in out], soar._stream(None))
    assert st == 0, soar._lib.soar_status_string(st)
    return [t.cpu().numpy() for t in out]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp8"])
def test_noalloc_matches_workspace_call(prec):
    import paper_2404_00774_amd as soar
    soar._lib.soar_assign_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                              ctypes.c_void_p, ctypes.c_int32,
                                              ctypes.POINTER(soar.AssignOpts)] + \
        [ctypes.c_void_p] * 5
    soar._lib.soar_assign_noalloc.restype = ctypes.c_int
    for n, K, seed in ((30_000, 700, 1), (5_000, 300, 2)):   # the second call is smaller
        print(f"noalloc {prec} n={n} K={K}", flush=True)
        X = gen_mixture(MixtureSpec(n, 96, 256, ("loguniform", 0.05, 0.5), "unit", seed))
        C = X[np.random.default_rng(seed).choice(n, K, replace=False)].copy()
        Xg, Cg = _t(X), _t(C)
        ref = [t.cpu().numpy() for t in soar.assign(Xg, Cg, 1.0, prec)]
        got = _noalloc(soar, Xg, Cg, 1.0, prec)
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)


def test_noalloc_rejects_beyond_limit():
    import paper_2404_00774_amd as soar
    lim = soar._lib.soar_assign_noalloc_limit
    lim.restype = ctypes.c_size_t
    n, d, K = 2_000_000, 128, 1000
    assert soar.assign_workspace_size(n, d, K, 1.0, "bf16") > lim()
    o = soar._opts(1.0, "bf16", 0, 0.0, 0)
    # sizes only: the call is rejected before any launch, so no buffer of that size is needed
    import torch
    X = torch.zeros((8, d), dtype=torch.float32, device="cuda")
    p = torch.zeros(8, dtype=torch.int32, device="cuda")
    st = soar._lib.soar_assign_noalloc(soar._ptr(X), n, d, soar._ptr(X), K, ctypes.byref(o),
                                       soar._ptr(p), soar._ptr(p), None, None, None)
    assert st == -2
