"""rbf_knn_noalloc (the kNN entry point for callers that cannot allocate
device memory) against rbf_knn, through the C ABI: bit-identical stencils on
two calls in a row, the second smaller than the first (the shared scratch
array keeps the first call's contents, so stale data would show), and sizes
beyond the scratch array refused with RBF_E_ARG before any search."""
import ctypes

import numpy as np
import pytest

import rbf_inputs as ri
from tests.helpers import to_dev

pytestmark = pytest.mark.gpu


def _call(fn, xq, xs, k, gpu):
    import torch
    nq, ns = xq.shape[1], xs.shape[1]
    idx = torch.full((k, nq), -9, dtype=torch.int32, device=gpu)
    rc = fn(ctypes.c_void_p(xq.data_ptr()), nq, ctypes.c_void_p(xs.data_ptr()), ns, k,
            ctypes.c_void_p(idx.data_ptr()), None)
    torch.cuda.synchronize()
    return rc, idx.cpu().numpy()


def test_knn_noalloc_matches_knn(gpu):
    from paper_2206_06495_amd import _lib
    lib = _lib.lib
    fn = lib.rbf_knn_noalloc
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    big = ri.square_nodes(300, 0.3, 1)      # 90,000 + 90,000 nodes
    small = ri.cavity_nodes(9, 0.3, 2)      # 261 V + 100 P nodes
    for name, nd, k in (("large", big, 28), ("small", small, 17)):
        print("knn_noalloc", name, nd.n_v, nd.n_p, k, flush=True)
        for xq, xs in ((nd.xp, nd.xv), (nd.xv, nd.xv)):
            dq, ds = to_dev(xq, gpu), to_dev(xs, gpu)
            rc_a, ref = _call(lib.rbf_knn, dq, ds, k, gpu)
            rc_b, got = _call(fn, dq, ds, k, gpu)
            assert rc_a == 0 and rc_b == 0, (rc_a, rc_b, lib.rbf_last_error())
            assert np.array_equal(got, ref), name


def test_knn_noalloc_rejects_oversize(gpu):
    import torch
    from paper_2206_06495_amd import _lib
    lib = _lib.lib
    fn = lib.rbf_knn_noalloc
    fn.restype = ctypes.c_int32
    fn.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    print("knn_noalloc oversize", flush=True)
    ns = 2_500_000  # about 30 bytes of scratch per source: 75 MB > 64 MiB
    xs = torch.rand((2, ns), dtype=torch.float64, device=gpu)
    xq = xs[:, :1000].contiguous()
    rc, idx = _call(fn, xq, xs, 28, gpu)
    assert rc == _lib.RBF_E_ARG
    assert "scratch" in lib.rbf_last_error().decode()
    assert (idx == -9).all()
