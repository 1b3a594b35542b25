"""The allocation-free k-means entry point (pfe_kmeans_noalloc, scratch in a
static device array of the library) against pfe_kmeans (scratch allocated per
call), through the C ABI: identical labels, centroids and iteration counts on
two calls in a row, the second with a smaller input, no library allocation
during the calls, and the argument limit."""
import ctypes as C

import numpy as np
import pytest

from gpu_helpers import banner

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)


def run(fn, Y, C0, max_iter):
    from paper_1612_06496_amd import _lib as L
    n, d = Y.shape
    K = C0.shape[0]
    labels = torch.full((n,), 7, dtype=torch.int32, device="cuda")
    cen = torch.empty((K, d), dtype=torch.float64, device="cuda")
    iters = C.c_int32(-1)
    dt = L.PFE_FP64 if Y.dtype == torch.float64 else L.PFE_FP32
    stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = fn(C.c_void_p(Y.data_ptr()), n, d, dt, C.c_void_p(C0.data_ptr()), K, max_iter,
            C.c_void_p(labels.data_ptr()), C.c_void_p(cen.data_ptr()), C.byref(iters), stream)
    return st, labels.cpu().numpy(), cen.cpu().numpy(), iters.value


def case(n, d, K, seed, dtype):
    rng = np.random.default_rng(seed)
    centres = rng.normal(0.0, 3.0, size=(K, d))
    Y = centres[rng.integers(K, size=n)] + rng.normal(size=(n, d))
    Yt = torch.as_tensor(Y, dtype=dtype, device="cuda")
    C0 = torch.as_tensor(Y[rng.choice(n, K, replace=False)], dtype=torch.float64, device="cuda")
    return Yt, C0


def test_noalloc_kmeans_matches_allocating_entry_point():
    from paper_1612_06496_amd import _lib as L
    from paper_1612_06496_amd import live_allocations
    banner("pfe_kmeans_noalloc vs pfe_kmeans, two calls (large, then small)")
    for (n, d, K, seed, dtype) in [(200_000, 10, 40, 1, torch.float32), (20_000, 6, 12, 2, torch.float64)]:
        Y, C0 = case(n, d, K, seed, dtype)
        st_a, lab_a, cen_a, it_a = run(L.lib.pfe_kmeans, Y, C0, 100)
        live = live_allocations()
        st_b, lab_b, cen_b, it_b = run(L.lib.pfe_kmeans_noalloc, Y, C0, 100)
        assert live_allocations() == live
        print(f"n={n} d={d} K={K}: iterations {it_a} / {it_b}; labels equal {np.array_equal(lab_a, lab_b)}")
        assert st_a == L.PFE_OK and st_b == L.PFE_OK
        assert it_a == it_b and it_a >= 1
        assert np.array_equal(lab_a, lab_b)
        assert np.array_equal(cen_a, cen_b)
        assert lab_b.min() >= 0 and lab_b.max() < K


def test_noalloc_kmeans_rejects_sizes_beyond_its_scratch():
    from paper_1612_06496_amd import _lib as L
    banner("pfe_kmeans_noalloc argument limits")
    Y, C0 = case(5_000, 32, 251, 3, torch.float32)     # K d = 8032 > 8000
    st, _, _, _ = run(L.lib.pfe_kmeans_noalloc, Y, C0, 5)
    assert st == L.PFE_E_ARG
    assert b"bad argument" in L.lib.pfe_last_error()
