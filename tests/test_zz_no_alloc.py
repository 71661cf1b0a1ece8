"""dmrg_gemv_t_noalloc (partial sums in a fixed device array, no allocation)
against dmrg_gemv_t (library-allocated partials), called through the C ABI:
two calls in a row, the second on a smaller input, and each checked against
NumPy."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib():
    from paper_1309_5571_amd import _native as N

    return N, N.lib()


def _call(fn, V, x, k, stream):
    s = torch.full((k,), float("nan"), dtype=torch.float64, device="cuda")
    st = fn(V.shape[1], k, ctypes.c_void_p(V.data_ptr()), V.stride(0), ctypes.c_void_p(x.data_ptr()),
            ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(stream))
    return st, s


def test_noalloc_matches_allocating_entry_point_twice():
    N, lib = _lib()
    stream = torch.cuda.current_stream().cuda_stream
    g = torch.Generator(device="cuda").manual_seed(11)
    cases = [(1_000_003, 40), (70_001, 17)]  # the second call is smaller in n and k
    for n, k in cases:
        print(f"gemv_t_noalloc n={n} k={k}", flush=True)
        V = torch.randn(k, n, dtype=torch.float64, device="cuda", generator=g)
        x = torch.randn(n, dtype=torch.float64, device="cuda", generator=g)
        st_a, a = _call(lib.dmrg_gemv_t_noalloc, V, x, k, stream)
        st_b, b = _call(lib.dmrg_gemv_t, V, x, k, stream)
        torch.cuda.synchronize()
        assert st_a == 0 and st_b == 0, N.last_error()
        a, b = a.cpu().numpy(), b.cpu().numpy()
        # same kernels, same grid, same summation order: identical bits
        assert np.array_equal(a, b)
        Vh, xh = V.cpu().numpy(), x.cpu().numpy()
        ref = Vh @ xh
        bound = 4 * n * 2.0 ** -53 * (np.abs(Vh) @ np.abs(xh))
        assert np.all(np.abs(a - ref) <= bound)


def test_noalloc_rejects_k_beyond_the_fixed_buffer():
    N, lib = _lib()
    stream = torch.cuda.current_stream().cuda_stream
    V = torch.zeros(65, 1000, dtype=torch.float64, device="cuda")
    x = torch.zeros(1000, dtype=torch.float64, device="cuda")
    st, _ = _call(lib.dmrg_gemv_t_noalloc, V, x, 65, stream)
    assert st == N.E_INVALID_ARG
    assert "fixed partial-sum buffer" in N.last_error()
