// dmrg_gemv_t_noalloc: s = V^T x with its partial sums in a fixed device
// array instead of memory the library allocates, for callers that cannot
// allocate (code under graph capture, tight serving loops).
//
// The array is a file-scope __device__ object: every device the library runs
// on holds its own copy, at its own address, until the process ends.  In host
// code its name is only a stand-in, so the address each device uses is taken
// once per device with hipGetSymbolAddress (that device current) and kept;
// kernels receive that address.  Calls on one device share the array: calls
// that overlap in time on one device (other streams, other threads) race on
// it.  Every partial a call reads was written by the same call, so nothing
// needs to start at zero.
#include <map>
#include <mutex>

#include "gemv.h"
#include "internal.h"

using namespace dmrg;

namespace {

__device__ __align__(256) double scratch[GEMV_PART_BLOCKS * GEMV_PART_COLS];  // 512 KiB

std::map<int, double *> g_scratch_ptr;  // device -> address of its copy of scratch
std::mutex g_scratch_mutex;

dmrg_status scratch_ptr(double **out) {
    int dev = 0;
    DMRG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void *ptr = nullptr;
        DMRG_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return set_error(DMRG_E_HIP, "hipGetSymbolAddress returned no address for device %d", dev);
        it = g_scratch_ptr.emplace(dev, (double *)ptr).first;
    }
    *out = it->second;
    return DMRG_OK;
}

}  // namespace

extern "C" dmrg_status dmrg_gemv_t_noalloc(int64_t n, int32_t k, const double *V, int64_t ldv, const double *x,
                                           double *s, void *stream) {
    clear_error();
    if (n < 1 || ldv < n || !V || !x || !s)
        return set_error(DMRG_E_INVALID_ARG, "need n >= 1, ldv >= n and non-null pointers");
    if (k < 1 || k > GEMV_PART_COLS)
        return set_error(DMRG_E_INVALID_ARG, "k = %d outside 1..%d: the fixed partial-sum buffer holds %d columns", k,
                         GEMV_PART_COLS, GEMV_PART_COLS);
    const int nblk = (int)std::min<int64_t>((n + GEMV_THREADS - 1) / GEMV_THREADS, GEMV_PART_BLOCKS);
    if ((size_t)nblk * GEMV_PART_COLS > sizeof(scratch) / sizeof(double))
        return set_error(DMRG_E_INVALID_ARG, "partial sums of %d blocks exceed the fixed buffer", nblk);
    double *part = nullptr;
    DMRG_TRY(scratch_ptr(&part));
    return gemv_t_launch(n, k, V, ldv, x, s, nblk, part, (hipStream_t)stream);
}
