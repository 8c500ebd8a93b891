// tqr_factor_noalloc: the tiled QR factorisation (Sec. 3.1, Algorithm 1)
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).
//
// The workspace that tqr_factor takes as an argument (the tile copy of A, the
// dense diagonal V blocks, the scheduler's counters, queues and mailboxes,
// and the R_kk chain's progress words) lives here in a file-scope device
// array of TQR_NOALLOC_SCRATCH_BYTES.  Each GPU holds its own copy of the
// array, at its own address, from the first call on that GPU until the
// process ends.  The factorisation path itself clears everything it needs
// cleared with kernels on the caller's stream (scheduler state, progress
// words) and writes every tile before reading it, so the contents left by an
// earlier call do not matter.  Calls that overlap on one GPU share the array
// and race; calls on one stream, or ordered by events, do not.
#include <mutex>

#include "tqr_impl.h"

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[TQR_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, or null before its first call

// The array's device address on the current device.  Host code must use this
// address, never the array's name (on the host the name is a stand-in, not a
// device address).
tqr_status scratch_on_current_device(void **out) {
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return tqr::set_err(TQR_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return tqr::set_err(TQR_EDEVICE, "hipGetSymbolAddress returned a null address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return TQR_OK;
}

}  // namespace

using tqr::set_err;

extern "C" tqr_status tqr_factor_noalloc(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib,
                                         double *T, hipStream_t stream) {
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (m == 0 || n == 0) return TQR_OK;
    if (!A) return set_err(-3, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-4, "lda < max(1, m)");
    if (!(tile_b == 16 || tile_b == 32 || tile_b == 64 || tile_b == 128 || tile_b == 256))
        return set_err(-5, "tile_b must be one of 16, 32, 64, 128, 256");
    if (!tqr::tiles_ok(tile_b, inner_ib))
        return set_err(-6, "inner_ib must be 16, 32 or 64, divide tile_b, and ib*(b+ib) <= 9216");
    if (!T) return set_err(-7, "T is null");
    const int64_t need = tqr_workspace_bytes(m, n, 0, tile_b, inner_ib);
    if (need < 0 || need > (int64_t)TQR_NOALLOC_SCRATCH_BYTES)
        return set_err(TQR_ESCRATCH, "tqr_factor_noalloc: this factorisation needs " + std::to_string(need) +
                                         " bytes of workspace, more than the library's fixed scratch of " +
                                         std::to_string((int64_t)TQR_NOALLOC_SCRATCH_BYTES) +
                                         " bytes; call tqr_factor with a workspace instead");
    void *work = nullptr;
    const tqr_status st = scratch_on_current_device(&work);
    if (st != TQR_OK) return st;
    return tqr_factor(m, n, A, lda, tile_b, inner_ib, T, work, (int64_t)TQR_NOALLOC_SCRATCH_BYTES, stream);
}
