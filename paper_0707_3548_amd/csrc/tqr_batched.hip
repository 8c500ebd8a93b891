// tqr: batched factorisation -- many independent problems in one persistent
// launch (each factorised as tqr_factor does it, Sec. 3.1, Algorithm 1).
#include "tqr_impl.h"

namespace tqr {

template <int B, int IB, bool F32>
__device__ void batch_one(const tqr_batch_problem &pr, char *work, double *smem) {
    const int64_t m = pr.m, n = pr.n;
    if (m <= 0 || n <= 0) return;
    const int p = (int)((m + B - 1) / B), q = (int)((n + B - 1) / B);
    double *W = reinterpret_cast<double *>(work + pr.work_offset);
    double *Vd = W + (int64_t)p * q * B * B;
    const int64_t tile_elems = (int64_t)B * B, total = (int64_t)p * q * tile_elems;
    for (int64_t idx = threadIdx.x; idx < total; idx += NT) {
        const int64_t t = idx / tile_elems, e = idx - t * tile_elems;
        const int i = (int)(t % p), j = (int)(t / p), r = (int)(e % B), c = (int)(e / B);
        const int64_t gr = (int64_t)i * B + r, gc = (int64_t)j * B + c;
        W[idx] = (gr < m && gc < n) ? pr.A[gc * pr.lda + gr] : 0.0;
    }
    __syncthreads();
    const FactorBody<B, IB, F32> body{W, pr.T, Vd, p};
    const FactorGraph g(p, q, B);
    const int K = p < q ? p : q;
    for (int k = 0; k < K; ++k) {
        body.run(g.decode(g.encode(GEQRT, k, k, k, 0)), smem);
        __syncthreads();
        for (int j = k + 1; j < q; ++j)
            for (int c = 0; c < (int)g.S; ++c) {
                body.run(g.decode(g.encode(LARFB, k, j, k, c)), smem);
                __syncthreads();
            }
        for (int i = k + 1; i < p; ++i) {
            body.run(g.decode(g.encode(TSQRT, i, k, k, 0)), smem);
            __syncthreads();
            for (int j = k + 1; j < q; ++j)
                for (int c = 0; c < (int)g.S; ++c) {
                    body.run(g.decode(g.encode(SSRFB, i, j, k, c)), smem);
                    __syncthreads();
                }
        }
    }
    for (int64_t idx = threadIdx.x; idx < total; idx += NT) {
        const int64_t t = idx / tile_elems, e = idx - t * tile_elems;
        const int i = (int)(t % p), j = (int)(t / p), r = (int)(e % B), c = (int)(e / B);
        const int64_t gr = (int64_t)i * B + r, gc = (int64_t)j * B + c;
        if (gr < m && gc < n) pr.A[gc * pr.lda + gr] = W[idx];
    }
    __syncthreads();
}

constexpr size_t kBatchLds = std::max(
    {TileKernels<16, 16>::LDS_BYTES, TileKernels<32, 16>::LDS_BYTES, TileKernels<32, 32>::LDS_BYTES,
     TileKernels<64, 16>::LDS_BYTES, TileKernels<64, 32>::LDS_BYTES, TileKernels<64, 64>::LDS_BYTES,
     TileKernels<128, 16>::LDS_BYTES, TileKernels<128, 32>::LDS_BYTES});

inline bool batch_pair_ok(int b, int ib) {
    const int i = ib == 0 ? 16 : ib;
    return (b == 16 && i == 16) || (b == 32 && (i == 16 || i == 32)) || (b == 64 && (i == 16 || i == 32 || i == 64)) ||
           (b == 128 && (i == 16 || i == 32));
}

// Persistent launch over the problems; *counter (cleared before the launch)
// hands out problem indices.  Every workgroup leaves once the counter passes
// the count.
template <bool F32>
__global__ void __launch_bounds__(NT) k_batched(const tqr_batch_problem *problems, int64_t count, char *work,
                                                int32_t *counter, int32_t *status) {
    extern __shared__ double smem[];
    __shared__ int32_t s_next;
    for (;;) {
        if (threadIdx.x == 0) s_next = __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int64_t pi = __builtin_amdgcn_readfirstlane(s_next);
        __syncthreads();
        if (pi >= count) break;
        const tqr_batch_problem pr = problems[pi];
        const int ib = pr.inner_ib == 0 ? 16 : pr.inner_ib;
        const int key = pr.tile_b * 1000 + ib;
        bool done = true;
        if constexpr (F32) {
            switch (key) {
            case 16016: batch_one<16, 16, true>(pr, work, smem); break;
            case 32016: batch_one<32, 16, true>(pr, work, smem); break;
            case 64016: batch_one<64, 16, true>(pr, work, smem); break;
            case 128016: batch_one<128, 16, true>(pr, work, smem); break;
            default: done = false; break;
            }
        } else {
            switch (key) {
            case 16016: batch_one<16, 16, false>(pr, work, smem); break;
            case 32016: batch_one<32, 16, false>(pr, work, smem); break;
            case 32032: batch_one<32, 32, false>(pr, work, smem); break;
            case 64016: batch_one<64, 16, false>(pr, work, smem); break;
            case 64032: batch_one<64, 32, false>(pr, work, smem); break;
            case 64064: batch_one<64, 64, false>(pr, work, smem); break;
            case 128016: batch_one<128, 16, false>(pr, work, smem); break;
            case 128032: batch_one<128, 32, false>(pr, work, smem); break;
            default: done = false; break;
            }
        }
        if (!done && threadIdx.x == 0 && status) *status = (int32_t)(pi + 1);
    }
}

int64_t batch_problem_bytes(const tqr_batch_problem &pr) {
    const int64_t b = pr.tile_b;
    const int64_t p = (pr.m + b - 1) / b, q = (pr.n + b - 1) / b;
    return ((p * q * b * b + q * b * b) * 8 + 255) / 256 * 256;
}


}  // namespace tqr

using namespace tqr;

extern "C" {

int64_t tqr_batch_plan(int64_t count, tqr_batch_problem *problems) {
    g_err.clear();
    if (count < 0) return set_err(-1, "count < 0");
    if (count > 0 && !problems) return set_err(-2, "problems is null");
    int64_t off = 256;  // the first 256 bytes hold the problem counter
    for (int64_t i = 0; i < count; ++i) {
        tqr_batch_problem &pr = problems[i];
        const bool bad = pr.n < 0 || pr.m < pr.n || pr.lda < std::max<int64_t>(1, pr.m) ||
                         !batch_pair_ok(pr.tile_b, pr.inner_ib) || (pr.m * pr.n > 0 && (!pr.A || !pr.T));
        if (bad) {
            static thread_local char msg[160];
            snprintf(msg, sizeof msg,
                     "problem %lld: bad m, n, lda, A, T or (tile_b, inner_ib) (16/16, 32/16, 32/32, 64/16, 64/32, "
                     "64/64, 128/16, 128/32)",
                     (long long)i);
            return set_err(-2, msg);
        }
        pr.work_offset = off;
        off += batch_problem_bytes(pr);
    }
    return off;
}

tqr_status tqr_factor_batched(int64_t count, const tqr_batch_problem *d_problems, void *work, int64_t work_bytes,
                              int32_t *d_status, int32_t workgroups, int32_t precision, hipStream_t stream) {
    g_err.clear();
    if (count < 0) return set_err(-1, "count < 0");
    if (count > 0 && !d_problems) return set_err(-2, "d_problems is null");
    if (!work) return set_err(-3, "work is null");
    if (work_bytes < 256) return set_err(-4, "work_bytes < 256");
    if (workgroups < 0) return set_err(-6, "workgroups < 0");
    if (precision != TQR_PRECISION_FP64 && precision != TQR_PRECISION_FP32_UPDATES)
        return set_err(-7, "precision must be TQR_PRECISION_FP64 or TQR_PRECISION_FP32_UPDATES");
    int32_t *counter = reinterpret_cast<int32_t *>(work);
    if (d_status) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_status, 0);
    if (count == 0) {
        HIPCHK(hipGetLastError());
        return TQR_OK;
    }
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, stream, counter, (int64_t)1, 0);
    const bool f32 = precision == TQR_PRECISION_FP32_UPDATES;
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    static int per_cu[2] = {0, 0};
    std::call_once(once, [&] {
        const void *ks[2] = {(const void *)k_batched<false>, (const void *)k_batched<true>};
        for (int v = 0; v < 2 && attr_err == hipSuccess; ++v) {
            attr_err = hipFuncSetAttribute(ks[v], hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLds);
            if (attr_err == hipSuccess)
                attr_err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu[v], ks[v], NT, kBatchLds);
        }
    });
    HIPCHK(attr_err);
    int64_t wg = (int64_t)std::max(per_cu[f32 ? 1 : 0], 1) * cu_count();
    if (workgroups > 0) wg = std::min<int64_t>(wg, workgroups);
    wg = std::min<int64_t>(wg, count);
    if (f32)
        hipLaunchKernelGGL(k_batched<true>, dim3((unsigned)wg), dim3(NT), kBatchLds, stream, d_problems, count,
                           reinterpret_cast<char *>(work), counter, d_status);
    else
        hipLaunchKernelGGL(k_batched<false>, dim3((unsigned)wg), dim3(NT), kBatchLds, stream, d_problems, count,
                           reinterpret_cast<char *>(work), counter, d_status);
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

}  // extern "C"
