// tqr: batched factorisation -- many independent problems in one persistent
// launch (each factorised as tqr_factor does it, Sec. 3.1, Algorithm 1).
#include "tqr_impl.h"

namespace tqr {

template <int B>
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
    const FactorBody<B, 16> body{W, pr.T, Vd, p};
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

constexpr size_t kBatchLds =
    std::max(std::max(TileKernels<16, 16>::LDS_BYTES, TileKernels<32, 16>::LDS_BYTES),
             std::max(TileKernels<64, 16>::LDS_BYTES, TileKernels<128, 16>::LDS_BYTES));

// Persistent launch over the problems; *counter (cleared before the launch)
// hands out problem indices.  Every workgroup leaves once the counter passes
// the count.
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
        switch (pr.tile_b) {
        case 16: batch_one<16>(pr, work, smem); break;
        case 32: batch_one<32>(pr, work, smem); break;
        case 64: batch_one<64>(pr, work, smem); break;
        case 128: batch_one<128>(pr, work, smem); break;
        default:
            if (threadIdx.x == 0 && status) *status = (int32_t)(pi + 1);
            break;
        }
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
        const bool tile_ok = pr.tile_b == 16 || pr.tile_b == 32 || pr.tile_b == 64 || pr.tile_b == 128;
        const bool bad = pr.n < 0 || pr.m < pr.n || pr.lda < std::max<int64_t>(1, pr.m) || !tile_ok ||
                         (pr.m * pr.n > 0 && (!pr.A || !pr.T)) || pr.reserved != 0;
        if (bad) {
            static thread_local char msg[128];
            snprintf(msg, sizeof msg, "problem %lld: bad m, n, lda, tile_b (16, 32, 64, 128), A, T or reserved",
                     (long long)i);
            return set_err(-2, msg);
        }
        pr.work_offset = off;
        off += batch_problem_bytes(pr);
    }
    return off;
}

tqr_status tqr_factor_batched(int64_t count, const tqr_batch_problem *d_problems, void *work, int64_t work_bytes,
                              int32_t *d_status, int32_t workgroups, hipStream_t stream) {
    g_err.clear();
    if (count < 0) return set_err(-1, "count < 0");
    if (count > 0 && !d_problems) return set_err(-2, "d_problems is null");
    if (!work) return set_err(-3, "work is null");
    if (work_bytes < 256) return set_err(-4, "work_bytes < 256");
    if (workgroups < 0) return set_err(-7, "workgroups < 0");
    int32_t *counter = reinterpret_cast<int32_t *>(work);
    if (d_status) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_status, 0);
    if (count == 0) {
        HIPCHK(hipGetLastError());
        return TQR_OK;
    }
    hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, stream, counter, (int64_t)1, 0);
    static std::once_flag once;
    static hipError_t attr_err = hipSuccess;
    static int per_cu = 0;
    std::call_once(once, [&] {
        attr_err = hipFuncSetAttribute((const void *)k_batched, hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBatchLds);
        if (attr_err == hipSuccess)
            attr_err = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_batched, NT, kBatchLds);
    });
    HIPCHK(attr_err);
    int64_t wg = (int64_t)std::max(per_cu, 1) * cu_count();
    if (workgroups > 0) wg = std::min<int64_t>(wg, workgroups);
    wg = std::min<int64_t>(wg, count);
    hipLaunchKernelGGL(k_batched, dim3((unsigned)wg), dim3(NT), kBatchLds, stream, d_problems, count,
                       reinterpret_cast<char *>(work), counter, d_status);
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

}  // extern "C"
