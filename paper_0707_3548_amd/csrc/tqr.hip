// tqr: tiled QR (Buttari, Langou, Kurzak, Dongarra) on one MI355X.
//
// The C entry points of include/tqr.h, the small layout and bookkeeping
// kernels, and the reference (Algorithm 1) task orders.  The tile kernels and
// the persistent scheduler are in tqr_impl.h, instantiated per (tile_b,
// inner_ib) pair in tqr_inst.hip; the batched launch is in tqr_batched.hip.
#include "tqr_impl.h"

namespace tqr {

thread_local std::string g_err;

// ===========================================================================
// Layout: column-major <-> tiles (Block Data Layout, Sec. 3.4)
// ===========================================================================
__global__ void k_cm_to_tiles(const double *__restrict__ A, int64_t lda, int64_t m, int64_t n,
                              double *__restrict__ W, int p, int b, int tw) {
    const int i = blockIdx.x, j = blockIdx.y;
    double *t = W + ((int64_t)j * p + i) * b * tw;
    const int64_t r0 = (int64_t)i * b, c0 = (int64_t)j * tw;
    for (int idx = threadIdx.x; idx < b * tw; idx += blockDim.x) {
        const int r = idx % b, c = idx / b;
        const int64_t gr = r0 + r, gc = c0 + c;
        t[idx] = (gr < m && gc < n) ? A[gc * lda + gr] : 0.0;
    }
}

__global__ void k_tiles_to_cm(const double *__restrict__ W, int p, int b, int tw, double *__restrict__ A,
                              int64_t lda, int64_t m, int64_t n) {
    const int i = blockIdx.x, j = blockIdx.y;
    const double *t = W + ((int64_t)j * p + i) * b * tw;
    const int64_t r0 = (int64_t)i * b, c0 = (int64_t)j * tw;
    for (int idx = threadIdx.x; idx < b * tw; idx += blockDim.x) {
        const int r = idx % b, c = idx / b;
        const int64_t gr = r0 + r, gc = c0 + c;
        if (gr < m && gc < n) A[gc * lda + gr] = t[idx];
    }
}

// Copies the launch's status word; with only_errors a zero status leaves
// *out as it is (so a later phase does not hide an earlier phase's abort).
__global__ void k_copy_status(const SchedState *st, int32_t *out, int only_errors) {
    const int32_t v = st->status;
    if (!only_errors || v != 0) *out = v;
}

__global__ void k_set_int(int32_t *out, int32_t v) { *out = v; }
__global__ void k_fill_u64(uint64_t *out, int64_t n, uint64_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}
__global__ void k_fill_int(int32_t *out, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = v;
}

// Dense unit-lower copy of the reflectors of diagonal tile k (block k of the
// grid): zeros above the diagonal, ones on it, V_kk below.
__global__ void k_unit_lower(const double *__restrict__ W, int p, int b, double *__restrict__ Vd) {
    const int k = blockIdx.x;
    const double *t = W + ((int64_t)k * p + k) * b * b;
    double *v = Vd + (int64_t)k * b * b;
    for (int idx = threadIdx.x; idx < b * b; idx += blockDim.x) {
        const int r = idx % b, c = idx / b;
        v[idx] = r < c ? 0.0 : (r == c ? 1.0 : t[idx]);
    }
}

// Q[0:m, 0:n] = [I_n; 0] (column-major, leading dimension ldq); grid
// (ceil(m / 256), n).
__global__ void k_eye(double *Q, int64_t ldq, int64_t m) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x, c = blockIdx.y;
    if (r < m) Q[c * ldq + r] = r == c ? 1.0 : 0.0;
}

// d_info: smallest 1-based index k with R(k,k) == 0, else 0.
// ---- FP64 residual kernels of least-squares refinement -------------------
// F = B - Rv - A X (m x nrhs, all column-major); the sum over A's columns is
// split over gridDim.y blocks of columns into Part (gridDim.y x m x nrhs),
// which k_resid_reduce adds in a fixed order.
__global__ void k_resid_partial(const double *A, int64_t lda, int64_t m, int64_t n, const double *X, int64_t ldx,
                                int nrhs, double *Part, const int32_t *skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || (skip && *skip)) return;
    const int64_t per = (n + gridDim.y - 1) / gridDim.y, j0 = blockIdx.y * per, j1 = min(n, j0 + per);
    for (int c0 = 0; c0 < nrhs; c0 += 4) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int64_t j = j0; j < j1; ++j) {
            const double a = A[j * lda + i];
#pragma unroll
            for (int c = 0; c < 4; ++c)
                if (c0 + c < nrhs) acc[c] += a * X[(c0 + c) * ldx + j];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (c0 + c < nrhs) Part[((int64_t)blockIdx.y * nrhs + c0 + c) * m + i] = acc[c];
    }
}
// Q = sum over the column chunks of Part (chunks x m x nrhs), in a fixed order.
__global__ void k_sum_chunks(const double *Part, int chunks, int64_t m, int nrhs, double *Q) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * nrhs) return;
    const int64_t i = idx % m, c = idx / m;
    double s = 0.0;
    for (int k = 0; k < chunks; ++k) s += Part[((int64_t)k * nrhs + c) * m + i];
    Q[c * m + i] = s;
}

// Rv = B - (sum over the column chunks of Part) for the columns still
// iterating (fixed-order sum).
__global__ void k_resid_replace(const double *Bm, int64_t ldb, const double *Part, int chunks, int64_t m, int nrhs,
                                double *Rv, const CglsState *st) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= m * nrhs) return;
    const int64_t i = idx % m, c = idx / m;
    if (st[c].alpha == 0.0) return;
    double s = 0.0;
    for (int k = 0; k < chunks; ++k) s += Part[((int64_t)k * nrhs + c) * m + i];
    Rv[c * m + i] = Bm[c * ldb + i] - s;
}

// G = A^T Rv (n x nrhs, leading dimension n; Rv m x nrhs, leading dimension
// m): one block per column of A, a fixed-order tree sum.
__global__ void k_gemv_t(const double *A, int64_t lda, int64_t m, const double *Rv, int nrhs, double *G, int64_t n,
                         const int32_t *skip) {
    __shared__ double red[NWAVES][kNarrowRhs];
    if (skip && *skip) return;
    const int64_t j = blockIdx.x;
    const double *a = A + j * lda;
    double s[kNarrowRhs] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = threadIdx.x; i < m; i += NT) {
        const double v = a[i];
#pragma unroll
        for (int c = 0; c < kNarrowRhs; ++c)
            if (c < nrhs) s[c] += v * Rv[c * m + i];
    }
#pragma unroll
    for (int c = 0; c < kNarrowRhs; ++c) {
        const double w = wave_sum(s[c]);
        if (lane_id() == 0) red[wave_id()][c] = w;
    }
    __syncthreads();
    if (threadIdx.x < (unsigned)nrhs) {
        double t = 0.0;
        for (int w = 0; w < NWAVES; ++w) t += red[w][threadIdx.x];
        G[threadIdx.x * n + j] = t;
    }
}

// out[j] = sum of squares of column j of A (one block per column).
__global__ void k_col_sumsq(const double *A, int64_t lda, int64_t m, double *out) {
    __shared__ double red[NWAVES];
    const double *a = A + (int64_t)blockIdx.x * lda;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += NT) s += a[i] * a[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

// *out = sum of v[0:n] (one block, fixed order).
__global__ void k_sum_vec(const double *v, int64_t n, double *out) {
    __shared__ double red[NWAVES];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += NT) s += v[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// ---- CGLS on A R^{-1} (mixed-precision least squares) ----------------------
// One block per right-hand side c for the reductions; sums in a fixed order.
__device__ double col_dot(const double *u, const double *v, int64_t rows) {
    __shared__ double red[NWAVES];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += NT) s += u[i] * v[i];
    return block_sum(s, red);
}

// p = s, gamma = ||s||^2; every column active.
__global__ void k_cgls_start(const double *S, int64_t n, double *P, const double *Rv, int64_t m, int nrhs,
                             CglsState *st, int max_iter) {
    const int c = blockIdx.x;
    const double *sc = S + (int64_t)c * n;
    for (int64_t i = threadIdx.x; i < n; i += NT) P[(int64_t)c * n + i] = sc[i];
    const double g = col_dot(sc, sc, n);
    if (threadIdx.x == 0) {
        CglsState z{};
        z.gamma = g;
        z.best = g;
        z.eta = -1.0;
        z.active = (g > 0.0 && max_iter > 0) ? 1 : 0;
        z.stop = g > 0.0 ? (max_iter > 0 ? 0 : TQR_REFINE_MAX_ITERATIONS) : TQR_REFINE_CONVERGED;
        st[c] = z;
    }
}

// alpha = gamma / ||q||^2 (q = A R^{-1} p).
__global__ void k_cgls_step(const double *Q, int64_t m, int nrhs, CglsState *st) {
    const int c = blockIdx.x;
    const double *qc = Q + (int64_t)c * m;
    const double qq = col_dot(qc, qc, m);
    if (threadIdx.x == 0) {
        CglsState &z = st[c];
        if (!z.active) {
            z.alpha = 0.0;
        } else if (!(qq > 0.0)) {
            z.alpha = 0.0;
            z.active = 0;
            z.stop = TQR_REFINE_BREAKDOWN;
        } else {
            z.alpha = z.gamma / qq;
            z.iters += 1;
        }
    }
}

// x += alpha t, r -= alpha q for the active columns.
__global__ void k_cgls_update_xr(double *Xv, const double *Tv, int64_t n, double *Rv, const double *Q, int64_t m,
                                 int nrhs, const CglsState *st) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t rows = m > n ? m : n;
    if (idx >= rows * nrhs) return;
    const int64_t i = idx % rows, c = idx / rows;
    const double a = st[c].alpha;
    if (a == 0.0) return;
    if (i < n) Xv[c * n + i] += a * Tv[c * n + i];
    if (i < m) Rv[c * m + i] -= a * Q[c * m + i];
}

// beta = ||s||^2 / gamma and the stopping test on
// eta = ||s|| / (||A||_F ||x||) (s = R^{-T} A^T r, the backward-error
// estimate of Karlson and Walden with R for the triangle of [A; mu I],
// exact when mu = ||r|| / ||x|| is below A's smallest singular value):
// converged when eta <= TQR_REFINE_ETA_TOL; stagnated when three iterations
// in a row have not halved the smallest ||s|| seen (rounding then decides s).
__global__ void k_cgls_next(const double *S, const double *Xv, const double *Rv, int64_t n, int64_t m, int nrhs,
                            const double *fro2, CglsState *st, int iter) {
    const int c = blockIdx.x;
    const double *sc = S + (int64_t)c * n;
    const double ss = col_dot(sc, sc, n);
    const double xx = col_dot(Xv + (int64_t)c * n, Xv + (int64_t)c * n, n);
    if (threadIdx.x == 0) {
        CglsState &z = st[c];
        if (!z.active) {
            z.beta = 0.0;
            return;
        }
        const double den = sqrt(*fro2) * sqrt(xx);
        z.eta = den > 0.0 ? sqrt(ss) / den : -1.0;
        z.beta = z.gamma > 0.0 ? ss / z.gamma : 0.0;
        z.gamma = ss;
        // progress: ||s|| at least halved since the best value so far
        if (ss < 0.25 * z.best) {
            z.best = ss;
            z.since = 0;
        } else {
            z.since += 1;
        }
        if (!(ss > 0.0) || (z.eta >= 0.0 && z.eta <= TQR_REFINE_ETA_TOL)) {
            z.active = 0;
            z.stop = TQR_REFINE_CONVERGED;
        } else if (z.since >= 3) {
            z.active = 0;
            z.stop = TQR_REFINE_STAGNATED;
        }
    }
}

// p = s + beta p for the active columns.
__global__ void k_cgls_update_p(double *P, const double *S, int64_t n, int nrhs, const CglsState *st) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * nrhs) return;
    const int64_t c = idx / n;
    if (!st[c].active) return;
    P[idx] = S[idx] + st[c].beta * P[idx];
}

// *done = 1 when no column of the chunk is still iterating.
__global__ void k_cgls_alldone(const CglsState *st, int nrhs, int32_t *done) {
    if (threadIdx.x != 0) return;
    int any = 0;
    for (int c = 0; c < nrhs; ++c) any |= st[c].active;
    *done = any ? 0 : 1;
}

// Statistics of an empty problem (nothing to refine).
__global__ void k_refine_stats_empty(tqr_refine_stats *out, int64_t nrhs) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c < nrhs) out[c] = tqr_refine_stats{0, TQR_REFINE_CONVERGED, 0.0};
}

// Per-column statistics for the caller; a column still active ran out of
// iterations.
__global__ void k_cgls_report(const CglsState *st, int nrhs, tqr_refine_stats *out) {
    const int c = threadIdx.x;
    if (c >= nrhs) return;
    tqr_refine_stats r;
    r.iterations = st[c].iters;
    r.stop = st[c].active ? TQR_REFINE_MAX_ITERATIONS : st[c].stop;
    r.eta = st[c].eta;
    out[c] = r;
}

__global__ void k_copy_cm(const double *S, int64_t lds, double *D, int64_t ldd, int64_t rows, int nrhs, double scale) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * nrhs) return;
    const int64_t r = idx % rows, c = idx / rows;
    D[c * ldd + r] = S ? scale * S[c * lds + r] : 0.0;
}

__global__ void k_diag_info(const double *W, int p, int b, int64_t n, int32_t *info) {
    __shared__ int32_t best;
    if (threadIdx.x == 0) best = 0x7fffffff;
    __syncthreads();
    for (int64_t d = threadIdx.x; d < n; d += blockDim.x) {
        const int64_t ti = d / b, r = d % b;
        const double v = W[(ti * p + ti) * b * b + r * b + r];
        if (v == 0.0) atomicMin(&best, (int32_t)(d + 1));
    }
    __syncthreads();
    if (threadIdx.x == 0) *info = best == 0x7fffffff ? 0 : best;
}

std::vector<int64_t> serial_order(const FactorGraph &g) {
    std::vector<int64_t> out;
    out.reserve((size_t)g.num_tasks());
    for (int64_t k = 0; k < g.K; ++k) {
        out.push_back(g.encode(GEQRT, k, k, k, 0));
        for (int64_t j = k + 1; j < g.q; ++j)
            for (int64_t c = 0; c < g.S; ++c) out.push_back(g.encode(LARFB, k, j, k, c));
        for (int64_t i = k + 1; i < g.p; ++i) {
            out.push_back(g.encode(TSQRT, i, k, k, 0));
            for (int64_t j = k + 1; j < g.q; ++j)
                for (int64_t c = 0; c < g.S; ++c) out.push_back(g.encode(SSRFB, i, j, k, c));
        }
    }
    return out;
}
std::vector<int64_t> serial_order(const ApplyGraph &g) {
    std::vector<int64_t> out;
    if (g.forward) {
        for (int64_t k = 0; k < g.K; ++k)
            for (int64_t i = k; i < g.p; ++i)
                for (int64_t c = 0; c < g.S; ++c) out.push_back(g.encode(i, k, c));
    } else {
        for (int64_t k = g.K - 1; k >= 0; --k) {
            for (int64_t i = g.p - 1; i > k; --i)
                for (int64_t c = 0; c < g.S; ++c) out.push_back(g.encode(i, k, c));
            for (int64_t c = 0; c < g.S; ++c) out.push_back(g.encode(k, k, c));
        }
    }
    return out;
}
std::vector<int64_t> serial_order(const TrsmGraph &g) {
    std::vector<int64_t> out;
    for (int64_t i = g.q - 1; i >= 0; --i) {
        for (int64_t j = g.q - 1; j > i; --j) out.push_back(g.encode_g(i, j));
        out.push_back(g.encode_d(i));
    }
    // G(i,j) needs D(j): rows are solved bottom-up, so D(j) precedes every G(i,j)
    return out;
}
template <class F>
tqr_status dispatch(int b, int ib, F &&f) {
#define TQR_CASE(BB, II) \
    if (b == BB && ib == II) return f(pair_fns<BB, II>());
    TQR_PAIRS(TQR_CASE)
#undef TQR_CASE
    return set_err(-5, "unsupported tile_b / inner_ib pair");
}

}  // namespace tqr

using namespace tqr;

// ===========================================================================
// C entry points
// ===========================================================================
extern "C" {

int64_t tqr_t_elems(int64_t m, int64_t n, int tile_b, int inner_ib) {
    if (m < 0 || n < 0 || m < n || !tiles_ok(tile_b, inner_ib)) return -1;
    return cdiv(std::max<int64_t>(m, 1), tile_b) * cdiv(std::max<int64_t>(n, 1), tile_b) * inner_ib * tile_b;
}

int64_t tqr_workspace_bytes(int64_t m, int64_t n, int64_t nrhs, int tile_b, int inner_ib) {
    if (m < 0 || n < 0 || m < n || nrhs < 0 || !tiles_ok(tile_b, inner_ib)) return -1;
    return sizes_of(m, n, nrhs, tile_b).total;
}

const char *tqr_last_error_string(void) { return g_err.c_str(); }

tqr_status tqr_factor_ex(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib, double *T, void *work,
                         int64_t work_bytes, hipStream_t stream, const tqr_options *options) {
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (m == 0 || n == 0) return TQR_OK;
    if (!A) return set_err(-3, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-4, "lda < max(1, m)");
    if (!(tile_b == 16 || tile_b == 32 || tile_b == 64 || tile_b == 128 || tile_b == 256))
        return set_err(-5, "tile_b must be one of 16, 32, 64, 128, 256");
    if (!tiles_ok(tile_b, inner_ib)) return set_err(-6, "inner_ib must be 16, 32 or 64, divide tile_b, and ib*(b+ib) <= 9216");
    if (!T) return set_err(-7, "T is null");
    if (!work) return set_err(-8, "work is null");
    if (work_bytes < tqr_workspace_bytes(m, n, 0, tile_b, inner_ib)) return set_err(-9, "work_bytes too small");
    if (check_opts(options) != TQR_OK) return set_err(-11, "bad tqr_options");
    if (options && options->precision == TQR_PRECISION_FP32_UPDATES && inner_ib != 16)
        return set_err(-11, "TQR_PRECISION_FP32_UPDATES needs inner_ib 16");
    if (options && options->precision == TQR_PRECISION_BF16_UPDATES && (inner_ib != 16 || tile_b < 64))
        return set_err(-11, "TQR_PRECISION_BF16_UPDATES needs inner_ib 16 and tile_b 64, 128 or 256");
    return dispatch(tile_b, inner_ib,
                    [&](const PairFns &f) { return f.factor(m, n, A, lda, T, work, stream, options, true); });
}

tqr_status tqr_factor(int64_t m, int64_t n, double *A, int64_t lda, int tile_b, int inner_ib, double *T, void *work,
                      int64_t work_bytes, hipStream_t stream) {
    return tqr_factor_ex(m, n, A, lda, tile_b, inner_ib, T, work, work_bytes, stream, nullptr);
}

static tqr_status apply_common(bool trans, int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda,
                               const double *T, int tile_b, int inner_ib, double *B, int64_t ldb, void *work,
                               int64_t work_bytes, hipStream_t stream) {
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (nrhs < 0) return set_err(-3, "nrhs must be >= 0");
    if (m == 0 || n == 0 || nrhs == 0) return TQR_OK;
    if (!A) return set_err(-4, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-5, "lda < max(1, m)");
    if (!T) return set_err(-6, "T is null");
    if (!(tile_b == 16 || tile_b == 32 || tile_b == 64 || tile_b == 128 || tile_b == 256))
        return set_err(-7, "tile_b must be one of 16, 32, 64, 128, 256");
    if (!tiles_ok(tile_b, inner_ib)) return set_err(-8, "unsupported inner_ib");
    if (!B) return set_err(-9, "B is null");
    if (ldb < std::max<int64_t>(1, m)) return set_err(-10, "ldb < max(1, m)");
    if (!work) return set_err(-11, "work is null");
    if (work_bytes < tqr_workspace_bytes(m, n, nrhs, tile_b, inner_ib)) return set_err(-12, "work_bytes too small");
    const Sizes z = sizes_of(m, n, nrhs, tile_b);
    double *W = reinterpret_cast<double *>(work);
    double *Vd = reinterpret_cast<double *>(reinterpret_cast<char *>(work) + z.tiles_bytes);
    double *Bt = reinterpret_cast<double *>(reinterpret_cast<char *>(work) + z.tiles_bytes + z.vd_bytes);
    void *sched = reinterpret_cast<char *>(work) + z.tiles_bytes + z.vd_bytes + z.btiles_bytes;
    hipLaunchKernelGGL(k_cm_to_tiles, dim3((unsigned)z.p, (unsigned)z.q), dim3(256), 0, stream, A, lda, m, n, W,
                       (int)z.p, tile_b, tile_b);
    hipLaunchKernelGGL(k_unit_lower, dim3((unsigned)std::min(z.p, z.q)), dim3(256), 0, stream, W, (int)z.p, tile_b, Vd);
    if (narrow_ok(tile_b, inner_ib, nrhs)) {
        // in place on B, one workgroup per row tile (no B tiles)
        const NarrowMem nm = narrow_mem(work, z, tile_b);
        return dispatch(tile_b, inner_ib, [&](const PairFns &f) {
            return f.apply_narrow(trans, m, n, nrhs, T, W, Vd, B, ldb, nm, stream, nullptr);
        });
    }
    tqr_status st = dispatch(tile_b, inner_ib, [&](const PairFns &f) {
        return f.apply(trans, m, n, nrhs, T, W, Vd, B, ldb, Bt, sched, stream, nullptr);
    });
    if (st != TQR_OK) return st;
    hipLaunchKernelGGL(k_tiles_to_cm, dim3((unsigned)z.p, 1), dim3(256), 0, stream, Bt, (int)z.p, tile_b,
                       (int)wb_of(nrhs), B, ldb, m, nrhs);
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

tqr_status tqr_apply_qt(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *T, int tile_b,
                        int inner_ib, double *B, int64_t ldb, void *work, int64_t work_bytes, hipStream_t stream) {
    return apply_common(true, m, n, nrhs, A, lda, T, tile_b, inner_ib, B, ldb, work, work_bytes, stream);
}

tqr_status tqr_apply_q(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *T, int tile_b,
                       int inner_ib, double *B, int64_t ldb, void *work, int64_t work_bytes, hipStream_t stream) {
    return apply_common(false, m, n, nrhs, A, lda, T, tile_b, inner_ib, B, ldb, work, work_bytes, stream);
}

tqr_status tqr_form_q(int64_t m, int64_t n, const double *A, int64_t lda, const double *T, int tile_b, int inner_ib,
                      double *Q, int64_t ldq, void *work, int64_t work_bytes, hipStream_t stream) {
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (m == 0 || n == 0) return TQR_OK;
    if (!A) return set_err(-3, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-4, "lda < max(1, m)");
    if (!T) return set_err(-5, "T is null");
    if (!(tile_b == 16 || tile_b == 32 || tile_b == 64 || tile_b == 128 || tile_b == 256))
        return set_err(-6, "tile_b must be one of 16, 32, 64, 128, 256");
    if (!tiles_ok(tile_b, inner_ib)) return set_err(-7, "unsupported inner_ib");
    if (!Q) return set_err(-8, "Q is null");
    if (ldq < std::max<int64_t>(1, m)) return set_err(-9, "ldq < max(1, m)");
    if (!work) return set_err(-10, "work is null");
    if (work_bytes < tqr_workspace_bytes(m, n, n, tile_b, inner_ib)) return set_err(-11, "work_bytes too small");
    if (n > 65535) return set_err(-2, "n > 65535 columns");
    hipLaunchKernelGGL(k_eye, dim3((unsigned)cdiv(m, 256), (unsigned)n), dim3(256), 0, stream, Q, ldq, m);
    HIPCHK(hipGetLastError());
    return apply_common(false, m, n, n, A, lda, T, tile_b, inner_ib, Q, ldq, work, work_bytes, stream);
}

tqr_status tqr_solve_ls(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb, int tile_b,
                        int inner_ib, double *T, void *work, int64_t work_bytes, int32_t *d_info, hipStream_t stream) {
    return tqr_solve_ls_ex(m, n, nrhs, A, lda, B, ldb, tile_b, inner_ib, T, work, work_bytes, d_info, stream, nullptr);
}

tqr_status tqr_solve_ls_ex(int64_t m, int64_t n, int64_t nrhs, double *A, int64_t lda, double *B, int64_t ldb,
                           int tile_b, int inner_ib, double *T, void *work, int64_t work_bytes, int32_t *d_info,
                           hipStream_t stream, const tqr_options *options) {
    // the three phases share the worker count, wait bound, abort flag and
    // status; the events bracket the whole solve; no per-task trace
    tqr_options o{};
    if (options) {
        o = *options;
        o.trace = nullptr;
        o.event_begin = o.event_end = nullptr;
    }
    const tqr_options *po = options ? &o : nullptr;
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (nrhs < 0) return set_err(-3, "nrhs must be >= 0");
    if (!A && m > 0 && n > 0) return set_err(-4, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-5, "lda < max(1, m)");
    if (!B && m > 0 && nrhs > 0) return set_err(-6, "B is null");
    if (ldb < std::max<int64_t>(1, m)) return set_err(-7, "ldb < max(1, m)");
    if (!(tile_b == 16 || tile_b == 32 || tile_b == 64 || tile_b == 128 || tile_b == 256))
        return set_err(-8, "tile_b must be one of 16, 32, 64, 128, 256");
    if (!tiles_ok(tile_b, inner_ib)) return set_err(-9, "unsupported inner_ib");
    if (!T && m > 0 && n > 0) return set_err(-10, "T is null");
    if (!work && m > 0 && n > 0) return set_err(-11, "work is null");
    if (m > 0 && n > 0 && work_bytes < tqr_workspace_bytes(m, n, nrhs, tile_b, inner_ib))
        return set_err(-12, "work_bytes too small");
    if (!d_info) return set_err(-13, "d_info is null");
    if (options && (options->struct_size != (int32_t)sizeof(tqr_options) || options->mode != TQR_MODE_PERSISTENT))
        return set_err(-15, "bad options (struct_size, or a mode other than TQR_MODE_PERSISTENT)");
    if (options && options->event_begin) HIPCHK(hipEventRecord((hipEvent_t)options->event_begin, stream));
    if (m == 0 || n == 0) {
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_info, 0);
        if (options && options->status) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, options->status, 0);
        if (options && options->event_end) HIPCHK(hipEventRecord((hipEvent_t)options->event_end, stream));
        HIPCHK(hipGetLastError());
        return TQR_OK;
    }
    tqr_status st = dispatch(tile_b, inner_ib, [&](const PairFns &f) {
        return f.solve(m, n, nrhs, A, lda, B, ldb, T, work, d_info, stream, po);
    });
    if (st != TQR_OK) return st;
    if (nrhs == 0) hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_info, 0);
    if (options && options->event_end) HIPCHK(hipEventRecord((hipEvent_t)options->event_end, stream));
    HIPCHK(hipGetLastError());
    return TQR_OK;
}

int64_t tqr_ls_mixed_workspace_bytes(int64_t m, int64_t n, int64_t nrhs, int tile_b) {
    if (m < 0 || n < 0 || m < n || nrhs < 1 || !(tile_b == 64 || tile_b == 128 || tile_b == 256)) return -1;
    return mixed_sizes(m, n, nrhs, tile_b).total;
}

tqr_status tqr_solve_ls_mixed(int64_t m, int64_t n, int64_t nrhs, const double *A, int64_t lda, const double *B,
                              int64_t ldb, double *X, int64_t ldx, int tile_b, int iterations, double *T, void *work,
                              int64_t work_bytes, int32_t *d_info, tqr_refine_stats *d_stats, hipStream_t stream,
                              const tqr_options *options) {
    g_err.clear();
    if (m < 0 || m < n) return set_err(-1, "m must be >= max(n, 0)");
    if (n < 0) return set_err(-2, "n must be >= 0");
    if (nrhs < 1) return set_err(-3, "nrhs must be >= 1");
    if (!A && m * n > 0) return set_err(-4, "A is null");
    if (lda < std::max<int64_t>(1, m)) return set_err(-5, "lda < max(1, m)");
    if (!B) return set_err(-6, "B is null");
    if (ldb < std::max<int64_t>(1, m)) return set_err(-7, "ldb < max(1, m)");
    if (!X) return set_err(-8, "X is null");
    if (ldx < std::max<int64_t>(1, n)) return set_err(-9, "ldx < max(1, n)");
    if (!(tile_b == 64 || tile_b == 128 || tile_b == 256)) return set_err(-10, "tile_b must be 64, 128 or 256");
    if (iterations < 0 || iterations > 200) return set_err(-11, "iterations must be in 0..200");
    if (!T) return set_err(-12, "T is null");
    if (!work) return set_err(-13, "work is null");
    const MixedSizes ms = mixed_sizes(std::max<int64_t>(m, 1), std::max<int64_t>(n, 1), nrhs, tile_b);
    if (work_bytes < ms.total) return set_err(-14, "work_bytes too small");
    if (!d_info) return set_err(-15, "d_info is null");
    if (check_opts(options) != TQR_OK || (options && options->mode != TQR_MODE_PERSISTENT))
        return set_err(-17, "bad options (struct_size, precision, or a mode other than TQR_MODE_PERSISTENT)");
    if (m == 0 || n == 0) {
        hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, stream, d_info, 0);
        if (n > 0)
            hipLaunchKernelGGL(k_copy_cm, dim3((unsigned)cdiv(n * nrhs, 256)), dim3(256), 0, stream, nullptr, 0, X, ldx,
                               n, (int)nrhs, 0.0);
        if (d_stats)
            hipLaunchKernelGGL(k_refine_stats_empty, dim3((unsigned)cdiv(nrhs, 256)), dim3(256), 0, stream, d_stats,
                               nrhs);
        HIPCHK(hipGetLastError());
        return TQR_OK;
    }
    tqr_options o{};
    if (options) o = *options;
    else {
        o.struct_size = (int32_t)sizeof(tqr_options);
        o.precision = TQR_PRECISION_FP32_UPDATES;
        o.policy = TQR_POLICY_COLUMN;
    }
    o.trace = nullptr;
    o.event_begin = o.event_end = nullptr;
    if (options && options->event_begin) HIPCHK(hipEventRecord((hipEvent_t)options->event_begin, stream));
    tqr_status st = dispatch(tile_b, 16, [&](const PairFns &f) {
        return f.mixed(m, n, nrhs, A, lda, B, ldb, X, ldx, iterations, T, work, d_info, d_stats, stream, o);
    });
    if (st != TQR_OK) return st;
    if (options && options->event_end) HIPCHK(hipEventRecord((hipEvent_t)options->event_end, stream));
    HIPCHK(hipGetLastError());
    return TQR_OK;
}
int64_t tqr_graph_tasks(int64_t p, int64_t q, int tile_b) {
    if (p < 1 || q < 1 || q > p || tile_b < 1) return -1;
    return FactorGraph(p, q, tile_b).num_tasks();
}

int tqr_graph_task(int64_t p, int64_t q, int tile_b, int64_t task, int32_t out[5]) {
    const int64_t nt = tqr_graph_tasks(p, q, tile_b);
    if (nt < 0 || task < 0 || task >= nt || !out) return -1;
    const Task t = FactorGraph(p, q, tile_b).decode(task);
    out[0] = t.kind; out[1] = t.i; out[2] = t.j; out[3] = t.k; out[4] = t.c;
    return 0;
}

int tqr_graph_indegree(int64_t p, int64_t q, int tile_b, int64_t task) {
    const int64_t nt = tqr_graph_tasks(p, q, tile_b);
    if (nt < 0 || task < 0 || task >= nt) return -1;
    FactorGraph g(p, q, tile_b);
    return g.indegree(g.decode(task));
}

int tqr_graph_successors(int64_t p, int64_t q, int tile_b, int64_t task, int64_t *out, int max_out) {
    const int64_t nt = tqr_graph_tasks(p, q, tile_b);
    if (nt < 0 || task < 0 || task >= nt) return -1;
    FactorGraph g(p, q, tile_b);
    const Task t = g.decode(task);
    const int ns = g.num_successors(t);
    for (int n = 0; n < ns && n < max_out; ++n) out[n] = g.successor(t, n);
    return ns;
}

}  // extern "C"
