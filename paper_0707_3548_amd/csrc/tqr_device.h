// Device building blocks of the tiled QR: tile addressing, reductions,
// the FP64 matrix-core (MFMA) block-reflector updates and the panel
// factorisation used by GEQRT and TSQRT.
//
// Tile storage (Block Data Layout, Sec. 3.4): tile (i,j) of a p x q grid is a
// contiguous b x b column-major block at offset ((j*p)+i) * b*b.  Edge tiles
// are zero padded.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace tqr {

constexpr int NT = 256;           // threads of every workgroup (4 wave64)
constexpr int NWAVES = NT / 64;

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// Four elements 4 apart (one lane's share of a 16-row block in the
// matrix-core accumulator layout); `stride` is 4 for a column, 4*ld across
// columns.
__device__ __forceinline__ d4 ld4s(const double *p, int stride) {
    return d4{p[0], p[stride], p[2 * stride], p[3 * stride]};
}
__device__ __forceinline__ void st4s(double *p, int stride, d4 v) {
    p[0] = v.x; p[stride] = v.y; p[2 * stride] = v.z; p[3 * stride] = v.w;
}

// D = A * B + C on a 16x16x4 FP64 matrix-core tile.  Lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; element r of C/D in lane l is
// D[4r + l/16][l%16] (the four rows a lane holds are 4 apart).
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Keeps the instruction scheduler from hoisting the next row block's operand
// loads above this point, which would hold many fragments live at once.
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the workgroup; every thread gets the result.  `red` holds NWAVES doubles.
__device__ __forceinline__ double block_sum(double v, double *red) {
    v = wave_sum(v);
    if (lane_id() == 0) red[wave_id()] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < NWAVES; ++w) s += red[w];
    __syncthreads();
    return s;
}

// ---------------------------------------------------------------------------
// A 16-column strip of a b-row tile held by one wave in matrix-core
// accumulator layout: element r of v[rb] holds row 16rb + 4r + l/16 of strip
// column l%16.  The same registers serve as the B operand of a product that
// sums over the strip's rows: element r is the k-slice of rows
// 16rb + 4r .. 16rb + 4r + 3 (lane group l/16 supplies k = l/16).
// ---------------------------------------------------------------------------
template <int B>
struct Strip {
    d4 v[B / 16];
};

template <int B>
__device__ __forceinline__ void strip_load(Strip<B> &s, const double *col0, int ld) {
    const int l = lane_id();
    const double *p = col0 + (size_t)(l & 15) * ld + (l >> 4);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) s.v[rb] = ld4s(p + 16 * rb, 4);
}

template <int B>
__device__ __forceinline__ void strip_store(const Strip<B> &s, double *col0, int ld, int rb0 = 0) {
    const int l = lane_id();
    double *p = col0 + (size_t)(l & 15) * ld + (l >> 4);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb)
        if (rb >= rb0) st4s(p + 16 * rb, 4, s.v[rb]);
}

// One wave applies the block reflector of one inner block (IB columns) to its
// 16-column strip C (all B rows, in registers).  V and T come from LDS:
//   V(row, a) = Vl[a * ldv + row]  for the block's column a (0..IB-1) and the
//               tile row `row`; T(r, c) = Tl[c * IB + r].
// TS (the TSQRT/SSRFB form, reflectors [I; V]):
//   W = top[c0:c0+IB] + V^T C,  W = op(T) W,  top[c0:c0+IB] -= W,  C -= V W
//   with `top` column 0 of the strip in the upper tile (global, ld B).
// !TS (the GEQRT/LARFB form, V dense unit lower, zero above row c0):
//   W = V^T C,  W = op(T) W,  C -= V W, over rows c0..B-1 only.
// op(T) = T^T applies Q^T (factorisation); T applies Q.  A wave that only
// duplicates another wave's columns passes write_top = false.
template <int B, int IB, bool TRANS, bool TS>
__device__ __forceinline__ void panel_update(Strip<B> &C, double *top, const double *Vl, int ldv, const double *Tl,
                                             int c0, bool write_top = true) {
    constexpr int NA = IB / 16;
    const int l = lane_id();
    const int rb0 = TS ? 0 : c0 / 16;
    d4 W[NA], W2[NA];
    double *tp = TS ? top + (size_t)(l & 15) * B + c0 + (l >> 4) : nullptr;
#pragma unroll
    for (int a = 0; a < NA; ++a) W[a] = TS ? ld4s(tp + 16 * a, 4) : d4{0.0, 0.0, 0.0, 0.0};
    // k-slice (rb, r): rows 16rb + 4r + {0..3}; A operand V^T[16a + l%16][16rb + 4r + l/16]
    const double *vp = Vl + (l & 15) * ldv + (l >> 4);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) continue;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const double *q = vp + 16 * a * ldv + 16 * rb;
            W[a] = mfma(q[0], C.v[rb].x, W[a]);
            W[a] = mfma(q[4], C.v[rb].y, W[a]);
            W[a] = mfma(q[8], C.v[rb].z, W[a]);
            W[a] = mfma(q[12], C.v[rb].w, W[a]);
        }
        sched_fence();
    }
    // W2 = op(T) W; A operand of k-slice (a, r): op(T)[16o + l%16][16a + 4r + l/16]
#pragma unroll
    for (int o = 0; o < NA; ++o) W2[o] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < NA; ++o) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            if (TRANS ? (a > o) : (a < o)) continue;  // T is upper triangular
            const double *tq = TRANS ? Tl + (16 * o + (l & 15)) * IB + 16 * a + (l >> 4)
                                     : Tl + (16 * a + (l >> 4)) * IB + 16 * o + (l & 15);
            const int st = TRANS ? 4 : 4 * IB;
            W2[o] = mfma(tq[0], W[a].x, W2[o]);
            W2[o] = mfma(tq[st], W[a].y, W2[o]);
            W2[o] = mfma(tq[2 * st], W[a].z, W2[o]);
            W2[o] = mfma(tq[3 * st], W[a].w, W2[o]);
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        if (TS && write_top) st4s(tp + 16 * a, 4, ld4s(tp + 16 * a, 4) - W2[a]);
        W2[a] = -W2[a];
    }
    // C -= V W2; A operand of k-slice (a, r): V[16rb + l%16][16a + 4r + l/16]
    const double *vq = Vl + (l >> 4) * ldv + (l & 15);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) continue;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const double *q = vq + 16 * a * ldv + 16 * rb;
            C.v[rb] = mfma(q[0], W2[a].x, C.v[rb]);
            C.v[rb] = mfma(q[4 * ldv], W2[a].y, C.v[rb]);
            C.v[rb] = mfma(q[8 * ldv], W2[a].z, C.v[rb]);
            C.v[rb] = mfma(q[12 * ldv], W2[a].w, C.v[rb]);
        }
        sched_fence();
    }
}

// ---------------------------------------------------------------------------
// Panel factorisation in LDS.  P holds hp rows and IB columns (ld = ldp);
// column jj's reflector has its pivot in row jj and acts on rows jj..hp-1.
// For GEQRT the panel is rows c0..b-1 of the diagonal tile; for TSQRT it is
// the IB rows of R_kk (upper triangle, zeros below) stacked on the b rows of
// A_ik, so that the rows between the pivot and A_ik are exact zeros and the
// same column loop yields DTSQT2's reflectors [e_j; v_j].
//
// Reflector (as the unblocked algorithm of Sec. 2.1, LAPACK convention):
//   sigma^2 = sum of squares below the pivot; sigma^2 == 0 -> tau = 0, H = I;
//   else beta = -sgn(alpha) sqrt(alpha^2 + sigma^2), tau = (beta - alpha)/beta,
//   v = x / (alpha - beta), pivot <- beta.
// ---------------------------------------------------------------------------
template <int IB>
__device__ void panel_factor(double *P, int hp, int ldp, double *tau, double *wv, double *red) {
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    for (int jj = 0; jj < IB; ++jj) {
        double *col = P + (size_t)jj * ldp;
        double s = 0.0;
        for (int r = jj + 1 + tid; r < hp; r += NT) s += col[r] * col[r];
        const double sigma2 = block_sum(s, red);
        const double alpha = col[jj];
        double t = 0.0, beta = alpha, denom = 1.0;
        if (sigma2 != 0.0) {
            const double nrm = sqrt(alpha * alpha + sigma2);
            beta = alpha >= 0.0 ? -nrm : nrm;
            t = (beta - alpha) / beta;
            denom = alpha - beta;
        }
        if (sigma2 != 0.0) {
            for (int r = jj + 1 + tid; r < hp; r += NT) col[r] = col[r] / denom;
        }
        __syncthreads();
        if (tid == 0) {
            col[jj] = beta;
            tau[jj] = t;
        }
        // every thread computed the same t; make the branch around the
        // barriers below visibly uniform to the compiler
        const int update = __builtin_amdgcn_readfirstlane((t != 0.0 && jj + 1 < IB) ? 1 : 0);
        if (update) {
            for (int c = jj + 1 + wave; c < IB; c += NWAVES) {
                const double *pc = P + (size_t)c * ldp;
                double d = 0.0;
                for (int r = jj + 1 + lane; r < hp; r += 64) d += col[r] * pc[r];
                d = wave_sum(d);
                if (lane == 0) wv[c] = t * (pc[jj] + d);
            }
            __syncthreads();
            const int nr = hp - jj, nc = IB - 1 - jj;
            for (int idx = tid; idx < nr * nc; idx += NT) {
                const int r = jj + idx % nr, c = jj + 1 + idx / nr;
                const double v = (r == jj) ? 1.0 : col[r];
                P[(size_t)c * ldp + r] -= wv[c] * v;
            }
        }
        __syncthreads();
    }
}

// T of the factored panel (compact WY, forward and column-wise):
//   T[c][c] = tau_c,  T[0:c, c] = -tau_c T[0:c, 0:c] (V[:, 0:c]^T v_c).
// G = V^T V (strict upper part) is formed first, with V unit lower in P.
template <int IB>
__device__ void panel_t(const double *P, int hp, int ldp, const double *tau, double *Ts, double *G) {
    const int tid = threadIdx.x, lane = lane_id(), wave = wave_id();
    for (int pr = wave; pr < IB * IB; pr += NWAVES) {
        const int a = pr % IB, c = pr / IB;
        if (a >= c) continue;
        const double *pa = P + (size_t)a * ldp, *pc = P + (size_t)c * ldp;
        double d = 0.0;
        for (int r = c + 1 + lane; r < hp; r += 64) d += pa[r] * pc[r];
        d = wave_sum(d);
        if (lane == 0) G[a + c * IB] = pa[c] + d;
    }
    for (int idx = tid; idx < IB * IB; idx += NT) Ts[idx] = 0.0;
    __syncthreads();
    for (int c = 0; c < IB; ++c) {
        if (tid < c) {
            double acc = 0.0;
            for (int d = tid; d < c; ++d) acc += Ts[tid + d * IB] * G[d + c * IB];
            Ts[tid + c * IB] = -tau[c] * acc;
        } else if (tid == c) {
            Ts[c + c * IB] = tau[c];
        }
        __syncthreads();
    }
}

}  // namespace tqr
