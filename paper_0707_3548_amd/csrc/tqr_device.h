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

#include "tqr_offsets.h"

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
// loads above this point, which would hold many fragments live at once (used
// for inner blocks wider than 16; with 16 the early loads hide LDS latency).
__device__ __forceinline__ void sched_fence() { __builtin_amdgcn_sched_barrier(0); }

// ---------------------------------------------------------------------------
// Cross-lane exchanges of doubles without the LDS unit.  Inside a 16-lane
// row: DPP quad_perm [1,0,3,2] (lane ^ 1), quad_perm [2,3,0,1] (lane ^ 2),
// row_half_mirror (lane i <-> 7 - i inside each group of 8) and row_ror:8
// (lane ^ 8).  Across rows: the gfx950 permlane16/32 swaps, which given the
// same register twice return the two rows (halves) of each pair, so their
// sum is the sum over lane ^ 16 (lane ^ 32).  Every step adds a lane's value
// and its partner's, so both lanes of a pair hold the same bits.
// ---------------------------------------------------------------------------
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppRor8 = 0x128;

template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    int2 w = __builtin_bit_cast(int2, v);
    w.x = __builtin_amdgcn_update_dpp(0, w.x, CTRL, 0xf, 0xf, false);
    w.y = __builtin_amdgcn_update_dpp(0, w.y, CTRL, 0xf, 0xf, false);
    return __builtin_bit_cast(double, w);
}

__device__ __forceinline__ double sum_xor16(double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    const auto lo = __builtin_amdgcn_permlane16_swap(w.x, w.x, false, false);
    const auto hi = __builtin_amdgcn_permlane16_swap(w.y, w.y, false, false);
    return __builtin_bit_cast(double, int2{(int)lo[0], (int)hi[0]}) + __builtin_bit_cast(double, int2{(int)lo[1], (int)hi[1]});
}

__device__ __forceinline__ double sum_xor32(double v) {
    const int2 w = __builtin_bit_cast(int2, v);
    const auto lo = __builtin_amdgcn_permlane32_swap(w.x, w.x, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap(w.y, w.y, false, false);
    return __builtin_bit_cast(double, int2{(int)lo[0], (int)hi[0]}) + __builtin_bit_cast(double, int2{(int)lo[1], (int)hi[1]});
}

// Sum over the wave, the same value in every lane.
__device__ __forceinline__ double wave_sum(double v) {
    v += dpp_d<kDppXor1>(v);
    v += dpp_d<kDppXor2>(v);
    v += dpp_d<kDppHalfMirror>(v);
    v += dpp_d<kDppRor8>(v);
    v = sum_xor16(v);
    return sum_xor32(v);
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
// A 16-column strip of a b-row tile held by one wave: element r of v[rb]
// holds row 16rb + 4(l/16) + r of strip column l%16, four consecutive rows
// per lane, so that a strip moves to and from memory in 32-byte pieces.
// As the B operand of a product that sums over the strip's rows, element r
// of v[rb] is the k-slice of rows {16rb + 4g + r : g = 0..3} (lane group
// g = l/16 supplies k = g).  As an accumulator, the matrix core returns row
// 4r + l/16 of its 16-row result in element r; a product whose A operand
// takes its rows through strip_row_perm lands row 16rb + 4(l/16) + r there.
// ---------------------------------------------------------------------------
template <int B>
struct Strip {
    d4 v[B / 16];
};

// (strip_row_perm and the operand offsets of the strip updates are in
// tqr_offsets.h, shared with a host-side bounds check.)

template <int B>
__device__ __forceinline__ void strip_load(Strip<B> &s, const double *col0, int ld) {
    const int l = lane_id();
    const d4 *p = reinterpret_cast<const d4 *>(col0 + (size_t)(l & 15) * ld + 4 * (l >> 4));
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) s.v[rb] = p[4 * rb];
}

template <int B>
__device__ __forceinline__ void strip_store(const Strip<B> &s, double *col0, int ld, int rb0 = 0) {
    const int l = lane_id();
    d4 *p = reinterpret_cast<d4 *>(col0 + (size_t)(l & 15) * ld + 4 * (l >> 4));
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb)
        if (rb >= rb0) p[4 * rb] = s.v[rb];
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
// The IB top rows of the wave's 16 columns in the upper tile (the TS form's
// W initial value), in the accumulator layout.
template <int B, int IB>
__device__ __forceinline__ void load_top(d4 (&W)[IB / 16], const double *top, int c0) {
    const int l = lane_id();
    const double *tp = top + (size_t)(l & 15) * B + c0 + (l >> 4);
#pragma unroll
    for (int a = 0; a < IB / 16; ++a) W[a] = ld4s(tp + 16 * a, 4);
}

// With `Wtop` the TS form takes the top rows already loaded by load_top
// (so that their load can be issued ahead of other memory traffic).
// `issue(rb)` is called once per row block rb (0 .. B/16-1) during the V^T C
// products, so that a caller can spread the issue of its global loads over
// them instead of stalling the wave's instruction stream with a burst.
struct NoIssue {
    __device__ __forceinline__ void operator()(int) const {}
};
template <int B, int IB, bool TRANS, bool TS, class Issue = NoIssue>
__device__ __forceinline__ void panel_update(Strip<B> &C, double *top, const double *Vl, int ldv, const double *Tl,
                                             int c0, bool write_top = true, const d4 *Wtop = nullptr,
                                             const Issue &issue = Issue{}) {
    constexpr int NA = IB / 16;
    const int l = lane_id();
    const int rb0 = TS ? 0 : c0 / 16;
    d4 W[NA], W2[NA], Wt[NA];
    double *tp = TS ? top + (size_t)(l & 15) * B + c0 + (l >> 4) : nullptr;
    // the top rows are added after V^T C, so that their load latency is
    // hidden behind the matrix-core products
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        if (TS) Wt[a] = Wtop ? Wtop[a] : ld4s(tp + 16 * a, 4);
        W[a] = d4{0.0, 0.0, 0.0, 0.0};
    }
    // k-slice (rb, r): rows 16rb + 4g + r; A operand V^T[16a + l%16][16rb + 4(l/16) + r].
    // The operands of row block rb+1 are read from LDS before the products of
    // row block rb are issued (the scheduling fences keep that order): with
    // one wave per SIMD nothing else hides the LDS latency.
    auto read_vt = [&](int rb, double (&o)[NA][4]) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) o[a][r] = Vl[upd_vt_off(l, ldv, a, rb, r)];
    };
    // op(T) operands of the W2 = op(T) W products, read ahead of them
    double tv[NA][NA][4];
#pragma unroll
    for (int o = 0; o < NA; ++o)
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            if (TRANS ? (a > o) : (a < o)) continue;  // T is upper triangular
#pragma unroll
            for (int r = 0; r < 4; ++r) tv[o][a][r] = Tl[upd_t_off(TRANS, l, IB, o, a, r)];
        }
    double va[NA][4], vn[NA][4];
    read_vt(rb0, va);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) {
            issue(rb);
            continue;
        }
        if (rb + 1 < B / 16) read_vt(rb + 1, vn);
        issue(rb);
        sched_fence();
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            W[a] = mfma(va[a][0], C.v[rb].x, W[a]);
            W[a] = mfma(va[a][1], C.v[rb].y, W[a]);
            W[a] = mfma(va[a][2], C.v[rb].z, W[a]);
            W[a] = mfma(va[a][3], C.v[rb].w, W[a]);
        }
        sched_fence();
        if (rb + 1 < B / 16) {
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) va[a][r] = vn[a][r];
        }
    }
    // A operand of the update C -= V W2, k-slice (a, r):
    // V[16rb + strip_row_perm(l%16)][16a + 4r + l/16]
    auto read_v = [&](int rb, double (&o)[NA][4]) {
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int r = 0; r < 4; ++r) o[a][r] = Vl[upd_v_off(l, ldv, a, rb, r)];
    };
    read_v(rb0, va);
    if (TS) {
#pragma unroll
        for (int a = 0; a < NA; ++a) W[a] += Wt[a];
    }
    // W2 = op(T) W; A operand of k-slice (a, r): op(T)[16o + l%16][16a + 4r + l/16]
#pragma unroll
    for (int o = 0; o < NA; ++o) W2[o] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int o = 0; o < NA; ++o) {
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            if (TRANS ? (a > o) : (a < o)) continue;
            W2[o] = mfma(tv[o][a][0], W[a].x, W2[o]);
            W2[o] = mfma(tv[o][a][1], W[a].y, W2[o]);
            W2[o] = mfma(tv[o][a][2], W[a].z, W2[o]);
            W2[o] = mfma(tv[o][a][3], W[a].w, W2[o]);
        }
    }
#pragma unroll
    for (int a = 0; a < NA; ++a) {
        if (TS && write_top) st4s(tp + 16 * a, 4, Wt[a] - W2[a]);
        W2[a] = -W2[a];
    }
    // C -= V W2, with the same one-row-block-ahead operand reads
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) continue;
        if (rb + 1 < B / 16) read_v(rb + 1, vn);
        sched_fence();
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            C.v[rb] = mfma(va[a][0], W2[a].x, C.v[rb]);
            C.v[rb] = mfma(va[a][1], W2[a].y, C.v[rb]);
            C.v[rb] = mfma(va[a][2], W2[a].z, C.v[rb]);
            C.v[rb] = mfma(va[a][3], W2[a].w, C.v[rb]);
        }
        sched_fence();
        if (rb + 1 < B / 16) {
#pragma unroll
            for (int a = 0; a < NA; ++a)
#pragma unroll
                for (int r = 0; r < 4; ++r) va[a][r] = vn[a][r];
        }
    }
}

// ---------------------------------------------------------------------------
// FP32 precision tier of the update kernels (LARFB / SSRFB): the strip is
// held as floats in the same rows-by-lane layout as Strip<B>, V and T are
// staged in LDS as floats, and every product runs on v_mfma_f32_16x16x4f32
// (twice the FP64 matrix rate).  That instruction takes its operands in the
// lanes of the FP64 one (lane l supplies A[l%16][l/16] and B[l/16][l%16]) but
// returns D[4(l/16)+i][l%16] in element i, four consecutive rows per lane.
// Results that feed the next product keep that layout (W, op(T) W), and the
// final C -= V W reads V's rows through the permutation 4a+b -> 4b+a, so that
// output element i of lane l lands on strip row 16rb + 4i + l/16, as stored.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma32(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int B>
struct StripF {
    f4 v[B / 16];
};

template <int B>
__device__ __forceinline__ void strip_load_f(StripF<B> &s, const double *col0, int ld) {
    const int l = lane_id();
    const double *p = col0 + (size_t)(l & 15) * ld + (l >> 4);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        const d4 x = ld4s(p + 16 * rb, 4);
        s.v[rb] = f4{(float)x.x, (float)x.y, (float)x.z, (float)x.w};
    }
}

template <int B>
__device__ __forceinline__ void strip_store_f(const StripF<B> &s, double *col0, int ld) {
    const int l = lane_id();
    double *p = col0 + (size_t)(l & 15) * ld + (l >> 4);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb)
        st4s(p + 16 * rb, 4, d4{(double)s.v[rb].x, (double)s.v[rb].y, (double)s.v[rb].z, (double)s.v[rb].w});
}

// The block reflector of one inner block of 16 columns (the forms of
// panel_update) applied to a float strip.  Vl: V(row, a) = Vl[a * ldv + row]
// (floats); Tl: T(r, c) = Tl[16 c + r] (floats).  The TS form's top rows stay
// FP64 in memory: W takes their float value and they are updated in FP64 by
// the float correction.
// BF16 operands for v_mfma_f32_16x16x16bf16_1k, which takes in lane l the
// four K values 4(l/16) .. 4(l/16)+3 of row l%16 of A and of column l%16 of
// B and accumulates in FP32 with the output layout of the FP32 instruction.
// The conversion rounds to nearest even (the gfx950 packed conversion, two
// floats per instruction).
typedef short bf4 __attribute__((ext_vector_type(4)));
typedef float fl2 __attribute__((ext_vector_type(2)));
typedef __bf16 bh2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ bf4 bf16x4(float a, float b, float c, float d) {
    const bh2 lo = __builtin_convertvector(fl2{a, b}, bh2), hi = __builtin_convertvector(fl2{c, d}, bh2);
    const uint32_t ulo = __builtin_bit_cast(uint32_t, lo), uhi = __builtin_bit_cast(uint32_t, hi);
    return __builtin_bit_cast(bf4, (uint64_t)ulo | ((uint64_t)uhi << 32));
}
__device__ __forceinline__ f4 mfma_bf16(bf4 a, bf4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// BF16 variant (BF16 = true): the two large products take their operands in
// BF16 (V, C, and W after op(T)) with FP32 accumulation, one instruction per
// 16-row block where the FP32 form issues four: the four K-slices of the FP32
// form are the four K values each lane group supplies, so the operands are
// the same registers and LDS words, converted.  op(T) W stays FP32.
template <int B, bool TRANS, bool TS, bool BF16 = false>
__device__ __forceinline__ void panel_update_f32(StripF<B> &C, double *top, const float *Vl, int ldv, const float *Tl,
                                                 int c0, bool write_top = true) {
    const int l = lane_id();
    const int rb0 = TS ? 0 : c0 / 16;
    // W = V^T C; k-slice (rb, r): rows 16rb + 4r + {0..3}; W row a in lane
    // group a/4, element a%4
    f4 W = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) continue;
        float q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) q[r] = Vl[updf_vt_off(l, ldv, rb, r)];
        if constexpr (BF16) {
            W = mfma_bf16(bf16x4(q[0], q[1], q[2], q[3]), bf16x4(C.v[rb].x, C.v[rb].y, C.v[rb].z, C.v[rb].w), W);
        } else {
            W = mfma32(q[0], C.v[rb].x, W);
            W = mfma32(q[1], C.v[rb].y, W);
            W = mfma32(q[2], C.v[rb].z, W);
            W = mfma32(q[3], C.v[rb].w, W);
        }
    }
    double *tp = nullptr;
    d4 t = {0.0, 0.0, 0.0, 0.0};
    if (TS) {
        tp = top + (size_t)(l & 15) * B + c0 + 4 * (l >> 4);
        t = d4{tp[0], tp[1], tp[2], tp[3]};
        W += f4{(float)t.x, (float)t.y, (float)t.z, (float)t.w};
    }
    // W2 = op(T) W; k-slice r: W rows {4j + r}; A[d][j] = op(T)[d][4j + r]
    f4 W2 = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const float a = Tl[updf_t_off(TRANS, l, r)];
        W2 = mfma32(a, W[r], W2);
    }
    if (TS && write_top) {
        tp[0] = t.x - (double)W2.x;
        tp[1] = t.y - (double)W2.y;
        tp[2] = t.z - (double)W2.z;
        tp[3] = t.w - (double)W2.w;
    }
    W2 = -W2;
    // C -= V W2; output row d of an MFMA is strip row 16rb + perm(d),
    // perm(4a + b) = 4b + a
    bf4 w2b = {};
    if constexpr (BF16) w2b = bf16x4(W2.x, W2.y, W2.z, W2.w);
#pragma unroll
    for (int rb = 0; rb < B / 16; ++rb) {
        if (!TS && rb < rb0) continue;
        float q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) q[r] = Vl[updf_v_off(l, ldv, rb, r)];
        if constexpr (BF16) {
            C.v[rb] = mfma_bf16(bf16x4(q[0], q[1], q[2], q[3]), w2b, C.v[rb]);
        } else {
            C.v[rb] = mfma32(q[0], W2.x, C.v[rb]);
            C.v[rb] = mfma32(q[1], W2.y, C.v[rb]);
            C.v[rb] = mfma32(q[2], W2.z, C.v[rb]);
            C.v[rb] = mfma32(q[3], W2.w, C.v[rb]);
        }
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

// ---------------------------------------------------------------------------
// One-wave panel factorisation of an inner block of 16 columns.
//
// The panel sits in the registers of a single wave, one row per lane and
// step (row lane + 64 i, i < RPL), all 16 columns per row: x[i][c].  A column
// step then needs only wave-level reductions: the squared norm below the
// pivot, and one batched reduction that yields, in a single pass over the
// rows, both the products v_jj^T A(:, c) for the columns right of the pivot
// (the rank-1 update) and v_c^T v_jj for the columns left of it (the next
// column of the compact-WY T, Sec. 2.1).  No workgroup barrier is involved, so
// the other waves of the workgroup keep updating trailing columns meanwhile.
// ---------------------------------------------------------------------------
// Lane `lane`'s v in every lane, through the cross-lane permute (the result
// stays in vector registers).
__device__ __forceinline__ double bcast_lane_d(double v, int lane) {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_ds_bpermute(lane << 2, w.x);
    r.y = __builtin_amdgcn_ds_bpermute(lane << 2, w.y);
    return __builtin_bit_cast(double, r);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(w.x, lane);
    r.y = __builtin_amdgcn_readlane(w.y, lane);
    return __builtin_bit_cast(double, r);
}

// out[c] = sum over the wave of v[c], c < 16, uniform in every lane, and
// lds_out[c] = the same totals in LDS.  Reduce-scatter inside each 16-lane
// row by halving exchanges (the lane ^ 8 pair keeps values 0..7 / 8..15 by
// lane bit 3, the half-mirror pair by bit 2, then bits 1 and 0), after which
// lane l holds its row's partial of value l & 15; the four rows are summed
// with the two swaps and the totals read from lanes 0..15.
__device__ __forceinline__ void wave_allsum16(const double (&v)[16], double (&out)[16], double *lds_out) {
    const int l = lane_id();
    double a[8], b[4], c[2];
    bool hi = (l & 8) != 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) a[i] = (hi ? v[8 + i] : v[i]) + dpp_d<kDppRor8>(hi ? v[i] : v[8 + i]);
    hi = (l & 4) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) b[i] = (hi ? a[4 + i] : a[i]) + dpp_d<kDppHalfMirror>(hi ? a[i] : a[4 + i]);
    hi = (l & 2) != 0;
#pragma unroll
    for (int i = 0; i < 2; ++i) c[i] = (hi ? b[2 + i] : b[i]) + dpp_d<kDppXor2>(hi ? b[i] : b[2 + i]);
    hi = (l & 1) != 0;
    double d = (hi ? c[1] : c[0]) + dpp_d<kDppXor1>(hi ? c[0] : c[1]);
    d = sum_xor32(sum_xor16(d));
    if (l < 16) lds_out[l] = d;
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = readlane_d(d, i);
}

// Householder reflector of the column with pivot alpha and squared norm
// sigma2 below the pivot (the unblocked algorithm of Sec. 2.1, LAPACK
// convention): sigma2 == 0 gives tau = 0 (H = I); else
// beta = -sgn(alpha) sqrt(alpha^2 + sigma2), tau = (beta - alpha) / beta and
// the entries below the pivot are scaled by 1 / (alpha - beta).
struct Reflector {
    double tau, beta, scale;
};
__device__ __forceinline__ Reflector make_reflector(double alpha, double sigma2) {
    Reflector h{0.0, alpha, 1.0};
    if (sigma2 != 0.0) {
        const double nrm = sqrt(alpha * alpha + sigma2);
        h.beta = alpha >= 0.0 ? -nrm : nrm;
        h.tau = (h.beta - alpha) / h.beta;
        h.scale = 1.0 / (alpha - h.beta);
    }
    return h;
}

// Both panel kernels keep the pivot column in x[.][0]: after each step the
// columns rotate left by one, so the step is the same code for every column
// (no unrolling over columns, which keeps the code small).  At step jj
// columns 1 .. 15-jj are the ones right of the pivot and columns 16-jj .. 15
// hold v_0 .. v_jj-1; after 16 steps the columns are back in order.
template <int RPL>
__device__ __forceinline__ void rotate_left(double (&x)[RPL][16]) {
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        const double t = x[i][0];
#pragma unroll
        for (int c = 0; c < 15; ++c) x[i][c] = x[i][c + 1];
        x[i][15] = t;
    }
}

// LDS scratch of a one-wave panel: the per-lane partial products (64 rows of
// kPartStride doubles: the padding spreads both the row writes and the
// column reads over all banks), the Gram columns G (16 x 16, step jj writes
// column jj in rotated order) and the taus.
constexpr int kPartStride = 18;
constexpr int kPanelScratch = 64 * kPartStride + 256 + 16;

// Batched products of a step, P[c] = sum over the wave of v . x[.][c], the
// same in every lane; the 16 totals also go to Gcol (LDS).  Each lane writes
// its 16 partial sums as one row of the scratch; lane l then adds column
// l & 15 over the 16 rows of its quarter, the two swaps add the quarters,
// lanes 0..15 write the totals, and every lane reads them back.
template <int RPL>
__device__ __forceinline__ void panel_products(const double (&x)[RPL][16], const double (&v)[RPL], double (&P)[16],
                                               double *part, double *Gcol) {
    const int l = lane_id();
    double pv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) acc += v[i] * x[i][c];
        pv[c] = acc;
    }
    double2 *row = reinterpret_cast<double2 *>(part + l * kPartStride);
#pragma unroll
    for (int i = 0; i < 8; ++i) row[i] = double2{pv[2 * i], pv[2 * i + 1]};
    const double *col = part + (l >> 4) * 16 * kPartStride + (l & 15);
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += col[k * kPartStride];
    s = sum_xor32(sum_xor16(s));
    if (l < 16) Gcol[l] = s;
    const double2 *g = reinterpret_cast<const double2 *>(Gcol);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 t = g[i];
        P[2 * i] = t.x;
        P[2 * i + 1] = t.y;
    }
}

// T of the block from the Gram columns and taus (compact WY, forward and
// column-wise, Sec. 2.1): T[j][j] = tau_j,
// T[0:j, j] = -tau_j T[0:j, 0:j] G[0:j, j], where the step-j column is stored
// rotated: G(d, j) = Gs[16 j + 16 - j + d].  Column j is computed from the
// columns before it in LDS, lane l < 16 computing row l (T's zeros left of
// the diagonal make the sum over d < j exact).  A runtime loop over j keeps
// only one column's lane masks live.
__device__ __forceinline__ void panel_t_from_gram(const double *Gs, const double *taus, double *Tl) {
    const int l = lane_id(), r = l & 15;
#pragma unroll 1
    for (int j = 0; j < 16; ++j) {
        const double tau = taus[j];
        const double *g = Gs + 16 * j + 16 - j;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < 15; ++d)
            if (d < j) acc += Tl[r + 16 * d] * g[d];
        if (l < 16) Tl[l + 16 * j] = l < j ? -tau * acc : (l == j ? tau : 0.0);
    }
}

// DTSQT2 on one inner block: x holds the b rows of A_ik (rows >= b zero) and
// Rr (LDS) the upper-triangular diagonal block of R_kk, row-major with each
// row r rotated left by r (Rr[16 r + c] = R[r][(r + c) mod 16], zeros where
// the column wraps), so that at step jj row jj lines up with the rotated
// columns of x.  Reflector jj is [e_jj; v_jj] (Sec. 3.1): it touches row jj
// of R and all of x.  On exit x holds V (the A_ik part of the reflectors), Rr
// the new triangle (same layout), Tl the block's T.  scr: kPanelScratch
// doubles of LDS.
template <int RPL>
__device__ __forceinline__ void ts_panel16(double (&x)[RPL][16], double *Rr, double *Tl, double *scr) {
    const int l = lane_id();
    double *part = scr, *Gs = scr + 64 * kPartStride, *taus = Gs + 256;
#pragma unroll 1
    for (int jj = 0; jj < 16; ++jj) {
        // row jj of R, rotated: rr[0] is the pivot, rr[c] is column jj + c
        double rr[16];
        const double2 *rp = reinterpret_cast<const double2 *>(Rr + 16 * jj);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const double2 t = rp[i];
            rr[2 * i] = t.x;
            rr[2 * i + 1] = t.y;
        }
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i) s += x[i][0] * x[i][0];
        const double sigma2 = wave_sum(s);
        const Reflector h = make_reflector(rr[0], sigma2);
        double v[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) v[i] = x[i][0] * h.scale;
        double P[16];
        panel_products<RPL>(x, v, P, part, Gs + 16 * jj);
        // w_c = R[jj][jj+c] + v^T A(:, jj+c);  R[jj][jj+c] -= tau w_c;
        // A(:, jj+c) -= tau w_c v, for c = 1 .. 15-jj (the columns past
        // 15-jj hold earlier reflectors: their factor is zero, and groups of
        // four such columns are skipped by a uniform branch)
        const int nright = 15 - jj;
        double tw[16];
#pragma unroll
        for (int c = 1; c < 16; ++c) tw[c] = c <= nright ? h.tau * (rr[c] + P[c]) : 0.0;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g > 0 && 4 * g > nright) continue;
#pragma unroll
            for (int c = 4 * g; c < 4 * g + 4; ++c) {
                if (c == 0) continue;
#pragma unroll
                for (int i = 0; i < RPL; ++i) x[i][c] -= tw[c] * v[i];
            }
        }
        if (l == 0) {
            rr[0] = h.beta;
#pragma unroll
            for (int c = 1; c < 16; ++c) rr[c] -= tw[c];
            double2 *wp = reinterpret_cast<double2 *>(Rr + 16 * jj);
#pragma unroll
            for (int i = 0; i < 8; ++i) wp[i] = double2{rr[2 * i], rr[2 * i + 1]};
            taus[jj] = h.tau;
        }
#pragma unroll
        for (int i = 0; i < RPL; ++i) x[i][0] = v[i];
        rotate_left<RPL>(x);
    }
    panel_t_from_gram(Gs, taus, Tl);
}

// DGEQT2 on one inner block whose pivots are rows c0 .. c0+15 of the tile:
// x holds rows c0 + lane + 64 i (rows >= b zero).  Pivot jj is in lane jj,
// i = 0.  On exit the rows at and below each pivot hold beta and v, the rows
// above the pivots are R entries, and Tl holds T.  scr as ts_panel16.
template <int RPL>
__device__ __forceinline__ void ge_panel16(double (&x)[RPL][16], double *Tl, double *scr) {
    const int l = lane_id();
    double *part = scr, *Gs = scr + 64 * kPartStride, *taus = Gs + 256;
#pragma unroll 1
    for (int jj = 0; jj < 16; ++jj) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < RPL; ++i)
            if (l + 64 * i > jj) s += x[i][0] * x[i][0];
        const double sigma2 = wave_sum(s);
        const Reflector h = make_reflector(readlane_d(x[0][0], jj), sigma2);
        // v with its unit pivot and zeros above
        double v[RPL];
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = l + 64 * i;
            v[i] = r > jj ? x[i][0] * h.scale : (r == jj ? 1.0 : 0.0);
        }
        double P[16];
        panel_products<RPL>(x, v, P, part, Gs + 16 * jj);
        const int nright = 15 - jj;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
            if (g > 0 && 4 * g > nright) continue;
#pragma unroll
            for (int c = 4 * g; c < 4 * g + 4; ++c) {
                if (c == 0) continue;
                const double tw = c <= nright ? h.tau * P[c] : 0.0;
#pragma unroll
                for (int i = 0; i < RPL; ++i) x[i][c] -= tw * v[i];
            }
        }
        if (l == 0) taus[jj] = h.tau;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int r = l + 64 * i;
            x[i][0] = r > jj ? v[i] : (r == jj ? h.beta : x[i][0]);
        }
        rotate_left<RPL>(x);
    }
    panel_t_from_gram(Gs, taus, Tl);
}

// ---------------------------------------------------------------------------
// Unrolled one-wave panels.  The 16 column steps run in groups of U
// (U = 4, 8 or 16) with the step inside a group a compile-time constant, so
// the pivot, the columns right of it and the columns holding earlier
// reflectors are known statically and the columns rotate left by U only
// after each group (not at all for U = 16).  Relative column c of group g is
// panel column (c + U g) mod 16.  Compared with the rotating panels above:
// the row of R that TSQRT updates is added into the batched products by the
// lanes of the first quarter (so the reduction yields w = R row + v^T A
// directly), the update is x -= w (tau v) on the live columns only, and the
// reflector takes one division.
// ---------------------------------------------------------------------------

// beta = -sgn(alpha) sqrt(alpha^2 + sigma2), d = alpha - beta (no
// cancellation: |d| = |alpha| + |beta|), q = 1 / (beta d): 1/beta = d q and
// 1/d = beta q, so tau = (beta - alpha) / beta = -d^2 q and scale = beta q.
__device__ __forceinline__ Reflector make_reflector_1div(double alpha, double sigma2) {
    Reflector h{0.0, alpha, 1.0};
    if (sigma2 != 0.0) {
        const double nrm = sqrt(fma(alpha, alpha, sigma2));
        h.beta = alpha >= 0.0 ? -nrm : nrm;
        const double d = alpha - h.beta;
        const double q = 1.0 / (h.beta * d);
        h.tau = -(d * d) * q;
        h.scale = h.beta * q;
    }
    return h;
}

// Rotation (in columns) in force at step r of a panel unrolled by U.
template <int U>
__device__ __forceinline__ int panel_rot(int r) { return (r / U) * U & 15; }

template <int RPL, int U>
__device__ __forceinline__ void rotate_left_by(double (&x)[RPL][16]) {
    if constexpr (U < 16) {
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            double t[U];
#pragma unroll
            for (int c = 0; c < U; ++c) t[c] = x[i][c];
#pragma unroll
            for (int c = 0; c + U < 16; ++c) x[i][c] = x[i][c + U];
#pragma unroll
            for (int c = 0; c < U; ++c) x[i][16 - U + c] = t[c];
        }
    }
}

// Batched products of one step: lane l ends with P[c] = add(c) + sum over
// the wave of v . x[.][c] for every c (the same in all lanes), where add(c)
// is the value lane c (< 16) passes in `add`; the totals also go to Gcol.
// `own` is the total of column l & 15.  SKIP is a column whose product is
// not needed (its partial is taken as 0).
template <int RPL, int SKIP>
__device__ __forceinline__ void panel_products_add(const double (&x)[RPL][16], const double (&v)[RPL], double add,
                                                   double (&P)[16], double &own, double *part, double *Gcol) {
    const int l = lane_id();
    double pv[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        double acc = 0.0;
        if (c != SKIP) {
#pragma unroll
            for (int i = 0; i < RPL; ++i) acc = fma(v[i], x[i][c], acc);
        }
        pv[c] = acc;
    }
    double2 *row = reinterpret_cast<double2 *>(part + l * kPartStride);
#pragma unroll
    for (int i = 0; i < 8; ++i) row[i] = double2{pv[2 * i], pv[2 * i + 1]};
    const double *col = part + (l >> 4) * 16 * kPartStride + (l & 15);
    double s4[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) s4[a] = col[a * kPartStride];
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int a = 0; a < 4; ++a) s4[a] += col[(4 * k + a) * kPartStride];
    double s = ((s4[0] + s4[1]) + (s4[2] + s4[3])) + add;
    s = sum_xor32(sum_xor16(s));
    own = s;
    if (l < 16) Gcol[l] = s;
    const double2 *g = reinterpret_cast<const double2 *>(Gcol);
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 t = g[i];
        P[2 * i] = t.x;
        P[2 * i + 1] = t.y;
    }
}

// T from the Gram columns of an unrolled panel: step j stored column j with
// the rotation of its group, G(d, j) = Gs[16 j + ((d - rot(j)) & 15)].
// Row r of T only involves row r (T[r][j] = -tau_j sum_{d<j} T[r][d] G(d, j)
// for r < j), so lane r keeps its row in registers: no LDS round trip per
// column, and the same operations in the same order as column by column.
template <int U>
__device__ __forceinline__ void panel_t_from_gram_u(const double *Gs, const double *taus, double *Tl) {
    const int l = lane_id(), r = l & 15;
    double t[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const double tau = taus[j];
        const int rot = panel_rot<U>(j);
        const double *g = Gs + 16 * j;
        double acc = 0.0;
#pragma unroll
        for (int d = 0; d < j; ++d) acc += t[d] * g[(d - rot) & 15];
        t[j] = r < j ? -tau * acc : (r == j ? tau : 0.0);
    }
    if (l < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) Tl[l + 16 * j] = t[j];
    }
}

// One step of the unrolled TSQRT panel: step jj = U g + u, pivot in relative
// column u.  Rr holds the diagonal block of R row-major with row r rotated
// left by rot(r) (Rr[16 r + c] = R[r][(c + rot(r)) mod 16], zero where that
// column is left of r).  One batched reduction gives g_c = x_u . x_c over the
// A rows for every column c: g_u is the sigma^2 of the reflector and, with
// v = scale x_u, w_c = R[jj][c] + scale g_c (also the Gram column of jj for
// T, as R row jj is zero in the columns of earlier reflectors).
template <int RPL, int U, int u>
__device__ __forceinline__ void ts_step(double (&x)[RPL][16], int g, double *Rr, double *part, double *Gs, double *taus) {
    const int l = lane_id();
    const int jj = U * g + u;
    double *rrow = Rr + 16 * jj, *Gcol = Gs + 16 * jj;
    double rr[16];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double2 t = reinterpret_cast<const double2 *>(rrow)[i];
        rr[2 * i] = t.x;
        rr[2 * i + 1] = t.y;
    }
    double xu[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) xu[i] = x[i][u];
    double gm[16], gown;
    panel_products_add<RPL, -1>(x, xu, 0.0, gm, gown, part, Gcol);
    const Reflector h = make_reflector_1div(rr[u], gm[u]);
    double v[RPL], tv[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        v[i] = xu[i] * h.scale;
        tv[i] = h.tau * v[i];
    }
    double P[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) P[c] = fma(h.scale, gm[c], rr[c]);
    // live columns right of the pivot: relative u+1 .. 15 - U g
    const int last = 15 - U * g;
    if (l == 0) {
        double nr[16];
#pragma unroll
        for (int c = 0; c < 16; ++c) nr[c] = c > u && c <= last ? fma(-h.tau, P[c], rr[c]) : (c == u ? h.beta : rr[c]);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            reinterpret_cast<double2 *>(Gcol)[i] = double2{P[2 * i], P[2 * i + 1]};
            reinterpret_cast<double2 *>(rrow)[i] = double2{nr[2 * i], nr[2 * i + 1]};
        }
        taus[jj] = h.tau;
    }
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        // groups wholly left of the pivot are skipped statically; since U is a
        // multiple of 4, a group past `last` holds only earlier reflectors
        if (4 * grp + 3 <= u) continue;
        if (4 * grp > last) continue;
#pragma unroll
        for (int c = 4 * grp; c < 4 * grp + 4; ++c) {
            if (c <= u) continue;
#pragma unroll
            for (int i = 0; i < RPL; ++i) x[i][c] = fma(-P[c], tv[i], x[i][c]);
        }
    }
#pragma unroll
    for (int i = 0; i < RPL; ++i) x[i][u] = v[i];
}

template <int RPL, int U, int u = 0>
__device__ __forceinline__ void ts_group(double (&x)[RPL][16], int g, double *Rr, double *part, double *Gs, double *taus) {
    if constexpr (u < U) {
        ts_step<RPL, U, u>(x, g, Rr, part, Gs, taus);
        ts_group<RPL, U, u + 1>(x, g, Rr, part, Gs, taus);
    }
}

// DTSQT2 on one inner block, unrolled by U (see ts_panel16 for the roles of
// x, Tl and scr; Rr in the layout of ts_step).
template <int RPL, int U>
__device__ __forceinline__ void ts_panel16u(double (&x)[RPL][16], double *Rr, double *Tl, double *scr) {
    static_assert(U % 4 == 0 && 16 % U == 0, "U must be 4, 8 or 16");
    double *part = scr, *Gs = scr + 64 * kPartStride, *taus = Gs + 256;
#pragma unroll 1
    for (int g = 0; g < 16 / U; ++g) {
        ts_group<RPL, U>(x, g, Rr, part, Gs, taus);
        rotate_left_by<RPL, U>(x);
    }
    panel_t_from_gram_u<U>(Gs, taus, Tl);
}

// One step of the unrolled GEQRT panel (pivot: relative row jj of the panel,
// lane jj of x[0]).  One batched reduction gives g_c = x_u . x_c over the
// rows below the pivot for every column c: g_u is sigma^2 and, with
// v = e_jj + scale x_u (below the pivot), w_c = x[jj][c] + scale g_c.
template <int RPL, int U, int u>
__device__ __forceinline__ void ge_step(double (&x)[RPL][16], int g, double *part, double *Gs, double *taus) {
    const int l = lane_id();
    const int jj = U * g + u;
    const bool below = l > jj, at = l == jj;
    double pr[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) pr[c] = bcast_lane_d(x[0][c], jj);
    double xu[RPL];
    xu[0] = below ? x[0][u] : 0.0;
#pragma unroll
    for (int i = 1; i < RPL; ++i) xu[i] = x[i][u];
    double gm[16], gown;
    double *Gcol = Gs + 16 * jj;
    panel_products_add<RPL, -1>(x, xu, 0.0, gm, gown, part, Gcol);
    const Reflector h = make_reflector_1div(pr[u], gm[u]);
    double v[RPL], tv[RPL];
#pragma unroll
    for (int i = 0; i < RPL; ++i) {
        v[i] = i == 0 ? (below ? xu[0] * h.scale : (at ? 1.0 : 0.0)) : xu[i] * h.scale;
        tv[i] = h.tau * v[i];
    }
    double P[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) P[c] = fma(h.scale, gm[c], pr[c]);
    if (l == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) reinterpret_cast<double2 *>(Gcol)[i] = double2{P[2 * i], P[2 * i + 1]};
        taus[jj] = h.tau;
    }
    const int last = 15 - U * g;
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        if (4 * grp + 3 <= u) continue;
        if (4 * grp > last) continue;
#pragma unroll
        for (int c = 4 * grp; c < 4 * grp + 4; ++c) {
            if (c <= u) continue;
#pragma unroll
            for (int i = 0; i < RPL; ++i) x[i][c] = fma(-P[c], tv[i], x[i][c]);
        }
    }
    x[0][u] = below ? v[0] : (at ? h.beta : x[0][u]);
#pragma unroll
    for (int i = 1; i < RPL; ++i) x[i][u] = v[i];
}

template <int RPL, int U, int u = 0>
__device__ __forceinline__ void ge_group(double (&x)[RPL][16], int g, double *part, double *Gs, double *taus) {
    if constexpr (u < U) {
        ge_step<RPL, U, u>(x, g, part, Gs, taus);
        ge_group<RPL, U, u + 1>(x, g, part, Gs, taus);
    }
}

// DGEQT2 on one inner block, unrolled by U (roles as in ge_panel16).
template <int RPL, int U>
__device__ __forceinline__ void ge_panel16u(double (&x)[RPL][16], double *Tl, double *scr) {
    static_assert(U % 4 == 0 && 16 % U == 0, "U must be 4, 8 or 16");
    double *part = scr, *Gs = scr + 64 * kPartStride, *taus = Gs + 256;
#pragma unroll 1
    for (int g = 0; g < 16 / U; ++g) {
        ge_group<RPL, U>(x, g, part, Gs, taus);
        rotate_left_by<RPL, U>(x);
    }
    panel_t_from_gram_u<U>(Gs, taus, Tl);
}

}  // namespace tqr
