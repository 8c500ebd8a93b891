// tqr: narrow right-hand sides (at most kNarrowRhs columns).
//
// Applying Q^T or Q of the tiled factorisation (the transformations of
// Algorithm 1 in their own order, as tqr_apply_qt does) and the two
// triangular solves with R, for a block B of 1 to 4 columns, as pipelines of
// workgroups instead of graphs of tile tasks.  With so few columns every tile
// task is a few microseconds of work behind a task's fixed costs, and the
// flat tree chains them: in column k, every pair (k, i) rewrites row tile k
// of B, so the graph's tasks run one after another.  Here one workgroup owns
// each row tile i of B (its rows in registers, one row per thread) for the
// whole launch and walks its part of Algorithm 1; what passes from one
// workgroup to the next is row block s of tile k (ib rows), handed over
// through a small buffer and a flag per (k, i, s).
//
// Q^T, column k (Sec. 3.1): the owner of row tile k applies the reflectors of
// GEQRT(k) (inner blocks s = 0, 1, ...), publishing row block s of tile k as
// soon as block s has been applied (later blocks of the tile do not touch
// it); the owner of row tile i > k applies the inner blocks of TSQRT(i, k) to
// the pair (row block s of tile k, tile i):
//     W = T_s^T (B_k[s] + V_s^T B_i),  B_k[s] -= W,  B_i -= V_s W,
// taking B_k[s] from the owner of tile i-1 and handing it to tile i+1; the
// last tile row writes the finished block to B.  V_s^T B_i does not depend
// on B_k[s], so each workgroup forms it before waiting.  Q runs the same
// steps transposed and in reverse (columns, rows and inner blocks in
// descending order, W = T_s (...)), with row tile k flowing up from the last
// tile row to its owner, which applies GEQRT(k) last.
//
// The triangular solves work on blocks of 64 rows: the owner of block j
// accumulates the products of the off-diagonal blocks of R with the solution
// blocks as their owners publish them, then solves its diagonal block in one
// wavefront and publishes its own solution block.
//
// Ordering and progress.  A workgroup takes its place in the pipeline from a
// ticket counter, not from its block index, so every workgroup it waits for
// has already started and holds its compute unit: the launch cannot wait on a
// workgroup that is not resident.  Hand-over buffers are filled with a
// "pending" bit pattern (a signalling NaN, which no arithmetic result has:
// results of operations are quiet) before the launch; a writer stores each
// value with a relaxed system-scope atomic (which goes to memory rather than
// to a compute unit's or an XCD's cache), and a reader polls the value itself
// until it is no longer pending, so a hand-over costs one trip to memory on
// each side and no separate flag.  Every wait is bounded (device clock and
// spin count): a wait that runs out sets the abort word, which every waiting
// thread also watches, and TQR_EABORTED in the status word.
// Included by tqr_impl.h inside namespace tqr, after the scheduler's flag
// helpers.
#pragma once

constexpr int kNarrowRhs = 4;   // widest block of right-hand sides handled here
constexpr int kTrsvRows = 64;   // rows per block of the triangular solves

// Control words of one narrow launch (zeroed before it): ticket, abort.
struct NarrowCtl {
    int32_t *ticket;
    int32_t *abort;
    int32_t *status;   // caller's status word or null
    int64_t timeout;   // per-wait bound in device clock ticks
};

__device__ __forceinline__ double coh_load(const double *p) {
    const uint64_t u = __hip_atomic_load(reinterpret_cast<uint64_t *>(const_cast<double *>(p)), __ATOMIC_RELAXED,
                                         TQR_FLAG_SCOPE);
    return __builtin_bit_cast(double, u);
}
__device__ __forceinline__ void coh_store(double *p, double v) {
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                       TQR_FLAG_SCOPE);
}

// The "pending" pattern of hand-over buffers: a signalling NaN.
constexpr uint64_t kPendingBits = 0x7FF4D1A5C0FFEE01ull;

// Waits until *p holds a value (not the pending pattern) and returns it in
// `out`; false when the launch was aborted (here or elsewhere).  Each calling
// thread polls its own value.
__device__ bool narrow_take(const double *p, double &out, const NarrowCtl &c) {
    uint64_t u = __hip_atomic_load(reinterpret_cast<uint64_t *>(const_cast<double *>(p)), __ATOMIC_RELAXED,
                                   TQR_FLAG_SCOPE);
    if (u != kPendingBits) {
        out = __builtin_bit_cast(double, u);
        return true;
    }
    const uint64_t deadline = rt_clock() + (uint64_t)c.timeout;
    uint32_t n = 0;
    while (true) {
        __builtin_amdgcn_s_sleep(1);
        u = __hip_atomic_load(reinterpret_cast<uint64_t *>(const_cast<double *>(p)), __ATOMIC_RELAXED,
                              TQR_FLAG_SCOPE);
        if (u != kPendingBits) break;
        if (flag_load(c.abort) != 0) return false;
        if (rt_clock() > deadline || ++n > kMaxSpins) {
            __hip_atomic_store(c.abort, 1, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            if (c.status) __hip_atomic_store(c.status, (int32_t)TQR_EABORTED, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
            return false;
        }
    }
    out = __builtin_bit_cast(double, u);
    return true;
}

// Lane l ends with the wave's total of v[l & 15] (every lane of the wave
// takes part): the halving exchanges of wave_allsum16, without the final
// broadcast.
__device__ __forceinline__ double wave_reduce16(const double (&v)[16]) {
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
    const double d = (hi ? c[1] : c[0]) + dpp_d<kDppXor1>(hi ? c[0] : c[1]);
    return sum_xor32(sum_xor16(d));
}

// ---------------------------------------------------------------------------
// Q^T B (TRANS) or Q B for nrhs <= NR columns, tiles of the factorisation in
// W (p x q grid of b x b tiles), the dense unit-lower V of each diagonal
// tile in Vd, T as tqr_factor writes it.  B is column-major m x nrhs.
// ---------------------------------------------------------------------------
struct NarrowApplyArgs {
    const double *W, *Vd, *T;
    double *Bm;
    int64_t ldb, m;
    int nrhs, p, q;
    double *H;        // hand-over blocks: slot (k, i, s) holds ib x NR doubles, pending on entry
    NarrowCtl ctl;
};

template <int B, int IB, int NR, bool TRANS>
__global__ __launch_bounds__(B) void k_narrow_apply(NarrowApplyArgs a) {
    static_assert(IB == 16 && B % 64 == 0 && IB * NR <= 64, "one wave forms W");
    constexpr int NWV = B / 64, NB = B / IB;
    __shared__ double zpart[NWV][NR][IB];
    __shared__ double wsh[NR][IB];
    __shared__ double ush[NR][IB];
    __shared__ int s_row, s_ok;
    const int t = threadIdx.x, l = lane_id(), wv = wave_id();
    const int p = a.p, q = a.q;
    if (t == 0) {
        const int tk = __hip_atomic_fetch_add(a.ctl.ticket, 1, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
        s_row = TRANS ? tk : p - 1 - tk;
        s_ok = 1;
    }
    __syncthreads();
    const int i = s_row;
    const int64_t grow = (int64_t)i * B + t;
    double bi[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) bi[r] = (grow < a.m && r < a.nrhs) ? a.Bm[r * a.ldb + grow] : 0.0;
    auto slot = [&](int k, int ii, int s) { return ((int64_t)k * p + ii) * NB + s; };
    // lanes of wave 0 that form W: column c of the inner block, right-hand side r
    const int wc = l % IB, wr = l / IB;
    const bool former = wv == 0 && l < IB * NR;

    const int kmax = i < q - 1 ? i : q - 1;
    for (int kk = 0; kk <= kmax; ++kk) {
        const int k = TRANS ? kk : kmax - kk;
        const bool top = k == i;
        const double *V = top ? a.Vd + (int64_t)k * B * B : a.W + ((int64_t)k * p + i) * B * B;
        const double *Ts = a.T + ((int64_t)k * p + i) * IB * B;
        for (int si = 0; si < NB; ++si) {
            const int s = TRANS ? si : NB - 1 - si;
            // Q, top: row block s of tile k arrives from the row below (or is
            // the input itself when there is no row below)
            if (!TRANS && top && k + 1 < p) {
                const int owner = (s * IB) / 64;
                if (wv == owner && t >= s * IB && t < s * IB + IB) {
                    const double *h = a.H + slot(k, k + 1, s) * IB * NR;
#pragma unroll
                    for (int r = 0; r < NR; ++r)
                        if (!narrow_take(h + r * IB + (t - s * IB), bi[r], a.ctl)) s_ok = 0;
                }
            }
            double v[IB];
#pragma unroll
            for (int c = 0; c < IB; ++c) v[c] = V[(int64_t)(s * IB + c) * B + t];
            double tcol[IB] = {};
            if (former) {
#pragma unroll
                for (int c2 = 0; c2 < IB; ++c2)
                    tcol[c2] = TRANS ? Ts[(s * IB + wc) * IB + c2] : Ts[(s * IB + c2) * IB + wc];
            }
            // Z = V_s^T B_i (this tile's rows), summed over the workgroup
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double pv[IB];
#pragma unroll
                for (int c = 0; c < IB; ++c) pv[c] = (top && t < s * IB) ? 0.0 : v[c] * bi[r];
                const double d = wave_reduce16(pv);
                if (l < IB) zpart[wv][r][l] = d;
            }
            __syncthreads();
            if (!s_ok) break;
            if (wv == 0) {
                double bk = 0.0;
                if (!top && former) {
                    // row block s of tile k from the previous workgroup of the chain
                    const bool first = TRANS ? false : i == p - 1;
                    if (first) {
                        const int64_t row = (int64_t)k * B + s * IB + wc;
                        bk = (row < a.m && wr < a.nrhs) ? a.Bm[wr * a.ldb + row] : 0.0;
                    } else {
                        const int64_t in = TRANS ? slot(k, i - 1, s) : slot(k, i + 1, s);
                        if (!narrow_take(a.H + in * IB * NR + wr * IB + wc, bk, a.ctl)) s_ok = 0;
                    }
                }
                if (former) {
                    double z = 0.0;
#pragma unroll
                    for (int w = 0; w < NWV; ++w) z += zpart[w][wr][wc];
                    ush[wr][wc] = bk + z;
                }
                // W = T_s^T U (Q^T) or T_s U (Q); T_s upper triangular
                if (former) {
                    double w = 0.0;
#pragma unroll
                    for (int c2 = 0; c2 < IB; ++c2) {
                        const bool in_tri = TRANS ? c2 <= wc : c2 >= wc;
                        if (in_tri) w += tcol[c2] * ush[wr][c2];
                    }
                    wsh[wr][wc] = w;
                    if (!top) {
                        const double out = bk - w;
                        if (TRANS && i == p - 1) {
                            const int64_t row = (int64_t)k * B + s * IB + wc;
                            if (row < a.m && wr < a.nrhs) a.Bm[wr * a.ldb + row] = out;
                        } else {
                            coh_store(a.H + slot(k, i, s) * IB * NR + wr * IB + wc, out);
                        }
                    }
                }
            }
            __syncthreads();
            if (!s_ok) break;
            // B_i -= V_s W
#pragma unroll
            for (int r = 0; r < NR; ++r) {
                double acc = bi[r];
#pragma unroll
                for (int c = 0; c < IB; ++c) acc -= v[c] * wsh[r][c];
                bi[r] = acc;
            }
            // Q^T, top: row block s of tile k is final for this column
            if (TRANS && top) {
                const int owner = (s * IB) / 64;
                if (wv == owner && t >= s * IB && t < s * IB + IB) {
                    if (k == p - 1) {
#pragma unroll
                        for (int r = 0; r < NR; ++r)
                            if (grow < a.m && r < a.nrhs) a.Bm[r * a.ldb + grow] = bi[r];
                    } else {
                        double *h = a.H + slot(k, k, s) * IB * NR;
#pragma unroll
                        for (int r = 0; r < NR; ++r) coh_store(h + r * IB + (t - s * IB), bi[r]);
                    }
                }
            }
        }
        if (!s_ok) return;
    }
    // rows whose final value this workgroup holds
    const bool store = TRANS ? i >= q : true;
    if (store) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (grow < a.m && r < a.nrhs) a.Bm[r * a.ldb + grow] = bi[r];
    }
}

// ---------------------------------------------------------------------------
// Triangular solves with the n x n upper-triangular R of the tiles:
// R X = Y (back substitution) or R^T X = Y (TRANS, forward substitution),
// Y (n x nrhs, column-major, leading dimension ldy) overwritten by X.
// ---------------------------------------------------------------------------
struct NarrowTrsvArgs {
    const double *W;
    int p;
    int64_t n;
    double *Y;
    int64_t ldy;
    int nrhs;
    double *X;        // published solution blocks: block j at X + j * 64 * NR (by rhs), pending on entry
    const int32_t *skip;  // nonzero: return at once (or null)
    NarrowCtl ctl;
};

template <int B>
__device__ __forceinline__ double r_at(const double *W, int p, int64_t r, int64_t c) {
    return W[((c / B) * p + r / B) * (int64_t)B * B + (c % B) * B + r % B];
}

template <int B, int NR, bool TRANS>
__global__ __launch_bounds__(256) void k_narrow_trsv(NarrowTrsvArgs a) {
    constexpr int RB = kTrsvRows, NW = 4;
    __shared__ double xs[NR][RB];            // the arriving solution block
    __shared__ double part[NW][NR][RB];      // per-wave partial sums
    __shared__ double dsh[RB][RB + 1];       // the diagonal block R_jj (padded rows)
    __shared__ int s_blk, s_ok;
    const int t = threadIdx.x, l = lane_id(), wv = wave_id();
    const int nb = (int)((a.n + RB - 1) / RB);
    if (a.skip && *a.skip) return;
    if (t == 0) {
        const int tk = __hip_atomic_fetch_add(a.ctl.ticket, 1, __ATOMIC_RELAXED, TQR_FLAG_SCOPE);
        s_blk = TRANS ? tk : nb - 1 - tk;
        s_ok = 1;
    }
    __syncthreads();
    const int j = s_blk;
    const int64_t r0 = (int64_t)j * RB;
    // stage the diagonal block while the earlier blocks are being solved
    for (int idx = t; idx < RB * RB; idx += 256) {
        const int rr = idx % RB, cc = idx / RB;
        dsh[rr][cc] = (r0 + rr < a.n && r0 + cc < a.n) ? r_at<B>(a.W, a.p, r0 + rr, r0 + cc) : 0.0;
    }
    // Back substitution: lane l of every wave owns row r0 + l and wave w
    // takes columns 16w .. 16w+15 of each arriving block.  Forward: lane l
    // is row l of the arriving block and wave w accumulates the products for
    // this block's columns 16w .. 16w+15 (16 per lane, summed at the end).
    double acc[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) acc[r] = 0.0;
    double pacc[TRANS ? 16 : 1][NR];
#pragma unroll
    for (int c = 0; c < (TRANS ? 16 : 1); ++c)
#pragma unroll
        for (int r = 0; r < NR; ++r) pacc[c][r] = 0.0;
    const int cnt = TRANS ? j : nb - 1 - j;   // arriving blocks
    double rv[16];
    auto load_block = [&](int c) {
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            int64_t rr, cc;
            if (TRANS) {
                rr = (int64_t)c * RB + l;
                cc = r0 + 16 * wv + u;
            } else {
                rr = r0 + l;
                cc = (int64_t)c * RB + 16 * wv + u;
            }
            rv[u] = (rr < a.n && cc < a.n) ? r_at<B>(a.W, a.p, rr, cc) : 0.0;
        }
    };
    if (cnt > 0) load_block(TRANS ? 0 : nb - 1);
    for (int e = 0; e < cnt; ++e) {
        const int c = TRANS ? e : nb - 1 - e;
        if (t < RB * NR) {
            double v = 0.0;
            if (!narrow_take(a.X + (int64_t)c * RB * NR + t, v, a.ctl)) s_ok = 0;
            xs[t / RB][t % RB] = v;
        }
        __syncthreads();
        if (!s_ok) return;
        double cur[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) cur[u] = rv[u];
        if (e + 1 < cnt) load_block(TRANS ? e + 1 : nb - 2 - e);
        if (TRANS) {
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int r = 0; r < NR; ++r) pacc[u][r] += cur[u] * xs[r][l];
        } else {
#pragma unroll
            for (int u = 0; u < 16; ++u)
#pragma unroll
                for (int r = 0; r < NR; ++r) acc[r] += cur[u] * xs[r][16 * wv + u];
        }
        __syncthreads();   // xs is rewritten by the next block
    }
    // combine the waves' sums: part[w][r][row]
    if (TRANS) {
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            double v16[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) v16[u] = pacc[u][r];
            const double d = wave_reduce16(v16);
            if (l < 16) part[0][r][16 * wv + l] = d;
        }
    } else {
#pragma unroll
        for (int r = 0; r < NR; ++r) part[wv][r][l] = acc[r];
    }
    __syncthreads();
    if (wv != 0) return;
    // diagonal block: lane l holds row l (back) or column l (forward) of R_jj
    double dg[RB];
    const int64_t myrow = r0 + l;
#pragma unroll
    for (int u = 0; u < RB; ++u) dg[u] = TRANS ? dsh[u][l] : dsh[l][u];
    double y[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        double s = 0.0;
        if (TRANS) {
            s = part[0][r][l];
        } else {
#pragma unroll
            for (int w = 0; w < NW; ++w) s += part[w][r][l];
        }
        const double yin = (myrow < a.n && r < a.nrhs) ? a.Y[r * a.ldy + myrow] : 0.0;
        y[r] = yin - s;
    }
    double dii = 0.0;
#pragma unroll
    for (int u = 0; u < RB; ++u)
        if (u == l) dii = dg[u];
    const double rinv = (myrow < a.n) ? 1.0 / dii : 0.0;
    // column sweep in one wave: step u finishes row u
#pragma unroll
    for (int si = 0; si < RB; ++si) {
        const int u = TRANS ? si : RB - 1 - si;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            const double xu = readlane_d(y[r] * rinv, u);
            if (l == u) y[r] = xu;
            else if (TRANS ? l > u : l < u) y[r] -= dg[u] * xu;
        }
    }
    // publish and store the solution block
    if (myrow < a.n) {
#pragma unroll
        for (int r = 0; r < NR; ++r)
            if (r < a.nrhs) a.Y[r * a.ldy + myrow] = y[r];
    }
    const bool others = TRANS ? j + 1 < nb : j > 0;
    if (others) {
#pragma unroll
        for (int r = 0; r < NR; ++r) coh_store(a.X + (int64_t)j * RB * NR + r * RB + l, myrow < a.n ? y[r] : 0.0);
    }
}
