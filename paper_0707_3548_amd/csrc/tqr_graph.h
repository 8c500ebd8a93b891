// Task graphs run by the persistent scheduler: closed-form numbering,
// dependency counts and successor lists, usable on the host and the device.
//
// Factorisation (Algorithm 1, Sec. 3.1; graph of Sec. 3.3).  Step k works on
// the (p-k) x (q-k) trailing tiles.  Its tasks are
//   GEQRT(k)                       factor diagonal tile (k,k)
//   TSQRT(i,k),   i > k            factor [R_kk; A_ik]
//   LARFB(k,j,c), j > k            apply GEQRT(k) to strip c of tile (k,j)
//   SSRFB(i,j,k,c), i,j > k        apply TSQRT(i,k) to strip c of (k,j),(i,j)
// A strip is a group of 64 columns of a tile (one strip when b <= 64):
// the two update kernels act on columns independently, so splitting them
// by columns leaves the arithmetic of every column unchanged.
//
// Dependencies (flat elimination tree; the diagonal tile's strict lower part
// V_kk and upper triangle R_kk are tracked apart, because TSQRT rewrites
// only R_kk while LARFB only reads V_kk):
//   GEQRT(k)        <- every strip of SSRFB(k,k,k-1)
//   TSQRT(i,k)      <- GEQRT(k) if i = k+1 else TSQRT(i-1,k);
//                      every strip of SSRFB(i,k,k-1)
//   LARFB(k,j,c)    <- GEQRT(k);  SSRFB(k,j,k-1,c)
//   SSRFB(i,j,k,c)  <- TSQRT(i,k); LARFB(k,j,c) if i = k+1 else
//                      SSRFB(i-1,j,k,c);  SSRFB(i,j,k-1,c)
// (terms with k-1 < 0 are absent).  Priorities (Sec. 3.3): GEQRT highest,
// then TSQRT, LARFB, SSRFB.
//
// Application of Q^T (or Q) to a block of right-hand sides B (p row tiles,
// strips of 64 columns): task (i,k,c) is LARFB on B_k when i == k and the
// SSRFB form on (B_k, B_i) when i > k, with the reflectors of tile (i,k).
//
// Back substitution with the tiled R: G(i,j), j > i: B_i -= R_ij X_j;
// D(i): X_i = R_ii^{-1} B_i.  G(i,j) <- D(j), G(i,j+1);  D(i) <- G(i,i+1).
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#define TQR_HD __host__ __device__ inline
#else
#define TQR_HD inline
#endif

namespace tqr {

enum Kind : int { GEQRT = 0, TSQRT = 1, LARFB = 2, SSRFB = 3, TSQRT_HELP = 4 };
constexpr int kStripCols = 64;   // columns of one update strip (one workgroup)
constexpr int kLevels = 8;       // ready-queue priority levels

struct Task {
    int kind, i, j, k, c;
};

TQR_HD int strips_of(int b) { return b > kStripCols ? b / kStripCols : 1; }

// ---------------------------------------------------------------------------
// Factorisation graph
// ---------------------------------------------------------------------------
struct FactorGraph {
    int64_t p, q, K, S;
    // With `helpers`, every TSQRT(i,k) has a helper task TSQRT_HELP(i,k)
    // (released when the TSQRT starts, no successors) that may take over part
    // of its trailing updates; helper ids follow the paper's tasks.
    bool helpers;

    TQR_HD FactorGraph(int64_t p_, int64_t q_, int b, bool helpers_ = false)
        : p(p_), q(q_), K(p_ < q_ ? p_ : q_), S(strips_of(b)), helpers(helpers_) {}

    // tasks of step k: (p-k) + (q-k-1)(p-k) S
    TQR_HD int64_t step_size(int64_t k) const { return (p - k) * (1 + S * (q - k - 1)); }
    // sum of step_size(t) for t < k, in closed form
    TQR_HD int64_t offset(int64_t k) const {
        const int64_t alpha = 1 + S * (q - 1);
        return p * alpha * k - (alpha + p * S) * (k * (k - 1) / 2) + S * ((k - 1) * k * (2 * k - 1) / 6);
    }
    TQR_HD int64_t num_paper_tasks() const { return offset(K); }
    // TSQRT tasks of steps before k: the sum over k' < k of (p - 1 - k')
    TQR_HD int64_t help_offset(int64_t k) const { return k * (p - 1) - k * (k - 1) / 2; }
    TQR_HD int64_t num_tasks() const { return offset(K) + (helpers ? help_offset(K) : 0); }
    TQR_HD int64_t encode_help(int64_t i, int64_t k) const { return offset(K) + help_offset(k) + (i - k - 1); }

    TQR_HD int64_t encode(int kind, int64_t i, int64_t j, int64_t k, int64_t c) const {
        const int64_t P = p - k;
        int64_t local;
        if (kind == GEQRT)
            local = 0;
        else if (kind == TSQRT)
            local = i - k;
        else
            local = P + (((j - k - 1) * P + (i - k)) * S + c);
        return offset(k) + local;
    }

    TQR_HD Task decode(int64_t t) const {
        if (t >= offset(K)) {
            const int64_t h = t - offset(K);
            int64_t lo = 0, hi = K - 1;  // largest k with help_offset(k) <= h
            while (lo < hi) {
                int64_t mid = (lo + hi + 1) / 2;
                if (help_offset(mid) <= h)
                    lo = mid;
                else
                    hi = mid - 1;
            }
            Task r;
            r.kind = TSQRT_HELP;
            r.k = (int)lo;
            r.j = (int)lo;
            r.i = (int)(lo + 1 + (h - help_offset(lo)));
            r.c = 0;
            return r;
        }
        int64_t lo = 0, hi = K - 1;  // largest k with offset(k) <= t
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (offset(mid) <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t k = lo, P = p - k;
        int64_t local = t - offset(k);
        Task r;
        r.k = (int)k;
        r.c = 0;
        if (local == 0) {
            r.kind = GEQRT; r.i = (int)k; r.j = (int)k;
        } else if (local < P) {
            r.kind = TSQRT; r.i = (int)(k + local); r.j = (int)k;
        } else {
            local -= P;
            r.c = (int)(local % S);
            local /= S;
            r.i = (int)(k + local % P);
            r.j = (int)(k + 1 + local / P);
            r.kind = (r.i == k) ? LARFB : SSRFB;
        }
        return r;
    }

    TQR_HD int indegree(const Task &t) const {
        const int prev = t.k > 0 ? 1 : 0;
        if (t.kind == TSQRT_HELP) return 1;
        switch (t.kind) {
        case GEQRT: return prev * (int)S;
        case TSQRT: return 1 + prev * (int)S;
        case LARFB: return 1 + prev;
        default: return 2 + prev;
        }
    }

    TQR_HD int num_successors(const Task &t) const {
        switch (t.kind) {
        case TSQRT_HELP: return 0;
        case GEQRT: return (t.i + 1 < p ? 1 : 0) + (int)((q - t.k - 1) * S);
        case TSQRT: return (helpers ? 1 : 0) + (t.i + 1 < p ? 1 : 0) + (int)((q - t.k - 1) * S);
        case LARFB: return t.k + 1 < p ? 1 : 0;
        default: return (t.i + 1 < p ? 1 : 0) + 1;
        }
    }

    // successor number n (0 <= n < num_successors)
    TQR_HD int64_t successor(const Task &t, int n) const {
        const int64_t k = t.k;
        switch (t.kind) {
        case GEQRT:
        case TSQRT: {
            if (t.kind == TSQRT && helpers) {
                if (n == 0) return encode_help(t.i, k);
                --n;
            }
            if (t.i + 1 < p) {
                if (n == 0) return encode(TSQRT, t.i + 1, k, k, 0);
                --n;
            }
            const int64_t j = k + 1 + n / S, c = n % S;
            return t.kind == GEQRT ? encode(LARFB, k, j, k, c) : encode(SSRFB, t.i, j, k, c);
        }
        case LARFB:
            return encode(SSRFB, k + 1, t.j, k, t.c);
        default: {
            if (t.i + 1 < p) {
                if (n == 0) return encode(SSRFB, t.i + 1, t.j, k, t.c);
            }
            const int64_t k1 = k + 1;
            if (t.j == k1) return t.i == k1 ? encode(GEQRT, k1, k1, k1, 0) : encode(TSQRT, t.i, k1, k1, 0);
            return t.i == k1 ? encode(LARFB, k1, t.j, k1, t.c) : encode(SSRFB, t.i, t.j, k1, t.c);
        }
        }
    }

    // priority level: 0 is served first.  Policy 0 (the paper's): by kind;
    // 1: the updates of tile column k+1 (the next panel) before the other
    // updates; 2: updates by the distance of their tile column j from the
    // next panel, levels 2..7 (the last holds every column from 6 on).  The
    // next panel is column k+1 for a task of step k, or `panel` (the number
    // of GEQRT tasks started so far) when the factorisation is further
    // ahead: an update whose column the panels are approaching becomes
    // more urgent than its step alone says.
    TQR_HD int level(const Task &t, int policy, int panel = 0) const {
        if (t.kind == GEQRT) return 0;
        if (t.kind == TSQRT || t.kind == TSQRT_HELP) return 1;
        if (policy == 2) {
            const int ref = panel > t.k + 1 ? panel : t.k + 1;
            const int d = t.j - ref;
            return 2 + (d < 0 ? 0 : (d < 5 ? d : 5));
        }
        if (t.kind == LARFB) return (policy == 1 && t.j == t.k + 1) ? 2 : 3;
        return (policy == 1 && t.j == t.k + 1) ? 2 : 4;
    }
};

// ---------------------------------------------------------------------------
// Application of Q^T (forward) or Q (backward) to p row tiles of B
// ---------------------------------------------------------------------------
struct ApplyGraph {
    int64_t p, K, S;
    bool forward;  // true: Q^T, false: Q

    TQR_HD ApplyGraph(int64_t p_, int64_t q_, int64_t strips, bool fwd) : p(p_), K(p_ < q_ ? p_ : q_), S(strips), forward(fwd) {}

    TQR_HD int64_t offset(int64_t k) const { return S * (p * k - k * (k - 1) / 2); }
    TQR_HD int64_t num_tasks() const { return offset(K); }
    TQR_HD int64_t encode(int64_t i, int64_t k, int64_t c) const { return offset(k) + (i - k) * S + c; }
    TQR_HD Task decode(int64_t t) const {
        int64_t lo = 0, hi = K - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (offset(mid) <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        int64_t local = t - offset(lo);
        Task r;
        r.k = (int)lo;
        r.c = (int)(local % S);
        r.i = (int)(lo + local / S);
        r.j = -1;
        r.kind = r.i == r.k ? LARFB : SSRFB;
        return r;
    }
    TQR_HD int indegree(const Task &t) const {
        if (forward)
            return (t.i > t.k ? 1 : 0) + (t.k > 0 ? 1 : 0);
        if (t.i == t.k) return t.k + 1 < p ? 1 : 0;
        return (t.i + 1 < p ? 1 : 0) + (t.k + 1 < K ? 1 : 0);
    }
    TQR_HD int num_successors(const Task &t) const {
        if (forward) {
            if (t.i == t.k) return t.k + 1 < p ? 1 : 0;
            return (t.i + 1 < p ? 1 : 0) + (t.k + 1 < K ? 1 : 0);
        }
        if (t.i == t.k) return t.k >= 1 ? 1 : 0;
        return 1 + (t.k >= 1 ? 1 : 0);
    }
    TQR_HD int64_t successor(const Task &t, int n) const {
        const int64_t k = t.k, i = t.i, c = t.c;
        if (forward) {
            if (i == k) return encode(k + 1, k, c);
            if (i + 1 < p) {
                if (n == 0) return encode(i + 1, k, c);
            }
            return encode(i, k + 1, c);  // i >= k+1: LARFB when i == k+1
        }
        if (i == k) return encode(k, k - 1, c);
        if (n == 0) return encode(i - 1, k, c);  // LARFB_Q(k) when i-1 == k
        return encode(i, k - 1, c);
    }
};

// ---------------------------------------------------------------------------
// Tiled back substitution with the q x q upper-triangular tiles of R
// ---------------------------------------------------------------------------
struct TrsmGraph {
    int64_t q;
    TQR_HD explicit TrsmGraph(int64_t q_) : q(q_) {}
    // row i holds G(i, q-1), ..., G(i, i+1), D(i): q - i tasks
    TQR_HD int64_t offset(int64_t i) const { return q * i - i * (i - 1) / 2; }
    TQR_HD int64_t num_tasks() const { return offset(q); }
    TQR_HD int64_t encode_g(int64_t i, int64_t j) const { return offset(i) + (q - 1 - j); }
    TQR_HD int64_t encode_d(int64_t i) const { return offset(i) + (q - 1 - i); }
    // kind 0 = D (diagonal solve), 1 = G (update)
    TQR_HD Task decode(int64_t t) const {
        int64_t lo = 0, hi = q - 1;
        while (lo < hi) {
            int64_t mid = (lo + hi + 1) / 2;
            if (offset(mid) <= t)
                lo = mid;
            else
                hi = mid - 1;
        }
        int64_t local = t - offset(lo);
        Task r;
        r.i = (int)lo;
        r.k = 0;
        r.c = 0;
        r.j = (int)(q - 1 - local);
        r.kind = (r.j == r.i) ? 0 : 1;
        return r;
    }
    TQR_HD int indegree(const Task &t) const {
        if (t.kind == 0) return t.i < q - 1 ? 1 : 0;
        return 1 + (t.j < q - 1 ? 1 : 0);
    }
    TQR_HD int num_successors(const Task &t) const { return t.kind == 0 ? t.i : 1; }
    TQR_HD int64_t successor(const Task &t, int n) const {
        if (t.kind == 0) return encode_g(n, t.i);  // G(n, i) for n < i
        return (t.j - 1 > t.i) ? encode_g(t.i, t.j - 1) : encode_d(t.i);
    }
};

}  // namespace tqr
