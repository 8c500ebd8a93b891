// Host-side bounds check of the strip updates' LDS operand reads: for every
// (tile_b, inner_ib) pair the library instantiates, both forms (TS / not),
// both directions, every inner block start c0 and every lane, enumerate the
// reads panel_update and panel_update_f32 issue (the offsets come from the
// kernels' own tqr_offsets.h; the row blocks read are rb0 .. B/16-1, which
// covers the one-row-block-ahead prefetch, guarded by rb + 1 < B/16) and
// check that each lands inside the staged buffer it is meant to read:
//   * staged V/T (leading dimension B + 1): V element (row, col) with
//     row < B, col < IB; T element < IB * IB;
//   * the generic ib = 32/64 panel in LDS (leading dimension IB + B + 1):
//     the GEQRT form reads it shifted by -c0 (rows c0.. only), the TSQRT form
//     shifted by +IB (below the IB rows of R).
// Prints the number of reads checked; exits 1 at the first violation.
#include <cstdio>
#include <cstdlib>

#include "tqr_offsets.h"

using namespace tqr;

static long g_reads = 0;

static void fail(const char *what, int B, int IB, int trans, int ts, int c0, int l, int a, int rb, int r, long off) {
    std::printf("VIOLATION %s: B=%d IB=%d trans=%d ts=%d c0=%d lane=%d a=%d rb=%d r=%d offset=%ld\n", what, B, IB,
                trans, ts, c0, l, a, rb, r, off);
    std::exit(1);
}

// layout: 0 staged (ldv = B+1, base 0); 1 generic GEQRT form (ldv = IB+B+1,
// base -c0); 2 generic TSQRT form (ldv = IB+B+1, base +IB)
static void check_fp64(int B, int IB, int layout) {
    const int ldv = layout == 0 ? B + 1 : IB + B + 1;
    const long region = (long)ldv * IB;
    const int NA = IB / 16;
    for (int trans = 0; trans < 2; ++trans)
        for (int ts = 0; ts < 2; ++ts) {
            if (layout == 1 && ts) continue;
            if (layout == 2 && !ts) continue;
            for (int c0 = 0; c0 + IB <= B; c0 += IB) {
                const int rb0 = ts ? 0 : c0 / 16;
                const long base = layout == 1 ? -c0 : (layout == 2 ? IB : 0);
                for (int l = 0; l < 64; ++l)
                    for (int rb = rb0; rb < B / 16; ++rb)
                        for (int a = 0; a < NA; ++a)
                            for (int r = 0; r < 4; ++r) {
                                const long offs[2] = {upd_vt_off(l, ldv, a, rb, r), upd_v_off(l, ldv, a, rb, r)};
                                for (int w = 0; w < 2; ++w) {
                                    const long off = offs[w];
                                    const long col = off / ldv, row = off % ldv;
                                    const long phys = off + base;
                                    ++g_reads;
                                    if (col < 0 || col >= IB || row < 16 * rb0 || row >= B)
                                        fail(w ? "V (C -= V W)" : "V (V^T C)", B, IB, trans, ts, c0, l, a, rb, r, off);
                                    if (phys < 0 || phys >= region)
                                        fail("V outside its LDS buffer", B, IB, trans, ts, c0, l, a, rb, r, phys);
                                }
                            }
                if (layout != 0) continue;
                for (int l = 0; l < 64; ++l)
                    for (int o = 0; o < NA; ++o)
                        for (int a = 0; a < NA; ++a) {
                            if (trans ? (a > o) : (a < o)) continue;
                            for (int r = 0; r < 4; ++r) {
                                const long off = upd_t_off(trans != 0, l, IB, o, a, r);
                                ++g_reads;
                                if (off < 0 || off >= (long)IB * IB) fail("T", B, IB, trans, ts, c0, l, a, o, r, off);
                            }
                        }
            }
        }
}

static void check_f32(int B) {
    const int ldv = B + 1, IB = 16;
    for (int trans = 0; trans < 2; ++trans)
        for (int ts = 0; ts < 2; ++ts)
            for (int c0 = 0; c0 + IB <= B; c0 += IB) {
                const int rb0 = ts ? 0 : c0 / 16;
                for (int l = 0; l < 64; ++l) {
                    for (int rb = rb0; rb < B / 16; ++rb)
                        for (int r = 0; r < 4; ++r) {
                            const long offs[2] = {updf_vt_off(l, ldv, rb, r), updf_v_off(l, ldv, rb, r)};
                            for (int w = 0; w < 2; ++w) {
                                const long off = offs[w], col = off / ldv, row = off % ldv;
                                ++g_reads;
                                if (col < 0 || col >= IB || row < 16 * rb0 || row >= B)
                                    fail(w ? "V f32 (C -= V W)" : "V f32 (V^T C)", B, IB, trans, ts, c0, l, 0, rb, r, off);
                            }
                        }
                    for (int r = 0; r < 4; ++r) {
                        const long off = updf_t_off(trans != 0, l, r);
                        ++g_reads;
                        if (off < 0 || off >= 256) fail("T f32", B, IB, trans, ts, c0, l, 0, 0, r, off);
                    }
                }
            }
}

int main() {
    // the (tile_b, inner_ib) pairs the library instantiates
    const int pairs[][2] = {{16, 16}, {32, 16}, {32, 32}, {64, 16}, {64, 32}, {64, 64},
                            {128, 16}, {128, 32}, {256, 16}, {256, 32}};
    for (const auto &pr : pairs) {
        check_fp64(pr[0], pr[1], 0);
        if (pr[1] > 16) {
            check_fp64(pr[0], pr[1], 1);
            check_fp64(pr[0], pr[1], 2);
        }
        if (pr[1] == 16) check_f32(pr[0]);
    }
    std::printf("OK %ld reads checked\n", g_reads);
    return 0;
}
