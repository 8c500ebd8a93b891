// tqr: LDS element offsets of the strip update's operand reads.
//
// The strip updates (panel_update in FP64, panel_update_f32 in the FP32 and
// BF16 tiers) read the staged V of one inner block (IB columns of B rows,
// column-major with leading dimension ldv) and its IB x IB T (column-major,
// leading dimension IB) from LDS.  The offsets are computed here, in plain
// C++ shared by the kernels and a host-side bounds check, so that the check
// enumerates exactly the reads the kernels issue.
//
// Lane l (0..63) of the wave; a: 16-column group of V (0..IB/16-1); rb: the
// strip's 16-row block (0..B/16-1); r: k-slice (0..3); o: 16-row group of
// op(T).
#pragma once

#if defined(__HIPCC__)
#define TQR_OFF_HD __host__ __device__ inline
#else
#define TQR_OFF_HD inline
#endif

namespace tqr {

// A-operand row m (0..15) of a product accumulated into a strip's row block
// reads source row strip_row_perm(m) = 4(m % 4) + m / 4 of that block.
TQR_OFF_HD int strip_row_perm(int m) { return 4 * (m & 3) + (m >> 2); }

// ---- FP64 form (v_mfma_f64_16x16x4f64) --------------------------------------
// V^T C: A operand V^T[16a + l%16][16rb + 4(l/16) + r] = V(16rb + 4(l/16) + r, 16a + l%16)
TQR_OFF_HD int upd_vt_off(int l, int ldv, int a, int rb, int r) {
    return (16 * a + (l & 15)) * ldv + 16 * rb + 4 * (l >> 4) + r;
}
// C -= V W2: A operand V(16rb + strip_row_perm(l%16), 16a + 4r + l/16)
TQR_OFF_HD int upd_v_off(int l, int ldv, int a, int rb, int r) {
    return (16 * a + 4 * r + (l >> 4)) * ldv + 16 * rb + strip_row_perm(l & 15);
}
// W2 = op(T) W: A operand op(T)[16o + l%16][16a + 4r + l/16] (op(T) = T^T
// when trans), read only where T's triangle is nonzero (a <= o for T^T, a >= o
// for T)
TQR_OFF_HD int upd_t_off(bool trans, int l, int ib, int o, int a, int r) {
    return trans ? (16 * o + (l & 15)) * ib + 16 * a + (l >> 4) + 4 * r
                 : (16 * a + (l >> 4) + 4 * r) * ib + 16 * o + (l & 15);
}

// ---- FP32 / BF16 form (inner block 16, v_mfma_f32_16x16x4f32) --------------
// V^T C: k-slice r of row block rb uses V rows 16rb + 4r + l/16, column l%16
TQR_OFF_HD int updf_vt_off(int l, int ldv, int rb, int r) { return (l & 15) * ldv + 16 * rb + 4 * r + (l >> 4); }
// C -= V W2: V(16rb + perm(l%16), 4(l/16) + r), perm(4a + b) = 4b + a
TQR_OFF_HD int updf_v_off(int l, int ldv, int rb, int r) {
    return (4 * (l >> 4) + r) * ldv + 16 * rb + 4 * (l & 3) + ((l & 15) >> 2);
}
// W2 = op(T) W: k-slice r reads op(T)[l%16][4(l/16) + r]
TQR_OFF_HD int updf_t_off(bool trans, int l, int r) {
    return trans ? (l & 15) * 16 + 4 * (l >> 4) + r : (4 * (l >> 4) + r) * 16 + (l & 15);
}

}  // namespace tqr
