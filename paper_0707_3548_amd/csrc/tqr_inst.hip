// tqr: the kernels and host launchers of one (tile_b, inner_ib) pair, chosen
// at compile time by TQR_INST_B and TQR_INST_IB (the build compiles this file
// once per supported pair, in parallel).
#include "tqr_impl.h"

#if !defined(TQR_INST_B) || !defined(TQR_INST_IB)
#error "compile with -DTQR_INST_B=<tile_b> -DTQR_INST_IB=<inner_ib>"
#endif

namespace tqr {

template <int B, int IB>
static PairFns make_pair_fns() {
    PairFns f{};
    f.factor = &factor_impl<B, IB>;
    f.apply = &apply_impl<B, IB>;
    f.solve = &solve_impl<B, IB>;
    if constexpr (IB == 16 && B >= 64) {
        f.mixed = &mixed_impl<B>;
        f.apply_narrow = &narrow_apply<B, IB>;
    }
    return f;
}

template <>
const PairFns &pair_fns<TQR_INST_B, TQR_INST_IB>() {
    static const PairFns f = make_pair_fns<TQR_INST_B, TQR_INST_IB>();
    return f;
}

}  // namespace tqr
