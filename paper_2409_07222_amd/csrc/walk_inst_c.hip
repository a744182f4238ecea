// Instantiations of the first-step walker for NW in {8, 9, 10}.
#include "walk_impl.h"

namespace labsdev {

namespace {
template <int NW, int R, int RB>
void fill(WalkKernels* o) {
    o->plain = walkimpl::k_walk<NW, R, RB>;
    o->bloom = walkimpl::k_walk_bloom<NW, R, RB>;
    o->persistent = walkimpl::k_walk_persistent<NW, R, RB>;
    o->R = R;
    o->RB = RB;
}

// R in {ceil(NW/2), ceil(NW/2)+1}; RB in {R, ceil(R/2)}.
template <int NW>
bool pick(int R, int RB, WalkKernels* o) {
    constexpr int R0 = (NW + 1) / 2, R1 = R0 + 1;
    constexpr int H0 = (R0 + 1) / 2, H1 = (R1 + 1) / 2;
    if (R <= R0) {
        if (RB < R0) fill<NW, R0, H0>(o); else fill<NW, R0, R0>(o);
        return true;
    }
    if (R == R1) {
        if (RB < R1) fill<NW, R1, H1>(o); else fill<NW, R1, R1>(o);
        return true;
    }
    return false;
}
}  // namespace

bool walk_kernels_c(int NW, int R, int RB, WalkKernels* o) {
    switch (NW) {
        case 8: return pick<8>(R, RB, o);
        case 9: return pick<9>(R, RB, o);
        case 10: return pick<10>(R, RB, o);
        default: return false;
    }
}

}  // namespace labsdev
