// Instantiations of the first-step walker for NW in {5, 6, 7}.
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

template <int NW, int R>
void fill_rb(int RB, WalkKernels* o) {
    constexpr int H = (R + 1) / 2;
    if (RB < R) fill<NW, R, H>(o); else fill<NW, R, R>(o);
}

// Slot groups R (64 free positions each) in {ceil(NW/2) - 1, ceil(NW/2),
// ceil(NW/2) + 1}: with k in (32(NW-1), 32NW] and the prefixes in use these hold
// R = ceil((k+1-p)/64) exactly, so no group of 64 slots is scanned for nothing;
// a smaller R (a long prefix) runs in the smallest group count.  RB in {R, ceil(R/2)}.
template <int NW>
bool pick(int R, int RB, WalkKernels* o) {
    constexpr int R0 = (NW + 1) / 2;
    constexpr int Rm = R0 > 1 ? R0 - 1 : 1;
    if (R <= Rm) {
        fill_rb<NW, Rm>(RB, o);
        return true;
    }
    if (R == R0) {
        fill_rb<NW, R0>(RB, o);
        return true;
    }
    if (R == R0 + 1) {
        fill_rb<NW, R0 + 1>(RB, o);
        return true;
    }
    return false;
}
}  // namespace

bool walk_kernels_b(int NW, int R, int RB, WalkKernels* o) {
    switch (NW) {
        case 5: return pick<5>(R, RB, o);
        case 6: return pick<6>(R, RB, o);
        case 7: return pick<7>(R, RB, o);
        default: return false;
    }
}

}  // namespace labsdev
