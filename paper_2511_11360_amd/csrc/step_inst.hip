// One instantiation set of the step kernel: lattice pair PFK_PAIR (0: D2Q9 +
// D2Q5, 1: D3Q19 + D3Q7, 2: D3Q27 + D3Q7) and model PFK_MODEL (0: AC, 1: CH, 2:
// nonlocal, 3: Liang2018, 4: Liang2014 with its hydrodynamics), every storage
// form, mode and tile. The build compiles this file
// once per pair and model, in parallel.
#include "step.h"

#define PFK_CAT2(a, b, c, d) a##b##c##d
#define PFK_CAT(a, b, c, d) PFK_CAT2(a, b, c, d)

namespace pfk {

#if PFK_PAIR == 0
using InstPair = Pair2D;
#elif PFK_PAIR == 1
using InstPair = Pair3D;
#else
using InstPair = Pair3D27;
#endif

hipError_t PFK_CAT(launch_step_p, PFK_PAIR, _m, PFK_MODEL)(int precision, int mode, const KArgs& a, hipStream_t s) {
    return step_prec<InstPair, PFK_MODEL>(precision, mode, a, s);
}

int PFK_CAT(occupancy_step_p, PFK_PAIR, _m, PFK_MODEL)(int precision, int tile, int walls) {
    return step_occupancy<InstPair, PFK_MODEL>(precision, tile, walls);
}

}  // namespace pfk
