// Alternative tile shapes for the 7x7 and 9x9 windows with 3 or 4 sources
// (for the autotuner): 4 x 8 and 2 x 8 (more waves per workgroup), 16 x 4 and
// 8 x 2, and FP16 staging with 4 x 8 and 8 x 4.
#include "sweep_common.h"

namespace psw {
#define PSW_E(W, R, NW, S, ST) \
    {W, R, NW, S, ST, false, 0, (const void *)&sweep_grid_kernel<W, R, NW, S, ST, false>, \
     Tile<W, R, NW, S, ST, false>::lds_bytes()}
#define PSW_WS(R, NW, ST) \
    PSW_E(7, R, NW, 3, ST), PSW_E(7, R, NW, 4, ST), PSW_E(9, R, NW, 3, ST), PSW_E(9, R, NW, 4, ST)
static const KernelEntry kSmall[] = {
    PSW_WS(4, 8, 0), PSW_WS(2, 8, 0), PSW_WS(16, 4, 0), PSW_WS(8, 2, 0), PSW_WS(4, 8, 1), PSW_WS(8, 4, 1),
};
}  // namespace psw

extern "C" int psw_kernels_small(const psw::KernelEntry **out) {
    *out = psw::kSmall;
    return (int)(sizeof(psw::kSmall) / sizeof(psw::kSmall[0]));
}
