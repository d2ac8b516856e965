// Per-level sweep launches, FP32 staging, 8 rows x 4 waves per tile: fewer
// warped halo rows per output row than the default tile, at the price of
// twice the per-row registers (for the autotuner).
#include "sweep_common.h"

namespace psw {
#define PSW_E(W, R, NW, S, ST, SOFT) \
    {W, R, NW, S, ST, SOFT, 0, (const void *)&sweep_grid_kernel<W, R, NW, S, ST, SOFT>, \
     Tile<W, R, NW, S, ST, SOFT>::lds_bytes()}
#define PSW_S4(W, R, NW, ST, SOFT) \
    PSW_E(W, R, NW, 1, ST, SOFT), PSW_E(W, R, NW, 2, ST, SOFT), PSW_E(W, R, NW, 3, ST, SOFT), PSW_E(W, R, NW, 4, ST, SOFT)
static const KernelEntry kGrid8[] = {
    PSW_S4(3, 8, 4, 0, false),  PSW_S4(5, 8, 4, 0, false),  PSW_S4(7, 8, 4, 0, false), PSW_S4(9, 8, 4, 0, false),
    PSW_S4(11, 8, 4, 0, false), PSW_S4(13, 8, 4, 0, false), PSW_S4(15, 8, 4, 0, false),
};
}  // namespace psw

extern "C" int psw_kernels_grid8(const psw::KernelEntry **out) {
    *out = psw::kGrid8;
    return (int)(sizeof(psw::kGrid8) / sizeof(psw::kGrid8[0]));
}
