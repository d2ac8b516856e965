// Plain per-level sweep launches, FP32 staging, default tile (4 rows x 4 waves).
#include "sweep_common.h"

namespace psw {
#define PSW_E(W, R, NW, S, ST, SOFT) \
    {W, R, NW, S, ST, SOFT, 0, (const void *)&sweep_grid_kernel<W, R, NW, S, ST, SOFT>, \
     Tile<W, R, NW, S, ST, SOFT>::lds_bytes()}
#define PSW_S4(W, R, NW, ST, SOFT) \
    PSW_E(W, R, NW, 1, ST, SOFT), PSW_E(W, R, NW, 2, ST, SOFT), PSW_E(W, R, NW, 3, ST, SOFT), PSW_E(W, R, NW, 4, ST, SOFT)
static const KernelEntry kGrid[] = {
    PSW_S4(3, 4, 4, 0, false),  PSW_S4(5, 4, 4, 0, false),  PSW_S4(7, 4, 4, 0, false), PSW_S4(9, 4, 4, 0, false),
    PSW_S4(11, 4, 4, 0, false), PSW_S4(13, 4, 4, 0, false), PSW_S4(15, 4, 4, 0, false),
};
}  // namespace psw

extern "C" int psw_kernels_grid(const psw::KernelEntry **out) {
    *out = psw::kGrid;
    return (int)(sizeof(psw::kGrid) / sizeof(psw::kGrid[0]));
}
