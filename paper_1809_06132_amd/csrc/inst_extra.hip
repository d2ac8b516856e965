// Half-precision staging and the soft-argmin sweep, default tile (4 x 4).
#include "sweep_common.h"

namespace psw {
#define PSW_E(W, R, NW, S, ST, SOFT) \
    {W, R, NW, S, ST, SOFT, 0, (const void *)&sweep_grid_kernel<W, R, NW, S, ST, SOFT>, \
     Tile<W, R, NW, S, ST, SOFT>::lds_bytes()}
#define PSW_S4(W, R, NW, ST, SOFT) \
    PSW_E(W, R, NW, 1, ST, SOFT), PSW_E(W, R, NW, 2, ST, SOFT), PSW_E(W, R, NW, 3, ST, SOFT), PSW_E(W, R, NW, 4, ST, SOFT)
static const KernelEntry kExtra[] = {
    // FP16 / BF16 staging
    PSW_S4(7, 4, 4, 1, false), PSW_S4(9, 4, 4, 1, false), PSW_S4(7, 4, 4, 2, false), PSW_S4(9, 4, 4, 2, false),
    // soft-argmin
    PSW_S4(5, 4, 4, 0, true), PSW_S4(7, 4, 4, 0, true), PSW_S4(9, 4, 4, 0, true),
};
}  // namespace psw

extern "C" int psw_kernels_extra(const psw::KernelEntry **out) {
    *out = psw::kExtra;
    return (int)(sizeof(psw::kExtra) / sizeof(psw::kExtra[0]));
}
