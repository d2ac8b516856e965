// Sweep kernels for float frame images (four floats per quad texel, FP64
// reference window statistics), default tile (4 rows x 4 waves), FP32
// staging: winner-take-all for every window, soft-argmin for 5, 7 and 9.
#include "sweep_common.h"

namespace psw {
#define PSW_E(W, S, SOFT)                                                                        \
    {W, 4, 4, S, 0, SOFT, 0, (const void *)&sweep_grid_kernel<W, 4, 4, S, 0, SOFT, 1>,        \
     Tile<W, 4, 4, S, 0, SOFT, 1>::lds_bytes(), 1}
#define PSW_S4(W, SOFT) PSW_E(W, 1, SOFT), PSW_E(W, 2, SOFT), PSW_E(W, 3, SOFT), PSW_E(W, 4, SOFT)
static const KernelEntry kF32Img[] = {
    PSW_S4(3, false), PSW_S4(5, false), PSW_S4(7, false), PSW_S4(9, false),
    PSW_S4(11, false), PSW_S4(13, false), PSW_S4(15, false),
    PSW_S4(5, true), PSW_S4(7, true), PSW_S4(9, true),
};
}  // namespace psw

extern "C" int psw_kernels_f32img(const psw::KernelEntry **out) {
    *out = psw::kF32Img;
    return (int)(sizeof(psw::kF32Img) / sizeof(psw::kF32Img[0]));
}
