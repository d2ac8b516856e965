// One persistent launch over every (frame, level, tile) of a run; windows 7
// and 9 (the low level and the crop level of the two-level sweep).
#include "sweep_common.h"

namespace psw {
template <int R, int NW, int S, int ST>
constexpr size_t persistent_lds() {
    return Tile<7, R, NW, S, ST, false>::lds_bytes() > Tile<9, R, NW, S, ST, false>::lds_bytes()
               ? Tile<7, R, NW, S, ST, false>::lds_bytes()
               : Tile<9, R, NW, S, ST, false>::lds_bytes();
}
#define PSW_P(R, NW, S, ST) {0, R, NW, S, ST, 0, 1, (const void *)&sweep_persistent_kernel<R, NW, S, ST>, persistent_lds<R, NW, S, ST>()}
#define PSW_P4(R, NW, ST) PSW_P(R, NW, 1, ST), PSW_P(R, NW, 2, ST), PSW_P(R, NW, 3, ST), PSW_P(R, NW, 4, ST)
static const KernelEntry kPersistent[] = {
    PSW_P4(4, 4, 0), PSW_P4(4, 4, 1), PSW_P4(4, 4, 2), PSW_P4(8, 4, 0), PSW_P(8, 4, 4, 1),
    // 8-wave tiles (fewer warped halo rows per output row); two workgroups
    // fill a CU, except four sources in FP32 (80 KB of LDS), left out
    PSW_P(4, 8, 3, 0), PSW_P(4, 8, 3, 1), PSW_P(4, 8, 3, 2), PSW_P(4, 8, 4, 1), PSW_P(4, 8, 4, 2),
};
}  // namespace psw

extern "C" int psw_kernels_persistent(const psw::KernelEntry **out) {
    *out = psw::kPersistent;
    return (int)(sizeof(psw::kPersistent) / sizeof(psw::kPersistent[0]));
}
