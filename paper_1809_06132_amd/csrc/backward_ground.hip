// Soft-argmin backward pass, the forms for levels with ground planes (their
// own translation unit: they compile beside the fronto-only forms).
#include <hip/hip_runtime.h>

#include "backward_impl.h"

extern "C" const void *psw_backward_ground_kernel(int win, int n_src, int img, int image_grads) {
#define PSW_B(W, I, G)                                                                      \
    if (win == W && img == I && (image_grads != 0) == G) {                                  \
        if (n_src == 1) return (const void *)&psw::backward_kernel<W, 1, I, G, true>;      \
        if (n_src == 2) return (const void *)&psw::backward_kernel<W, 2, I, G, true>;      \
        if (n_src == 3) return (const void *)&psw::backward_kernel<W, 3, I, G, true>;      \
        if (n_src == 4) return (const void *)&psw::backward_kernel<W, 4, I, G, true>;      \
    }
    PSW_B(5, 0, true) PSW_B(7, 0, true) PSW_B(9, 0, true) PSW_B(5, 1, true) PSW_B(7, 1, true) PSW_B(9, 1, true)
    PSW_B(5, 0, false) PSW_B(7, 0, false) PSW_B(9, 0, false) PSW_B(5, 1, false) PSW_B(7, 1, false)
    PSW_B(9, 1, false)
#undef PSW_B
    return nullptr;
}
