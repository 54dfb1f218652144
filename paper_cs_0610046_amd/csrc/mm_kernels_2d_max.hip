// Fused 2-D kernels with the max output only (a max-only filter, erosion /
// dilation), one translation unit so they compile beside the others.
#include "mm_f2d.hpp"

namespace mm {

template hipError_t f2d_launch<false, 1>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                         void*, void*, int64_t, int64_t, hipStream_t);
template hipError_t f2d_launch<true, 1>(int, const void*, const void*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        void*, void*, int64_t, int64_t, hipStream_t);

}  // namespace mm
