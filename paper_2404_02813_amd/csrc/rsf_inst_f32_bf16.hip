// Pass launchers for radii 4..12, image type float, storage type __bf16
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(4, float, __bf16)
RSF_INSTANTIATE(5, float, __bf16)
RSF_INSTANTIATE(6, float, __bf16)
RSF_INSTANTIATE(7, float, __bf16)
RSF_INSTANTIATE(8, float, __bf16)
RSF_INSTANTIATE(9, float, __bf16)
RSF_INSTANTIATE(10, float, __bf16)
RSF_INSTANTIATE(11, float, __bf16)
RSF_INSTANTIATE(12, float, __bf16)
RSF_INSTANTIATE_PAPER(float, __bf16)
}  // namespace rsf
