// Pass launchers for radii 4..12, image type float, storage type _Float16
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(4, float, _Float16)
RSF_INSTANTIATE(5, float, _Float16)
RSF_INSTANTIATE(6, float, _Float16)
RSF_INSTANTIATE(7, float, _Float16)
RSF_INSTANTIATE(8, float, _Float16)
RSF_INSTANTIATE(9, float, _Float16)
RSF_INSTANTIATE(10, float, _Float16)
RSF_INSTANTIATE(11, float, _Float16)
RSF_INSTANTIATE(12, float, _Float16)
RSF_INSTANTIATE_PAPER(float, _Float16)
}  // namespace rsf
