// Pass launchers for radii 10..12, image type float, storage type float
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(10, float, float)
RSF_INSTANTIATE(11, float, float)
RSF_INSTANTIATE(12, float, float)
}  // namespace rsf
