// Pass launchers for radii 7..9, image type float, storage type float
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(7, float, float)
RSF_INSTANTIATE(8, float, float)
RSF_INSTANTIATE(9, float, float)
}  // namespace rsf
