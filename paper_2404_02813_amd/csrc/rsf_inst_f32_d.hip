// Pass launchers for radii 13..16, image type float, storage type float
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(13, float, float)
RSF_INSTANTIATE(14, float, float)
RSF_INSTANTIATE(15, float, float)
RSF_INSTANTIATE(16, float, float)
}  // namespace rsf
