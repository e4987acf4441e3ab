// Pass launchers for radii 1..6, image type float, storage type float
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(1, float, float)
RSF_INSTANTIATE(2, float, float)
RSF_INSTANTIATE(3, float, float)
RSF_INSTANTIATE(4, float, float)
RSF_INSTANTIATE(5, float, float)
RSF_INSTANTIATE(6, float, float)
RSF_INSTANTIATE_PAPER(float, float)
}  // namespace rsf
