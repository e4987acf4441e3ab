// Pass launchers for radii 4..12, image type uint16_t, storage type float
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(4, uint16_t, float)
RSF_INSTANTIATE(5, uint16_t, float)
RSF_INSTANTIATE(6, uint16_t, float)
RSF_INSTANTIATE(7, uint16_t, float)
RSF_INSTANTIATE(8, uint16_t, float)
RSF_INSTANTIATE(9, uint16_t, float)
RSF_INSTANTIATE(10, uint16_t, float)
RSF_INSTANTIATE(11, uint16_t, float)
RSF_INSTANTIATE(12, uint16_t, float)
RSF_INSTANTIATE_PAPER(uint16_t, float)
}  // namespace rsf
