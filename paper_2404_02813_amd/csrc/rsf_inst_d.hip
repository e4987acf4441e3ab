// Instantiation of the pass templates for Gaussian radii 13..16
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(13)
RSF_INSTANTIATE(14)
RSF_INSTANTIATE(15)
RSF_INSTANTIATE(16)
}  // namespace rsf
