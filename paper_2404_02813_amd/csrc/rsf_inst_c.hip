// Instantiation of the pass templates for Gaussian radii 10..12
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(10)
RSF_INSTANTIATE(11)
RSF_INSTANTIATE(12)
}  // namespace rsf
