// Instantiation of the pass templates for Gaussian radii 1..6
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(1)
RSF_INSTANTIATE(2)
RSF_INSTANTIATE(3)
RSF_INSTANTIATE(4)
RSF_INSTANTIATE(5)
RSF_INSTANTIATE(6)
}  // namespace rsf
