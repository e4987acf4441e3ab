// Instantiation of the pass templates for Gaussian radii 7..9
// (split over several files so the build compiles them in parallel).
#include "rsf_kernels.hpp"

namespace rsf {
RSF_INSTANTIATE(7)
RSF_INSTANTIATE(8)
RSF_INSTANTIATE(9)
}  // namespace rsf
