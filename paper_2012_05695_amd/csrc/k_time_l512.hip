// Time kernel instantiation for transform length 512.
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(512)
}  // namespace ddm
