// Time kernel instantiation for transform length 256.
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(256)
}  // namespace ddm
