// Time kernel instantiation for transform length 4096.
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(4096)
}  // namespace ddm
