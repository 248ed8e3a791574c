// Time kernel instantiation for transform length 1024.
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(1024)
}  // namespace ddm
