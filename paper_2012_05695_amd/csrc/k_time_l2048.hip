// Time kernel instantiation for transform length 2048.
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(2048)
}  // namespace ddm
