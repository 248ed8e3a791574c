// Time kernel instantiation for transform length 1536 (3 * 2^9).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(1536)
}  // namespace ddm
