// Time kernel instantiation for transform length 384 (3 * 2^7).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(384)
}  // namespace ddm
