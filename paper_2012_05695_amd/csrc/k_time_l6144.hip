// Time kernel instantiation for transform length 6144 (3 * 2^11).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(6144)
}  // namespace ddm
