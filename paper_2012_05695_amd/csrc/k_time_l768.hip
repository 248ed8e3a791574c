// Time kernel instantiation for transform length 768 (3 * 2^8).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(768)
}  // namespace ddm
