// Time kernel instantiation for transform length 3072 (3 * 2^10).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(3072)
}  // namespace ddm
