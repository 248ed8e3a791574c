// Time kernel instantiations for the short transform lengths (N <= 128).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(16)
DDM_TIME_INSTANTIATE(32)
DDM_TIME_INSTANTIATE(64)
DDM_TIME_INSTANTIATE(128)
}  // namespace ddm
