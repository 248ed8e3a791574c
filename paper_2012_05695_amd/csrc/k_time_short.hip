// Time kernel instantiations for the short transform lengths (N <= 192).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(16)
DDM_TIME_INSTANTIATE(32)
DDM_TIME_INSTANTIATE(64)
DDM_TIME_INSTANTIATE(128)
DDM_TIME_INSTANTIATE(192)
}  // namespace ddm
