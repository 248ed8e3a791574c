// Time kernel instantiation for transform length 8192 (N up to 8192: one wave
// vector per workgroup of 512 threads, 140 KB of LDS).
#include "time_kernel.hpp"

namespace ddm {
DDM_TIME_INSTANTIATE(8192)
}  // namespace ddm
