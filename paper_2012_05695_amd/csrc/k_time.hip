// Step two launcher: picks the time-transform length L for N and hands the
// launch to that length's instantiation (time_kernel.hpp, one translation unit
// per length).
#include "internal.hpp"

namespace ddm {

template <int L>
hipError_t time_run(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M, const float2* twN2,
                    const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D, TimeShape shape);

hipError_t launch_time(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M,
                       const float2* twN2, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D,
                       TimeShape shape) {
  int L = 16;
  while (L < N) L <<= 1;
  switch (L) {
#define TIME_CASE(n) case n: return time_run<n>(s, spec, qb, nq, N, M, twN2, ramp, qmap, qexp, D, shape);
    TIME_CASE(16) TIME_CASE(32) TIME_CASE(64) TIME_CASE(128) TIME_CASE(256) TIME_CASE(512) TIME_CASE(1024)
    TIME_CASE(2048) TIME_CASE(4096)
#undef TIME_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddm
