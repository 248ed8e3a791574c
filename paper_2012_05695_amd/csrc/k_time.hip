// Step two launcher: picks the time-transform length L for N and hands the
// launch to that length's instantiation (time_kernel.hpp, one translation unit
// per length).
#include "internal.hpp"

namespace ddm {

template <int L>
hipError_t time_run(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M, const float2* twN2,
                    const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D, TimeShape shape);
hipError_t time_run_long(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M, const float2* twN2,
                         const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D);

int time_length(int N, int minimal) {
  int L = 16;
  while (L < N) L <<= 1;
  if (!minimal) return L;
  // 3 * 2^k (192 to 6144) where it lies in [N, L): the padded length 2 L' >= 2 N - 1 keeps the
  // result exact (Eq. (B4) with any padding of at least N - 1 zeros)
  const int L3 = 3 * (L / 4);
  if (L3 >= N && L3 >= 192 && L3 <= 6144) return L3;
  return L;
}

hipError_t launch_time(hipStream_t s, int L, const void* spec, int qb, int64_t nq, int N, int M,
                       const float2* twN2, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D,
                       TimeShape shape) {
  if (L < N) return hipErrorInvalidValue;
  switch (L) {
#define TIME_CASE(n) case n: return time_run<n>(s, spec, qb, nq, N, M, twN2, ramp, qmap, qexp, D, shape);
    TIME_CASE(16) TIME_CASE(32) TIME_CASE(64) TIME_CASE(128) TIME_CASE(256) TIME_CASE(512) TIME_CASE(1024)
    TIME_CASE(2048) TIME_CASE(4096) TIME_CASE(8192)
    TIME_CASE(192) TIME_CASE(384) TIME_CASE(768) TIME_CASE(1536) TIME_CASE(3072) TIME_CASE(6144)
#undef TIME_CASE
    case 16384: return time_run_long(s, spec, qb, nq, N, M, twN2, ramp, qmap, qexp, D);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddm
