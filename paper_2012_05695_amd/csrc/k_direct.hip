// Step two by direct differences: D(q, m) = mean over n < N - m of
// |F_{n+m}(q) - F_n(q)|^2, Eq. (1) evaluated term by term on the stored image
// spectra.  This is the scheme the paper compares its Fourier method against
// (section "The algorithm": the difference of two image spectra is the spectrum
// of the difference image, so the direct scheme needs no image transforms per
// pair), at O(N M) work per wave vector instead of O(N log N): cheaper than the
// time transform when few lags are wanted, and the crossover reference when all
// are.
//
// Layout: one thread per (slot, tile of LG consecutive lags).  A workgroup is
// 64 slots (one per lane; four blocks of the blocked store, so every load is
// four 128-byte rows) x up to 4 consecutive lag tiles (one per wave; fewer
// where that leaves no wave idle): the waves read the same
// slots' time series, which the L1 and the XCD's L2 serve after the first.
// Each step of S time points holds the S base values F_n and a window of
// S + LG - 1 values F_{n+m} in registers: S x LG pairs for 2S loads.  Sums run in FP32 over
// 64 time points, then add into FP64 totals (the paper's definition sums N - m
// positive terms; the FP64 totals keep the error independent of N).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "internal.hpp"

namespace ddm {
namespace {

constexpr int kDirSlots = 64;   // slots per workgroup (lanes)
constexpr int kDirWaves = 4;    // most lag tiles (waves) per workgroup
constexpr int kDirChunk = 64;   // time points per FP32 partial sum

template <bool F16>
__device__ __forceinline__ float2 dir_val(const void* p, float sc) {
  if constexpr (F16) {
    const __half2 h = __builtin_bit_cast(__half2, *reinterpret_cast<const uint32_t*>(p));
    return make_float2(__low2float(h) * sc, __high2float(h) * sc);
  } else {
    return *reinterpret_cast<const float2*>(p);
  }
}

// QB: 1 for the plain store [s][N], 16 for the blocked store [s / 16][N][16].
// qmap[s]: the row of D of slot s (-1: none; null: slot s is row s).  F16: the
// blocked FP16 store scaled by 2^qexp[row], unscaled on load (exact).
template <int QB, bool F16, int S, int LG>
__global__ void __launch_bounds__(kDirSlots * kDirWaves) k_direct(const void* __restrict__ spec, int64_t nslots,
                                                                  int N, int M, int ntiles, int64_t nwork,
                                                                  int64_t per_xcd, const int32_t* __restrict__ qmap,
                                                                  const int32_t* __restrict__ qexp,
                                                                  float* __restrict__ D) {
  // consecutive work items on one XCD (workgroups are dealt to the 8 XCDs in
  // turn), so that the lag tiles of one group of slots share that XCD's L2
  const int64_t w = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (w >= nwork) return;
  const int waves = (int)(blockDim.x / kDirSlots);
  const int tgroups = (ntiles + waves - 1) / waves;
  const int64_t sg = w / tgroups;
  const int tile = (int)(w % tgroups) * waves + (int)(threadIdx.x / kDirSlots);
  const int64_t s = sg * kDirSlots + (threadIdx.x % kDirSlots);
  if (tile >= ntiles || s >= nslots) return;  // no barriers below: a lane may leave
  const int row = qmap ? qmap[s] : (int)s;
  if (row < 0) return;
  const float sc = F16 ? ldexpf(1.0f, -qexp[row]) : 1.0f;
  const int64_t base = (QB == 1) ? s * (int64_t)N : (s / QB) * (int64_t)N * QB + (s % QB);
  using Elem = typename std::conditional<F16, uint32_t, float2>::type;
  const Elem* ser = reinterpret_cast<const Elem*>(spec) + base;  // F_t of this slot is ser[t QB]
  const int mb = tile * LG;  // this thread's lags mb .. mb + LG - 1 (those below M)
  const int nend = N - mb;  // pairs exist for n < N - m <= nend
  auto ld = [&](int t) { return dir_val<F16>(ser + (int64_t)(t < N ? t : N - 1) * QB, sc); };

  static_assert(kDirChunk % S == 0, "steps divide the FP32 partial sums");
  double tot[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) tot[j] = 0.0;
  // v[i] = F_{n + mb + i} (i < LG + S - 1) for the step starting at n; the
  // next step's window is this one shifted by S plus S new values
  float2 v[LG + S];
#pragma unroll
  for (int i = 0; i < LG; ++i) v[S + i] = ld(mb + i);
  for (int n0 = 0; n0 < nend; n0 += kDirChunk) {
    float acc[LG];
#pragma unroll
    for (int j = 0; j < LG; ++j) acc[j] = 0.0f;
    const int n1 = (n0 + kDirChunk < nend) ? n0 + kDirChunk : nend;
    for (int n = n0; n < n1; n += S) {
      float2 b[S];
#pragma unroll
      for (int i = 0; i < LG; ++i) v[i] = v[i + S];
      if (n + mb + LG + S - 1 < N) {
        // every load in range and every pair of the step exists: two row
        // pointers with constant offsets
        const Elem* pb = ser + (int64_t)n * QB;
        const Elem* pw = ser + (int64_t)(n + mb + LG) * QB;
#pragma unroll
        for (int i = 0; i < S; ++i) {
          v[LG + i] = dir_val<F16>(pw + i * QB, sc);
          b[i] = dir_val<F16>(pb + i * QB, sc);
        }
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
          for (int j = 0; j < LG; ++j) {
            const float dx = v[i + j].x - b[i].x, dy = v[i + j].y - b[i].y;
            acc[j] = fmaf(dx, dx, fmaf(dy, dy, acc[j]));
          }
      } else {
        // the last steps: loads clamped to F_{N-1}; pair (n + i, mb + j)
        // exists while n + i + mb + j < N
#pragma unroll
        for (int i = 0; i < S; ++i) {
          v[LG + i] = ld(n + mb + LG + i);
          b[i] = ld(n + i);
        }
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
          for (int j = 0; j < LG; ++j) {
            const float dx = v[i + j].x - b[i].x, dy = v[i + j].y - b[i].y;
            const float t = fmaf(dx, dx, fmaf(dy, dy, acc[j]));
            acc[j] = (n + i + mb + j < N) ? t : acc[j];
          }
      }
    }
#pragma unroll
    for (int j = 0; j < LG; ++j) tot[j] += (double)acc[j];
  }
  float* out = D + (int64_t)row * M;
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const int m = mb + j;
    if (m < M) out[m] = (m == 0) ? 0.0f : (float)(tot[j] / (double)(N - m));
  }
}

template <int QB, bool F16, int LG>
hipError_t direct_go(hipStream_t s, const void* spec, int64_t nslots, int N, int M, const int32_t* qmap,
                     const int32_t* qexp, float* D) {
  constexpr int S = 8;
  const int ntiles = (M + LG - 1) / LG;
  // waves per workgroup: all tiles when there are at most 4, else 4, 3 or 2
  // where that divides the tiles (no idle waves in the last tile group)
  int waves = ntiles < kDirWaves ? ntiles : kDirWaves;
  if (ntiles > kDirWaves && ntiles % 4 != 0) waves = ntiles % 3 == 0 ? 3 : ntiles % 2 == 0 ? 2 : 4;
  const int64_t tgroups = (ntiles + waves - 1) / waves;
  const int64_t nwork = (nslots + kDirSlots - 1) / kDirSlots * tgroups;  // (slot group, tile group) items
  const int64_t per_xcd = (nwork + 7) / 8;
  const int64_t grid = per_xcd * 8;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_direct<QB, F16, S, LG>), dim3((unsigned)grid), dim3(kDirSlots * waves), 0, s, spec, nslots,
                     N, M, ntiles, nwork, per_xcd, qmap, qexp, D);
  return hipGetLastError();
}

}  // namespace

// Lags per lane: 16 (twice the pairs per load, and one wave streams a slot
// group once when M <= 16; measured 1.2-1.4x faster from 16 lags up at
// 512 x 512 x 1024), 8 for M <= 8 (more waves when there are few lags).
// Results are the same bits either way: each lag's pairs are summed in time
// order whichever lane holds it.  DDM_DIRECT_LAGS=8|16 (environment)
// overrides, for tuning.
static int direct_lags(int M) {
  static const int env = [] {
    const char* v = std::getenv("DDM_DIRECT_LAGS");
    const int x = v ? std::atoi(v) : 0;
    return (x == 8 || x == 16) ? x : 0;
  }();
  return env ? env : (M <= 8 ? 8 : 16);
}

template <int LG>
static hipError_t direct_lg(hipStream_t s, const void* spec, int qb, int64_t nslots, int N, int M,
                            const int32_t* qmap, const int32_t* qexp, float* D) {
  if (qb == 1) {
    if (qexp != nullptr) return hipErrorInvalidValue;
    return direct_go<1, false, LG>(s, spec, nslots, N, M, qmap, nullptr, D);
  }
  if (qb != 16) return hipErrorInvalidValue;
  if (qexp != nullptr) return direct_go<16, true, LG>(s, spec, nslots, N, M, qmap, qexp, D);
  return direct_go<16, false, LG>(s, spec, nslots, N, M, qmap, nullptr, D);
}

hipError_t launch_direct(hipStream_t s, const void* spec, int qb, int64_t nslots, int N, int M, const int32_t* qmap,
                         const int32_t* qexp, float* D) {
  if (nslots <= 0) return hipSuccess;
  if (N < 2 || M < 1 || M > N) return hipErrorInvalidValue;
  if (direct_lags(M) == 16) return direct_lg<16>(s, spec, qb, nslots, N, M, qmap, qexp, D);
  return direct_lg<8>(s, spec, qb, nslots, N, M, qmap, qexp, D);
}

}  // namespace ddm
