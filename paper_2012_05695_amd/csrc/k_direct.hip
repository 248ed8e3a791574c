// Step two by direct differences: D(q, m) = mean over n < N - m of
// |F_{n+m}(q) - F_n(q)|^2, Eq. (1) evaluated term by term on the stored image
// spectra.  This is the scheme the paper compares its Fourier method against
// (section "The algorithm": the difference of two image spectra is the spectrum
// of the difference image, so the direct scheme needs no image transforms per
// pair), at O(N M) work per wave vector instead of O(N log N): cheaper than the
// time transform when few lags are wanted, and the crossover reference when all
// are.
//
// Layout: one thread per (slot, tile of LG consecutive lags).  A work item is
// 64 slots (one per lane; four blocks of the blocked store, so every load is
// four 128-byte rows) x one lag tile; the items of one slot group run on one
// XCD in a row, so its lag tiles read the slots' time series from that XCD's L2
// after the first.  An item is one wave, or, where slot groups and lags give
// too few waves to fill the chip (few lags, or few wave vectors with long
// series), 2 or 4 waves that split the base points into ranges of whole
// 64-point chunks.  Each step of S time points holds a window of S + LG - 1
// values F_{n+m} and the S base values F_n in registers (lag tile 0 takes its
// base values from its window): S x LG pairs for at most 2S loads, issued one
// step ahead.  Sums run in FP32 over 64 time points, then add into FP64 totals
// (the paper's definition sums N - m positive terms; the FP64 totals keep the
// error independent of N).
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <type_traits>

#include "internal.hpp"

namespace ddm {
namespace {

constexpr int kDirSlots = 64;   // slots per work item (the lanes of a wave)
constexpr int kDirMaxParts = 4; // most time ranges (waves) per workgroup
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

// One lane's sums for lags mb .. mb + LG - 1 of one slot over base points
// [n_lo, n_hi) (n_lo a multiple of 64), added into tot[LG].  ser[t QB] is F_t.
// OWN: the lane holds lag tile 0 (mb = 0), whose base values F_n .. F_{n+S-1}
// are the first S values of its window, so it loads only the window.  Pair
// (n, m) adds to the FP32 sum of base points [64 c, 64 c + 64) that holds n,
// and those sums add into the FP64 totals in order of c.  (tot is taken by
// pointer: as an array reference it cost 30 more VGPRs.)
template <bool F16, int QB, int S, int LG, bool OWN, typename Elem>
__device__ __forceinline__ void direct_sums(const Elem* __restrict__ ser, float sc, int N, int mb, int n_lo,
                                            int n_hi, double* tot) {
  float acc[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) acc[j] = 0.0f;
  auto flush = [&]() {
#pragma unroll
    for (int j = 0; j < LG; ++j) {
      tot[j] += (double)acc[j];
      acc[j] = 0.0f;
    }
  };
  // v[i] = F_{n + mb + i} (i < LG + S - 1) for the step at n; the next step's
  // window is this one shifted by S plus S new values
  float2 v[LG + S];
  float2 b[S];
  auto pairs = [&](auto masked, int n) {
#pragma unroll
    for (int i = 0; i < S; ++i)
#pragma unroll
      for (int j = 0; j < LG; ++j) {
        const float2 bi = OWN ? v[i] : b[i];
        const float dx = v[i + j].x - bi.x, dy = v[i + j].y - bi.y;
        const float t = fmaf(dx, dx, fmaf(dy, dy, acc[j]));
        if constexpr (decltype(masked)::value)
          acc[j] = (n + i + mb + j < N) ? t : acc[j];  // pair (n + i, mb + j) exists
        else
          acc[j] = t;
      }
  };
  auto ld = [&](int t) { return dir_val<F16>(ser + (int64_t)(t < N ? t : N - 1) * QB, sc); };
#pragma unroll
  for (int i = 0; i < LG; ++i) v[S + i] = ld(n_lo + mb + i);
  int n = n_lo;
  // Main steps: this step's loads and the next one's are in range and every
  // pair exists.  nw / nb hold the step's new window values F_{n+mb+LG+i} and
  // base values F_{n+i}, loaded one step ahead so that they are in flight
  // while the previous step's pairs are summed.
  if (n_lo + mb + LG + 2 * S - 1 < N && n_lo < n_hi) {
    float2 nw[S], nb[S];
    auto fetch = [&](int t) {
      const Elem* pw = ser + (int64_t)(t + mb + LG) * QB;
#pragma unroll
      for (int i = 0; i < S; ++i) nw[i] = dir_val<F16>(pw + i * QB, sc);
      if constexpr (!OWN) {
        const Elem* pb = ser + (int64_t)t * QB;
#pragma unroll
        for (int i = 0; i < S; ++i) nb[i] = dir_val<F16>(pb + i * QB, sc);
      }
    };
    fetch(n);
    for (; n + mb + LG + 2 * S - 1 < N && n < n_hi; n += S) {
#pragma unroll
      for (int i = 0; i < LG; ++i) v[i] = v[i + S];
#pragma unroll
      for (int i = 0; i < S; ++i) {
        v[LG + i] = nw[i];
        if constexpr (!OWN) b[i] = nb[i];
      }
      fetch(n + S);
      pairs(std::false_type{}, n);
      if (((n + S) % kDirChunk) == 0) flush();
    }
  }
  // The last steps: loads clamped to F_{N-1}, pairs masked.
  for (; n < n_hi; n += S) {
#pragma unroll
    for (int i = 0; i < LG; ++i) v[i] = v[i + S];
#pragma unroll
    for (int i = 0; i < S; ++i) {
      v[LG + i] = ld(n + mb + LG + i);
      if constexpr (!OWN) b[i] = ld(n + i);
    }
    pairs(std::true_type{}, n);
    if (((n + S) % kDirChunk) == 0 || n + S >= n_hi) flush();
  }
}

// QB: 1 for the plain store [s][N], 16 for the blocked store [s / 16][N][16].
// qmap[s]: the row of D of slot s (-1: none; null: slot s is row s).  F16: the
// blocked FP16 store scaled by 2^qexp[row], unscaled on load (exact).
// A workgroup is one (slot group, lag tile) item; its `parts` waves each sum
// one range of 64-point chunks of the base points (chunks
// [p C / parts, (p + 1) C / parts) of C = ceil(N / 64)), and the ranges' FP64
// totals are added in order of p through LDS.
template <int QB, bool F16, int S, int LG>
__global__ void __launch_bounds__(kDirSlots * kDirMaxParts) k_direct(const void* __restrict__ spec, int64_t nslots,
                                                                     int N, int M, int ntiles, int parts,
                                                                     int64_t nwork, int64_t per_xcd,
                                                                     const int32_t* __restrict__ qmap,
                                                                     const int32_t* __restrict__ qexp,
                                                                     float* __restrict__ D) {
  // consecutive work items on one XCD (workgroups are dealt to the 8 XCDs in
  // turn), so that the lag tiles of one group of slots share that XCD's L2
  const int64_t w = (int64_t)(blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (w >= nwork) return;  // the whole workgroup
  const int64_t sg = w / ntiles;
  const int tile = (int)(w % ntiles);
  // the time range is the wave's (made explicit, so that loop bounds and the
  // choice of the step's path are scalar)
  const int part = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kDirSlots));
  const int64_t s = sg * kDirSlots + (threadIdx.x % kDirSlots);
  // lanes without a wave vector (past the last slot, or a hole of the store)
  // sum the last slot's, or their own, series like the others and write nothing:
  // every lane takes the same path, and every load stays inside the store
  const int64_t sl = s < nslots ? s : nslots - 1;
  const int row = s < nslots ? (qmap ? qmap[s] : (int)s) : -1;
  const int mb = tile * LG;  // this thread's lags mb .. mb + LG - 1 (those below M)
  static_assert(kDirChunk % S == 0, "steps divide the FP32 partial sums");
  double tot[LG];
#pragma unroll
  for (int j = 0; j < LG; ++j) tot[j] = 0.0;
  {
    const float sc = (F16 && row >= 0) ? ldexpf(1.0f, -qexp[row]) : 1.0f;
    const int64_t base = (QB == 1) ? sl * (int64_t)N : (sl / QB) * (int64_t)N * QB + (sl % QB);
    using Elem = typename std::conditional<F16, uint32_t, float2>::type;
    const Elem* ser = reinterpret_cast<const Elem*>(spec) + base;  // F_t of this slot is ser[t QB]
    const int nend = N - mb;  // pairs exist for n < N - m <= nend
    const int chunks = (N + kDirChunk - 1) / kDirChunk;
    const int n_lo = (int)((int64_t)part * chunks / parts) * kDirChunk;
    int n_hi = (int)((int64_t)(part + 1) * chunks / parts) * kDirChunk;
    n_hi = n_hi < nend ? n_hi : nend;
    if (mb == 0)
      direct_sums<F16, QB, S, LG, true>(ser, sc, N, mb, n_lo, n_hi, tot);
    else
      direct_sums<F16, QB, S, LG, false>(ser, sc, N, mb, n_lo, n_hi, tot);
  }
  if (parts > 1) {
    // ranges 1 .. parts - 1 hand their totals to range 0: red[p - 1][j][lane]
    extern __shared__ double red[];
    const int lane = threadIdx.x % kDirSlots;
    if (part > 0) {
#pragma unroll
      for (int j = 0; j < LG; ++j) red[((part - 1) * LG + j) * kDirSlots + lane] = tot[j];
    }
    __syncthreads();
    if (part > 0) return;
    for (int p = 1; p < parts; ++p)
#pragma unroll
      for (int j = 0; j < LG; ++j) tot[j] += red[((p - 1) * LG + j) * kDirSlots + lane];
  }
  if (row < 0) return;
  float* out = D + (int64_t)row * M;
#pragma unroll
  for (int j = 0; j < LG; ++j) {
    const int m = mb + j;
    if (m < M) out[m] = (m == 0) ? 0.0f : (float)(tot[j] / (double)(N - m));
  }
}

template <int QB, bool F16, int LG>
hipError_t direct_go(hipStream_t s, const void* spec, int64_t nslots, int N, int M, int parts, const int32_t* qmap,
                     const int32_t* qexp, float* D) {
  constexpr int S = 8;
  const int ntiles = (M + LG - 1) / LG;
  // (slot group, lag tile) items, one workgroup of `parts` waves each (one
  // wave per item measured as fast as, or up to 1.3x faster than, items of up
  // to 4 lag tiles sharing a workgroup, 64-1024 lags at 512 x 512 x 1024)
  const int64_t nwork = (nslots + kDirSlots - 1) / kDirSlots * ntiles;
  const size_t lds = (size_t)(parts - 1) * LG * kDirSlots * sizeof(double);
  const int64_t per_xcd = (nwork + 7) / 8;
  const int64_t grid = per_xcd * 8;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_direct<QB, F16, S, LG>), dim3((unsigned)grid), dim3(kDirSlots * parts), lds, s, spec,
                     nslots, N, M, ntiles, parts, nwork, per_xcd, qmap, qexp, D);
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

// Time ranges per (slot group, lag tile): the smallest power of two (at most
// 4, and at most the 64-point chunks of the series) for which the work
// (slot groups x 16-lag units x ranges) reaches 8192 waves, about two rounds
// of the chip's resident waves; 1 when the lags alone give that many.  It
// depends on N, M and the slot count only (not on the lags per lane), so the
// sums, and so the bits, are the same at 8 and 16 lags per lane.  (At most 4:
// with 8 the 512-thread bound let the compiler wait for all of a step's loads
// at once, 6% slower with one range; 8 ranges gained 4% on 256 x 256 x 16384.)
// DDM_DIRECT_PARTS=1|2|4 (environment) overrides, for tuning.
static int direct_parts(int64_t nslots, int N, int M) {
  static const int env = [] {
    const char* v = std::getenv("DDM_DIRECT_PARTS");
    const int x = v ? std::atoi(v) : 0;
    return (x == 1 || x == 2 || x == 4) ? x : 0;
  }();
  const int chunks = (N + kDirChunk - 1) / kDirChunk;
  if (env) return env < chunks ? env : 1;
  const int64_t units = (nslots + kDirSlots - 1) / kDirSlots * ((M + 15) / 16);
  int parts = 1;
  while (parts < kDirMaxParts && units * parts < 8192 && parts * 2 <= chunks) parts *= 2;
  return parts;
}

template <int LG>
static hipError_t direct_lg(hipStream_t s, const void* spec, int qb, int64_t nslots, int N, int M,
                            const int32_t* qmap, const int32_t* qexp, float* D) {
  const int parts = direct_parts(nslots, N, M);
  if (qb == 1) {
    if (qexp != nullptr) return hipErrorInvalidValue;
    return direct_go<1, false, LG>(s, spec, nslots, N, M, parts, qmap, nullptr, D);
  }
  if (qb != 16) return hipErrorInvalidValue;
  if (qexp != nullptr) return direct_go<16, true, LG>(s, spec, nslots, N, M, parts, qmap, qexp, D);
  return direct_go<16, false, LG>(s, spec, nslots, N, M, parts, qmap, nullptr, D);
}

hipError_t launch_direct(hipStream_t s, const void* spec, int qb, int64_t nslots, int N, int M, const int32_t* qmap,
                         const int32_t* qexp, float* D) {
  if (nslots <= 0) return hipSuccess;
  if (N < 2 || M < 1 || M > N) return hipErrorInvalidValue;
  if (direct_lags(M) == 16) return direct_lg<16>(s, spec, qb, nslots, N, M, qmap, qexp, D);
  return direct_lg<8>(s, spec, qb, nslots, N, M, qmap, qexp, D);
}

}  // namespace ddm
