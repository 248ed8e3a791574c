// Azimuthal |q| averaging of D(q, m) (standard DDM reduction; the paper
// computes D per wave vector and leaves binning to the analysis).
//
// Bin b holds the kept wave vectors with T[b] <= k2 < T[b+1], where
// k2 = kx^2 ca + ky_s^2 cc is the exact integer squared magnitude.  For a
// fixed ky row, k2 grows with kx, so the members of bin b in that row form one
// contiguous kx interval [lo, hi); it is found with integer arithmetic only,
// which makes bin membership bit-exact.
//
// One workgroup per (bin, lag tile); each thread owns one lag and sums
// w(q) D(q, m) over the bin's rows in q order in FP64 (fixed order, so the
// result is deterministic and independent of the launch geometry).
#include "internal.hpp"

namespace ddm {

// smallest kx in [0, cnt) with kx^2 * a >= r (a > 0), or cnt if none; exact
// integer result (the floating-point root is only a starting guess).
__device__ __forceinline__ int64_t first_kx(int64_t r, int64_t a, int64_t cnt) {
  if (r <= 0) return 0;
  if ((cnt - 1) * (cnt - 1) * a < r) return cnt;
  int64_t x = (int64_t)ceil(sqrt((double)r / (double)a));
  if (x > cnt - 1) x = cnt - 1;
  while (x > 0 && (x - 1) * (x - 1) * a >= r) --x;
  while (x * x * a < r) ++x;
  return x;
}

__global__ void __launch_bounds__(256) k_radial(const float* __restrict__ D, int M, int W, int H,
                                                int64_t ca, int64_t cc,
                                                const int32_t* __restrict__ qoff,
                                                const int32_t* __restrict__ kxcnt,
                                                const int64_t* __restrict__ thr, double* __restrict__ Dbar,
                                                int64_t* __restrict__ counts,
                                                int32_t* __restrict__ bin_of_q) {
  const int b = blockIdx.x;
  const int m = blockIdx.y * blockDim.x + threadIdx.x;
  const int64_t lo_t = thr[b], hi_t = thr[b + 1];
  double acc = 0.0;
  int64_t wsum = 0;
  for (int ky = 0; ky < H; ++ky) {
    const int64_t kys = (ky <= H / 2) ? ky : ky - H;
    const int64_t base = kys * kys * cc;
    const int64_t cnt = kxcnt[ky];
    if (cnt == 0 || base >= hi_t) continue;
    const int64_t lo = first_kx(lo_t - base, ca, cnt);
    const int64_t hi = first_kx(hi_t - base, ca, cnt);
    if (lo >= hi) continue;
    const int64_t q0 = qoff[ky];
    for (int64_t kx = lo; kx < hi; ++kx) {
      const int w = (kx > 0 && kx < W / 2) ? 2 : 1;
      wsum += w;
      if (m < M) acc += (double)w * (double)D[(size_t)(q0 + kx) * M + m];
    }
    if (bin_of_q != nullptr && blockIdx.y == 0) {
      for (int64_t kx = lo + threadIdx.x; kx < hi; kx += blockDim.x) bin_of_q[q0 + kx] = b;
    }
  }
  if (m < M) Dbar[(size_t)b * M + m] = (wsum > 0) ? acc / (double)wsum : 0.0;
  if (blockIdx.y == 0 && threadIdx.x == 0) counts[b] = wsum;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

hipError_t launch_radial(hipStream_t s, const float* D, int64_t nq, int M, int W, int H, int64_t ca,
                         int64_t cc, QTable qt, const int64_t* thr, int nbins, double* Dbar,
                         int64_t* counts, int32_t* bin_of_q) {
  if (bin_of_q != nullptr && nq > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, bin_of_q, nq, -1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (nbins == 0) return hipSuccess;
  const int mt = 256;
  dim3 grid(nbins, (M + mt - 1) / mt);
  hipLaunchKernelGGL(k_radial, grid, dim3(mt), 0, s, D, M, W, H, ca, cc, qt.qoff, qt.kxcnt, thr,
                     Dbar, counts, bin_of_q);
  return hipGetLastError();
}

}  // namespace ddm
