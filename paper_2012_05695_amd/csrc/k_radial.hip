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
  // the bin's kx interval of every ky row, computed once per workgroup in
  // chunks of blockDim rows and compacted (in ky order) into LDS
  __shared__ int2 rows[256];
  __shared__ int nrows_s;
  double acc = 0.0;
  int64_t wsum = 0;
  for (int ky0 = 0; ky0 < H; ky0 += blockDim.x) {
    if (threadIdx.x == 0) nrows_s = 0;
    __syncthreads();
    const int ky = ky0 + (int)threadIdx.x;
    int2 iv = make_int2(0, 0);
    if (ky < H) {
      const int64_t kys = (ky <= H / 2) ? ky : ky - H;
      const int64_t base = kys * kys * cc;
      const int64_t cnt = kxcnt[ky];
      if (cnt > 0 && base < hi_t) {
        iv.x = (int)first_kx(lo_t - base, ca, cnt);
        iv.y = (int)first_kx(hi_t - base, ca, cnt);
      }
    }
    // compaction that keeps ky order: prefix count over the workgroup
    const bool has = iv.x < iv.y;
    const unsigned long long ball = __ballot(has);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __shared__ int wcount[4];
    if (lane == 0) wcount[wave] = __popcll(ball);
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wcount[w];
    before += __popcll(ball & ((1ull << lane) - 1ull));
    if (has) rows[before] = make_int2(ky, (iv.y - iv.x) << 16 | iv.x);
    if (threadIdx.x == blockDim.x - 1) nrows_s = before + (has ? 1 : 0);
    __syncthreads();
    const int nr = nrows_s;
    for (int r = 0; r < nr; ++r) {
    const int2 rr = rows[r];
    const int ky_r = rr.x;
    const int64_t lo = rr.y & 0xFFFF, hi = lo + (rr.y >> 16);
    const int64_t q0 = qoff[ky_r];
    for (int64_t kx = lo; kx < hi; ++kx) wsum += (kx > 0 && kx < W / 2) ? 2 : 1;
    if (m < M) {
      // eight rows in flight per step; the sum itself stays in q order
      const float* col = D + (size_t)q0 * M + m;
      int64_t kx = lo;
      for (; kx + 8 <= hi; kx += 8) {
        float d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) d[u] = col[(size_t)(kx + u) * M];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int64_t k = kx + u;
          acc += ((k > 0 && k < W / 2) ? 2.0 : 1.0) * (double)d[u];
        }
      }
      for (; kx < hi; ++kx) acc += ((kx > 0 && kx < W / 2) ? 2.0 : 1.0) * (double)col[(size_t)kx * M];
    }
    if (bin_of_q != nullptr && blockIdx.y == 0) {
      for (int64_t kx = lo + threadIdx.x; kx < hi; kx += blockDim.x) bin_of_q[q0 + kx] = b;
    }
    }
    __syncthreads();  // rows[] is rewritten by the next chunk
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
