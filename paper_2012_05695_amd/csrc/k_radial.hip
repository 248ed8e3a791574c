// Azimuthal |q| averaging of D(q, m) (standard DDM reduction; the paper
// computes D per wave vector and leaves binning to the analysis).
//
// Bin b holds the kept wave vectors with T[b] <= k2 < T[b+1], where
// k2 = kx^2 ca + ky_s^2 cc is the exact integer squared magnitude.  For a
// fixed ky row, k2 grows with kx, so the members of bin b in that row form one
// contiguous kx interval [lo, hi); it is found with integer arithmetic only,
// which makes bin membership bit-exact.
//
// One workgroup per (bin, tile of 64 LPT lags); each lane owns LPT
// consecutive lags (LPT = 4 when rows of D are 16-byte aligned, so that a
// wave reads 1 KiB of a row at once; else 1).  The bin's rows are taken in
// chunks of 256; the members of a chunk are flattened, in q order, into an
// LDS list (q index and weight), a window of kListCap entries at a time.
// Wave w of the four sums the entries j = w (mod 4) of each window for its
// lags in FP64, with 16 loads in flight, and the four partials are added in
// wave order at the end: a fixed order that depends neither on the launch
// geometry (LPT included) nor on timing, so results are deterministic.
#include "internal.hpp"

namespace ddm {

namespace {
constexpr int kRadThreads = 256;
constexpr int kRadLags = 64;
constexpr int kListCap = 4096;
constexpr int kUnroll = 16;
}  // namespace

// LPT consecutive values of one row of D: one 16-byte load for 4 (the
// address is 16-byte aligned), a plain load for 1.
template <int LPT> struct Lags;
template <> struct Lags<1> {
  float v[1];
  __device__ __forceinline__ static Lags load(const float* p) { return Lags{{*p}}; }
};
template <> struct Lags<4> {
  float v[4];
  __device__ __forceinline__ static Lags load(const float* p) {
    const float4 f = *reinterpret_cast<const float4*>(p);
    return Lags{{f.x, f.y, f.z, f.w}};
  }
};

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

template <int LPT>
__global__ void __launch_bounds__(kRadThreads) k_radial(const float* __restrict__ D, int M, int W, int H,
                                                        int64_t ca, int64_t cc,
                                                        const int32_t* __restrict__ qoff,
                                                        const int32_t* __restrict__ kxcnt,
                                                        const int64_t* __restrict__ thr,
                                                        double* __restrict__ Dbar,
                                                        int64_t* __restrict__ counts,
                                                        int32_t* __restrict__ bin_of_q) {
  const int b = blockIdx.x;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int m = (blockIdx.y * kRadLags + lane) * LPT;  // first of this lane's lags
  const bool lag_ok = m < M;  // LPT = 4: M % 4 == 0, so all four are lags
  const bool write_bins = bin_of_q != nullptr && blockIdx.y == 0;
  const int64_t lo_t = thr[b], hi_t = thr[b + 1];
  const int half = W / 2;

  __shared__ int32_t row_q[kRadThreads];   // q index of the row's first member
  __shared__ int32_t row_kx[kRadThreads];  // kx of the row's first member
  __shared__ int32_t row_off[kRadThreads + 1];
  __shared__ int32_t wpart[4];
  __shared__ uint32_t list[kListCap];      // q | (weight 2) << 31
  __shared__ double part[4][kRadLags * LPT];
  __shared__ int64_t wpart64[4];

  double acc[LPT];
#pragma unroll
  for (int i = 0; i < LPT; ++i) acc[i] = 0.0;
  int64_t wsum = 0;
  const float* Dm = D + m;
  for (int ky0 = 0; ky0 < H; ky0 += kRadThreads) {
    // this thread's row: the bin's kx interval, its weight sum
    const int ky = ky0 + tid;
    int lo = 0, len = 0;
    if (ky < H) {
      const int64_t kys = (ky <= H / 2) ? ky : ky - H;
      const int64_t base = kys * kys * cc;
      const int64_t cnt = kxcnt[ky];
      if (cnt > 0 && base < hi_t) {
        lo = (int)first_kx(lo_t - base, ca, cnt);
        len = (int)first_kx(hi_t - base, ca, cnt) - lo;
      }
      if (len > 0) {
        // kx in [lo, lo + len): weight 2 for 0 < kx < W/2, else 1
        const int a = lo > 1 ? lo : 1, z = (lo + len) < half ? (lo + len) : half;
        wsum += len + (z > a ? z - a : 0);
      }
    }
    // exclusive prefix of the interval lengths over the workgroup (ky order)
    int incl = len;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int v = __shfl_up(incl, d, 64);
      if (lane >= d) incl += v;
    }
    if (lane == 63) wpart[wave] = incl;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wave; ++w) before += wpart[w];
    const int total = wpart[0] + wpart[1] + wpart[2] + wpart[3];
    row_off[tid] = before + incl - len;
    row_q[tid] = (ky < H ? qoff[ky] : 0) + lo;
    row_kx[tid] = lo;
    if (tid == 0) row_off[kRadThreads] = total;
    __syncthreads();
    for (int s = 0; s < total; s += kListCap) {
      const int n = (total - s) < kListCap ? (total - s) : kListCap;
      for (int i = tid; i < n; i += kRadThreads) {
        // row holding entry e: the last r with row_off[r] <= e (it is non-empty)
        const int e = s + i;
        int r0 = 0, r1 = kRadThreads;  // row_off[r0] <= e < row_off[r1]
        while (r1 - r0 > 1) {
          const int mid = (r0 + r1) >> 1;
          if (row_off[mid] <= e) r0 = mid; else r1 = mid;
        }
        const int d = e - row_off[r0];
        const int kx = row_kx[r0] + d;
        const uint32_t q = (uint32_t)(row_q[r0] + d);
        list[i] = q | ((kx > 0 && kx < half) ? 0x80000000u : 0u);
        if (write_bins) bin_of_q[q] = b;
      }
      __syncthreads();
      if (lag_ok) {
        int j = wave;
        for (; j + 4 * (kUnroll - 1) < n; j += 4 * kUnroll) {
          Lags<LPT> v[kUnroll];
          uint32_t e[kUnroll];
#pragma unroll
          for (int u = 0; u < kUnroll; ++u) {
            e[u] = list[j + 4 * u];
            v[u] = Lags<LPT>::load(Dm + (size_t)(e[u] & 0x7FFFFFFFu) * (size_t)M);
          }
#pragma unroll
          for (int u = 0; u < kUnroll; ++u)
#pragma unroll
            for (int i = 0; i < LPT; ++i) acc[i] += ((e[u] >> 31) ? 2.0 : 1.0) * (double)v[u].v[i];
        }
        for (; j < n; j += 4) {
          const uint32_t e = list[j];
          const Lags<LPT> v = Lags<LPT>::load(Dm + (size_t)(e & 0x7FFFFFFFu) * (size_t)M);
#pragma unroll
          for (int i = 0; i < LPT; ++i) acc[i] += ((e >> 31) ? 2.0 : 1.0) * (double)v.v[i];
        }
      }
      __syncthreads();  // list[] is rewritten by the next window
    }
  }
  // partials of the four waves, added in wave order; weight sum over threads
#pragma unroll
  for (int i = 0; i < LPT; ++i) part[wave][lane * LPT + i] = acc[i];
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) wsum += __shfl_xor(wsum, d, 64);
  if (lane == 0) wpart64[wave] = wsum;
  __syncthreads();
  if (wave == 0) {
    const int64_t ws = wpart64[0] + wpart64[1] + wpart64[2] + wpart64[3];
#pragma unroll
    for (int i = 0; i < LPT; ++i) {
      const int c = lane * LPT + i;
      const double sum = ((part[0][c] + part[1][c]) + part[2][c]) + part[3][c];
      if (lag_ok) Dbar[(size_t)b * M + m + i] = (ws > 0) ? sum / (double)ws : 0.0;
    }
    if (blockIdx.y == 0 && lane == 0) counts[b] = ws;
  }
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
  if (M % 4 == 0 && ((uintptr_t)D & 15) == 0) {
    dim3 grid(nbins, (M / 4 + kRadLags - 1) / kRadLags);
    hipLaunchKernelGGL(k_radial<4>, grid, dim3(kRadThreads), 0, s, D, M, W, H, ca, cc, qt.qoff, qt.kxcnt, thr,
                       Dbar, counts, bin_of_q);
  } else {
    dim3 grid(nbins, (M + kRadLags - 1) / kRadLags);
    hipLaunchKernelGGL(k_radial<1>, grid, dim3(kRadThreads), 0, s, D, M, W, H, ca, cc, qt.qoff, qt.kxcnt, thr,
                       Dbar, counts, bin_of_q);
  }
  return hipGetLastError();
}

}  // namespace ddm
