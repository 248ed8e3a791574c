// Step two for time-transform length L = 16384 (N2 = 32768, so 8192 < N <=
// 16384): the structure function of one wave vector's time sequence via a
// Fourier transform in time (paper, Eq. (2), Appendix B with the padding of
// Eq. (B4)).  The arithmetic is that of k_time (time_kernel.hpp): per-q mean
// removal, the N2-point forward FFT of the half-zero sequence as two L-point
// FFTs (X_2j = FFT_L(x)_j, X_2j+1 = FFT_L(x_n w^n)_j, w = e^{-2 pi i / N2}), one
// packed L-point inverse of the power spectrum, prefix sums with FP64 offsets
// (wave-local parts rounded to floats) and an FP64 combination, the kTailLags
// largest lags summed from Eq. (1) directly.
//
// Layout for this length: one wave vector per workgroup of 1024 threads, 16
// values per thread held in registers.  LDS holds a single L-element buffer
// (136 KB with padding) that serves, in turn, every FFT pass's exchange, the
// inverse's mirrored reads, then 2 Re c(m) and the prefix sums, instead of a
// staged sequence plus an exchange buffer (which would need 272 KB); the
// sequence is read three times instead (for each forward transform and for
// the prefix sums), the re-reads from lines that the L2 still holds.
#include "time_kernel.hpp"

namespace ddm {

namespace {

constexpr int kLongL = 16384;
constexpr int kLongE = 16;                  // values per thread
constexpr int kLongT = kLongL / kLongE;     // threads per workgroup

// The twiddle table's address, opaque to the compiler at each use: the three
// transforms read the same twiddles, and loads it could prove equal would be
// merged and their values held in registers across all three (more than the
// 128 registers a thread of a 1024-thread workgroup has).
__device__ __forceinline__ const float2* opaque(const float2* p) {
  asm volatile("" : "+s"(p));
  return p;
}
// Likewise the thread index handed to each transform, so that the per-thread
// twiddle and LDS offsets it derives are recomputed per transform rather than
// kept live from the first to the last.
__device__ __forceinline__ int opaque(int t) {
  asm volatile("" : "+v"(t));
  return t;
}

// The FFT passes of length kLongL, their twiddles w_L^j = e^{-2 pi i j / L}
// taken as th[j >> 7] * tl[j & 127] from two 128-entry LDS tables (th[h] =
// w_L^{128 h}, tl[l] = w_L^l) instead of scattered reads of the global table.
template <int NS>
struct LongPasses {
  static constexpr int R = pick_radix(kLongL / NS, kLongE);
  __device__ __forceinline__ static void run(float2 (&v)[kLongE], LdsView<1, true> buf, int tid,
                                             const float2* th, const float2* tl) {
    stockham_pass_g<kLongL, kLongE, R, NS, 1, true, false>(v, buf, tid, [&](int, int k, int jm) {
      const int j = k * jm * (kLongL / (NS * R));
      return cmul(th[j >> 7], tl[j & 127]);
    });
    if constexpr (NS * R < kLongL) LongPasses<NS * R>::run(v, buf, tid, th, tl);
  }
};
static_assert(kLongL == 128 * 128, "two-level twiddle tables of 128 entries");

template <int QB, bool F16>
__global__ void __launch_bounds__(kLongT) k_time_long(const void* __restrict__ spec, int64_t nq, int N, int M,
                                                    const float2* __restrict__ twN2,
                                                    const double* __restrict__ ramp,
                                                    const int32_t* __restrict__ qmap,
                                                    const int32_t* __restrict__ qexp, float* __restrict__ D) {
  constexpr int L = kLongL;
  constexpr int E = kLongE;
  constexpr int T = L / E;  // 1024 threads, 16 waves
  constexpr uint32_t ES = F16 ? 4u : 8u;
  __shared__ float2 buf[lds_len<true>(L)];
  __shared__ double wtot[E * (T / 64)];  // per (chunk, wave) sums of |x'|^2, then their offsets
  __shared__ double wtot4[4];
  __shared__ float redf[T / 64];
  __shared__ float2 ends[2 * kTailLags];  // x'_n for n < kTailLags and N - kTailLags <= n < N
  __shared__ float2 th[128], tl[128];     // two-level twiddle tables (LongPasses)

  // uniform per workgroup: a padding id or a slot without a row of D
  const int64_t q0 = time_q0<1, QB>(blockIdx.x);
  if (q0 >= nq) return;
  const int qd = qmap ? qmap[q0] : (int)q0;
  if (qd < 0) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  LdsView<1, true> yb{buf};
  if (tid < 128) {  // twN2[2 j] = w_L^j; read before the first transform (group_sum synchronises)
    th[tid] = twN2[2 * 128 * tid];
    tl[tid] = twN2[2 * tid];
  }

  // ---- load x_n, n = tid + e T (zero for n >= N: reads past the range return 0) ----
  __amdgpu_buffer_rsrc_t in_r;
  if constexpr (QB == 1)
    in_r = make_rsrc((const float2*)spec + (size_t)q0 * N, (uint32_t)N * 8u);
  else
    in_r = make_rsrc((const char*)spec + ((size_t)(q0 / QB) * N * QB + (size_t)(q0 % QB)) * ES,
                     (uint32_t)(((size_t)(N - 1) * QB + 1) * ES));
  const float sc = F16 ? ldexpf(1.0f, -qexp[qd]) : 1.0f;
  // x_n for this thread's n = tid + e T; the thread index is made opaque per
  // call so that the three reads stay three reads (the sequence is not kept in
  // registers across the transforms: the re-reads hit the L2 lines that the 16
  // workgroups of one block share)
  auto load_x = [&](float2 (&x)[E]) {
    int t = tid;
    asm volatile("" : "+v"(t));
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const uint32_t off = (uint32_t)(t + e * T) * (uint32_t)(QB * ES);
      if constexpr (F16) {
        const __half2 h = __builtin_bit_cast(__half2, __builtin_amdgcn_raw_buffer_load_b32(in_r, off, 0, 0));
        x[e] = make_float2(__low2float(h) * sc, __high2float(h) * sc);
      } else {
        x[e] = ld_f2(in_r, off);
      }
    }
  };

  // ---- offset: FP32 mean in a fixed order (per thread over e, then the group);
  // x'_n = x_n - mean for n < N, 0 beyond ----
  float2 v[E];
  load_x(v);
  float mr, mi;
  {
    float sr = 0.0f, si = 0.0f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      sr += v[e].x;
      si += v[e].y;
    }
    const float inv_n = 1.0f / (float)N;
    mr = group_sum<T>(sr, tid, redf) * inv_n;
    mi = group_sum<T>(si, tid, redf) * inv_n;
  }
  auto offset_free = [&](float2 (&x)[E]) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = tid + e * T;
      x[e] = (n < N) ? make_float2(x[e].x - mr, x[e].y - mi) : make_float2(0.0f, 0.0f);
    }
  };
  offset_free(v);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = tid + e * T;
    if (n < kTailLags) ends[n] = v[e];
    if (n >= N - kTailLags && n < N) ends[n - N + 2 * kTailLags] = v[e];
  }

  // ---- X_even = FFT_L(x'), X_odd = FFT_L(x' w^n); z = IFFT_L(P_even + i P_odd) ----
  LongPasses<1>::run(v, yb, opaque(tid), th, tl);
  float pe[E];
#pragma unroll
  for (int e = 0; e < E; ++e) pe[e] = v[e].x * v[e].x + v[e].y * v[e].y;
  load_x(v);
  offset_free(v);
  {
    const float2* tw = opaque(twN2);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cmul(v[e], tw[tid + e * T]);
  }
  LongPasses<1>::run(v, yb, opaque(tid), th, tl);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = make_float2(pe[e], v[e].x * v[e].x + v[e].y * v[e].y);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);  // inverse by conjugation
  LongPasses<1>::run(v, yb, opaque(tid), th, tl);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
#pragma unroll
  for (int e = 0; e < E; ++e) yb[tid + e * T] = v[e];
  __syncthreads();

  // ---- 2 Re c(m) = (2/N2) Re sum_k P_k e^{2 pi i k m / N2} for m = tid + e T,
  // from z_m and z_{L-m}; kept in the first quarter of the buffer (as floats,
  // element m) once every z has been read ----
  const float inv_l = 1.0f / (float)L;  // 2 / N2
  float* tcl = reinterpret_cast<float*>(buf);      // 2 Re c(m), m < L
  float* sl = reinterpret_cast<float*>(buf) + L;   // wave-local parts of S(n), n < L
  {
    const float2* tw = opaque(twN2);
    float two_c[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int m = tid + e * T;
      const float2 zm = v[e];
      const float2 zr = yb[m == 0 ? 0 : L - m];
      const float2 w = tw[m];  // (cos th, -sin th), th = 2 pi m / N2
      two_c[e] = 0.5f * ((zm.x + zr.x) + w.x * (zm.y + zr.y) - w.y * (zm.x - zr.x)) * inv_l;
    }
    __syncthreads();  // every z has been read: the buffer holds 2 Re c and S from here on
#pragma unroll
    for (int e = 0; e < E; ++e) tcl[tid + e * T] = two_c[e];
  }

  // ---- prefix sums S(n) = sum_{j<n} |x'_j|^2 for n = tid + e T: a wave scan in
  // FP64 per chunk e, whose exclusive part (a sum of at most 63 terms) is kept
  // as a float in the buffer, then the FP64 exclusive scan of the (chunk, wave)
  // totals in n order; S(n) = wave part + offset of its (chunk, wave).  The
  // float rounding of the wave part (a relative 2^-24 of at most 63 |x'|^2) is
  // far below the FP32 transform route's error in 2 Re c(m). ----
  load_x(v);
  offset_free(v);
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const double d = (double)v[e].x * v[e].x + (double)v[e].y * v[e].y;
    double incl = d;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const double excl = __shfl_up(incl, 1, 64);
    sl[tid + e * T] = (lane == 0) ? 0.0f : (float)excl;
    if (lane == 63) wtot[e * (T / 64) + wave] = incl;
  }
  __syncthreads();
  static_assert(E * (T / 64) == 256, "four waves scan the (chunk, wave) totals");
  double off = 0.0;
  if (tid < E * (T / 64)) {  // waves 0-3, whole waves
    double incl = wtot[tid];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const double y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    const double excl = __shfl_up(incl, 1, 64);
    off = (lane == 0) ? 0.0 : excl;
    if (lane == 63) wtot4[wave] = incl;
  }
  __syncthreads();
  if (tid < E * (T / 64)) {
    double before = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < wave) before += wtot4[i];
    wtot[tid] = before + off;
  }
  const double sN = ((wtot4[0] + wtot4[1]) + wtot4[2]) + wtot4[3];  // S(N)
  __syncthreads();
  // S(n), 0 <= n < L (S(n) = S(N) for n >= N)
  auto S = [&](int n) { return (double)sl[n] + wtot[(n / T) * (T / 64) + (n % T) / 64]; };

  // ---- D(m) = (S(N-m) + S(N) - S(m) - 2 Re c(m)) / (N - m); D(q, 0) = 0 ----
  float* drow = D + (size_t)qd * M;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int m = tid + e * T;
    if (m < M) {
      if (m == 0) {
        drow[0] = 0.0f;  // lag 0 pairs every frame with itself
        continue;
      }
      double sum = (S(N - m) + sN) - S(m) - (double)tcl[m];
      if (m >= N - kTailLags) {
        // fewer than kTailLags pairs: Eq. (1) summed directly, in order
        float acc = 0.0f;
        for (int j = 0; j < N - m; ++j) {
          const float2 p = ends[m + j - N + 2 * kTailLags], b = ends[j];
          const float dx = p.x - b.x, dy = p.y - b.y;
          acc += fmaf(dx, dx, dy * dy);
        }
        sum = (double)acc;
      }
      drow[m] = (float)(sum * ramp[m]);
    }
  }
}

}  // namespace

// Launch of the length-16384 kernel: one workgroup per slot id (ids of the
// blocked store that share a block's cache lines are congruent mod 8, so the
// round-robin dispatcher keeps them on one XCD).
hipError_t time_run_long(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M, const float2* twN2,
                         const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D) {
  if (N <= kTailLags || N > kLongL || M < 1 || M > N) return hipErrorInvalidValue;
  if (qb == 1 && qexp == nullptr) {
    const int64_t nids = time_ids<1, 1>(nq);
    if (nids == 0) return hipSuccess;
    hipLaunchKernelGGL((k_time_long<1, false>), dim3((unsigned)nids), dim3(kLongT), 0, s, spec, nq, N, M, twN2, ramp,
                       qmap, nullptr, D);
    return hipGetLastError();
  }
  if (qb != kSpecQB) return hipErrorInvalidValue;
  const int64_t nids = time_ids<1, kSpecQB>(nq);
  if (nids == 0) return hipSuccess;
  if (qexp != nullptr)
    hipLaunchKernelGGL((k_time_long<kSpecQB, true>), dim3((unsigned)nids), dim3(kLongT), 0, s, spec, nq, N, M, twN2,
                       ramp, qmap, qexp, D);
  else
    hipLaunchKernelGGL((k_time_long<kSpecQB, false>), dim3((unsigned)nids), dim3(kLongT), 0, s, spec, nq, N, M, twN2,
                       ramp, qmap, nullptr, D);
  return hipGetLastError();
}

}  // namespace ddm
