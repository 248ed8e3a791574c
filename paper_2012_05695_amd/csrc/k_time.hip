// Step two: the structure function of one time sequence via a Fourier
// transform in time (paper, Eq. (2) and Appendix B).
//
// For the time sequence x_n = F(q, n), n < N, of one wave vector:
//   D(m) (N-m) = sum_{n=m}^{N-1} |x_n|^2 + |x_{n-m}|^2 - 2 Re(conj(x_{n-m}) x_n)
//              = S(N-m) + S(N) - S(m) - 2 Re c(m),
// with prefix sums S(k) = sum_{j<k} |x_j|^2 (the closed form of the recursion
// Eq. (B3)) and the acyclic autocorrelation c(m) = sum_n conj(x_n) x_{n+m},
// obtained by zero padding to N2 = 2L (Eq. (B4), L = 2^ceil(log2 N)), a
// forward FFT, squared modulus, inverse FFT (Appendix B, the five steps).
//
// MI355X formulation of the same computation:
//  * the per-q FP64 temporal mean is subtracted first (D depends only on
//    differences of x, so any per-q constant offset cancels exactly; removing
//    it keeps the FP32 transforms away from cancellation);
//  * the N2-point forward FFT of the half-zero sequence is done as two L-point
//    FFTs: X_{2j} = FFT_L(x)_j and X_{2j+1} = FFT_L(x_n w^n)_j, w = e^{-2 pi i/N2};
//  * the real power spectrum P is inverted with one complex L-point IFFT of
//    P_even + i P_odd, separated afterwards by conjugate symmetry:
//    with z = IFFT(P_e + i P_o), a_m = (z_m + conj z_{L-m})/2 and
//    b_m = (z_m - conj z_{L-m})/(2i), sum_k P_k e^{2 pi i k m/N2} = a_m + e^{2 pi i m/N2} b_m;
//  * S and the final combination are FP64; D is rounded to FP32 once.
#include "fft.hpp"
#include "internal.hpp"

namespace ddm {

template <int L, int E>
__global__ void __launch_bounds__(512) k_time(const float2* __restrict__ spec, int qb, int qpw,
                                               int64_t nq, int N, int M,
                                               const float2* __restrict__ twN2,
                                               float* __restrict__ D) {
  constexpr int T = L / E;
  constexpr int XS = L + 1;  // per-q stride of the complex buffer (breaks bank aliasing)
  extern __shared__ __align__(16) unsigned char lds_raw[];
  float2* xbuf = reinterpret_cast<float2*>(lds_raw);
  double* sbuf = reinterpret_cast<double*>(lds_raw + sizeof(float2) * (size_t)XS * qpw);

  // Workgroup -> first wave vector.  When a workgroup covers only part of a
  // layout block (qpw < qb), the qb/qpw workgroups that share the block's
  // cache lines get ids that the round-robin dispatcher sends to the same XCD.
  const int64_t id = blockIdx.x;
  int64_t q0;
  if (qpw >= qb) {
    q0 = id * qpw;
  } else {
    const int nsub = qb / qpw;
    const int64_t G = 8LL * nsub;
    const int64_t r = id % G;
    q0 = ((id / G) * 8 + (r % 8)) * qb + (r / 8) * qpw;
  }
  if (q0 >= nq) return;  // uniform for the whole workgroup

  const int qi = threadIdx.x / T;
  const int tid = threadIdx.x % T;
  const int64_t q = q0 + qi;
  const bool qvalid = q < nq;

  // ---- cooperative load of qpw time sequences into LDS, [q][t] ----
  // element (q, t) of the store sits at ((q / qb) * N + t) * qb + q % qb:
  // qb = 1 is plain q-major input, qb > 1 the blocked store.
  {
    const int total = N * qpw;
    const int nthr = blockDim.x;
    for (int f = threadIdx.x; f < total; f += nthr) {
      int t, i;
      if (qb == 1) { i = f / N; t = f - i * N; }
      else { t = f / qpw; i = f - t * qpw; }
      const int64_t qq = q0 + i;
      float2 val = make_float2(0.f, 0.f);
      if (qq < nq) val = spec[((size_t)(qq / qb) * N + t) * qb + (qq % qb)];
      xbuf[i * XS + t] = val;
    }
    for (int f = threadIdx.x; f < (L - N) * qpw; f += nthr) {
      const int i = f / (L - N), t = N + (f - i * (L - N));
      xbuf[i * XS + t] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();

  float2* xb = xbuf + qi * XS;
  double* sb = sbuf + (size_t)qi * L;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = xb[tid + e * T];

  // ---- FP64 temporal mean, reduced in a fixed order ----
  double sr = 0.0, si = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    sr += (double)v[e].x;
    si += (double)v[e].y;
  }
  sb[tid] = sr;
  sb[T + tid] = si;
  __syncthreads();
  double mr = 0.0, mi = 0.0;
  for (int k = 0; k < T; ++k) {
    mr += sb[k];
    mi += sb[T + k];
  }
  mr /= (double)N;
  mi /= (double)N;
  __syncthreads();

  // ---- offset-free sequence x' (FP32) and |x'|^2 (exact in FP64) ----
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int n = tid + e * T;
    if (n < N) {
      v[e] = make_float2((float)((double)v[e].x - mr), (float)((double)v[e].y - mi));
    } else {
      v[e] = make_float2(0.f, 0.f);
    }
    sb[n] = (double)v[e].x * (double)v[e].x + (double)v[e].y * (double)v[e].y;
  }
  __syncthreads();

  // ---- prefix sums S(k) = sum_{j<k} |x'_j|^2, FP64, fixed order ----
  // each thread owns the contiguous chunk [tid*E, tid*E + E)
  double chunk[E];
  double ctot = 0.0;
#pragma unroll
  for (int i = 0; i < E; ++i) {
    chunk[i] = ctot;  // exclusive within the chunk
    ctot += sb[tid * E + i];
  }
  double* tots = reinterpret_cast<double*>(xb);  // xb is free: data lives in v[]
  tots[tid] = ctot;
  __syncthreads();
  double before = 0.0, total = 0.0;
  for (int k = 0; k < T; ++k) {
    const double tk = tots[k];
    if (k < tid) before += tk;
    total += tk;
  }
#pragma unroll
  for (int i = 0; i < E; ++i) sb[tid * E + i] = before + chunk[i];
  __syncthreads();  // sb holds S(k), k < L; tots no longer needed

  // ---- X_odd = FFT_L(x' w^n), w = e^{-2 pi i / N2}; X_even = FFT_L(x') ----
  LdsView<1> buf{xb};
  float2 u[E];
#pragma unroll
  for (int e = 0; e < E; ++e) u[e] = cmul(v[e], twN2[tid + e * T]);
  fft_forward<L, E, 1>(u, buf, tid, twN2, 2);
  float po[E];
#pragma unroll
  for (int e = 0; e < E; ++e) po[e] = u[e].x * u[e].x + u[e].y * u[e].y;
  fft_forward<L, E, 1>(v, buf, tid, twN2, 2);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = make_float2(v[e].x * v[e].x + v[e].y * v[e].y, po[e]);

  // ---- z = IFFT_L(P_even + i P_odd), unnormalised ----
  fft_inverse<L, E, 1>(v, buf, tid, twN2, 2);
#pragma unroll
  for (int e = 0; e < E; ++e) buf[tid + e * T] = v[e];
  __syncthreads();

  // ---- combination: D(m) = (S(N-m) + S(N) - S(m) - 2 Re c(m)) / (N-m) ----
  if (qvalid) {
    const double inv_n2 = 1.0 / (2.0 * (double)L);
    float* drow = D + (size_t)q * M;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int m = tid + e * T;
      if (m < M) {
        const float2 zm = buf[m];
        const float2 zr = buf[(L - m) & (L - 1)];
        const float2 w = twN2[m];  // (cos th, -sin th), th = 2 pi m / N2
        const double p = zm.x, qq = zm.y, uu = zr.x, vv = zr.y;
        const double re_R = 0.5 * ((p + uu) + (double)w.x * (qq + vv) - (double)w.y * (p - uu));
        const double cm = re_R * inv_n2;
        const double s_nm = (N - m < L) ? sb[N - m] : total;
        const double s_m = sb[m];
        const double dm = ((s_nm + total - s_m) - 2.0 * cm) / (double)(N - m);
        // lag 0 pairs every frame with itself: D(q, 0) = 0 exactly by definition
        drow[m] = (m == 0) ? 0.0f : (float)dm;
      }
    }
  }
}

TimeCfg time_cfg(int L) {
  TimeCfg c;
  c.L = L;
  c.E = 16;
  c.T = L / c.E;
  const size_t per_q = sizeof(float2) * (size_t)(L + 1) + sizeof(double) * (size_t)L;
  int qpw = 16;
  while (qpw > 1 && per_q * qpw > 163840) qpw >>= 1;
  while (qpw > 1 && qpw * c.T > 512) qpw >>= 1;
  c.qpw = qpw;
  c.lds = per_q * qpw;
  return c;
}

template <int L>
static hipError_t time_go(hipStream_t s, const float2* spec, int qb, int64_t nq, int N, int M,
                          const float2* tw, float* D) {
  TimeCfg c = time_cfg(L);
  const int qpw = c.qpw;
  int64_t nwg;
  if (qpw >= qb) {
    nwg = (nq + qpw - 1) / qpw;
  } else {
    const int64_t nblocks = (nq + qb - 1) / qb;
    nwg = ((nblocks + 7) / 8) * 8 * (qb / qpw);
  }
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL((k_time<L, 16>), dim3((unsigned)nwg), dim3(qpw * c.T), c.lds, s, spec, qb, qpw,
                     nq, N, M, tw, D);
  return hipGetLastError();
}

hipError_t launch_time(hipStream_t s, const float2* spec, int qb, int64_t nq, int N, int M,
                       const float2* twN2, float* D) {
  int L = 16;
  while (L < N) L <<= 1;
  switch (L) {
    case 16: return time_go<16>(s, spec, qb, nq, N, M, twN2, D);
    case 32: return time_go<32>(s, spec, qb, nq, N, M, twN2, D);
    case 64: return time_go<64>(s, spec, qb, nq, N, M, twN2, D);
    case 128: return time_go<128>(s, spec, qb, nq, N, M, twN2, D);
    case 256: return time_go<256>(s, spec, qb, nq, N, M, twN2, D);
    case 512: return time_go<512>(s, spec, qb, nq, N, M, twN2, D);
    case 1024: return time_go<1024>(s, spec, qb, nq, N, M, twN2, D);
    case 2048: return time_go<2048>(s, spec, qb, nq, N, M, twN2, D);
    case 4096: return time_go<4096>(s, spec, qb, nq, N, M, twN2, D);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace ddm
