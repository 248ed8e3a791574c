// Fit of D(q, m) = A (1 - exp(-m / tau)) + B per wave vector (standard DDM
// model; the paper stops at D).
//
//   k_sample: one wavefront per row of D, one lane per fractional lag m_j:
//             linear interpolation between the integer lags around m_j, then
//             normalisation by the row maximum c (returned).
//   k_lm:     one thread per curve, Marquardt's damped Gauss-Newton on
//             p = (A, B, log tau): residuals in FP32, J^T J and J^T r
//             accumulated and the 3x3 system solved in FP64; lambda x10 on a
//             rejected step, /10 on an accepted one; stop on a relative cost
//             decrease <= ftol, a step <= xtol (|p| + xtol), the iteration
//             limit, or a damping overflow (converged if the residual is then
//             orthogonal to the Jacobian columns to within gtol).
#include <cmath>

#include "internal.hpp"

namespace ddm {

constexpr int kMaxK = 64;

__global__ void __launch_bounds__(256) k_sample(const float* __restrict__ D, int64_t n, int M,
                                                LagSet lags, float* __restrict__ Y,
                                                float* __restrict__ scale) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (row >= n) return;  // uniform per wavefront
  const float* d = D + (size_t)row * M;
  float y = -INFINITY;
  if (lane < lags.K) {
    const float m = lags.m[lane];
    int i0 = (int)floorf(m);
    if (i0 > M - 1) i0 = M - 1;
    const int i1 = (i0 + 1 < M) ? i0 + 1 : M - 1;
    const float f = m - (float)i0;
    const float a = d[i0], b = d[i1];
    y = a + f * (b - a);
  }
  float c = y;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) c = fmaxf(c, __shfl_xor(c, o, 64));
  if (!(c > 0.0f) || !isfinite(c)) c = 1.0f;
  if (lane < lags.K) Y[(size_t)row * lags.K + lane] = y / c;
  if (lane == 0 && scale != nullptr) scale[row] = c;
}

template <int K>
__device__ __forceinline__ double lm_cost(const float (&y)[K], const LagSet& lags, int k, double A,
                                          double B, double th) {
  const float a = (float)A, b = (float)B, inv_tau = (float)exp(-th);
  double c = 0.0;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (j < k) {
      const float r = a * (1.0f - expf(-lags.m[j] * inv_tau)) + b - y[j];
      c += (double)r * (double)r;
    }
  }
  return c;
}

// start_mode with init given: 0 start from init; 1 from whichever of init and
// the default start has the lower cost; 2 from init when its tau lies within
// [m_1 / 4, 4 m_K] and its A is at least 5% of |A| + |B| (a decay the sampled
// lags can resolve), else from the default start.  LM_FLAG_DEFAULT_START when
// the default start is used.
__global__ void __launch_bounds__(64) k_lm(const float* __restrict__ Y, int64_t n, LagSet lags,
                                           const float* __restrict__ init, LmParams prm,
                                           const int32_t* only_if_flag_clear,  // may alias flags
                                           float* __restrict__ params, int32_t* iters,
                                           int32_t* flags, int start_mode) {
  constexpr int K = kMaxK;
  __shared__ float tile[64 * (K + 1)];
  const int64_t c0 = (int64_t)blockIdx.x * 64;
  const int k = lags.K;
  // coalesced load of 64 curves, transposed through LDS
  for (int f = threadIdx.x; f < 64 * k; f += 64) {
    const int64_t cv = c0 + f / k;
    tile[(f / k) * (K + 1) + (f % k)] = (cv < n) ? Y[(size_t)c0 * k + f] : 0.0f;
  }
  __syncthreads();
  const int64_t cid = c0 + threadIdx.x;
  if (cid >= n) return;
  if (only_if_flag_clear != nullptr && (only_if_flag_clear[cid] & LM_FLAG_CONVERGED)) return;
  float y[K];
#pragma unroll
  for (int j = 0; j < K; ++j) y[j] = (j < k) ? tile[threadIdx.x * (K + 1) + j] : 0.0f;

  double yy = 0.0, ymax = -INFINITY;
  bool finite = true;
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (j < k) {
      yy += (double)y[j] * (double)y[j];
      ymax = fmax(ymax, (double)y[j]);
      finite = finite && isfinite(y[j]);
    }
  // default initialisation on the curve normalised by its maximum
  const double c = (isfinite(ymax) && ymax > 0.0) ? ymax : 1.0;
  const double B0 = (double)y[0] / c;
  double A = (1.0 - B0) * c, B = B0 * c, th = 0.5 * (log((double)lags.m[0]) + log((double)lags.m[k - 1]));
  int32_t fl = 0, it = 0;
  if (init != nullptr && only_if_flag_clear == nullptr) {
    const double Ai = init[cid * 3 + 0], Bi = init[cid * 3 + 1], thi = init[cid * 3 + 2];
    bool take = true;
    if (start_mode == 1) {
      const double ci = lm_cost<K>(y, lags, k, Ai, Bi, thi), cd = lm_cost<K>(y, lags, k, A, B, th);
      take = isfinite(ci) && !(cd < ci);  // ties go to the given start
    } else if (start_mode == 2) {
      // a decay the sampled lags can resolve: tau inside the window and an
      // amplitude of at least 5% of the curve (below it the curve is noise)
      const double ln4 = 1.3862943611198906;
      take = thi >= log((double)lags.m[0]) - ln4 && thi <= log((double)lags.m[k - 1]) + ln4 &&
             Ai >= 0.05 * (fabs(Ai) + fabs(Bi));
    }
    if (take) {
      A = Ai;
      B = Bi;
      th = thi;
    } else {
      fl |= LM_FLAG_DEFAULT_START;
    }
  }
  if (!finite || !isfinite(A) || !isfinite(B) || !isfinite(th)) {
    fl = LM_FLAG_NONFINITE;
  } else {
    double cost = lm_cost<K>(y, lags, k, A, B, th);
    double lam = prm.lambda0;
    while (true) {
      if (it >= prm.max_iter) {
        fl |= LM_FLAG_MAXITER;
        break;
      }
      // J^T J and J^T r at p (FP32 model, FP64 sums)
      const float a = (float)A, b = (float)B, inv_tau = (float)exp(-th);
      double h00 = 0, h01 = 0, h02 = 0, h11 = 0, h12 = 0, h22 = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll
      for (int j = 0; j < K; ++j) {
        if (j < k) {
          const float e = expf(-lags.m[j] * inv_tau);
          const float r = a * (1.0f - e) + b - y[j];
          const double j0 = 1.0 - (double)e, j2 = -(double)a * (double)e * (double)lags.m[j] * (double)inv_tau;
          h00 += j0 * j0; h01 += j0; h02 += j0 * j2;
          h11 += 1.0; h12 += j2; h22 += j2 * j2;
          g0 += j0 * r; g1 += r; g2 += j2 * r;
        }
      }
      ++it;
      bool accepted = false, small_f = false, small_x = false;
      while (lam <= prm.lambda_max) {
        // (H + lam diag H) delta = -g, by Cramer's rule in FP64
        const double a00 = h00 * (1 + lam), a11 = h11 * (1 + lam), a22 = h22 * (1 + lam);
        const double det = a00 * (a11 * a22 - h12 * h12) - h01 * (h01 * a22 - h12 * h02) +
                           h02 * (h01 * h12 - a11 * h02);
        if (!(fabs(det) > 0.0) || !isfinite(det)) {
          lam *= 10.0;
          continue;
        }
        const double b0 = -g0, b1 = -g1, b2 = -g2;
        const double d0 = (b0 * (a11 * a22 - h12 * h12) - h01 * (b1 * a22 - h12 * b2) +
                           h02 * (b1 * h12 - a11 * b2)) / det;
        const double d1 = (a00 * (b1 * a22 - h12 * b2) - b0 * (h01 * a22 - h12 * h02) +
                           h02 * (h01 * b2 - b1 * h02)) / det;
        const double d2 = (a00 * (a11 * b2 - b1 * h12) - h01 * (h01 * b2 - b1 * h02) +
                           b0 * (h01 * h12 - a11 * h02)) / det;
        const double An = A + d0, Bn = B + d1, thn = th + d2;
        const double cn = lm_cost<K>(y, lags, k, An, Bn, thn);
        if (isfinite(cn) && cn < cost) {
          small_f = (cost - cn) <= prm.ftol * cost;
          const double dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
          const double pn = sqrt(A * A + B * B + th * th);
          small_x = dn <= prm.xtol * (pn + prm.xtol);
          A = An; B = Bn; th = thn; cost = cn;
          lam /= 10.0;
          accepted = true;
          break;
        }
        lam *= 10.0;
      }
      if (!accepted) {
        // No decreasing step at any damping: p is stationary to the precision
        // of the FP32 cost.  Converged if the fit is exact or the residual is
        // orthogonal to every Jacobian column to within gtol (cosine test).
        const double rn = sqrt(cost);
        const bool orth = fabs(g0) <= prm.gtol * sqrt(h00) * rn && fabs(g1) <= prm.gtol * sqrt(h11) * rn &&
                          fabs(g2) <= prm.gtol * sqrt(h22) * rn;
        fl |= (cost <= prm.exact_fit * yy || orth) ? LM_FLAG_CONVERGED : LM_FLAG_STALLED;
        break;
      }
      if (small_f || small_x) {
        fl |= LM_FLAG_CONVERGED;
        break;
      }
    }
    if (!isfinite(A) || !isfinite(B) || !isfinite(th)) fl |= LM_FLAG_NONFINITE;
  }
  params[cid * 3 + 0] = (float)A;
  params[cid * 3 + 1] = (float)B;
  params[cid * 3 + 2] = (float)exp(th);
  if (only_if_flag_clear != nullptr) {
    // second pass from the default start: count both passes' iterations
    fl |= LM_FLAG_FALLBACK;
    if (iters) iters[cid] += it;
  } else if (iters) {
    iters[cid] = it;
  }
  if (flags) flags[cid] = fl;
}

hipError_t launch_sample(hipStream_t s, const float* D, int64_t n, int M, const LagSet& lags, float* Y,
                         float* scale) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, D, n, M, lags, Y, scale);
  return hipGetLastError();
}

hipError_t launch_lm(hipStream_t s, const float* Y, int64_t n, const LagSet& lags, const float* init,
                     const LmParams& prm, const int32_t* only_if_flag_clear, float* params,
                     int32_t* iters, int32_t* flags, int start_mode) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_lm, dim3((unsigned)((n + 63) / 64)), dim3(64), 0, s, Y, n, lags, init, prm,
                     only_if_flag_clear, params, iters, flags, start_mode);
  return hipGetLastError();
}

}  // namespace ddm
