// Fit of D(q, m) = A (1 - exp(-m / tau)) + B per wave vector (standard DDM
// model; the paper stops at D).
//
//   k_sample: one wavefront per row of D, one lane per fractional lag m_j:
//             linear interpolation between the integer lags around m_j, then
//             normalisation by the row maximum c (returned).
//   k_lm:     one lane per curve at a time, Marquardt's damped Gauss-Newton on
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

// ys[j * 64]: sample j of the lane's curve (LDS, one column per lane).  The
// loops over the samples run to k, unrolled by 8, in order of j: unrolled over
// all 64 with the samples in registers, the lags held in scalar registers
// spilled (470 of them) into the hot loops, at 1.8x the time.
template <int K>
__device__ __forceinline__ double lm_cost(const float* ys, const LagSet& lags, int k, double A, double B,
                                          double th) {
  const float a = (float)A, b = (float)B, inv_tau = (float)exp(-th);
  double c = 0.0;
#pragma unroll 8
  for (int j = 0; j < k; ++j) {
    const float r = a * (1.0f - expf(-lags.m[j] * inv_tau)) + b - ys[j * 64];
    c += (double)r * (double)r;
  }
  return c;
}

// start_mode with init given: 0 start from init; 1 from whichever of init and
// the default start has the lower cost; 2 from init when its tau lies within
// [m_1 / 4, 4 m_K] and its A is at least 5% of |A| + |B| (a decay the sampled
// lags can resolve), else from the default start.  LM_FLAG_DEFAULT_START when
// the default start is used.
//
// Each wave owns per_wave consecutive curves.  A lane whose curve has finished
// takes the block's next unassigned curve (idle lanes in lane order, counted
// by a ballot), so a wave runs for about the sum of its curves' iterations over
// 64 rather than for its slowest curve's, and the lanes of a wave that still
// iterates stay busy.  Each curve's arithmetic is the same whichever lane fits it.
__global__ void __launch_bounds__(64) k_lm(const float* __restrict__ Y, int64_t n, int64_t per_wave, LagSet lags,
                                           const float* __restrict__ init, LmParams prm,
                                           const int32_t* only_if_flag_clear,  // may alias flags
                                           float* __restrict__ params, int32_t* iters,
                                           int32_t* flags, int start_mode) {
  constexpr int K = kMaxK;
  const int k = lags.K;
  const int lane = (int)threadIdx.x;
  const int64_t b0 = (int64_t)blockIdx.x * per_wave;
  const int64_t b1 = (b0 + per_wave < n) ? b0 + per_wave : n;
  int64_t next = b0;  // the block's next unassigned curve (the same in every lane)
  int64_t cid = -1;   // this lane's curve; -1: idle
  __shared__ float ycol[K * 64];  // ycol[j * 64 + lane]: sample j of the lane's curve
  float* const ys = ycol + lane;
  double yy = 0.0, A = 0.0, B = 0.0, th = 0.0, cost = 0.0, lam = 0.0;
  int32_t fl = 0, it = 0;

  auto finish = [&]() {
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
    cid = -1;
  };

  // Take curve c: its samples, the start, the first cost.  Leaves the lane
  // idle again when the curve is skipped or cannot be fitted.
  auto start = [&](int64_t c) {
    if (only_if_flag_clear != nullptr && (only_if_flag_clear[c] & LM_FLAG_CONVERGED)) return;
    cid = c;
    const float* yc = Y + (size_t)c * k;
    yy = 0.0;
    double ymax = -INFINITY;
    bool finite = true;
#pragma unroll 8
    for (int j = 0; j < k; ++j) {
        const float v = yc[j];
        ys[j * 64] = v;
        yy += (double)v * (double)v;
        ymax = fmax(ymax, (double)v);
        finite = finite && isfinite(v);
      }
    // default initialisation on the curve normalised by its maximum
    const double cn = (isfinite(ymax) && ymax > 0.0) ? ymax : 1.0;
    const double B0 = (double)ys[0] / cn;
    A = (1.0 - B0) * cn;
    B = B0 * cn;
    th = 0.5 * (log((double)lags.m[0]) + log((double)lags.m[k - 1]));
    fl = 0;
    it = 0;
    if (init != nullptr && only_if_flag_clear == nullptr) {
      const double Ai = init[c * 3 + 0], Bi = init[c * 3 + 1], thi = init[c * 3 + 2];
      bool take = true;
      if (start_mode == 1) {
        const double ci = lm_cost<K>(ys, lags, k, Ai, Bi, thi), cd = lm_cost<K>(ys, lags, k, A, B, th);
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
      finish();
      return;
    }
    cost = lm_cost<K>(ys, lags, k, A, B, th);
    lam = prm.lambda0;
  };

  // One Jacobian evaluation and its damped step; finishes the curve when it stops.
  auto step = [&]() {
    bool done = false;
    if (it >= prm.max_iter) {
      fl |= LM_FLAG_MAXITER;
      done = true;
    } else {
      // J^T J and J^T r at p (FP32 model, FP64 sums)
      const float a = (float)A, b = (float)B, inv_tau = (float)exp(-th);
      double h00 = 0, h01 = 0, h02 = 0, h11 = 0, h12 = 0, h22 = 0, g0 = 0, g1 = 0, g2 = 0;
#pragma unroll 8
      for (int j = 0; j < k; ++j) {
        const float e = expf(-lags.m[j] * inv_tau);
        const float r = a * (1.0f - e) + b - ys[j * 64];
        const double j0 = 1.0 - (double)e, j2 = -(double)a * (double)e * (double)lags.m[j] * (double)inv_tau;
        h00 += j0 * j0; h01 += j0; h02 += j0 * j2;
        h11 += 1.0; h12 += j2; h22 += j2 * j2;
        g0 += j0 * r; g1 += r; g2 += j2 * r;
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
        const double r0 = -g0, r1 = -g1, r2 = -g2;
        const double d0 = (r0 * (a11 * a22 - h12 * h12) - h01 * (r1 * a22 - h12 * r2) +
                           h02 * (r1 * h12 - a11 * r2)) / det;
        const double d1 = (a00 * (r1 * a22 - h12 * r2) - r0 * (h01 * a22 - h12 * h02) +
                           h02 * (h01 * r2 - r1 * h02)) / det;
        const double d2 = (a00 * (a11 * r2 - r1 * h12) - h01 * (h01 * r2 - r1 * h02) +
                           r0 * (h01 * h12 - a11 * h02)) / det;
        const double An = A + d0, Bn = B + d1, thn = th + d2;
        const double cn = lm_cost<K>(ys, lags, k, An, Bn, thn);
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
        done = true;
      } else if (small_f || small_x) {
        fl |= LM_FLAG_CONVERGED;
        done = true;
      }
    }
    if (done) {
      if (!isfinite(A) || !isfinite(B) || !isfinite(th)) fl |= LM_FLAG_NONFINITE;
      finish();
    }
  };

  while (true) {
    const uint64_t idle = __ballot(cid < 0);
    if (idle != 0 && next < b1) {
      // idle lanes take the next curves of the block, in lane order
      const int64_t mine = next + __popcll(idle & ((1ull << lane) - 1ull));
      next += __popcll(idle);
      if (cid < 0 && mine < b1) start(mine);
      continue;  // a curve may end at its start: hand out again first
    }
    if (__ballot(cid >= 0) == 0) break;  // the block is handed out and every lane idle
    if (cid >= 0) step();
  }
}

hipError_t launch_sample(hipStream_t s, const float* D, int64_t n, int M, const LagSet& lags, float* Y,
                         float* scale) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sample, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, D, n, M, lags, Y, scale);
  return hipGetLastError();
}

// Curves per wave: enough that the waves fit in one round of the chip's
// resident waves (k_lm holds three waves per SIMD: 3072 on 256 CUs), at least 64.
constexpr int64_t kLmWaves = 3072;

hipError_t launch_lm(hipStream_t s, const float* Y, int64_t n, const LagSet& lags, const float* init,
                     const LmParams& prm, const int32_t* only_if_flag_clear, float* params,
                     int32_t* iters, int32_t* flags, int start_mode) {
  if (n == 0) return hipSuccess;
  const int64_t per_wave = 64 * ((n + 64 * kLmWaves - 1) / (64 * kLmWaves));
  const int64_t grid = (n + per_wave - 1) / per_wave;
  hipLaunchKernelGGL(k_lm, dim3((unsigned)grid), dim3(64), 0, s, Y, n, per_wave, lags, init, prm,
                     only_if_flag_clear, params, iters, flags, start_mode);
  return hipGetLastError();
}

}  // namespace ddm
