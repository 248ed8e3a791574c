// Kernels of the fit-initialisation MLP: x (64) -> 3 x [Linear(256), GELU]
// -> Linear(3), trained with Adam (not in the paper; it supplies the start of
// the per-q least-squares fit).
//
// Contractions run on the matrix cores: BF16 operands, FP32 accumulation,
// v_mfma_f32_32x32x16_bf16.  A workgroup computes a 64 x 64 tile of
// C = A B with four waves of 32 x 32; A(i,k) and B(k,j) are read with
// arbitrary strides so that forward (X W^T), input-gradient (dZ W) and
// weight-gradient (dZ^T H) products share one kernel.  Epilogues fuse the
// bias, the exact-erf GELU, and the GELU derivative of the backward pass.
#include <cmath>

#include "internal.hpp"

namespace ddm {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}
__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }  // round to nearest even

enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };

constexpr int TM = 64, TN = 64, TK = 32;
constexpr int AS = TK + 8;  // LDS row stride (bf16) of the A tile [TM][TK] and the B^T tile [TN][TK]

template <int EPI>
__global__ void __launch_bounds__(256) k_gemm(int M, int N, int K, const __bf16* __restrict__ A,
                                              int64_t sam, int64_t sak, const __bf16* __restrict__ B,
                                              int64_t sbk, int64_t sbn, const float* __restrict__ bias,
                                              float* __restrict__ C, int64_t ldc, __bf16* __restrict__ H,
                                              int64_t ldh, const float* __restrict__ Zin, int64_t ldz) {
  __shared__ __bf16 As[TM * AS];
  __shared__ __bf16 Bt[TN * AS];
  const int i0 = blockIdx.y * TM, j0 = blockIdx.x * TN;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave >> 1, wn = wave & 1;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;

  // unit stride along k with 16-byte aligned rows: each thread moves 8
  // consecutive k at once (one 16-byte load per operand and k step)
  const bool vecA = sak == 1 && (sam % 8) == 0 && (((uintptr_t)A) & 15) == 0;
  const bool vecB = sbk == 1 && (sbn % 8) == 0 && (((uintptr_t)B) & 15) == 0;
  static_assert(TM * TK / 8 == 256 && TN * TK / 8 == 256, "one 8-element chunk per thread");
  for (int k0 = 0; k0 < K; k0 += TK) {
    // tile loads, zero outside the matrices; the index order follows the
    // unit-stride dimension so that neighbouring threads read neighbouring bytes
    if (vecA) {
      const int i = threadIdx.x / (TK / 8), kc = 8 * (threadIdx.x % (TK / 8));
      const int gi = i0 + i, gk = k0 + kc;
      bf16x8 v;
      if (gi < M && gk + 8 <= K) {
        v = *reinterpret_cast<const bf16x8*>(A + (int64_t)gi * sam + gk);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = (gi < M && gk + t < K) ? A[(int64_t)gi * sam + gk + t] : (__bf16)0.0f;
      }
      *reinterpret_cast<bf16x8*>(&As[i * AS + kc]) = v;
    } else {
#pragma unroll
      for (int s = 0; s < (TM * TK) / 256; ++s) {
        const int f = threadIdx.x + s * 256;
        int i, k;
        if (sak == 1) { i = f / TK; k = f % TK; } else { i = f % TM; k = f / TM; }
        const int gi = i0 + i, gk = k0 + k;
        As[i * AS + k] = (gi < M && gk < K) ? A[gi * sam + gk * sak] : (__bf16)0.0f;
      }
    }
    if (vecB) {
      const int j = threadIdx.x / (TK / 8), kc = 8 * (threadIdx.x % (TK / 8));
      const int gj = j0 + j, gk = k0 + kc;
      bf16x8 v;
      if (gj < N && gk + 8 <= K) {
        v = *reinterpret_cast<const bf16x8*>(B + (int64_t)gj * sbn + gk);
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) v[t] = (gj < N && gk + t < K) ? B[(int64_t)gj * sbn + gk + t] : (__bf16)0.0f;
      }
      *reinterpret_cast<bf16x8*>(&Bt[j * AS + kc]) = v;
    } else {
#pragma unroll
      for (int s = 0; s < (TN * TK) / 256; ++s) {
        const int f = threadIdx.x + s * 256;
        int j, k;
        if (sbk == 1) { j = f / TK; k = f % TK; } else { j = f % TN; k = f / TN; }
        const int gj = j0 + j, gk = k0 + k;
        Bt[j * AS + k] = (gj < N && gk < K) ? B[gk * sbk + gj * sbn] : (__bf16)0.0f;
      }
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; kk += 16) {
      // A fragment: row (lane % 32), k = kk + 8 (lane / 32) .. +7 ; B likewise by column
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&As[(wm * 32 + (lane & 31)) * AS + kk + 8 * (lane >> 5)]);
      const bf16x8 b = *reinterpret_cast<const bf16x8*>(&Bt[(wn * 32 + (lane & 31)) * AS + kk + 8 * (lane >> 5)]);
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // accumulator r of a lane holds C[8 (r/4) + 4 (lane/32) + r%4][lane % 32] of the wave's 32 x 32 block
  const int gj = j0 + wn * 32 + (lane & 31);
  if (gj >= N) return;
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int gi = i0 + wm * 32 + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
    if (gi < M) {
      float z = acc[r];
      if (EPI == EPI_BIAS || EPI == EPI_BIAS_GELU) z += bias[gj];
      if (EPI == EPI_GELU_BWD) {
        H[gi * ldh + gj] = to_bf16(z * gelu_grad_f(Zin[gi * ldz + gj]));
      } else {
        if (C != nullptr) C[gi * ldc + gj] = z;
        if (EPI == EPI_BIAS_GELU && H != nullptr) H[gi * ldh + gj] = to_bf16(gelu_f(z));
      }
    }
  }
}

__global__ void k_to_bf16(const float* __restrict__ x, __bf16* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// Mean squared error over n values: per-workgroup partial sums (fixed order),
// and the BF16 output gradient 2 (y - t) / n.
__global__ void __launch_bounds__(256) k_mse(const float* __restrict__ Y, const float* __restrict__ T,
                                             int64_t n, __bf16* __restrict__ dY, float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  float d = 0.0f;
  if (i < n) {
    d = Y[i] - T[i];
    dY[i] = to_bf16(2.0f * d / (float)n);
  }
  red[threadIdx.x] = d * d;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) k_sum_partials(const float* __restrict__ partial, int np, int64_t n,
                                                      float* __restrict__ loss) {
  __shared__ float red[256];
  float s = 0.0f;
  for (int i = threadIdx.x; i < np; i += 256) s += partial[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) loss[0] = red[0] / (float)n;
}

// Bias gradient: column sums of dZ [B][N] (BF16) in FP32, one thread per column.
__global__ void k_colsum(const __bf16* __restrict__ dZ, int64_t B, int N, float* __restrict__ db) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= N) return;
  float s = 0.0f;
  for (int64_t b = 0; b < B; ++b) s += (float)dZ[b * N + j];
  db[j] = s;
}

// Adam with bias correction on the FP32 master parameters; refreshes the BF16 copy.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, __bf16* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
  p[i] = pi;
  pb[i] = to_bf16(pi);
}

// Inference of the whole network in one launch: a workgroup takes 64 rows,
// keeps their activations in LDS (rounded to BF16 as the layered forward
// rounds them between layers) and runs the four layers with k_gemm's MFMA
// fragments, k order and epilogues, reading the weights from L2; only x and y
// touch HBM.  The results are those of the layered forward.
constexpr int kInfRows = 64;
constexpr int kInfStride = DDM_MLP_HIDDEN + 8;  // LDS row stride (bf16): 528 bytes, rows 16-byte aligned

__global__ void __launch_bounds__(256) k_mlp_infer(const float* __restrict__ x, int64_t rows,
                                                   const __bf16* __restrict__ W1, const float* __restrict__ b1,
                                                   const __bf16* __restrict__ W2, const float* __restrict__ b2,
                                                   const __bf16* __restrict__ W3, const float* __restrict__ b3,
                                                   const __bf16* __restrict__ W4, const float* __restrict__ b4,
                                                   float* __restrict__ y) {
  constexpr int NI = DDM_MLP_IN, NHd = DDM_MLP_HIDDEN, NO = DDM_MLP_OUT;
  static_assert(NI % 16 == 0 && NHd == 4 * 64 && NO <= 32, "layer shapes of the fused inference");
  __shared__ __bf16 Hs[kInfRows * kInfStride];
  const int64_t r0 = (int64_t)blockIdx.x * kInfRows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  {
    // the input rows in BF16: thread t converts 16 consecutive inputs of row t / 4
    const int r = threadIdx.x >> 2, c0 = (threadIdx.x & 3) * 16;
    const int64_t gr = r0 + r;
#pragma unroll
    for (int c = 0; c < 16; ++c) Hs[r * kInfStride + c0 + c] = to_bf16(gr < rows ? x[gr * NI + c0 + c] : 0.0f);
  }
  __syncthreads();
  // hidden layers: wave w computes columns 64 w .. 64 w + 63 of all 64 rows
  // (2 x 2 blocks of 32 x 32); a lane's A fragment is row (lane % 32),
  // k = k0 + 8 (lane / 32) .. +7, its B fragment column (lane % 32) likewise
  for (int l = 0; l < 3; ++l) {
    const int K = l == 0 ? NI : NHd;
    const __bf16* W = l == 0 ? W1 : (l == 1 ? W2 : W3);
    const float* bias = l == 0 ? b1 : (l == 1 ? b2 : b3);
    f32x16 acc[2][2];
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[rb][cb][r] = 0.0f;
    for (int k0 = 0; k0 < K; k0 += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
        a[rb] = *reinterpret_cast<const bf16x8*>(&Hs[(32 * rb + (lane & 31)) * kInfStride + k0 + 8 * (lane >> 5)]);
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
        b[cb] = *reinterpret_cast<const bf16x8*>(W + (int64_t)(64 * wave + 32 * cb + (lane & 31)) * K + k0 +
                                                 8 * (lane >> 5));
#pragma unroll
      for (int rb = 0; rb < 2; ++rb)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[rb], b[cb], acc[rb][cb], 0, 0, 0);
    }
    __syncthreads();  // every wave has read this layer's input
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb) {
        const int col = 64 * wave + 32 * cb + (lane & 31);
        const float bc = bias[col];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = 32 * rb + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
          Hs[row * kInfStride + col] = to_bf16(gelu_f(acc[rb][cb][r] + bc));
        }
      }
    __syncthreads();
  }
  // output layer: waves 0 and 1 take 32 rows each, columns 0..31 with zero
  // weights past the NO outputs (as k_gemm pads its B tile)
  if (wave < 2) {
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
    const int col = lane & 31;
    for (int k0 = 0; k0 < NHd; k0 += 16) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(&Hs[(32 * wave + (lane & 31)) * kInfStride + k0 + 8 * (lane >> 5)]);
      bf16x8 b;
      if (col < NO) {
        b = *reinterpret_cast<const bf16x8*>(W4 + (int64_t)col * NHd + k0 + 8 * (lane >> 5));
      } else {
#pragma unroll
        for (int t = 0; t < 8; ++t) b[t] = (__bf16)0.0f;
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
    }
    if (col < NO) {
      const float bc = b4[col];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t gr = r0 + 32 * wave + 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3);
        if (gr < rows) y[gr * NO + col] = acc[r] + bc;
      }
    }
  }
}

// ---- launchers ----

hipError_t launch_gemm(hipStream_t s, int epi, int M, int N, int K, const void* A, int64_t sam, int64_t sak,
                       const void* B, int64_t sbk, int64_t sbn, const float* bias, float* C, int64_t ldc,
                       void* H, int64_t ldh, const float* Zin, int64_t ldz) {
  if (M <= 0 || N <= 0) return hipSuccess;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM);
  const __bf16* a = (const __bf16*)A;
  const __bf16* b = (const __bf16*)B;
  __bf16* h = (__bf16*)H;
  switch (epi) {
    case EPI_STORE:
      hipLaunchKernelGGL(k_gemm<EPI_STORE>, grid, dim3(256), 0, s, M, N, K, a, sam, sak, b, sbk, sbn, bias, C, ldc,
                         h, ldh, Zin, ldz);
      break;
    case EPI_BIAS:
      hipLaunchKernelGGL(k_gemm<EPI_BIAS>, grid, dim3(256), 0, s, M, N, K, a, sam, sak, b, sbk, sbn, bias, C, ldc,
                         h, ldh, Zin, ldz);
      break;
    case EPI_BIAS_GELU:
      hipLaunchKernelGGL(k_gemm<EPI_BIAS_GELU>, grid, dim3(256), 0, s, M, N, K, a, sam, sak, b, sbk, sbn, bias, C,
                         ldc, h, ldh, Zin, ldz);
      break;
    case EPI_GELU_BWD:
      hipLaunchKernelGGL(k_gemm<EPI_GELU_BWD>, grid, dim3(256), 0, s, M, N, K, a, sam, sak, b, sbk, sbn, bias, C,
                         ldc, h, ldh, Zin, ldz);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_to_bf16(hipStream_t s, const float* x, void* y, int64_t n) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_to_bf16, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, x, (__bf16*)y, n);
  return hipGetLastError();
}

hipError_t launch_mse(hipStream_t s, const float* Y, const float* T, int64_t n, void* dY, float* partial,
                      float* loss) {
  const int np = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_mse, dim3(np), dim3(256), 0, s, Y, T, n, (__bf16*)dY, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || loss == nullptr) return e;
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(256), 0, s, partial, np, n, loss);
  return hipGetLastError();
}

hipError_t launch_colsum(hipStream_t s, const void* dZ, int64_t B, int N, float* db) {
  hipLaunchKernelGGL(k_colsum, dim3((N + 255) / 256), dim3(256), 0, s, (const __bf16*)dZ, B, N, db);
  return hipGetLastError();
}

hipError_t launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, void* pb, int64_t n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2) {
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, (__bf16*)pb, n, lr, b1,
                     b2, eps, bc1, bc2);
  return hipGetLastError();
}

// w[l], b[l]: the BF16 weights and FP32 biases of layer l (row-major
// [out][in]); every weight pointer 16-byte aligned.
hipError_t launch_mlp_infer(hipStream_t s, const float* x, int64_t rows, const void* const* w,
                            const float* const* b, float* y) {
  if (rows <= 0) return hipSuccess;
  for (int l = 0; l < 4; ++l)
    if (((uintptr_t)w[l] & 15) != 0) return hipErrorInvalidValue;
  const int64_t grid = (rows + kInfRows - 1) / kInfRows;
  if (grid > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)grid), dim3(256), 0, s, x, rows, (const __bf16*)w[0], b[0],
                     (const __bf16*)w[1], b[1], (const __bf16*)w[2], b[2], (const __bf16*)w[3], b[3], y);
  return hipGetLastError();
}

}  // namespace ddm
