// Step one: the 2-D transform of every frame (paper, section "The algorithm":
// the FFTs of all images are computed once and stored, after which every wave
// vector is independent).
//
//   k_row: real rows -> half spectra along x.  Two real rows y, y+1 are packed
//          into one complex sequence z = r_y + i r_{y+1}; one complex FFT of
//          length W gives both: R_y(k) = (Z_k + conj Z_{W-k})/2 and
//          R_{y+1}(k) = (Z_k - conj Z_{W-k})/(2i).  Optionally subtracts frame 0
//          first (integer difference, exact in FP32).
//          Output: intermediate [frame][y][kxw] complex FP32.
//   k_col: complex FFT of length H down each kx column, then a direct write of
//          the kept wave vectors into the q-blocked spectra store
//          [block][t][QB] (the transpose to time series is this write).
#include <hip/hip_fp16.h>

#include "fft.hpp"
#include "internal.hpp"

namespace ddm {

// Unpack the pixels of one 16-byte load.
template <typename PIX> struct Pix16;
template <> struct Pix16<uint16_t> {
  static constexpr int n = 8;
  __device__ __forceinline__ static int get(const uint4& a, int k) {
    const uint32_t w = (k < 2) ? a.x : (k < 4) ? a.y : (k < 6) ? a.z : a.w;
    return (int)((w >> (16 * (k & 1))) & 0xFFFFu);
  }
};
template <> struct Pix16<uint8_t> {
  static constexpr int n = 16;
  __device__ __forceinline__ static int get(const uint4& a, int k) {
    const uint32_t w = (k < 4) ? a.x : (k < 8) ? a.y : (k < 12) ? a.z : a.w;
    return (int)((w >> (8 * (k & 3))) & 0xFFu);
  }
};

template <int W, int E, typename PIX>
__global__ void __launch_bounds__(256) k_row(const PIX* __restrict__ frames, int H, int64_t t0,
                                             int precondition, float2* __restrict__ inter, int kxw,
                                             const float2* __restrict__ tw, int tws) {
  constexpr int T = W / E;
  constexpr bool WAVE = (T <= 64) && (64 % T == 0);  // a transform inside one wavefront
  constexpr int WL = lds_len<true>(W);
  extern __shared__ float2 lds_row[];
  const int p = threadIdx.x / T;          // transform (row pair) within the workgroup
  const int tid = threadIdx.x % T;
  const int nt = blockDim.x / T;
  const int ybase = blockIdx.x * nt * 2;
  const int y0 = ybase + 2 * p;
  const int64_t t = t0 + blockIdx.y;

  // Stage rows [ybase, ybase + 2 nt) of frame t (minus frame 0) with 16-byte
  // loads: row 2p' + c of the block becomes component c of transform p'.
  {
    constexpr int V = Pix16<PIX>::n;
    const uint4* src = reinterpret_cast<const uint4*>(frames + ((size_t)t * H + ybase) * W);
    const uint4* ref = reinterpret_cast<const uint4*>(frames + (size_t)ybase * W);
    const int nvec = 2 * nt * W / V;
    float* f = reinterpret_cast<float*>(lds_row);
#pragma unroll 4
    for (int g = threadIdx.x; g < nvec; g += blockDim.x) {
      const uint4 a = src[g];
      uint4 b = make_uint4(0u, 0u, 0u, 0u);
      if (precondition) b = ref[g];
      const int pix = g * V;
      const int r = pix / W, n0 = pix % W;
      float* dst = f + 2 * ((r >> 1) * WL) + (r & 1);
#pragma unroll
      for (int k = 0; k < V; ++k) {
        const int n = n0 + k;
        dst[2 * LdsView<1, true>::slot(n)] = (float)(Pix16<PIX>::get(a, k) - Pix16<PIX>::get(b, k));
      }
    }
  }
  __syncthreads();

  LdsView<1, true> buf{lds_row + p * WL};
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = buf[tid + e * T];
  group_sync<WAVE>();
  fft_forward<W, E, 1, true, WAVE>(v, buf, tid, tw, tws);
#pragma unroll
  for (int e = 0; e < E; ++e) buf[tid + e * T] = v[e];
  group_sync<WAVE>();
  float2* o0 = inter + ((size_t)blockIdx.y * H + y0) * kxw;
  float2* o1 = o0 + kxw;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * T;
    if (k < kxw) {
      const float2 zk = buf[k];
      const float2 zm = buf[(W - k) % W];
      o0[k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
      o1[k] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
    }
  }
}

// F16: store complex FP16 scaled by 2^qexp[q] (round to nearest even),
// clamping |value| > 65504 and counting each clamped component in *sat.
template <int H, int E, int CW, bool F16>
__global__ void __launch_bounds__(1024) k_col(const float2* __restrict__ inter, int kxw, int64_t t0,
                                              int N, const int32_t* __restrict__ qoff,
                                              const int32_t* __restrict__ kxcnt, int64_t q_lo,
                                              int64_t q_hi, int qb, void* __restrict__ spec,
                                              const int32_t* __restrict__ qexp, int32_t* sat,
                                              const float2* __restrict__ tw, int tws) {
  constexpr int T = H / E;
  extern __shared__ float2 lds_col[];
  const int c = threadIdx.x % CW;
  const int tid = threadIdx.x / CW;
  const int kx = blockIdx.x * CW + c;
  const float2* src = inter + (size_t)blockIdx.y * H * kxw + kx;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[(size_t)(tid + e * T) * kxw];
  LdsView<CW> buf{lds_col + c};
  fft_forward<H, E, CW>(v, buf, tid, tw, tws);
  const int64_t t = t0 + blockIdx.y;
  int nsat = 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int ky = tid + e * T;
    if (kx < kxcnt[ky]) {
      const int64_t q = (int64_t)qoff[ky] + kx;
      if (q >= q_lo && q < q_hi) {
        const int64_t j = q - q_lo;
        const size_t at = ((j / qb) * N + t) * qb + (j % qb);
        if constexpr (F16) {
          float re = ldexpf(v[e].x, qexp[q]), im = ldexpf(v[e].y, qexp[q]);
          const float lim = 65504.0f;
          if (!(fabsf(re) <= lim)) { re = copysignf(lim, re); ++nsat; }
          if (!(fabsf(im) <= lim)) { im = copysignf(lim, im); ++nsat; }
          reinterpret_cast<__half2*>(spec)[at] = __halves2half2(__float2half_rn(re), __float2half_rn(im));
        } else {
          reinterpret_cast<float2*>(spec)[at] = v[e];
        }
      }
    }
  }
  if (F16 && nsat > 0) atomicAdd(sat, nsat);
}

// Per-q exponent of the FP16 store: the largest |component| over the pilot
// frames is mapped into (2^10, 2^11], leaving a factor 32 of headroom below
// the FP16 maximum for the other frames.  pilot: [nq][np] complex FP32.
__global__ void k_qexp(const float2* __restrict__ pilot, int np, int64_t nq, int32_t* __restrict__ qexp) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nq) return;
  float mx = 0.0f;
  for (int i = 0; i < np; ++i) {
    const float2 a = pilot[q * np + i];
    mx = fmaxf(mx, fmaxf(fabsf(a.x), fabsf(a.y)));
  }
  int e = 0;
  if (mx > 0.0f && isfinite(mx)) {
    int ex;
    const float m = frexpf(mx, &ex);  // mx = m 2^ex, m in [0.5, 1)
    const int c = (m == 0.5f) ? ex - 1 : ex;  // ceil(log2 mx)
    e = 11 - c;
  }
  qexp[q] = e;
}

__global__ void k_fill_i32s(int32_t* p, int64_t n, int32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

bool supported_spatial(int n) {
  switch (n) {
    case 16: case 32: case 64: case 128: case 256: case 512: case 1024: case 2048: case 4096:
    case 48: case 96: case 192: case 384: case 768: case 1536: case 3072:
      return true;
    default:
      return false;
  }
}

static int spatial_E(int n) { return (n % 3 == 0) ? 24 : 16; }

RowCfg row_cfg(int W, int H) {
  RowCfg c;
  c.W = W;
  c.E = spatial_E(W);
  c.T = W / c.E;
  int nt = 256 / c.T;
  if (nt < 1) nt = 1;
  while (nt > 1 && ((H / 2) % nt) != 0) nt >>= 1;
  c.nt = nt;
  c.lds = (size_t)nt * (W + W / 16) * sizeof(float2);
  return c;
}

ColCfg col_cfg(int H) {
  ColCfg c;
  c.H = H;
  c.E = spatial_E(H);
  c.T = H / c.E;
  int cw = 16;
  while (cw > 1 && (size_t)cw * H * sizeof(float2) > 131072) cw >>= 1;
  c.cw = cw;
  c.lds = (size_t)cw * H * sizeof(float2);
  return c;
}

template <int W, typename PIX>
static hipError_t row_go(hipStream_t s, const void* frames, int H, int64_t t0, int nframes,
                         int pre, float2* inter, int kxw, const float2* tw, int tws) {
  constexpr int E = (W % 3 == 0) ? 24 : 16;
  RowCfg c = row_cfg(W, H);
  dim3 grid(H / (2 * c.nt), nframes);
  hipLaunchKernelGGL((k_row<W, E, PIX>), grid, dim3(c.nt * c.T), c.lds, s,
                     (const PIX*)frames, H, t0, pre, inter, kxw, tw, tws);
  return hipGetLastError();
}

template <typename PIX>
static hipError_t row_dispatch(hipStream_t s, const void* f, int W, int H, int64_t t0, int nf, int pre,
                               float2* inter, int kxw, const float2* tw, int tws) {
  switch (W) {
#define ROW_CASE(n) case n: return row_go<n, PIX>(s, f, H, t0, nf, pre, inter, kxw, tw, tws);
    ROW_CASE(16) ROW_CASE(32) ROW_CASE(64) ROW_CASE(128) ROW_CASE(256) ROW_CASE(512)
    ROW_CASE(1024) ROW_CASE(2048) ROW_CASE(4096)
    ROW_CASE(48) ROW_CASE(96) ROW_CASE(192) ROW_CASE(384) ROW_CASE(768) ROW_CASE(1536) ROW_CASE(3072)
#undef ROW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_row(hipStream_t s, int pixel, const void* frames, int W, int H, int64_t t0,
                      int nframes, int precondition, float2* inter, int kxw, const float2* tw,
                      int tws) {
  if (pixel == DDM_PIX_U8)
    return row_dispatch<uint8_t>(s, frames, W, H, t0, nframes, precondition, inter, kxw, tw, tws);
  return row_dispatch<uint16_t>(s, frames, W, H, t0, nframes, precondition, inter, kxw, tw, tws);
}

template <int H>
static hipError_t col_go(hipStream_t s, const float2* inter, int kxw, int ntiles, int64_t t0,
                         int nframes, int N, QTable qt, int64_t q_lo, int64_t q_hi, int qb,
                         SpecOut out, const float2* tw, int tws) {
  constexpr int E = (H % 3 == 0) ? 24 : 16;
  constexpr int T = H / E;
  constexpr int CW = (16 * H * 8 <= 131072) ? 16 : (8 * H * 8 <= 131072) ? 8 : 4;
  dim3 grid(ntiles, nframes);
  if (out.qexp != nullptr)
    hipLaunchKernelGGL((k_col<H, E, CW, true>), grid, dim3(CW * T), (size_t)CW * H * sizeof(float2), s,
                       inter, kxw, t0, N, qt.qoff, qt.kxcnt, q_lo, q_hi, qb, out.spec, out.qexp, out.sat, tw,
                       tws);
  else
    hipLaunchKernelGGL((k_col<H, E, CW, false>), grid, dim3(CW * T), (size_t)CW * H * sizeof(float2), s,
                       inter, kxw, t0, N, qt.qoff, qt.kxcnt, q_lo, q_hi, qb, out.spec, nullptr, nullptr, tw,
                       tws);
  return hipGetLastError();
}

hipError_t launch_col(hipStream_t s, const float2* inter, int H, int kxw, int ntiles, int64_t t0,
                      int nframes, int N, QTable qt, int64_t q_lo, int64_t q_hi, int qb,
                      SpecOut out, const float2* tw, int tws) {
  switch (H) {
#define COL_CASE(n) case n: return col_go<n>(s, inter, kxw, ntiles, t0, nframes, N, qt, q_lo, q_hi, qb, out, tw, tws);
    COL_CASE(16) COL_CASE(32) COL_CASE(64) COL_CASE(128) COL_CASE(256) COL_CASE(512)
    COL_CASE(1024) COL_CASE(2048) COL_CASE(4096)
    COL_CASE(48) COL_CASE(96) COL_CASE(192) COL_CASE(384) COL_CASE(768) COL_CASE(1536) COL_CASE(3072)
#undef COL_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_qexp(hipStream_t s, const float2* pilot, int np, int64_t nq, int32_t* qexp) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qexp, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, pilot, np, nq, qexp);
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32s, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ddm
