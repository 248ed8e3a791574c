// Step one: the 2-D transform of every frame (paper, section "The algorithm":
// the FFTs of all images are computed once and stored, after which every wave
// vector is independent).
//
//   k_row: real rows -> half spectra along x.  Two real rows y, y+1 are packed
//          into one complex sequence z = r_y + i r_{y+1}; one complex FFT of
//          length W gives both: R_y(k) = (Z_k + conj Z_{W-k})/2 and
//          R_{y+1}(k) = (Z_k - conj Z_{W-k})/(2i).  Optionally subtracts frame 0
//          first (integer difference, exact in FP32).
//          Output: intermediate [frame][y][kxw] complex FP32.  When the Nyquist
//          column kx = W/2 is needed ("pack"), the two real values R_y(0) and
//          R_y(W/2) share slot 0 as R_y(0) + i R_y(W/2), so a row holds W/2
//          values instead of W/2 + 1.
//   k_col: complex FFT of length H down each kx column, then a direct write of
//          the kept wave vectors into the q-blocked spectra store
//          [block][t][QB] (the transpose to time series is this write).  A
//          packed column 0 is separated after its transform: with
//          C = FFT(a + i b) of two real columns, A_k = (C_k + conj C_{-k})/2 and
//          B_k = (C_k - conj C_{-k})/(2i).
#include <hip/hip_fp16.h>

#include "fft.hpp"
#include "internal.hpp"

namespace ddm {

// Eight pixels of one row, loaded at once (16 bytes of uint16, 8 of uint8).
template <typename PIX> struct Pix8;
template <> struct Pix8<uint16_t> {
  using vec = uint4;
  __device__ __forceinline__ static int get(const vec& a, int k) {
    const uint32_t w = (k < 2) ? a.x : (k < 4) ? a.y : (k < 6) ? a.z : a.w;
    return (int)((w >> (16 * (k & 1))) & 0xFFFFu);
  }
  __device__ __forceinline__ static vec zero() { return make_uint4(0u, 0u, 0u, 0u); }
};
template <> struct Pix8<uint8_t> {
  using vec = uint2;
  __device__ __forceinline__ static int get(const vec& a, int k) {
    const uint32_t w = (k < 4) ? a.x : a.y;
    return (int)((w >> (8 * (k & 3))) & 0xFFu);
  }
  __device__ __forceinline__ static vec zero() { return make_uint2(0u, 0u); }
};

template <int W, int E, typename PIX>
__global__ void __launch_bounds__(256) k_row(const PIX* __restrict__ frames, int H, int t0,
                                             int precondition, float2* __restrict__ inter, int kxw,
                                             int pack, const float2* __restrict__ tw, int tws) {
  constexpr int T = W / E;
  constexpr bool WAVE = (T <= 64) && (64 % T == 0);  // a transform inside one wavefront
  constexpr int WL = lds_len<true>(W);
  constexpr int CPR = W / 8;  // 8-pixel chunks per row
  using P8 = Pix8<PIX>;
  using vec = typename P8::vec;
  extern __shared__ float2 lds_row[];
  const int p = threadIdx.x / T;  // transform (row pair) within the workgroup
  const int tid = threadIdx.x % T;
  const int nt = blockDim.x / T;
  const int ybase = blockIdx.x * nt * 2;
  const int t = t0 + blockIdx.y;

  // Stage the rows of the block: chunk g = 8 pixels of rows 2p', 2p'+1 (minus
  // frame 0), written as 8 consecutive complex values of transform p' (inside
  // one padding group, so one contiguous 64-byte run).
  {
    const PIX* src = frames + ((size_t)t * H + ybase) * W;
    const PIX* ref = frames + (size_t)ybase * W;
    for (int g = threadIdx.x; g < nt * CPR; g += blockDim.x) {
      const int pp = g / CPR, n0 = (g % CPR) * 8;
      const int off = 2 * pp * W + n0;
      const vec a0 = *reinterpret_cast<const vec*>(src + off);
      const vec a1 = *reinterpret_cast<const vec*>(src + off + W);
      vec b0 = P8::zero(), b1 = P8::zero();
      if (precondition) {
        b0 = *reinterpret_cast<const vec*>(ref + off);
        b1 = *reinterpret_cast<const vec*>(ref + off + W);
      }
      float2* dst = lds_row + pp * WL + LdsView<1, true>::slot(n0);
#pragma unroll
      for (int k = 0; k < 8; ++k)
        dst[k] = make_float2((float)(P8::get(a0, k) - P8::get(b0, k)), (float)(P8::get(a1, k) - P8::get(b1, k)));
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
  const int y0 = ybase + 2 * p;
  float2* o0 = inter + ((size_t)blockIdx.y * H + y0) * kxw;
  float2* o1 = o0 + kxw;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * T;
    if (k < kxw) {
      const float2 zk = v[e];
      const float2 zm = buf[k == 0 ? 0 : W - k];
      if (k == 0 && pack) {
        const float2 zn = buf[W / 2];  // Z_{W/2}: R_y(W/2) = Re, R_{y+1}(W/2) = Im
        o0[0] = make_float2(zk.x, zn.x);
        o1[0] = make_float2(zk.y, zn.y);
      } else {
        o0[k] = make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y));
        o1[k] = make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x));
      }
    }
  }
}

// One value of the column transform into the spectra store: slot sl (group-
// local index j = sl - s_lo), time t, at [j / QB][N][QB].  F16: complex FP16
// scaled by 2^qexp[q] (round to nearest even), |value| > 65504 clamped and
// counted.
template <int QB, bool F16>
__device__ __forceinline__ void put_spec(void* __restrict__ spec, int sl, int s_lo, int s_hi, int N, int t,
                                         float2 val, int q, const int32_t* __restrict__ qexp, int& nsat) {
  if (sl < s_lo || sl >= s_hi) return;
  const int j = sl - s_lo;
  const size_t at = ((size_t)(j / QB) * (size_t)N + (size_t)t) * QB + (j % QB);
  if constexpr (F16) {
    const int ex = qexp[q];
    float re = ldexpf(val.x, ex), im = ldexpf(val.y, ex);
    const float lim = 65504.0f;
    if (!(fabsf(re) <= lim)) { re = copysignf(lim, re); ++nsat; }
    if (!(fabsf(im) <= lim)) { im = copysignf(lim, im); ++nsat; }
    reinterpret_cast<__half2*>(spec)[at] = __halves2half2(__float2half_rn(re), __float2half_rn(im));
  } else {
    reinterpret_cast<float2*>(spec)[at] = val;
  }
}

// Slots: kept (ky, kx) with kx < W/2 (or every kept kx without packing) sits
// in slot sbase[ky] + kx; the Nyquist value (ky, W/2) of a packed column sits
// in slot sN + ky, or sbase[ky] + W/2 when sN < 0.  kxnyq = W/2 when column 0
// of the intermediate carries R(0) + i R(W/2) (columns >= W/2 are then
// padding), else -1.  qoff[ky] + kx is the wave vector (FP16 scale index).
template <int H, int E, int CW, int QB, bool F16>
__global__ void __launch_bounds__(CW * (H / E)) k_col(const float2* __restrict__ inter, int kxw, int t0,
                                                      int N, const int32_t* __restrict__ qoff,
                                                      const int32_t* __restrict__ kxcnt,
                                                      const int32_t* __restrict__ sbase, int sN, int s_lo,
                                                      int s_hi, int kxnyq, void* __restrict__ spec,
                                                      const int32_t* __restrict__ qexp, int32_t* sat,
                                                      const float2* __restrict__ tw, int tws) {
  constexpr int T = H / E;
  extern __shared__ float2 lds_col[];
  const int c = threadIdx.x % CW;
  const int tid = threadIdx.x / CW;
  const int kx = blockIdx.x * CW + c;
  const int t = t0 + blockIdx.y;
  const float2* src = inter + (size_t)blockIdx.y * H * kxw + kx;
  float2 v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = src[(size_t)(tid + e * T) * kxw];
  // row tables of this thread's rows, fetched while the transform runs
  int rs[E], rc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    rs[e] = sbase[tid + e * T];
    rc[e] = kxcnt[tid + e * T];
  }
  LdsView<CW> buf{lds_col + c};
  fft_forward<H, E, CW>(v, buf, tid, tw, tws);
  int nsat = 0;
  const int kxlim = kxnyq > 0 ? kxnyq : 0x7FFFFFFF;  // packing: columns >= W/2 are padding
  const bool packed0 = kxnyq > 0 && blockIdx.x == 0;  // uniform over the workgroup
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (kx < rc[e] && kx < kxlim && !(packed0 && kx == 0))
      put_spec<QB, F16>(spec, rs[e] + kx, s_lo, s_hi, N, t, v[e], F16 ? qoff[tid + e * T] + kx : 0, qexp, nsat);
  }
  if (packed0) {
    // column 0 = FFT(R(0) + i R(W/2)): separate through LDS (every thread is
    // past the transform's last exchange once the barrier is passed)
    __syncthreads();
    if (c == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) buf[tid + e * T] = v[e];
    }
    __syncthreads();
    if (c == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int ky = tid + e * T;
        const float2 a = v[e], b = buf[ky == 0 ? 0 : H - ky];
        const int q0 = F16 ? qoff[ky] : 0;
        if (0 < rc[e])
          put_spec<QB, F16>(spec, rs[e], s_lo, s_hi, N, t,
                            make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y)), q0, qexp, nsat);
        if (kxnyq < rc[e])
          put_spec<QB, F16>(spec, sN >= 0 ? sN + ky : rs[e] + kxnyq, s_lo, s_hi, N, t,
                            make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x)), q0 + kxnyq, qexp, nsat);
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
static hipError_t row_go(hipStream_t s, const void* frames, int H, int t0, int nframes,
                         int pre, float2* inter, int kxw, int pack, const float2* tw, int tws) {
  constexpr int E = (W % 3 == 0) ? 24 : 16;
  RowCfg c = row_cfg(W, H);
  dim3 grid(H / (2 * c.nt), nframes);
  hipLaunchKernelGGL((k_row<W, E, PIX>), grid, dim3(c.nt * c.T), c.lds, s,
                     (const PIX*)frames, H, t0, pre, inter, kxw, pack, tw, tws);
  return hipGetLastError();
}

template <typename PIX>
static hipError_t row_dispatch(hipStream_t s, const void* f, int W, int H, int t0, int nf, int pre,
                               float2* inter, int kxw, int pack, const float2* tw, int tws) {
  switch (W) {
#define ROW_CASE(n) case n: return row_go<n, PIX>(s, f, H, t0, nf, pre, inter, kxw, pack, tw, tws);
    ROW_CASE(16) ROW_CASE(32) ROW_CASE(64) ROW_CASE(128) ROW_CASE(256) ROW_CASE(512)
    ROW_CASE(1024) ROW_CASE(2048) ROW_CASE(4096)
    ROW_CASE(48) ROW_CASE(96) ROW_CASE(192) ROW_CASE(384) ROW_CASE(768) ROW_CASE(1536) ROW_CASE(3072)
#undef ROW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_row(hipStream_t s, int pixel, const void* frames, int W, int H, int64_t t0,
                      int nframes, int precondition, float2* inter, int kxw, int pack, const float2* tw,
                      int tws) {
  if (pixel == DDM_PIX_U8)
    return row_dispatch<uint8_t>(s, frames, W, H, (int)t0, nframes, precondition, inter, kxw, pack, tw, tws);
  return row_dispatch<uint16_t>(s, frames, W, H, (int)t0, nframes, precondition, inter, kxw, pack, tw, tws);
}

template <int H>
static hipError_t col_go(hipStream_t s, const float2* inter, int kxw, int ntiles, int t0,
                         int nframes, int N, QTable qt, SlotMap sm, int s_lo, int s_hi, int qb, int kxnyq,
                         SpecOut out, const float2* tw, int tws) {
  constexpr int E = (H % 3 == 0) ? 24 : 16;
  constexpr int T = H / E;
  constexpr int CW = (16 * H * 8 <= 131072) ? 16 : (8 * H * 8 <= 131072) ? 8 : 4;
  static_assert(kSpecQB == 16, "the column transform is instantiated for blocks of 16");
  dim3 grid(ntiles, nframes);
  const size_t lds = (size_t)CW * H * sizeof(float2);
  if (out.qexp != nullptr) {
    if (qb != kSpecQB) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_col<H, E, CW, 16, true>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, out.qexp, out.sat, tw, tws);
  } else if (qb == kSpecQB) {
    hipLaunchKernelGGL((k_col<H, E, CW, 16, false>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, nullptr, nullptr, tw, tws);
  } else if (qb == 1) {
    hipLaunchKernelGGL((k_col<H, E, CW, 1, false>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, nullptr, nullptr, tw, tws);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_col(hipStream_t s, const float2* inter, int H, int kxw, int ntiles, int64_t t0,
                      int nframes, int N, QTable qt, SlotMap sm, int64_t s_lo, int64_t s_hi, int qb, int kxnyq,
                      SpecOut out, const float2* tw, int tws) {
  const int a = (int)t0, lo = (int)s_lo, hi = (int)s_hi;
  switch (H) {
#define COL_CASE(n) case n: return col_go<n>(s, inter, kxw, ntiles, a, nframes, N, qt, sm, lo, hi, qb, kxnyq, out, tw, tws);
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
