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

#include <algorithm>
#include <cstdlib>

#include "fft.hpp"
#include "internal.hpp"

namespace ddm {

typedef unsigned int v2u32 __attribute__((ext_vector_type(2)));

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

// Row item: rows [ybase, ybase + 2 nt) of frame t (nt row pairs, one per T
// threads; the caller's block holds nt * T threads) -> out rows [2 nt][kxw],
// out = the intermediate at row ybase.  lds: nt * lds_len(W) complex values.
// Non-temporal loads of the 8-pixel chunks (through native vector types).
__device__ __forceinline__ uint4 nt_load(const uint4* p) {
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  const u4 x = __builtin_nontemporal_load(reinterpret_cast<const u4*>(p));
  return make_uint4(x[0], x[1], x[2], x[3]);
}
__device__ __forceinline__ uint2 nt_load(const uint2* p) {
  const v2u32 x = __builtin_nontemporal_load(reinterpret_cast<const v2u32*>(p));
  return make_uint2(x[0], x[1]);
}

// ref0: frame 0 (subtracted when precondition).
template <int W, int E, typename PIX, bool NT = false>
__device__ __forceinline__ void row_item(const PIX* __restrict__ frames, const PIX* __restrict__ ref0, int H, int t,
                                         int ybase, int nt, int precondition, float2* __restrict__ out, int kxw,
                                         int pack, const float2* __restrict__ tw, int tws, float2* lds_row, int tx) {
  constexpr int T = W / E;
  constexpr bool WAVE = (T <= 64) && (64 % T == 0);  // a transform inside one wavefront
  constexpr int WL = lds_len<true>(W);
  constexpr int CPR = W / 8;  // 8-pixel chunks per row
  using P8 = Pix8<PIX>;
  using vec = typename P8::vec;
  const int p = tx / T;  // transform (row pair) within the block (tx = thread index)
  const int tid = tx % T;
  const int nthr = nt * T;

  // Stage the rows: chunk g = 8 pixels of rows 2p', 2p'+1 (minus frame 0),
  // written as 8 consecutive complex values of transform p' (inside one
  // padding group, so one contiguous 64-byte run).
  {
    const PIX* src = frames + ((size_t)t * H + ybase) * W;
    const PIX* ref = ref0 + (size_t)ybase * W;
    for (int g = tx; g < nt * CPR; g += nthr) {
      const int pp = g / CPR, n0 = (g % CPR) * 8;
      const int off = 2 * pp * W + n0;
      vec a0, a1;
      if constexpr (NT) {  // frames are read once: stream them past the L2
        a0 = nt_load(reinterpret_cast<const vec*>(src + off));
        a1 = nt_load(reinterpret_cast<const vec*>(src + off + W));
      } else {
        a0 = *reinterpret_cast<const vec*>(src + off);
        a1 = *reinterpret_cast<const vec*>(src + off + W);
      }
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
  float2* o0 = out + (size_t)(2 * p) * kxw;
  float2* o1 = o0 + kxw;
  auto put = [&](float2* o, int k, float2 val) { o[k] = val; };
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int k = tid + e * T;
    if (k < kxw) {
      const float2 zk = v[e];
      const float2 zm = buf[k == 0 ? 0 : W - k];
      if (k == 0 && pack) {
        const float2 zn = buf[W / 2];  // Z_{W/2}: R_y(W/2) = Re, R_{y+1}(W/2) = Im
        put(o0, 0, make_float2(zk.x, zn.x));
        put(o1, 0, make_float2(zk.y, zn.y));
      } else {
        put(o0, k, make_float2(0.5f * (zk.x + zm.x), 0.5f * (zk.y - zm.y)));
        put(o1, k, make_float2(0.5f * (zk.y + zm.y), -0.5f * (zk.x - zm.x)));
      }
    }
  }
}

template <int W, int E, typename PIX>
__global__ void __launch_bounds__(256) k_row(const PIX* __restrict__ frames, const PIX* __restrict__ ref0, int H,
                                             int t0,
                                             const int32_t* __restrict__ tsel, int precondition,
                                             float2* __restrict__ inter, int kxw, int pack,
                                             const float2* __restrict__ tw, int tws) {
  extern __shared__ float2 lds_row[];
  const int nt = blockDim.x / (W / E);
  const int ybase = blockIdx.x * nt * 2;
  // frame t0 + z, or the z-th entry of the frame list
  const int t = (tsel != nullptr) ? tsel[blockIdx.y] : t0 + (int)blockIdx.y;
  row_item<W, E, PIX>(frames, ref0, H, t, ybase, nt, precondition,
                      inter + ((size_t)blockIdx.y * H + ybase) * kxw, kxw, pack, tw, tws, lds_row, threadIdx.x);
}

// One value of the column transform into the spectra store: slot sl (group-
// local index j = sl - s_lo), time t, at [j / QB][N][QB].  F16: complex FP16
// scaled by 2^ex, ex the wave vector's exponent (round to nearest even),
// |value| > 65504 clamped and counted.
// NT: non-temporal stores (streamed past the L2 without displacing what it holds).
template <int QB, bool F16, bool NT = false>
__device__ __forceinline__ void put_spec(void* __restrict__ spec, int sl, int s_lo, int s_hi, int N, int t,
                                         float2 val, int ex, int& nsat) {
  if (sl < s_lo || sl >= s_hi) return;
  const int j = sl - s_lo;
  const size_t at = ((size_t)(j / QB) * (size_t)N + (size_t)t) * QB + (j % QB);
  if constexpr (F16) {
    float re = ldexpf(val.x, ex), im = ldexpf(val.y, ex);
    const float lim = 65504.0f;
    if (!(fabsf(re) <= lim)) { re = copysignf(lim, re); ++nsat; }
    if (!(fabsf(im) <= lim)) { im = copysignf(lim, im); ++nsat; }
    const __half2 h = __halves2half2(__float2half_rn(re), __float2half_rn(im));
    if constexpr (NT)
      __builtin_nontemporal_store(__builtin_bit_cast(uint32_t, h), reinterpret_cast<uint32_t*>(spec) + at);
    else
      reinterpret_cast<__half2*>(spec)[at] = h;
  } else {
    if constexpr (NT) {
      __builtin_nontemporal_store(val.x, reinterpret_cast<float*>(spec) + 2 * at);
      __builtin_nontemporal_store(val.y, reinterpret_cast<float*>(spec) + 2 * at + 1);
    } else {
      reinterpret_cast<float2*>(spec)[at] = val;
    }
  }
}

// Slots: kept (ky, kx) with kx < W/2 (or every kept kx without packing) sits
// in slot sbase[ky] + kx; the Nyquist value (ky, W/2) of a packed column sits
// in slot sN + ky, or sbase[ky] + W/2 when sN < 0.  kxnyq = W/2 when column 0
// of the intermediate carries R(0) + i R(W/2) (columns >= W/2 are then
// padding), else -1.  F16: qgrid[ky qgw + kx] (qgw = W/2 + 1) is the FP16
// exponent of wave vector (ky, kx).
// Column item, in two parts.  col_load: this thread's E values of column
// kx of one frame's intermediate (BYPASS: reads that skip the CU's L1, for
// data written by other workgroups during the same launch).
template <int H, int E, int CW, bool BYPASS>
__device__ __forceinline__ void col_load(float2 (&v)[E], const float2* __restrict__ frame_inter, int kxw, int kx,
                                         int tid) {
  constexpr int T = H / E;
  if constexpr (BYPASS) {
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float2*>(frame_inter), (short)0, (int)((size_t)H * kxw * sizeof(float2)), 0x00020000);
#pragma unroll
    for (int e = 0; e < E; ++e)
      v[e] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                            r, (uint32_t)(((tid + e * T) * kxw + kx) * 8), 0, 0x10 /* sc1 */));
  } else {
    const float2* src = frame_inter + kx;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[(size_t)(tid + e * T) * kxw];
  }
}

// col_fft_store: FFT of the loaded column tile (column c of CW), then the
// kept values into the spectra store at time t.
template <int H, int E, int CW, int QB, bool F16, bool NT = false>
__device__ __forceinline__ void col_fft_store(float2 (&v)[E], int tile, int t, int N,
                                              const int32_t* __restrict__ qoff, const int32_t* __restrict__ kxcnt,
                                              const int32_t* __restrict__ sbase, int sN, int s_lo, int s_hi,
                                              int kxnyq, void* __restrict__ spec, const int8_t* __restrict__ qgrid,
                                              int qgw, int& nsat, const float2* __restrict__ tw, int tws,
                                              float2* lds_col, int tx) {
  constexpr int T = H / E;
  const int c = tx % CW;
  const int tid = tx / CW;
  const int kx = tile * CW + c;
  // row tables of this thread's rows
  int rs[E], rc[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    rs[e] = sbase[tid + e * T];
    rc[e] = kxcnt[tid + e * T];
  }
  // F16: this thread's exponents, loaded before the transform so that their
  // latency hides behind it; four bytes per register
  uint32_t exq[(E + 3) / 4];
  if constexpr (F16) {
#pragma unroll
    for (int i = 0; i < (E + 3) / 4; ++i) exq[i] = 0u;
    if (kx < qgw) {
#pragma unroll
      for (int e = 0; e < E; ++e)
        exq[e / 4] |= (uint32_t)(uint8_t)qgrid[(size_t)(tid + e * T) * qgw + kx] << (8 * (e % 4));
    }
  }
  auto ex_of = [&](int e) { return F16 ? (int)(int8_t)(exq[e / 4] >> (8 * (e % 4))) : 0; };
  LdsView<CW> buf{lds_col + c};
  fft_forward<H, E, CW>(v, buf, tid, tw, tws);
  const int kxlim = kxnyq > 0 ? kxnyq : 0x7FFFFFFF;  // packing: columns >= W/2 are padding
  const bool packed0 = kxnyq > 0 && tile == 0;        // uniform over the workgroup
#pragma unroll
  for (int e = 0; e < E; ++e) {
    if (kx < rc[e] && kx < kxlim && !(packed0 && kx == 0))
      put_spec<QB, F16, NT>(spec, rs[e] + kx, s_lo, s_hi, N, t, v[e], ex_of(e), nsat);
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
        if (0 < rc[e])
          put_spec<QB, F16, NT>(spec, rs[e], s_lo, s_hi, N, t,
                            make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y)), ex_of(e), nsat);
        if (kxnyq < rc[e])
          put_spec<QB, F16, NT>(spec, sN >= 0 ? sN + ky : rs[e] + kxnyq, s_lo, s_hi, N, t,
                            make_float2(0.5f * (a.y + b.y), -0.5f * (a.x - b.x)),
                            F16 ? (int)qgrid[(size_t)ky * qgw + kxnyq] : 0, nsat);
      }
    }
  }
}

template <int H, int E, int CW, int QB, bool F16>
__global__ void __launch_bounds__(CW * (H / E)) k_col(const float2* __restrict__ inter, int kxw, int t0,
                                                      int N, const int32_t* __restrict__ qoff,
                                                      const int32_t* __restrict__ kxcnt,
                                                      const int32_t* __restrict__ sbase, int sN, int s_lo,
                                                      int s_hi, int kxnyq, void* __restrict__ spec,
                                                      const int8_t* __restrict__ qgrid, int qgw, int32_t* sat,
                                                      const float2* __restrict__ tw, int tws) {
  extern __shared__ float2 lds_col[];
  float2 v[E];
  col_load<H, E, CW, false>(v, inter + (size_t)blockIdx.y * H * kxw, kxw, blockIdx.x * CW + threadIdx.x % CW,
                            threadIdx.x / CW);
  int nsat = 0;
  col_fft_store<H, E, CW, QB, F16>(v, blockIdx.x, t0 + blockIdx.y, N, qoff, kxcnt, sbase, sN, s_lo, s_hi, kxnyq,
                                   spec, qgrid, qgw, nsat, tw, tws, lds_col, threadIdx.x);
  if (F16 && nsat > 0) atomicAdd(sat, nsat);
}

// ---------------------------------------------------------------------------
// Step one in one persistent launch, for square frames up to 512 x 512.  Each
// XCD runs its own ordered stream of items: step s holds the NR row items of
// slot s (a frame claimed from a global counter) and then the NC column items
// of slot s - lag, so that column items find their rows done instead of
// waiting for them.  Row items write the frame's intermediate into one of
// nbufs buffers of that XCD (nbufs > lag); column items read it back (loads
// that skip the CU's L1; from the XCD's L2 or the Infinity Cache) and write
// the spectra store.  A workgroup takes the
// next ticket of its XCD and waits only for items with lower tickets of the
// same XCD (column items: the slot's rows; row items: the columns of the slot
// that last used the buffer; a slot's frame claim: the previous slot's claim),
// so every wait ends whatever the residency; each
// wait is also bounded, and a wait that runs out sets *err (reported by the
// host) instead of hanging.  Control words per XCD: ticket, then per slot the
// claimed frame (kUnset until published), rows done and columns done.
// ---------------------------------------------------------------------------
// Default frame buffers per XCD and steps between a slot's rows and its
// columns (512x512 x 1024 frames: 3 buffers and lag 1 0.92 ms, 4 and 2 0.83 ms,
// 6 and 3 0.81 ms; 2 and 1 1.46 ms).  Buffers must exceed the lag.
constexpr int kStep1Bufs = 6;
constexpr int kStep1Lag = 3;
constexpr int kUnset = -2;
// bound of one wait, in ticks of the 100 MHz constant clock (0.2 s)
constexpr uint64_t kWaitTicks = 20000000ull;

// Every access to the control words is an atomic read-modify-write (a poll
// adds 0), so that writers and pollers meet at the same point of the memory
// system; a poll that bypassed the cache while the update sat in the XCD's L2
// would never see it.
// (the zero is opaque to the compiler, which would otherwise turn the add of 0
// into a plain load)
__device__ __forceinline__ int ctl_read(int* p) {
  int zero = 0;
  asm volatile("" : "+v"(zero));
  return atomicAdd(p, zero);
}

// Wait for *p != kUnset (returns it), or *p >= target; -1 / false once the
// error flag is set, by this wait running out or by any other.
__device__ __forceinline__ int spin_value(int* p, int* err) {
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int v = ctl_read(p);
    if (v != kUnset) return v;
    if (ctl_read(err) != 0) return -1;
    if (wall_clock64() - t0 > kWaitTicks) {
      atomicExch(err, 1);
      return -1;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

__device__ __forceinline__ bool spin_ge(int* p, int target, int* err) {
  const uint64_t t0 = wall_clock64();
  for (;;) {
    if (ctl_read(p) >= target) return true;
    if (ctl_read(err) != 0) return false;
    if (wall_clock64() - t0 > kWaitTicks) {
      atomicExch(err, 1);
      return false;
    }
    __builtin_amdgcn_s_sleep(4);
  }
}

template <int W, int E, typename PIX, bool F16>
__global__ void __launch_bounds__(16 * (W / E)) k_step1(const PIX* __restrict__ frames, int N, int precondition,
                                                         float2* __restrict__ bufs, int kxw, int ncol_tiles,
                                                         int pack, int kxnyq, const int32_t* __restrict__ qoff,
                                                         const int32_t* __restrict__ kxcnt,
                                                         const int32_t* __restrict__ sbase, int sN, int s_lo,
                                                         int s_hi, void* __restrict__ spec,
                                                         const int8_t* __restrict__ qgrid, int qgw, int32_t* sat,
                                                         const float2* __restrict__ twW,
                                                         const float2* __restrict__ twH, int* __restrict__ ctl,
                                                         int maxslots, int nbufs, int lag) {
  constexpr int H = W;
  constexpr int T = W / E;
  constexpr int CW = 16;
  constexpr int NTR = CW;  // row pairs per row item: the block has CW * T threads
  constexpr int NR = H / (2 * NTR);
  extern __shared__ float2 lds[];
  __shared__ int s_val, s_val2;
  const int NC = ncol_tiles;
  const int IPF = NR + NC;
  const size_t frame_elems = (size_t)H * kxw;
  // the XCD this wave runs on: hardware register XCC_ID (id 20), bits 3:0
  const int xcc = (int)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 7;
  int* mine = ctl + (size_t)xcc * (1 + 3 * maxslots);
  int* ticket = mine;
  int* fidx = mine + 1;
  int* rows = fidx + maxslots;
  int* cols = rows + maxslots;
  int* gframe = ctl + (size_t)8 * (1 + 3 * maxslots);
  int* err = gframe + 1;
  int nsat = 0;
  for (;;) {
    // ticket -> step s, position r: the row items of slot s, then the column
    // items of slot s - 1 (whose rows finished a step earlier)
    if (threadIdx.x == 0) s_val = atomicAdd(ticket, 1);
    __syncthreads();
    const int tk = s_val;
    __syncthreads();
    const int st = tk / IPF, r = tk % IPF;
    if (st + 1 >= maxslots) break;  // uniform
    if (threadIdx.x == 0) {
      if (r == 0) {
        // claims are in slot order per XCD: a slot claims a frame only after
        // the previous slot (a lower ticket) got one, so once a slot is left
        // without a frame every later slot is too
        int f = -1;
        const int prev = (st == 0) ? 0 : spin_value(&fidx[st - 1], err);
        if (prev >= 0) {
          f = atomicAdd(gframe, 1);
          if (f >= N) f = -1;
        }
        atomicExch(&fidx[st], f);
      }
      const int fs = spin_value(&fidx[st], err);
      const int fp = (st < lag) ? -1 : spin_value(&fidx[st - lag], err);
      s_val = fs;
      s_val2 = fp;
    }
    __syncthreads();
    const int fs = s_val, fp = s_val2;
    __syncthreads();
    if (fs < 0 && fp < 0) break;  // uniform: nothing left in this step or after it
    const bool is_row = r < NR;
    const int k = is_row ? st : st - lag;  // the slot this item works on
    const int f = is_row ? fs : fp;
    if (f < 0) continue;  // uniform: this item's slot has no frame
    float2* buf = bufs + (size_t)(xcc * nbufs + k % nbufs) * frame_elems;
    // the thread index, made opaque per item so that the per-thread addresses
    // of both item kinds are not hoisted out of the loop (they would all stay
    // live in registers)
    // (the mask restores its range, the workgroup size being a power of two)
    static_assert(((16 * (W / E)) & (16 * (W / E) - 1)) == 0, "workgroup size is a power of two");
    unsigned utx = threadIdx.x;
    asm volatile("" : "+v"(utx));
    const int tx = (int)(utx & (unsigned)(16 * (W / E) - 1));
    if (is_row) {
      // the buffer is free once the columns of the slot that last used it
      // have read it (that slot has a frame: claims are in slot order)
      if (threadIdx.x == 0) s_val = (k < nbufs || spin_ge(&cols[k - nbufs], NC, err)) ? 1 : 0;
      __syncthreads();
      if (s_val == 0) break;  // uniform: a wait ran out
      const int ybase = r * 2 * NTR;
      row_item<W, E, PIX, true>(frames, frames, H, f, ybase, NTR, precondition, buf + (size_t)ybase * kxw, kxw,
                                pack, twW, 1, lds, tx);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the rows have reached L2
      __syncthreads();
      if (threadIdx.x == 0) atomicAdd(&rows[k], 1);
    } else {
      const int tile = r - NR;
      if (threadIdx.x == 0) s_val = spin_ge(&rows[k], NR, err) ? 1 : 0;
      __syncthreads();
      if (s_val == 0) break;  // uniform: a wait ran out
      // device-scope loads: this CU's L1 may still hold lines of the buffer
      // from the slot that used it before (an acquire fence at device scope
      // instead, with plain loads, measured 50% slower)
      float2 v[E];
      col_load<H, E, CW, true>(v, buf, kxw, tile * CW + tx % CW, tx / CW);
      asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // the tile is in registers
      __syncthreads();
      if (threadIdx.x == 0) atomicAdd(&cols[k], 1);
      col_fft_store<H, E, CW, kSpecQB, F16, true>(v, tile, f, N, qoff, kxcnt, sbase, sN, s_lo, s_hi, kxnyq, spec,
                                                  qgrid, qgw, nsat, twH, 1, lds, tx);
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
    // within int8 for the (ky, kx) grid; pilot maxima below 2^-89 (never
    // reached by transforms of integer frames) keep the factor 2^100
    e = e > 100 ? 100 : (e < -100 ? -100 : e);
  }
  qexp[q] = e;
}

// The exponents on the (ky, kx) grid the column transform stores from:
// qgrid[ky qgw + kx] = qexp[qoff[ky] + kx] for kept kx, else 0.
__global__ void k_qgrid(const int32_t* __restrict__ qexp, const int32_t* __restrict__ qoff,
                        const int32_t* __restrict__ kxcnt, int H, int qgw, int8_t* __restrict__ qgrid) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H * qgw) return;
  const int ky = i / qgw, kx = i % qgw;
  qgrid[i] = (int8_t)(kx < kxcnt[ky] ? qexp[qoff[ky] + kx] : 0);
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
static hipError_t row_go(hipStream_t s, const void* frames, const void* ref, int H, int t0, const int32_t* tsel,
                         int nframes, int pre, float2* inter, int kxw, int pack, const float2* tw, int tws) {
  constexpr int E = (W % 3 == 0) ? 24 : 16;
  RowCfg c = row_cfg(W, H);
  dim3 grid(H / (2 * c.nt), nframes);
  hipLaunchKernelGGL((k_row<W, E, PIX>), grid, dim3(c.nt * c.T), c.lds, s,
                     (const PIX*)frames, (const PIX*)ref, H, t0, tsel, pre, inter, kxw, pack, tw, tws);
  return hipGetLastError();
}

template <typename PIX>
static hipError_t row_dispatch(hipStream_t s, const void* f, const void* ref, int W, int H, int t0,
                               const int32_t* tsel, int nf, int pre, float2* inter, int kxw, int pack,
                               const float2* tw, int tws) {
  switch (W) {
#define ROW_CASE(n) case n: return row_go<n, PIX>(s, f, ref, H, t0, tsel, nf, pre, inter, kxw, pack, tw, tws);
    ROW_CASE(16) ROW_CASE(32) ROW_CASE(64) ROW_CASE(128) ROW_CASE(256) ROW_CASE(512)
    ROW_CASE(1024) ROW_CASE(2048) ROW_CASE(4096)
    ROW_CASE(48) ROW_CASE(96) ROW_CASE(192) ROW_CASE(384) ROW_CASE(768) ROW_CASE(1536) ROW_CASE(3072)
#undef ROW_CASE
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_row(hipStream_t s, int pixel, const void* frames, int W, int H, int64_t t0,
                      const int32_t* tsel, int nframes, int precondition, float2* inter, int kxw, int pack,
                      const float2* tw, int tws, const void* ref) {
  if (ref == nullptr) ref = frames;
  if (pixel == DDM_PIX_U8)
    return row_dispatch<uint8_t>(s, frames, ref, W, H, (int)t0, tsel, nframes, precondition, inter, kxw, pack, tw,
                                 tws);
  return row_dispatch<uint16_t>(s, frames, ref, W, H, (int)t0, tsel, nframes, precondition, inter, kxw, pack, tw,
                                tws);
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
  if (out.qgrid != nullptr) {
    if (qb != kSpecQB) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_col<H, E, CW, 16, true>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, out.qgrid, out.qgw, out.sat, tw,
                       tws);
  } else if (qb == kSpecQB) {
    hipLaunchKernelGGL((k_col<H, E, CW, 16, false>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, nullptr, 0, nullptr, tw, tws);
  } else if (qb == 1) {
    hipLaunchKernelGGL((k_col<H, E, CW, 1, false>), grid, dim3(CW * T), lds, s, inter, kxw, t0, N, qt.qoff,
                       qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, kxnyq, out.spec, nullptr, 0, nullptr, tw, tws);
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

// ---- fused step one ----
__host__ __device__ size_t step1_ctl_words(int maxslots) { return (size_t)8 * (1 + 3 * (size_t)maxslots) + 2; }

int step1_lag() {
  static const int env = [] {
    const char* v = std::getenv("DDM_STEP1_LAG");
    return v ? std::atoi(v) : 0;
  }();
  return (env >= 1 && env <= 4) ? env : kStep1Lag;
}

int step1_bufs() {
  static const int env = [] {
    const char* v = std::getenv("DDM_STEP1_BUFS");
    return v ? std::atoi(v) : 0;
  }();
  return (env >= 2 && env <= 8) ? env : kStep1Bufs;
}

bool step1_fusable(int W, int H, int ncol_tiles, int kxw) {
  if (W != H || kxw != 16 * ncol_tiles) return false;
  return W == 64 || W == 128 || W == 256 || W == 512;
}

// control words: per XCD [ticket, fidx[maxslots] = kUnset, rows[maxslots], cols[maxslots]], then
// the global frame counter and the error flag, all 0 except fidx; the error
// flag is set to err_init when err_init >= 0, else left as it is
__global__ void k_step1_init(int* ctl, int maxslots, int err_init) {
  const int64_t words = (int64_t)step1_ctl_words(maxslots);
  const int64_t per = 1 + 3 * (int64_t)maxslots;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = i % per;
    if (i == words - 1) {
      if (err_init >= 0) ctl[i] = err_init;
    } else {
      ctl[i] = (i < 8 * per && o >= 1 && o <= maxslots) ? kUnset : 0;
    }
  }
}

__global__ void k_copy_i32(const int32_t* __restrict__ src, int32_t* __restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

template <int W, typename PIX>
static hipError_t step1_go(hipStream_t s, const void* frames, int N, int pre, float2* bufs, int kxw, int ntiles,
                           int pack, int kxnyq, QTable qt, SlotMap sm, int s_lo, int s_hi, SpecOut out,
                           const float2* twW, const float2* twH, int* ctl, int maxslots, int nwg, int nbufs,
                           int lag) {
  constexpr int E = 16, T = W / E, CW = 16;
  const size_t lds = std::max((size_t)CW * lds_len<true>(W) * sizeof(float2), (size_t)CW * W * sizeof(float2));
  if (out.qgrid != nullptr)
    hipLaunchKernelGGL((k_step1<W, E, PIX, true>), dim3(nwg), dim3(CW * T), lds, s, (const PIX*)frames, N, pre,
                       bufs, kxw, ntiles, pack, kxnyq, qt.qoff, qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, out.spec,
                       out.qgrid, out.qgw, out.sat, twW, twH, ctl, maxslots, nbufs, lag);
  else
    hipLaunchKernelGGL((k_step1<W, E, PIX, false>), dim3(nwg), dim3(CW * T), lds, s, (const PIX*)frames, N, pre,
                       bufs, kxw, ntiles, pack, kxnyq, qt.qoff, qt.kxcnt, sm.sbase, sm.sN, s_lo, s_hi, out.spec,
                       nullptr, 0, nullptr, twW, twH, ctl, maxslots, nbufs, lag);
  return hipGetLastError();
}

int step1_workgroups(int W) {
  const size_t lds = std::max((size_t)16 * lds_len<true>(W) * sizeof(float2), (size_t)16 * W * sizeof(float2));
  const int per_cu = (int)std::min<size_t>(8, (160 * 1024) / lds);
  return 256 * std::max(1, per_cu);
}

hipError_t launch_step1(hipStream_t s, int pixel, const void* frames, int W, int N, int precondition,
                        float2* bufs, int kxw, int ntiles, int kxnyq, QTable qt, SlotMap sm, int64_t s_lo,
                        int64_t s_hi, SpecOut out, const float2* twW, const float2* twH, int* ctl, int maxslots,
                        int nwg, int nbufs, int err_init) {
  const int lag = step1_lag();
  // a row item waits for the columns of slot k - nbufs, which are in step
  // k - nbufs + lag: that must be an earlier step
  if (nbufs <= lag) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_step1_init, dim3(64), dim3(256), 0, s, ctl, maxslots, err_init);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int pack = kxnyq > 0, lo = (int)s_lo, hi = (int)s_hi;
#define S1_CASE(n)                                                                                              \
  case n:                                                                                                       \
    return pixel == DDM_PIX_U8                                                                                  \
               ? step1_go<n, uint8_t>(s, frames, N, precondition, bufs, kxw, ntiles, pack, kxnyq, qt, sm, lo,  \
                                      hi, out, twW, twH, ctl, maxslots, nwg, nbufs, lag)                        \
               : step1_go<n, uint16_t>(s, frames, N, precondition, bufs, kxw, ntiles, pack, kxnyq, qt, sm, lo, \
                                       hi, out, twW, twH, ctl, maxslots, nwg, nbufs, lag);
  switch (W) {
    S1_CASE(64) S1_CASE(128) S1_CASE(256) S1_CASE(512)
    default:
      return hipErrorInvalidValue;
  }
#undef S1_CASE
}

hipError_t launch_qgrid(hipStream_t s, const int32_t* qexp, QTable qt, int H, int qgw, int8_t* qgrid) {
  const int n = H * qgw;
  hipLaunchKernelGGL(k_qgrid, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, qexp, qt.qoff, qt.kxcnt, H, qgw,
                     qgrid);
  return hipGetLastError();
}

hipError_t launch_qexp(hipStream_t s, const float2* pilot, int np, int64_t nq, int32_t* qexp) {
  if (nq == 0) return hipSuccess;
  hipLaunchKernelGGL(k_qexp, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, s, pilot, np, nq, qexp);
  return hipGetLastError();
}

hipError_t launch_copy_i32(hipStream_t s, const int32_t* src, int32_t* dst, int n) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32s, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace ddm
