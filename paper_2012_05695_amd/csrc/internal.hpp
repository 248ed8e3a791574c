// Host-side internals shared by the C-ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddm.h"

namespace ddm {

// Spectra store between step one and step two: blocks of QB consecutive wave
// vectors (q order), each block [N][QB] complex, so that one time step of a
// block is a 128-byte run (FP32) written by the column transform and read by
// the time transform.
constexpr int kSpecQB = 16;

// Static LDS of the time kernel with qpw wave vectors per workgroup: staging
// and exchange buffers per wave vector, the L-entry twiddle table (L <= 1024),
// and room for the reduction scratch.
constexpr size_t time_lds_bytes(int L, int qpw) {
  return (size_t)qpw * (2 * (size_t)L + L / 8 + 1) * 8 + (L <= 1024 ? (size_t)L * 8 : 8) + 1024;
}

struct RowCfg {
  int W, E, T, nt;  // transform length, values/thread, threads/transform, transforms/WG
  size_t lds;
};
RowCfg row_cfg(int W, int H);

struct ColCfg {
  int H, E, T, cw;  // transform length, values/thread, threads/column, columns/WG
  size_t lds;
};
ColCfg col_cfg(int H);

// Device-side description of the kept wave vectors: for each ky row, the
// first q index of the row and the number of kept kx (kept kx are 0..cnt-1
// because k2 grows with kx).
struct QTable {
  const int32_t* qoff;   // [H] (device)
  const int32_t* kxcnt;  // [H] (device)
};

bool supported_spatial(int n);

// Fractional lags of the fit (at most 64), passed by value to the kernels.
struct LagSet {
  int K;
  float m[64];
};

struct LmParams {
  double lambda0, lambda_max, ftol, xtol, gtol, exact_fit;
  int max_iter;
};

enum : int32_t {
  LM_FLAG_CONVERGED = 1,
  LM_FLAG_MAXITER = 2,
  LM_FLAG_NONFINITE = 4,
  LM_FLAG_STALLED = 8,
  LM_FLAG_FALLBACK = 16,
  LM_FLAG_DEFAULT_START = 32
};

// ---- launchers (each returns hipSuccess or the launch error) ----
// pack: slot 0 of every row carries R(0) + i R(W/2) (the Nyquist column is needed).
// Frames t0 .. t0 + nframes - 1, or, when tsel (device, nframes entries) is not
// NULL, frames tsel[0 .. nframes - 1]; intermediate frame z holds the z-th.
// ref: frame 0 (subtracted when precondition); NULL means frames itself.
hipError_t launch_row(hipStream_t s, int pixel, const void* frames, int W, int H, int64_t t0,
                      const int32_t* tsel, int nframes, int precondition, float2* inter, int kxw, int pack,
                      const float2* tw, int tws, const void* ref = nullptr);

// Destination of the column transform: complex FP32, or complex FP16 scaled
// by 2^qexp[q] when qgrid (the same exponents on the (ky, kx) grid) is
// non-null (saturations counted in *sat).
struct SpecOut {
  void* spec;
  const int8_t* qgrid;  // FP16 store: exponents on the (ky, kx) grid, row stride qgw = W/2 + 1; null for FP32
  int32_t* sat;         // FP16 store: saturation counter
  int qgw;
};

// Slot of each kept wave vector in the spectra store: (ky, kx < W/2, or any
// kept kx without packing) -> sbase[ky] + kx; the Nyquist value (ky, W/2) ->
// sN + ky, or sbase[ky] + W/2 when sN < 0.  The plain layout is sbase = qoff.
struct SlotMap {
  const int32_t* sbase;  // [H] (device)
  int sN;
};

// Writes slots [s_lo, s_hi) of frames t0..t0+nframes-1.  qb: 16 (the blocked
// store) or 1 (plain [slot][N]); kxnyq: W/2 when the rows are packed, else -1.
// Slot and q indices must fit in int32.
hipError_t launch_col(hipStream_t s, const float2* inter, int H, int kxw, int ntiles,
                      int64_t t0, int nframes, int N, QTable qt, SlotMap sm, int64_t s_lo, int64_t s_hi,
                      int qb, int kxnyq, SpecOut out, const float2* tw, int tws);

// Fused step one (one persistent launch; row intermediates kept per XCD in
// nbufs >= 2 frame buffers of each of 8 XCDs at bufs; step1_bufs() is the
// default, DDM_STEP1_BUFS overrides).  Applies to square
// frames W = H in {64, 128, 256, 512} with full column tiles.  ctl:
// step1_ctl_words(maxslots) ints of device memory (initialised by the launch);
// maxslots >= N + nwg / (items per frame) + 4; the last word is an error flag
// (non-zero if a wait ran out), set by the launch to err_init when err_init >= 0
// (0 clears it; 1 makes every wait give up at once, so the kernel exits with its
// result invalid), else kept from the previous launch (a later launch then does
// no work).
bool step1_fusable(int W, int H, int ncol_tiles, int kxw);
int step1_bufs();
int step1_lag();  // steps between a slot's row items and its column items (DDM_STEP1_LAG overrides)
int step1_workgroups(int W);
__host__ __device__ size_t step1_ctl_words(int maxslots);
hipError_t launch_step1(hipStream_t s, int pixel, const void* frames, int W, int N, int precondition,
                        float2* bufs, int kxw, int ntiles, int kxnyq, QTable qt, SlotMap sm, int64_t s_lo,
                        int64_t s_hi, SpecOut out, const float2* twW, const float2* twH, int* ctl, int maxslots,
                        int nwg, int nbufs, int err_init);

hipError_t launch_qexp(hipStream_t s, const float2* pilot, int np, int64_t nq, int32_t* qexp);
hipError_t launch_qgrid(hipStream_t s, const int32_t* qexp, QTable qt, int H, int qgw, int8_t* qgrid);
hipError_t launch_fill_i32(hipStream_t s, int32_t* p, int64_t n, int32_t v);
hipError_t launch_copy_i32(hipStream_t s, const int32_t* src, int32_t* dst, int n);

// spec: the group's slots, complex FP32, or complex FP16 scaled by 2^qexp[q]
// when qexp is non-null (qexp indexed by wave vector q).  qmap: wave vector of
// each of the group's slots (-1: none), or null when slot s is wave vector s;
// D_rows + q M is the output row of wave vector q.
// Launch shape of the time kernel: values per thread E (8 or 16) and wave
// vectors per workgroup; 0 picks the built-in choice for the length.
struct TimeShape {
  int E = 0;
  int qpw = 0;
};

// Time-transform length L for N frames: the smallest 2^k >= max(N, 16); with
// `minimal`, 3 * 2^k >= N instead when that is smaller (and at least 192).
// N2 = 2 L >= 2 N either way.
int time_length(int N, int minimal);

// L: the plan's transform length (time_length(N) when the plan was made; twN2
// holds 2 L entries).
// Step two by direct differences (Eq. (1) term by term) over slots [0, nslots)
// of a spectra store laid out as for launch_time (qb 16 blocked, 1 plain);
// qexp: the blocked FP16 store's per-row exponents, else null.
hipError_t launch_direct(hipStream_t s, const void* spec, int qb, int64_t nslots, int N, int M,
                         const int32_t* qmap, const int32_t* qexp, float* D);

hipError_t launch_time(hipStream_t s, int L, const void* spec, int qb, int64_t nslots_group, int N, int M,
                       const float2* twN2, const double* ramp, const int32_t* qmap,
                       const int32_t* qexp, float* D_rows,
                       TimeShape shape = TimeShape{});

hipError_t launch_radial(hipStream_t s, const float* D, int64_t nq, int M, int W, int H,
                         int64_t ca, int64_t cc, QTable qt, const int64_t* thr, int nbins,
                         double* Dbar, int64_t* counts, int32_t* bin_of_q);

hipError_t launch_sample(hipStream_t s, const float* D, int64_t n, int M, const LagSet& lags, float* Y,
                         float* scale);

hipError_t launch_lm(hipStream_t s, const float* Y, int64_t n, const LagSet& lags, const float* init,
                     const LmParams& prm, const int32_t* only_if_flag_clear, float* params,
                     int32_t* iters, int32_t* flags, int start_mode = 0);

}  // namespace ddm
