// Step two: the structure function of one time sequence via a Fourier
// transform in time (paper, Eq. (2) and Appendix B).
//
// For the time sequence x_n = F(q, n), n < N, of one wave vector:
//   D(m) (N-m) = sum_{n=m}^{N-1} |x_n|^2 + |x_{n-m}|^2 - 2 Re(conj(x_{n-m}) x_n)
//              = S(N-m) + S(N) - S(m) - 2 Re c(m),
// with prefix sums S(k) = sum_{j<k} |x_j|^2 (the closed form of the recursion
// Eq. (B3)) and the acyclic autocorrelation c(m) = sum_n conj(x_n) x_{n+m},
// obtained by zero padding to N2 = 2L (Eq. (B4), L = 2^ceil(log2 N)), a
// forward FFT, squared modulus, inverse FFT, and the ramp 1/(N-m)
// (Appendix B, the five steps).
//
// MI355X formulation of the same computation:
//  * a per-q constant close to the temporal mean is subtracted first.  D
//    depends only on differences of x, so any constant offset per q cancels
//    exactly; removing it keeps the FP32 transforms and the squared moduli
//    away from cancellation.  The constant is the FP32 mean (its own rounding
//    error is irrelevant: it is the same constant for every sample);
//  * the N2-point forward FFT of the half-zero sequence is done as two L-point
//    FFTs: X_{2j} = FFT_L(x)_j and X_{2j+1} = FFT_L(x_n w^n)_j, w = e^{-2 pi i/N2};
//  * the real power spectrum P is inverted with one complex L-point IFFT of
//    P_even + i P_odd, separated afterwards by conjugate symmetry:
//    with z = IFFT(P_e + i P_o), a_m = (z_m + conj z_{L-m})/2 and
//    b_m = (z_m - conj z_{L-m})/(2i), sum_k P_k e^{2 pi i k m/N2} = a_m + e^{2 pi i m/N2} b_m;
//  * the prefix sums S are accumulated in FP64 and the final combination
//    S(N-m) + S(N) - S(m) - 2 Re c(m) and the ramp are FP64 (the cancellation
//    at small lags needs it); D is rounded to FP32 once.
//
// Work layout: a workgroup holds QPW wave vectors; each is transformed by
// T = L/E threads with E values each (E = 16 by default).  For L <= 1024 a wave vector lives
// inside one wavefront, so after the cooperative load every wave runs on its
// own (wave-local sync, shuffle reductions); longer transforms span waves and
// synchronise the workgroup.  LDS per wave vector: the input sequence
// (later its prefix sums, as doubles) and one exchange buffer.  The twiddles
// of every FFT pass are fetched once per thread into registers and serve all
// three transforms.  Global reads
// use buffer loads (scalar base, 32-bit offsets; reads past the described
// range return 0, which supplies the zero padding).
#pragma once
#include <hip/hip_fp16.h>

#include <cstdlib>

#include "fft.hpp"
#include "internal.hpp"

namespace ddm {

namespace {

constexpr int kRsrcWord3 = 0x00020000;  // raw buffer descriptor, gfx9 family
constexpr int kTailLags = 16;           // lags summed directly from the definition

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kRsrcWord3);
}
__device__ __forceinline__ float2 ld_f2(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
__device__ __forceinline__ double ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

// Sum over the T consecutive threads of a group (tid = index in the group).
// T <= 64: xor butterfly inside the wave (every lane ends with the same bits).
// T > 64: per-wave butterfly, then the T/64 wave totals through LDS.
template <int T, typename V>
__device__ __forceinline__ V group_sum(V v, int tid, V* scratch) {
  constexpr int WT = T < 64 ? T : 64;
#pragma unroll
  for (int o = WT / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WT);
  if constexpr (T > 64) {
    if ((tid & 63) == 0) scratch[tid >> 6] = v;
    __syncthreads();
    V s = 0;
#pragma unroll
    for (int i = 0; i < T / 64; ++i) s += scratch[i];
    __syncthreads();
    v = s;
  }
  return v;
}

// Exclusive prefix sum over the group; *total receives the group sum.
template <int T>
__device__ __forceinline__ double group_excl_scan(double v, int tid, double* scratch, double* total) {
  constexpr int WT = T < 64 ? T : 64;
  const int l = tid % WT;
  double incl = v;
#pragma unroll
  for (int o = 1; o < WT; o <<= 1) {
    const double y = __shfl_up(incl, o, WT);
    if (l >= o) incl += y;
  }
  double excl = __shfl_up(incl, 1, WT);
  if (l == 0) excl = 0.0;
  double wtot = __shfl(incl, WT - 1, WT);
  if constexpr (T > 64) {
    if (l == WT - 1) scratch[tid >> 6] = wtot;
    __syncthreads();
    double before = 0.0, all = 0.0;
#pragma unroll
    for (int i = 0; i < T / 64; ++i) {
      const double s = scratch[i];
      if (i < (tid >> 6)) before += s;
      all += s;
    }
    __syncthreads();
    excl += before;
    wtot = all;
  }
  *total = wtot;
  return excl;
}

}  // namespace

// Work items of the time kernel: groups of QPW consecutive slots.  When a
// group covers only part of a layout block (QPW < QB), the QB/QPW groups that
// share the block's cache lines get ids congruent mod 8, which the round-robin
// dispatcher (and a persistent grid that is a multiple of 8) sends to one XCD.
// The id space is padded to whole sets of 8 blocks; ids past the last slot
// are skipped.
template <int QPW, int QB>
__host__ __device__ __forceinline__ int64_t time_ids(int64_t nq) {
  if constexpr (QPW >= QB) {
    return (nq + QPW - 1) / QPW;
  } else {
    const int64_t nblocks = (nq + QB - 1) / QB;
    return ((nblocks + 7) / 8) * 8 * (QB / QPW);
  }
}
template <int QPW, int QB>
__device__ __forceinline__ int64_t time_q0(int64_t id) {
  if constexpr (QPW >= QB) {
    return id * QPW;
  } else {
    constexpr int nsub = QB / QPW;
    const int64_t r = id % (8 * nsub);
    return ((id / (8 * nsub)) * 8 + (r % 8)) * QB + (r / 8) * QPW;
  }
}

// QB: layout of the input time series, indexed by slot s < nq.  QB == 1:
// plain [s][N].  QB > 1: the blocked store [s / QB][N][QB] written by the
// column transform.  qmap[s] is the wave vector (row of D) held by slot s, -1
// for a slot that holds none; a null qmap means slot s holds wave vector s.
// F16 (blocked store only): complex FP16 scaled by 2^qexp[q], unscaled on load
// (exact: a power of two).
//
// Workgroup b takes groups b, b + gridDim.x, ...  For L <= 1024 the grid is
// persistent and the loads of the next group are issued before the
// transforms of the current one, landing in registers while they run; longer
// transforms have no registers to spare for that (one wave per SIMD instead
// of two) and take one group per workgroup, loaded when it starts.
template <int L>
constexpr bool time_prefetch() { return L <= 1024; }

// Transform lengths: 2^k (16 <= L <= 8192, E = 16 or 8) and 3 * 2^k
// (192 <= L <= 6144, E = 12: radix-4 and radix-2 passes, then one radix-3
// pass; E = 24 would hold too many registers), so that the zero-padded length
// 2 L >= 2 N - 1 exceeds 2 N by at most a factor 4/3 instead of 2.
constexpr bool time_len_3(int L) { return L % 3 == 0; }

template <int L, int QPW, int QB, int E, bool FULL, bool F16>
__global__ void __launch_bounds__(QPW * (L / E)) k_time(const void* __restrict__ spec, int64_t nq,
                                                       int N, int M, const float2* __restrict__ twN2,
                                                       const double* __restrict__ ramp,
                                                       const int32_t* __restrict__ qmap,
                                                       const int32_t* __restrict__ qexp,
                                                       float* __restrict__ D) {
  // FULL: N == L and M == L (no padding, every lag), so no bounds tests.
  constexpr int T = L / E;
  constexpr bool WAVE = (T <= 64);
  constexpr int XS = lds_len<true>(L) + 1;  // staging stride (odd: spreads the transposed writes)
  constexpr int YS = lds_len<true>(L);      // exchange buffer stride
  constexpr int NT = QPW * T;
  static_assert((T & (T - 1)) == 0, "threads per transform must be a power of two");
  constexpr uint32_t ES = F16 ? 4u : 8u;    // bytes per stored complex value
  __shared__ float2 xall[QPW * XS];
  __shared__ float2 yall[QPW * YS];
  constexpr bool PF = time_prefetch<L>();
  // e^{-2 pi i n / N2}, n < L, where the group loop prefetches (its global
  // loads would wait for the prefetch); read from the table otherwise
  __shared__ float2 wtab[PF ? L : 1];
  __shared__ double red[QPW * (T > 64 ? T / 64 : 1)];
  __shared__ float redf[QPW * (T > 64 ? T / 64 : 1)];
  if (FULL && (N != L || M != L)) return;  // guarded by the launcher; uniform

  const int64_t nids = time_ids<QPW, QB>(nq);
  const __amdgpu_buffer_rsrc_t tw_r = make_rsrc(twN2, 2u * L * sizeof(float2));
  const __amdgpu_buffer_rsrc_t ramp_r = make_rsrc(ramp, (uint32_t)N * sizeof(double));
  // twiddles of every FFT pass, exp(-2 pi i j / L) = twN2[2 j], held in
  // registers and shared by the three transforms of every wave vector
  TwCache<L, E> tc;
  tc.load(threadIdx.x % T, [&](int j) { return ld_f2(tw_r, (uint32_t)(2 * j) * 8u); });
  if constexpr (PF)
    for (int j = threadIdx.x; j < L; j += NT) wtab[j] = ld_f2(tw_r, (uint32_t)j * 8u);
  auto w_n = [&](int n) { return PF ? wtab[n] : ld_f2(tw_r, (uint32_t)n * 8u); };

  // This thread's share of a group's input: element f = threadIdx.x + r NT of
  // the group's QPW sequences (raw: FP32 pairs, or the FP16 pair's bits in .x).
  float2 ld[E];
  // q0 < 0: no group (a range of 0 bytes: every load returns 0 and reads nothing)
  auto issue_loads = [&](int64_t q0, int tx) {
    __amdgpu_buffer_rsrc_t in_r;
    if (q0 < 0) {
      in_r = make_rsrc(spec, 0u);
    } else if constexpr (QB == 1) {
      const int64_t nvalid = (nq - q0) < QPW ? (nq - q0) : QPW;
      in_r = make_rsrc((const float2*)spec + (size_t)q0 * N, (uint32_t)(nvalid * N * sizeof(float2)));
    } else {
      // rows t < N of this sub-block; t >= N falls past the range and reads 0
      const int64_t blk = q0 / QB;
      const int sub = (int)(q0 % QB);
      in_r = make_rsrc((const char*)spec + ((size_t)blk * N * QB + sub) * ES,
                       (uint32_t)(((size_t)(N - 1) * QB + QPW) * ES));
    }
    // blocked layout: element f = tx + r NT is time tx / QPW + r T of sequence
    // tx % QPW, so its offset is a per-thread base plus a constant
    const uint32_t off0 = ((uint32_t)tx / QPW * QB + (uint32_t)tx % QPW) * ES;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int f = tx + r * NT;
      uint32_t off;
      if constexpr (QB == 1) {
        const int i = f / L, t = f % L;
        off = (FULL || t < N) ? (uint32_t)(i * N + t) * 8u : 0xFFFFFFF0u;
      } else {
        off = off0 + (uint32_t)(r * T * QB) * ES;
      }
      if constexpr (F16)
        ld[r].x = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(in_r, off, 0, 0));
      else
        ld[r] = ld_f2(in_r, off);
    }
  };

  int64_t id = blockIdx.x;
  if (PF) issue_loads((id < nids && time_q0<QPW, QB>(id) < nq) ? time_q0<QPW, QB>(id) : -1, threadIdx.x);
  for (; id < nids; id += gridDim.x) {
    // the thread index, made opaque per group so that the per-thread LDS
    // addresses of the whole group are not hoisted out of the loop (they
    // would all stay live in registers)
    int tx = threadIdx.x;
    asm volatile("" : "+v"(tx));
    const int qi = tx / T;
    const int tid = tx % T;
    const int64_t q0 = time_q0<QPW, QB>(id);
    const int64_t nid = id + gridDim.x;
    // the next group's first slot, -1 for none (past the end or a padding id)
    const int64_t q0n = (PF && nid < nids && time_q0<QPW, QB>(nid) < nq) ? time_q0<QPW, QB>(nid) : -1;
    const bool live = q0 < nq;  // uniform: false for a padding id
    if (!PF) {
      if (!live) continue;
      issue_loads(q0, tx);
    }
    __syncthreads();  // every wave is done with the previous group's LDS data

    // ---- stage the QPW sequences in LDS, [q][t] ----
    if (live) {
      float sc = 1.0f;  // 2^-qexp of this thread's wave vector (blocked layout: i = threadIdx.x % QPW)
      if constexpr (F16) {
        const int64_t ss = q0 + (tx % QPW);
        const int qq = (ss < nq) ? (qmap ? qmap[ss] : (int)ss) : -1;
        sc = (qq >= 0) ? ldexpf(1.0f, -qexp[qq]) : 1.0f;
      }
      // blocked layout: time tx / QPW + r T of sequence tx % QPW; T is a power
      // of two and tx / QPW < T, so the padded slot of that time is the slot of
      // tx / QPW plus the slot of r T
      float2* xs = xall + ((uint32_t)tx % QPW) * XS + LdsView<1, true>::slot((uint32_t)tx / QPW);
#pragma unroll
      for (int r = 0; r < E; ++r) {
        float2 val = ld[r];
        if constexpr (F16) {
          const __half2 h = __builtin_bit_cast(__half2, __builtin_bit_cast(uint32_t, ld[r].x));
          val = make_float2(__low2float(h) * sc, __high2float(h) * sc);
        }
        if constexpr (QB == 1) {
          const int f = tx + r * NT;
          xall[(f / L) * XS + LdsView<1, true>::slot(f % L)] = val;
        } else {
          xs[LdsView<1, true>::slot(r * T)] = val;
        }
      }
    }
    __syncthreads();

    // the next group's loads run during this group's transforms; issued on
    // every path (also for no group), so that the registers they fill are the
    // only values of `ld` that reach the next iteration
    if (PF) issue_loads(q0n, tx);
    if (!live) continue;
    const int64_t q = q0 + qi;  // slot of this wave vector in the store
    const int qd = (q < nq) ? (qmap ? qmap[q] : (int)q) : -1;  // its row of D (-1: a hole)

    LdsView<1, true> xb{xall + qi * XS};
    LdsView<1, true> yb{yall + qi * YS};
    double* xd = reinterpret_cast<double*>(xall + qi * XS);  // the same bytes, as doubles
    double* scratch = red + qi * (T > 64 ? T / 64 : 1);
    float* scratchf = redf + qi * (T > 64 ? T / 64 : 1);

    // ---- offset: FP32 mean over the contiguous chunk [tid*E, tid*E+E), fixed order ----
    float mr, mi;
    {
      float sr[E / 2], si[E / 2];
#pragma unroll
      for (int i = 0; i < E / 2; ++i) {
        const float2 a = xb[tid * E + 2 * i], b = xb[tid * E + 2 * i + 1];
        sr[i] = a.x + b.x;
        si[i] = a.y + b.y;
      }
      if constexpr (((E / 2) & (E / 2 - 1)) == 0) {
#pragma unroll
        for (int w = E / 4; w > 0; w >>= 1)
#pragma unroll
          for (int i = 0; i < w; ++i) {
            sr[i] += sr[i + w];
            si[i] += si[i + w];
          }
      } else {  // E / 2 not a power of two: fold the upper half onto the lower until one is left
#pragma unroll
        for (int n = E / 2; n > 1; n -= n / 2)
#pragma unroll
          for (int i = 0; i < n / 2; ++i) {
            sr[i] += sr[n - 1 - i];
            si[i] += si[n - 1 - i];
          }
      }
      const float inv_n = 1.0f / (float)N;
      mr = group_sum<T>(sr[0], tid, scratchf) * inv_n;
      mi = group_sum<T>(si[0], tid, scratchf) * inv_n;
    }
    // offset-free sequence x' = x - mean for n < N, 0 beyond
    auto xp = [&](float2 a, int n) {
      return (FULL || n < N) ? make_float2(a.x - mr, a.y - mi) : make_float2(0.f, 0.f);
    };

    // ---- X_odd = FFT_L(x' w^n), w = e^{-2 pi i / N2}; X_even = FFT_L(x') ----
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int n = tid + e * T;
      v[e] = cmul(xp(xb[n], n), w_n(n));
    }
    fft_forward_c<L, E, 1, true, WAVE>(v, yb, tid, tc);
    float po[E];
#pragma unroll
    for (int e = 0; e < E; ++e) po[e] = v[e].x * v[e].x + v[e].y * v[e].y;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = xp(xb[tid + e * T], tid + e * T);
    fft_forward_c<L, E, 1, true, WAVE>(v, yb, tid, tc);
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = make_float2(v[e].x * v[e].x + v[e].y * v[e].y, po[e]);

    // ---- z = IFFT_L(P_even + i P_odd), unnormalised; v[e] = z[tid + e*T] ----
    fft_inverse_c<L, E, 1, true, WAVE>(v, yb, tid, tc);
#pragma unroll
    for (int e = 0; e < E; ++e) yb[tid + e * T] = v[e];

    // ---- the kTailLags largest lags, where D averages fewer than kTailLags
    // pairs: Eq. (1) summed directly (FP32 differences of the raw sequence; a
    // constant offset cancels).  The FFT route's rounding error in c(m) is
    // spread evenly over the lags while D(m) divides by N - m, so it is largest
    // exactly there.  Read before the prefix sums overwrite the sequence. ----
    float dtail[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      dtail[e] = 0.0f;
      const int m = tid + e * T;
      // with N == L the candidates are the last e only (T >= kTailLags)
      if ((!FULL || T < kTailLags || e == E - 1) && m >= N - kTailLags && m > 0 && m < M) {
        // all kTailLags pairs at once (indices clamped into the sequence, the
        // pairs past N dropped), summed in order
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < kTailLags; ++j) {
          const float2 a = xb[min(m + j, N - 1)], b = xb[j];
          const float dx = a.x - b.x, dy = a.y - b.y;
          const float t = fmaf(dx, dx, dy * dy);
          acc += (j < N - m) ? t : 0.0f;
        }
        dtail[e] = acc;
      }
    }

    // ---- prefix sums S(k) = sum_{j<k} |x'_j|^2, accumulated in FP64 over the
    // contiguous chunk [tid*E, tid*E+E) of this thread, then across threads ----
    {
      double s[E];
      double run = 0.0;
#pragma unroll
      for (int i = 0; i < E; ++i) {
        const float2 a = xp(xb[tid * E + i], tid * E + i);
        s[i] = run;
        run += (double)(a.x * a.x + a.y * a.y);
      }
      double total;
      const double before = group_excl_scan<T>(run, tid, scratch, &total);
      // each thread rewrites only the chunk it has just read
#pragma unroll
      for (int i = 0; i < E; ++i) xd[LdsView<1, true>::slot(tid * E + i)] = before + s[i];
      // S(N) sits in slot L (one past the sequence) so that every lag reads the same way
      if (tid == 0) xd[LdsView<1, true>::slot(L)] = total;
    }
    group_sync<WAVE>();

    // ---- D(m) = (S(N-m) + S(N) - S(m) - 2 Re c(m)) / (N-m) ----
    if (qd >= 0) {
      const double sN = xd[LdsView<1, true>::slot(N)];
      const float inv_l = 1.0f / (float)L;  // 2 / N2 (exact for L a power of two)
      float* drow = D + (size_t)qd * M;
      // With T a multiple of 16, the padded slots of m = tid + e T, N - m and
      // L - m (for e >= 1, where L - m >= 1) are a per-thread slot plus or
      // minus the slot of e T.
      constexpr bool LIN = (T % 16 == 0);
      const int s_m = LdsView<1, true>::slot(tid);
      const int s_nm = LdsView<1, true>::slot(N - tid);
      const int s_lm = LdsView<1, true>::slot(L - tid);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int m = tid + e * T;
        if (FULL || m < M) {
          const int set = LdsView<1, true>::slot(e * T);
          const float2 zm = v[e];
          const float2 zr = (LIN && e > 0) ? yb.base[s_lm - set] : yb[m == 0 ? 0 : L - m];
          const float2 w = w_n(m);  // (cos th, -sin th), th = 2 pi m / N2
          // 2 Re c(m) = (2/N2) Re sum_k P_k e^{2 pi i k m / N2}
          const float two_c = 0.5f * ((zm.x + zr.x) + w.x * (zm.y + zr.y) - w.y * (zm.x - zr.x)) * inv_l;
          const double s_nmv = LIN ? xd[s_nm - set] : xd[LdsView<1, true>::slot(N - m)];
          const double s_mv = LIN ? xd[s_m + set] : xd[LdsView<1, true>::slot(m)];
          const double num = (s_nmv + sN) - s_mv - (double)two_c;
          const double sum = (m >= N - kTailLags) ? (double)dtail[e] : num;
          const double dm = sum * ld_f64(ramp_r, (uint32_t)m * 8u);
          // lag 0 pairs every frame with itself: D(q, 0) = 0 exactly by definition
          drow[m] = (m == 0) ? 0.0f : (float)dm;
        }
      }
      
    }
  }
}

// Launch shape of the time kernel for a transform length: values per thread
// E and wave vectors per workgroup QPW (DDM_TIME_E / DDM_TIME_QPW override,
// for tuning).
inline int env_int(const char* name) {
  const char* s = std::getenv(name);
  return s ? std::atoi(s) : 0;
}

inline int time_e(int L) {
  if (time_len_3(L)) return 12;
  static const int env = env_int("DDM_TIME_E");
  if ((env == 8 || env == 16) && L / env >= 1 && L % env == 0 && L >= 16) return env;
  return 16;
}

inline int time_qpw(int L, int E) {
  static const int env = env_int("DDM_TIME_QPW");
  int qpw;
  if (L <= 256) qpw = 16;
  else if (L <= 512) qpw = 8;
  else if (L <= 1024) qpw = 4;
  else if (L <= 2048) qpw = 2;
  else qpw = 1;
  if (env == 1 || env == 2 || env == 4 || env == 8 || env == 16) qpw = env;
  while (qpw > 1 && (qpw * (L / E) > 1024 || time_lds_bytes(L, qpw) > 160 * 1024))
    qpw >>= 1;
  return qpw;
}


// Workgroups of one kernel resident at once on the device (the persistent
// grid), looked up once per kernel.
inline int device_cus() {
  static const int n = [] {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    return cus;
  }();
  return n;
}

template <typename K>
int64_t resident_wgs(K kernel, int block) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  return (int64_t)per_cu * device_cus();
}

// Grid of the time kernel: one workgroup per id, or, where it prefetches, at
// most the resident workgroups, a multiple of 8 (so that every workgroup
// keeps to one XCD's ids).
template <int L, int QPW, int QB, int E, bool FULL, bool F16>
void time_launch_one(hipStream_t s, int64_t nids, dim3 block, const void* spec, int64_t nq, int N, int M,
                            const float2* tw, const double* ramp, const int32_t* qmap, const int32_t* qexp,
                            float* D) {
  static const int64_t res =
      time_prefetch<L>() ? resident_wgs(k_time<L, QPW, QB, E, FULL, F16>, (int)block.x) : INT64_MAX;
  int64_t g = res >= 8 ? res / 8 * 8 : res;
  if (g > nids) g = nids;
  hipLaunchKernelGGL((k_time<L, QPW, QB, E, FULL, F16>), dim3((unsigned)g), block, 0, s, spec, nq, N, M, tw, ramp,
                     qmap, qexp, D);
}

template <int L, int QPW, int QB, int E, bool FULL>
void time_launch(hipStream_t s, int64_t nids, dim3 block, const void* spec, int64_t nq, int N, int M,
                        const float2* tw, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D) {
  if constexpr (QB > 1) {
    if (qexp != nullptr) {
      time_launch_one<L, QPW, QB, E, FULL, true>(s, nids, block, spec, nq, N, M, tw, ramp, qmap, qexp, D);
      return;
    }
  }
  time_launch_one<L, QPW, QB, E, FULL, false>(s, nids, block, spec, nq, N, M, tw, ramp, qmap, nullptr, D);
}

template <int L, int QPW, int QB, int E>
hipError_t time_go(hipStream_t s, const void* spec, int64_t nq, int N, int M,
                          const float2* tw, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D) {
  const int64_t nids = time_ids<QPW, QB>(nq);
  if (nids == 0) return hipSuccess;
  const dim3 block(QPW * (L / E));
  if (N == L && M == L)
    time_launch<L, QPW, QB, E, true>(s, nids, block, spec, nq, N, M, tw, ramp, qmap, qexp, D);
  else
    time_launch<L, QPW, QB, E, false>(s, nids, block, spec, nq, N, M, tw, ramp, qmap, qexp, D);
  return hipGetLastError();
}

template <int L, int QPW, int E>
constexpr bool qpw_fits() {
  return QPW * (L / E) <= 1024 && time_lds_bytes(L, QPW) <= 163840;
}

template <int L, int QB, int E>
hipError_t time_qpw_go(hipStream_t s, int qpw, const void* spec, int64_t nq, int N, int M,
                              const float2* tw, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D) {
  switch (qpw) {
    case 16: if constexpr (qpw_fits<L, 16, E>()) return time_go<L, 16, QB, E>(s, spec, nq, N, M, tw, ramp, qmap, qexp, D);
             break;
    case 8: if constexpr (qpw_fits<L, 8, E>()) return time_go<L, 8, QB, E>(s, spec, nq, N, M, tw, ramp, qmap, qexp, D);
            break;
    case 4: if constexpr (qpw_fits<L, 4, E>()) return time_go<L, 4, QB, E>(s, spec, nq, N, M, tw, ramp, qmap, qexp, D);
            break;
    case 2: if constexpr (qpw_fits<L, 2, E>()) return time_go<L, 2, QB, E>(s, spec, nq, N, M, tw, ramp, qmap, qexp, D);
            break;
    case 1: return time_go<L, 1, QB, E>(s, spec, nq, N, M, tw, ramp, qmap, qexp, D);
  }
  return hipErrorInvalidValue;
}

template <int L, int QB>
hipError_t time_e_go(hipStream_t s, const void* spec, int64_t nq, int N, int M,
                            const float2* tw, const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D,
                            TimeShape shape) {
  if constexpr (time_len_3(L)) {
    int qpw = shape.qpw > 0 ? shape.qpw : time_qpw(L, 12);
    while (qpw > 1 && (qpw * (L / 12) > 1024 || time_lds_bytes(L, qpw) > 160 * 1024)) qpw >>= 1;
    return time_qpw_go<L, QB, 12>(s, qpw, spec, nq, N, M, tw, ramp, qmap, qexp, D);
  } else {
    const int E = (shape.E == 8 || shape.E == 16) ? shape.E : time_e(L);
    int qpw = shape.qpw > 0 ? shape.qpw : time_qpw(L, E);
    while (qpw > 1 && (qpw * (L / E) > 1024 || time_lds_bytes(L, qpw) > 160 * 1024))
      qpw >>= 1;
    if constexpr (L >= 512) {
      if (E == 8) return time_qpw_go<L, QB, 8>(s, qpw, spec, nq, N, M, tw, ramp, qmap, qexp, D);
    }
    return time_qpw_go<L, QB, 16>(s, qpw, spec, nq, N, M, tw, ramp, qmap, qexp, D);
  }
}

// Every launch of the time kernel for one transform length L (blocked or
// plain input layout); each length is instantiated in a translation unit of
// its own (k_time_l*.hip) so that they compile in parallel.
template <int L>
hipError_t time_run(hipStream_t s, const void* spec, int qb, int64_t nq, int N, int M, const float2* twN2,
                    const double* ramp, const int32_t* qmap, const int32_t* qexp, float* D, TimeShape shape) {
  if (qb == 1 && qexp == nullptr) return time_e_go<L, 1>(s, spec, nq, N, M, twN2, ramp, qmap, nullptr, D, shape);
  if (qb == kSpecQB) return time_e_go<L, kSpecQB>(s, spec, nq, N, M, twN2, ramp, qmap, qexp, D, shape);
  return hipErrorInvalidValue;
}

#define DDM_TIME_INSTANTIATE(L)                                                                                  \
  template hipError_t time_run<L>(hipStream_t, const void*, int, int64_t, int, int, const float2*, const double*, \
                                  const int32_t*, const int32_t*, float*, TimeShape);

}  // namespace ddm
