// Register/LDS Stockham FFT building blocks for gfx950 (wave64).
//
// A length-L transform is held by T = L/E threads, E complex values each.
// Thread `tid` holds v[e] = x[tid + e*T].  Each pass of radix R applies E/R
// radix-R butterflies in registers (butterfly j = tid + b*T reads
// x[j + k*L/R], k < R), then exchanges through LDS so that the next pass again
// finds its inputs in the same strided distribution.  The last pass needs no
// exchange: its outputs land in natural order, v[e] = X[tid + e*T].
//
// Pass radices are chosen at compile time among 16, 8, 4, 2 and 3; each must
// divide E.  Twiddles come from a table tw[j] = exp(-2 pi i j / L_tab) built
// in FP64 on the host and rounded once to FP32; a transform of length L reads
// it with stride L_tab / L.
#pragma once
#include <hip/hip_runtime.h>

namespace ddm {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i
__device__ __forceinline__ float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Forward DFT codelets (kernel exp(-2 pi i jk / R)) on x[0..R-1] in registers.
template <int R> struct Dft;

template <> struct Dft<2> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <> struct Dft<3> {
  __device__ __forceinline__ static void run(float2* x) {
    const float h = 0.86602540378443864676f;  // sqrt(3)/2
    float2 s = cadd(x[1], x[2]);
    float2 d = csub(x[1], x[2]);
    float2 m = make_float2(x[0].x - 0.5f * s.x, x[0].y - 0.5f * s.y);
    // -i * h * d
    float2 r = make_float2(h * d.y, -h * d.x);
    x[0] = cadd(x[0], s);
    x[1] = cadd(m, r);
    x[2] = csub(m, r);
  }
};

template <> struct Dft<4> {
  __device__ __forceinline__ static void run(float2* x) {
    float2 t0 = cadd(x[0], x[2]), t1 = csub(x[0], x[2]);
    float2 t2 = cadd(x[1], x[3]), t3 = cmul_mi(csub(x[1], x[3]));
    x[0] = cadd(t0, t2);
    x[2] = csub(t0, t2);
    x[1] = cadd(t1, t3);
    x[3] = csub(t1, t3);
  }
};

template <> struct Dft<8> {
  __device__ __forceinline__ static void run(float2* x) {
    const float c = 0.70710678118654752440f;
    float2 e[4] = {x[0], x[2], x[4], x[6]};
    float2 o[4] = {x[1], x[3], x[5], x[7]};
    Dft<4>::run(e);
    Dft<4>::run(o);
    // o[k] *= exp(-2 pi i k / 8)
    o[1] = make_float2(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
    o[2] = cmul_mi(o[2]);
    o[3] = make_float2(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      x[k] = cadd(e[k], o[k]);
      x[k + 4] = csub(e[k], o[k]);
    }
  }
};

template <> struct Dft<16> {
  __device__ __forceinline__ static void run(float2* x) {
    // exp(-2 pi i k / 16), k = 0..7
    const float c1 = 0.92387953251128675613f, s1 = 0.38268343236508977173f;
    const float c2 = 0.70710678118654752440f;
    float2 e[8], o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      e[k] = x[2 * k];
      o[k] = x[2 * k + 1];
    }
    Dft<8>::run(e);
    Dft<8>::run(o);
    // constant twiddles, with the trivial ones (k = 2, 4, 6) written out
    o[1] = cmul(o[1], make_float2(c1, -s1));
    o[2] = make_float2(c2 * (o[2].x + o[2].y), c2 * (o[2].y - o[2].x));
    o[3] = cmul(o[3], make_float2(s1, -c1));
    o[4] = cmul_mi(o[4]);
    o[5] = cmul(o[5], make_float2(-s1, -c1));
    o[6] = make_float2(c2 * (o[6].y - o[6].x), -c2 * (o[6].x + o[6].y));
    o[7] = cmul(o[7], make_float2(-c1, -s1));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      x[k] = cadd(e[k], o[k]);
      x[k + 8] = csub(e[k], o[k]);
    }
  }
};

// Largest radix for the remaining length `rem` that also divides E.
constexpr int pick_radix(int rem, int E) {
  return (rem % 16 == 0 && E % 16 == 0) ? 16
       : (rem % 8 == 0 && E % 8 == 0)   ? 8
       : (rem % 4 == 0 && E % 4 == 0)   ? 4
       : (rem % 2 == 0 && E % 2 == 0)   ? 2
       : (rem % 3 == 0 && E % 3 == 0)   ? 3
                                         : 0;
}

constexpr bool fft_schedule_ok(int L, int E, int ns = 1) {
  return ns == L ? true : (pick_radix(L / ns, E) == 0 ? false : fft_schedule_ok(L, E, ns * pick_radix(L / ns, E)));
}

// LDS view of one transform: element i lives at base[(i + pad(i)) * STR],
// pad(i) = i / 16 when PAD (one spare slot per 16 elements, which spreads the
// stride-16 writes of a radix-16 pass over the LDS banks).
template <int STR, bool PAD = false> struct LdsView {
  float2* base;
  __device__ __forceinline__ static int slot(int i) { return PAD ? i + (i >> 4) : i; }
  __device__ __forceinline__ float2& operator[](int i) const { return base[slot(i) * STR]; }
};

// Padded length of an L-element transform buffer.
template <bool PAD> constexpr int lds_len(int L) { return PAD ? L + L / 16 : L; }

// Synchronisation of the threads that share one transform: a whole workgroup,
// or only the wavefront when the transform lives inside one wave (LDS
// operations of one wave execute in order, so a compiler fence suffices).
template <bool WAVE> __device__ __forceinline__ void group_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// LDS addressing of one Stockham pass.  Butterfly b of thread tid (j = tid +
// b T) writes its k-th output to element (j / NS) NS R + (j mod NS) + k NS, and
// the next pass reads element tid + e T.  For the power-of-two thread counts
// used here every such slot (padding included) is the thread's first slot plus
// an offset that depends only on (b, k) or e; the check below proves it for
// every thread at compile time, and the pass then computes one base address per
// thread and uses constant offsets (otherwise it evaluates each index).
template <int L, int E, int R, int NS, bool PAD>
struct PassLayout {
  static constexpr int T = L / E;
  static constexpr int NB = E / R;
  static constexpr int sl(int i) { return PAD ? i + (i >> 4) : i; }
  static constexpr int widx(int tid, int b, int k) {
    return ((tid + b * T) / NS) * NS * R + (tid + b * T) % NS + k * NS;
  }
  static constexpr int woff(int b, int k) { return sl(widx(0, b, k)) - sl(widx(0, 0, 0)); }
  static constexpr int roff(int e) { return sl(e * T) - sl(0); }
  static constexpr bool check() {
    for (int tid = 0; tid < T; ++tid) {
      const int w0 = sl(widx(tid, 0, 0));
      for (int b = 0; b < NB; ++b)
        for (int k = 0; k < R; ++k)
          if (sl(widx(tid, b, k)) - w0 != woff(b, k)) return false;
      const int r0 = sl(tid);
      for (int e = 0; e < E; ++e)
        if (sl(tid + e * T) - r0 != roff(e)) return false;
    }
    return true;
  }
  static constexpr bool kLinear = ((T & (T - 1)) == 0) && ((NS & (NS - 1)) == 0) && check();
  // first write slot and first read slot of thread tid (< T)
  __device__ __forceinline__ static int wbase(unsigned tid) {
    const unsigned i = (tid / (unsigned)NS) * (unsigned)(NS * R) + tid % (unsigned)NS;
    return (int)(PAD ? i + (i >> 4) : i);
  }
  __device__ __forceinline__ static int rbase(unsigned tid) { return (int)(PAD ? tid + (tid >> 4) : tid); }
};

// Pass of radix R with span NS (product of the radices already applied).
// Exchanges through LDS unless it is the last pass.  Every thread of the
// workgroup must call it (it contains __syncthreads()).  twf(b, k, jm) gives
// the twiddle exp(-2 pi i k jm / (NS R)) of butterfly b of this thread.
template <int L, int E, int R, int NS, int STR, bool PAD, bool WAVE, typename TwF>
__device__ __forceinline__ void stockham_pass_g(float2 (&v)[E], LdsView<STR, PAD> buf, int tid, TwF twf) {
  constexpr int T = L / E;
  constexpr int NB = E / R;
  constexpr bool LAST = (NS * R == L);
  using PL = PassLayout<L, E, R, NS, PAD>;
  const unsigned ut = (unsigned)tid;
  float2* wp = nullptr;
  if constexpr (!LAST && PL::kLinear) wp = buf.base + PL::wbase(ut) * STR;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    float2 x[R];
#pragma unroll
    for (int k = 0; k < R; ++k) x[k] = v[b + k * NB];
    // j mod NS of butterfly j = tid + b T (NS and T are powers of two, or NS = 1)
    const int jm = (NS == 1) ? 0 : (int)((ut + (unsigned)(b * T)) % (unsigned)NS);
    if (NS > 1) {
#pragma unroll
      for (int k = 1; k < R; ++k) x[k] = cmul(x[k], twf(b, k, jm));
    }
    Dft<R>::run(x);
    if (LAST) {
#pragma unroll
      for (int k = 0; k < R; ++k) v[b + k * NB] = x[k];
    } else if constexpr (PL::kLinear) {
#pragma unroll
      for (int k = 0; k < R; ++k) wp[PL::woff(b, k) * STR] = x[k];
    } else {
      const int j = tid + b * T;
      const int base = (j / NS) * NS * R + jm;
#pragma unroll
      for (int k = 0; k < R; ++k) buf[base + k * NS] = x[k];
    }
  }
  if (!LAST) {
    group_sync<WAVE>();
    if constexpr (PL::kLinear) {
      const float2* rp = buf.base + PL::rbase(ut) * STR;
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = rp[PL::roff(e) * STR];
    } else {
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = buf[tid + e * T];
    }
    group_sync<WAVE>();
  }
}

// Twiddles from a table tw[j] = exp(-2 pi i j / L_tab), read at stride tws = L_tab / L.
template <int L, int E, int R, int NS, int STR, bool PAD, bool WAVE>
__device__ __forceinline__ void stockham_pass(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                              const float2* __restrict__ tw, int tws) {
  stockham_pass_g<L, E, R, NS, STR, PAD, WAVE>(
      v, buf, tid, [&](int, int k, int jm) { return tw[k * jm * (L / (NS * R)) * tws]; });
}

template <int L, int E, int NS, int STR, bool PAD, bool WAVE>
struct FftPasses {
  static constexpr int R = pick_radix(L / NS, E);
  static_assert(R != 0, "length not reachable with radices dividing E");
  __device__ __forceinline__ static void run(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                             const float2* __restrict__ tw, int tws) {
    stockham_pass<L, E, R, NS, STR, PAD, WAVE>(v, buf, tid, tw, tws);
    if constexpr (NS * R < L) FftPasses<L, E, NS * R, STR, PAD, WAVE>::run(v, buf, tid, tw, tws);
  }
};

// Forward transform, exp(-2 pi i n k / L), unnormalised.
template <int L, int E, int STR, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_forward(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                            const float2* __restrict__ tw, int tws) {
  static_assert(L % E == 0, "E must divide L");
  static_assert(fft_schedule_ok(L, E), "no radix schedule");
  FftPasses<L, E, 1, STR, PAD, WAVE>::run(v, buf, tid, tw, tws);
}

// The twiddles of every pass of a length-L transform, held in registers by
// the thread that applies them: for kernels that run several transforms with
// the same thread layout, they are fetched once instead of once per pass.
// Pass (R, NS) of butterfly j = tid + b*T uses exp(-2 pi i k (j mod NS) / (NS R)),
// k = 1..R-1.
template <int L, int E, int NS = 1, bool DONE = (NS == L)>
struct TwCache {
  static constexpr int R = pick_radix(L / NS, E);
  static constexpr int NB = E / R;
  float2 w[NS > 1 ? NB * (R - 1) : 1];
  TwCache<L, E, NS * R> next;
  // ld(i) = exp(-2 pi i i / L), 0 <= i < L
  template <typename Ld>
  __device__ __forceinline__ void load(int tid, Ld ld) {
    constexpr int T = L / E;
    if constexpr (NS > 1) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int jm = (tid + b * T) % NS;
#pragma unroll
        for (int k = 1; k < R; ++k) w[b * (R - 1) + k - 1] = ld(k * jm * (L / (NS * R)));
      }
    }
    next.load(tid, ld);
  }
};
template <int L, int E, int NS>
struct TwCache<L, E, NS, true> {
  template <typename Ld>
  __device__ __forceinline__ void load(int, Ld) {}
};

template <int L, int E, int NS, int STR, bool PAD, bool WAVE>
struct FftPassesC {
  static constexpr int R = pick_radix(L / NS, E);
  __device__ __forceinline__ static void run(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                             const TwCache<L, E, NS>& tc) {
    stockham_pass_g<L, E, R, NS, STR, PAD, WAVE>(
        v, buf, tid, [&](int b, int k, int) { return tc.w[NS > 1 ? b * (R - 1) + k - 1 : 0]; });
    if constexpr (NS * R < L) FftPassesC<L, E, NS * R, STR, PAD, WAVE>::run(v, buf, tid, tc.next);
  }
};

// Forward transform with the twiddles of a TwCache.
template <int L, int E, int STR, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_forward_c(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                              const TwCache<L, E>& tc) {
  static_assert(L % E == 0, "E must divide L");
  static_assert(fft_schedule_ok(L, E), "no radix schedule");
  FftPassesC<L, E, 1, STR, PAD, WAVE>::run(v, buf, tid, tc);
}

// Inverse transform with the twiddles of a TwCache (conjugation trick).
template <int L, int E, int STR, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_inverse_c(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                              const TwCache<L, E>& tc) {
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
  fft_forward_c<L, E, STR, PAD, WAVE>(v, buf, tid, tc);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
}

// Inverse transform, exp(+2 pi i n k / L), unnormalised (conjugation trick).
template <int L, int E, int STR, bool PAD = false, bool WAVE = false>
__device__ __forceinline__ void fft_inverse(float2 (&v)[E], LdsView<STR, PAD> buf, int tid,
                                            const float2* __restrict__ tw, int tws) {
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
  fft_forward<L, E, STR, PAD, WAVE>(v, buf, tid, tw, tws);
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = cconj(v[e]);
}

}  // namespace ddm
