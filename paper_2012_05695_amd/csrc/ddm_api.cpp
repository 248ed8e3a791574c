// C ABI of libddm: plans, validation, workspace partition and the launch
// sequence of the structure-function path.  No exception crosses the ABI;
// every entry point returns a ddm_status and records a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>
#include <string>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "internal.hpp"

using namespace ddm;

namespace {

thread_local std::string g_err;

ddm_status fail(ddm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

ddm_status hip_fail(hipError_t e, const char* what) {
  return fail(DDM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// DDM_LOG (environment, any value but 0): one line per plan, batch, workspace
// and autotune decision on stderr, prefixed "[ddm]".
bool log_on() {
  static const bool on = [] {
    const char* v = std::getenv("DDM_LOG");
    return v != nullptr && v[0] != '\0' && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void ddm_log(const char* fmt, ...) {
  if (!log_on()) return;
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "[ddm] %s\n", buf);
}

}  // namespace

namespace ddm {
// error reporting shared with the other ABI translation units
ddm_status api_fail(ddm_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}
}  // namespace ddm

namespace {

constexpr size_t kInterTargetBytes = 128u << 20;  // row-transform intermediate per batch (half the Infinity Cache)
constexpr int kReadback = 4;                      // calls in flight before the host waits

// Step two's cost model: the direct method evaluates N M - M (M - 1) / 2
// difference pairs per wave vector; the time transform of length L costs a
// time proportional to L log2 L per wave vector.  The constant is the measured
// crossover at 512 x 512 frames: direct faster at 48 lags and the transform
// faster at 56 for both N = 512 and N = 1024 (at 256 x 256, with fewer wave
// vectors, direct stays faster to about 80 lags at N = 2048 and 96 at 4096;
// the model keeps the larger frames' constant there, and autotune times both).
// The length-16384 kernel (one wave vector per workgroup) costs relatively
// more: at 512 x 512 x 16384 direct is faster at 192 lags and the transform at
// 256 (crossover near 224 lags), hence the constant 16 there.
bool direct_cheaper(int N, int M, int L) {
  const double pairs = (double)N * M - 0.5 * (double)M * (M - 1);
  const double c = L >= 16384 ? 16.0 : 5.2;
  return pairs < c * L * std::log2((double)L);
}

}  // namespace

struct ddm_plan_s {
  uint32_t magic;
  ddm_plan_desc d;
  int W, H, N, M;
  int L;         // time transform length (N2 / 2), >= 16
  int method;    // step two: DDM_METHOD_FOURIER or DDM_METHOD_DIRECT (AUTO resolved)
  int n2_paper;  // Eq. (B4) length
  int64_t nq;
  int64_t ca, cc;  // k2 = kx^2 ca + ky_s^2 cc
  std::vector<int32_t> qoff, kxcnt;
  int kx_needed, cw, kxw, ncol_tiles;
  int kxnyq;  // W/2 when the Nyquist column is kept (packed with kx = 0), else -1
  // step one in one launch (square frames up to 512): workgroups, control
  // slots, workspace frames it needs
  bool fused;
  int s1_nwg, s1_maxslots, s1_frames;
  size_t frame_inter_bytes;
  int fb_target;
  hipStream_t stream;
  // host-resident frames (ddm_structure_function_host): copies on s_copy into
  // two staging halves; events: a half's frames arrived, a half's frames read,
  // the plan's stream reached the call
  hipStream_t s_copy;
  hipEvent_t ev_h2d[2], ev_used[2], ev_start;
  // device tables (one allocation)
  void* dev_tables;
  float2 *twW, *twH, *twT;
  double* ramp;  // 1/(N-m), m < N, FP64 (the ramp vector of Appendix B)
  int32_t *qoff_d, *kxcnt_d;
  int32_t* pilot_d;  // FP16 store: the pilot frame numbers
  // blocked spectra store: slot tables (every row starts a new block of 16,
  // the Nyquist column has its own rows of blocks), slot -> wave vector
  int64_t nslots;
  int sN;
  std::vector<int32_t> sbase;
  int32_t *sbase_d, *qmap_d;
  // radial thresholds (grown on demand): device copy, pinned staging, the
  // last values sent, and an event after the last launch that read them
  int64_t* thr_d;
  int64_t* thr_pin;
  size_t thr_cap;
  std::vector<int64_t> thr_last;
  hipEvent_t thr_ev;
  // workspace
  void* ws;
  size_t ws_bytes;
  TimeShape tshape;  // time-kernel launch shape (autotuned or built-in)
  // FP16 spectrum store
  bool f16;
  std::vector<int> pilot;  // pilot frames that fix the per-q scale
  int64_t sat_total;       // saturation counts folded in so far
  // what a call hands back to the host (step-one error flag, FP16 saturation
  // count): a ring of pinned slots, each with the event after its copies.  A
  // slot is folded in once its event has completed, checked without waiting at
  // the start of each call; the host waits only to reuse a slot, i.e. when it
  // runs kReadback calls ahead of the device.
  int32_t* rb_host;  // pinned [kReadback][2]: error flag, saturation count
  hipEvent_t rb_ev[kReadback];
  bool rb_pending[kReadback];
  int rb_next;
  bool s1_failed;  // a folded slot carried a step-one error not yet reported
  int64_t sat_unreported;  // saturation counts folded in since the last report
  bool s1_force_err;  // DDM_STEP1_FAIL: the single-launch step one starts with its error flag raised
  int32_t* outcome_dev;  // when set (a batch's stack): each call leaves its step-one error flag here
  int32_t batch_nbins;   // a batch's stack: bins set by ddm_batch_set_bins (thresholds in thr_d), else 0
  // profiling: event pairs around launches of the kinds in prof_mask
  uint32_t prof_mask;
  struct Rec { uint32_t kind; hipEvent_t a, b; };
  std::vector<Rec> prof_recs;
  double prof_ms[5];
  int64_t prof_n[5];
};

static int kind_slot(uint32_t kind) {
  switch (kind) {
    case DDM_KERNEL_ROW: return 0;
    case DDM_KERNEL_COL: return 1;
    case DDM_KERNEL_TIME: return 2;
    case DDM_KERNEL_RADIAL: return 3;
    case DDM_KERNEL_STEP1: return 4;
    default: return -1;
  }
}

// Collect finished event pairs into the per-kind totals (waits for them).
static hipError_t prof_drain(ddm_plan_s* p) {
  hipError_t err = hipSuccess;
  for (auto& r : p->prof_recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipSuccess) {
      const int s = kind_slot(r.kind);
      p->prof_ms[s] += ms;
      p->prof_n[s] += 1;
    } else if (err == hipSuccess) {
      err = e;
    }
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  p->prof_recs.clear();
  return err;
}

// RAII bracket: records an event pair around one launch when profiled.
struct ProfScope {
  ddm_plan_s* p;
  uint32_t kind;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(ddm_plan_s* p_, uint32_t k) : p(p_), kind(k) {
    if (p->prof_mask & kind) {
      if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        a = b = nullptr;
        return;
      }
      hipEventRecord(a, p->stream);
    }
  }
  ~ProfScope() {
    if (a != nullptr) {
      hipEventRecord(b, p->stream);
      p->prof_recs.push_back({kind, a, b});
    }
  }
};

static constexpr uint32_t kPlanMagic = 0x44444d31u;  // "DDM1"

static ddm_status check_plan(ddm_plan_t p) {
  if (p == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "plan is NULL");
  if (p->magic != kPlanMagic) return fail(DDM_ERR_STATE, "plan handle is not a live plan");
  return DDM_OK;
}

static void fill_twiddles(std::vector<float2>& h, size_t off, int L) {
  // tw[j] = exp(-2 pi i j / L), evaluated in FP64, rounded once to FP32
  for (int j = 0; j < L; ++j) {
    const double a = 2.0 * M_PI * (double)j / (double)L;
    h[off + j] = make_float2((float)std::cos(a), (float)-std::sin(a));
  }
}

extern "C" {

void ddm_plan_desc_init(ddm_plan_desc* d) {
  if (d == nullptr) return;
  std::memset(d, 0, sizeof(*d));
  d->struct_size = sizeof(ddm_plan_desc);
  d->max_lag = 0;
  d->pixel = DDM_PIX_U16;
  d->spectrum = DDM_SPEC_F32;
  d->precondition = 1;
  d->k2_max = -1;
  d->stream = nullptr;
}

int32_t ddm_abi_version(void) { return DDM_ABI_VERSION; }

const char* ddm_last_error(void) { return g_err.c_str(); }

// Every descriptor rule that needs no device: the plan and batch constructors
// refuse a descriptor before any HIP call.
static ddm_status check_desc(const ddm_plan_desc* desc) {
  if (desc->struct_size != sizeof(ddm_plan_desc))
    return fail(DDM_ERR_INVALID_ARGUMENT, "desc.struct_size %u != %zu (header/library mismatch)",
                desc->struct_size, sizeof(ddm_plan_desc));
  const int W = desc->width, H = desc->height, N = desc->n_frames;
  if (W <= 0 || H <= 0) return fail(DDM_ERR_INVALID_ARGUMENT, "width/height must be positive");
  if (!supported_spatial(W) || !supported_spatial(H))
    return fail(DDM_ERR_UNSUPPORTED,
                "frame %dx%d: each side must be 2^k (16..4096) or 3*2^k (48..3072)", W, H);
  if (N < 2) return fail(DDM_ERR_INVALID_ARGUMENT, "n_frames must be >= 2");
  if (desc->method != DDM_METHOD_FOURIER && desc->method != DDM_METHOD_DIRECT && desc->method != DDM_METHOD_AUTO)
    return fail(DDM_ERR_INVALID_ARGUMENT, "method must be DDM_METHOD_FOURIER, _DIRECT or _AUTO");
  if (N > 65536) return fail(DDM_ERR_UNSUPPORTED, "n_frames > 65536");
  if (N > 16384 && desc->method == DDM_METHOD_FOURIER)
    return fail(DDM_ERR_UNSUPPORTED, "n_frames > 16384 (time FFT length > 32768) needs DDM_METHOD_DIRECT");
  if (desc->max_lag < 0 || desc->max_lag > N)
    return fail(DDM_ERR_INVALID_ARGUMENT, "max_lag must be in [0, n_frames]");
  if (desc->pixel != DDM_PIX_U8 && desc->pixel != DDM_PIX_U16)
    return fail(DDM_ERR_INVALID_ARGUMENT, "pixel must be DDM_PIX_U8 or DDM_PIX_U16");
  if (desc->spectrum != DDM_SPEC_F32 && desc->spectrum != DDM_SPEC_F16_QSCALED)
    return fail(DDM_ERR_INVALID_ARGUMENT, "unknown spectrum storage %d", desc->spectrum);
  if (desc->precondition != 0 && desc->precondition != 1)
    return fail(DDM_ERR_INVALID_ARGUMENT, "precondition must be 0 or 1");
  if (desc->k2_max < -1) return fail(DDM_ERR_INVALID_ARGUMENT, "k2_max must be >= -1");
  if (desc->padding != DDM_PAD_POW2 && desc->padding != DDM_PAD_MINIMAL)
    return fail(DDM_ERR_INVALID_ARGUMENT, "padding must be DDM_PAD_POW2 or DDM_PAD_MINIMAL");
  return DDM_OK;
}

ddm_status ddm_plan_create(const ddm_plan_desc* desc, ddm_plan_t* out) {
  if (out == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (desc == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "desc is NULL");
  ddm_status st0 = check_desc(desc);
  if (st0 != DDM_OK) return st0;
  const int W = desc->width, H = desc->height, N = desc->n_frames;

  ddm_plan_s* p = new (std::nothrow) ddm_plan_s();
  if (p == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "host allocation failed");
  p->magic = kPlanMagic;
  p->d = *desc;
  p->W = W;
  p->H = H;
  p->N = N;
  p->M = desc->max_lag == 0 ? N : desc->max_lag;
  int l = 1;
  while (l < N) l <<= 1;
  p->n2_paper = 2 * l;
  p->L = time_length(N, desc->padding);
  p->method = desc->method == DDM_METHOD_AUTO ? (N > 16384 || direct_cheaper(N, p->M, p->L) ? DDM_METHOD_DIRECT
                                                                                         : DDM_METHOD_FOURIER)
                                              : desc->method;
  const int64_t g = std::gcd(W, H);
  p->ca = (int64_t)(H / g) * (H / g);
  p->cc = (int64_t)(W / g) * (W / g);
  p->qoff.assign(H, 0);
  p->kxcnt.assign(H, 0);
  int64_t nq = 0;
  int kxn = 0;
  for (int ky = 0; ky < H; ++ky) {
    const int64_t kys = ky <= H / 2 ? ky : ky - H;
    int cnt = 0;
    for (int kx = 0; kx <= W / 2; ++kx) {
      const int64_t k2 = (int64_t)kx * kx * p->ca + kys * kys * p->cc;
      if (desc->k2_max >= 0 && k2 > desc->k2_max) break;  // k2 grows with kx
      ++cnt;
    }
    p->qoff[ky] = (int32_t)nq;
    p->kxcnt[ky] = cnt;
    nq += cnt;
    kxn = std::max(kxn, cnt);
  }
  p->nq = nq;
  p->kx_needed = kxn;
  const ColCfg cc = col_cfg(H);
  p->cw = cc.cw;
  // the real columns kx = 0 and kx = W/2 share one complex column when both are kept
  p->kxnyq = (kxn == W / 2 + 1) ? W / 2 : -1;
  const int ncols = p->kxnyq > 0 ? W / 2 : kxn;
  p->ncol_tiles = (ncols + p->cw - 1) / p->cw;
  p->kxw = p->ncol_tiles * p->cw;
  p->frame_inter_bytes = (size_t)H * p->kxw * sizeof(float2);
  size_t inter_target = kInterTargetBytes;
  if (const char* v = std::getenv("DDM_INTER_MB")) {  // tuning: row-intermediate bytes per batch
    const long mb = std::atol(v);
    if (mb >= 1 && mb <= 4096) inter_target = (size_t)mb << 20;
  }
  p->fb_target = (int)std::max<size_t>(1, std::min<size_t>(N, inter_target / p->frame_inter_bytes));
  // Step one in one launch where it applies (DDM_STEP1=split keeps the two
  // kernels): its intermediates (step1_bufs() frames per XCD) and control words
  // take the place of the batch of intermediates.
  p->fused = step1_fusable(W, H, p->ncol_tiles, p->kxw);
  if (const char* v = std::getenv("DDM_STEP1")) p->fused = p->fused && std::strcmp(v, "split") != 0;
  p->s1_nwg = p->s1_maxslots = p->s1_frames = 0;
  if (p->fused) {
    const int ipf = H / 32 + p->ncol_tiles;  // row items (32 rows each) + column items per frame
    p->s1_nwg = step1_workgroups(W);
    p->s1_maxslots = N + p->s1_nwg / ipf + 4 + step1_lag();
    const size_t ctl_bytes = step1_ctl_words(p->s1_maxslots) * sizeof(int32_t);
    p->s1_frames = 8 * step1_bufs() + (int)((ctl_bytes + p->frame_inter_bytes - 1) / p->frame_inter_bytes);
    p->fb_target = p->s1_frames;
  }
  // Slots of the blocked store: the kept kx < KR of row ky fill slots
  // sbase[ky] + kx, each row rounded up to whole blocks, so that a column tile
  // of 16 writes whole 128-byte lines; packed Nyquist values (ky, W/2) follow
  // in slots sN + ky.
  {
    const int KR = p->kxnyq > 0 ? W / 2 : kxn;
    p->sbase.assign(H, 0);
    int64_t acc = 0;
    for (int ky = 0; ky < H; ++ky) {
      p->sbase[ky] = (int32_t)acc;
      const int r = std::min(p->kxcnt[ky], KR);
      acc += (r + kSpecQB - 1) / kSpecQB * kSpecQB;
    }
    p->sN = -1;
    if (p->kxnyq > 0) {
      p->sN = (int)acc;
      acc += (H + kSpecQB - 1) / kSpecQB * kSpecQB;
    }
    p->nslots = acc;
  }
  if (p->nslots > INT32_MAX) {
    delete p;
    return fail(DDM_ERR_UNSUPPORTED, "too many wave vectors");
  }
  std::vector<int32_t> qmap((size_t)p->nslots, -1);
  for (int ky = 0; ky < H; ++ky) {
    const int r = std::min(p->kxcnt[ky], p->kxnyq > 0 ? W / 2 : kxn);
    for (int kx = 0; kx < r; ++kx) qmap[(size_t)p->sbase[ky] + kx] = p->qoff[ky] + kx;
    if (p->kxnyq > 0 && p->kxcnt[ky] == W / 2 + 1) qmap[(size_t)p->sN + ky] = p->qoff[ky] + W / 2;
  }
  p->stream = (hipStream_t)desc->stream;
  p->f16 = desc->spectrum == DDM_SPEC_F16_QSCALED;
  for (int j = 1; j <= 7; ++j) p->pilot.push_back((int)((int64_t)j * N / 8));
  p->pilot.push_back(N - 1);
  std::sort(p->pilot.begin(), p->pilot.end());
  p->pilot.erase(std::unique(p->pilot.begin(), p->pilot.end()), p->pilot.end());

  // device tables: twiddles for W, H, 2L; q offsets and counts per ky row;
  // slot map; pilot frames
  const size_t ntw = (size_t)W + H + 2 * (size_t)p->L;
  std::vector<float2> tw(ntw);
  fill_twiddles(tw, 0, W);
  fill_twiddles(tw, W, H);
  fill_twiddles(tw, W + H, 2 * p->L);
  const size_t tw_bytes = align256(ntw * sizeof(float2));
  const size_t ramp_bytes = align256((size_t)N * sizeof(double));
  std::vector<double> ramp(N);
  for (int m = 0; m < N; ++m) ramp[m] = 1.0 / (double)(N - m);
  const size_t qmap_bytes = align256((size_t)p->nslots * sizeof(int32_t));
  const size_t pilot_bytes = align256(p->pilot.size() * sizeof(int32_t));
  const size_t tab_bytes = tw_bytes + ramp_bytes + 3 * align256(H * sizeof(int32_t)) + qmap_bytes + pilot_bytes;
  hipError_t e = hipMalloc(&p->dev_tables, tab_bytes);
  if (e != hipSuccess) {
    delete p;
    return hip_fail(e, "hipMalloc(plan tables)");
  }
  char* base = (char*)p->dev_tables;
  p->twW = (float2*)base;
  p->twH = p->twW + W;
  p->twT = p->twH + H;
  p->ramp = (double*)(base + tw_bytes);
  p->qoff_d = (int32_t*)(base + tw_bytes + ramp_bytes);
  p->kxcnt_d = (int32_t*)(base + tw_bytes + ramp_bytes + align256(H * sizeof(int32_t)));
  p->sbase_d = (int32_t*)(base + tw_bytes + ramp_bytes + 2 * align256(H * sizeof(int32_t)));
  p->qmap_d = (int32_t*)(base + tw_bytes + ramp_bytes + 3 * align256(H * sizeof(int32_t)));
  p->pilot_d = (int32_t*)((char*)p->qmap_d + qmap_bytes);
  if ((e = hipMemcpy(p->twW, tw.data(), ntw * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->ramp, ramp.data(), N * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->qoff_d, p->qoff.data(), H * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->kxcnt_d, p->kxcnt.data(), H * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->sbase_d, p->sbase.data(), H * sizeof(int32_t), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(p->qmap_d, qmap.data(), (size_t)p->nslots * sizeof(int32_t), hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(p->pilot_d, p->pilot.data(), p->pilot.size() * sizeof(int32_t), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    hipFree(p->dev_tables);
    delete p;
    return hip_fail(e, "hipMemcpy(plan tables)");
  }
  p->thr_d = nullptr;
  p->thr_pin = nullptr;
  p->thr_cap = 0;
  p->thr_ev = nullptr;
  p->ws = nullptr;
  p->ws_bytes = 0;
  p->prof_mask = 0;
  for (int i = 0; i < 5; ++i) {
    p->prof_ms[i] = 0.0;
    p->prof_n[i] = 0;
  }
  p->sat_total = 0;
  p->rb_host = nullptr;
  p->rb_next = 0;
  p->s1_failed = false;
  p->sat_unreported = 0;
  p->outcome_dev = nullptr;
  p->batch_nbins = 0;
  {
    const char* v = std::getenv("DDM_STEP1_FAIL");
    p->s1_force_err = v != nullptr && std::strcmp(v, "1") == 0;
  }
  for (int i = 0; i < kReadback; ++i) {
    p->rb_ev[i] = nullptr;
    p->rb_pending[i] = false;
  }
  if (p->f16 || p->fused) {
    e = hipHostMalloc((void**)&p->rb_host, 2 * kReadback * sizeof(int32_t), hipHostMallocDefault);
    for (int i = 0; i < kReadback && e == hipSuccess; ++i)
      e = hipEventCreateWithFlags(&p->rb_ev[i], hipEventDisableTiming);
    if (e != hipSuccess) {
      for (int i = 0; i < kReadback; ++i)
        if (p->rb_ev[i]) hipEventDestroy(p->rb_ev[i]);
      if (p->rb_host) hipHostFree(p->rb_host);
      hipFree(p->dev_tables);
      delete p;
      return hip_fail(e, "readback setup");
    }
    std::memset(p->rb_host, 0, 2 * kReadback * sizeof(int32_t));
  }
  p->s_copy = nullptr;
  p->ev_start = nullptr;
  for (int i = 0; i < 2; ++i) p->ev_h2d[i] = p->ev_used[i] = nullptr;
  e = hipStreamCreateWithFlags(&p->s_copy, hipStreamNonBlocking);
  for (int i = 0; i < 2 && e == hipSuccess; ++i) {
    e = hipEventCreateWithFlags(&p->ev_h2d[i], hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_used[i], hipEventDisableTiming);
  }
  if (e == hipSuccess) e = hipEventCreateWithFlags(&p->ev_start, hipEventDisableTiming);
  if (e != hipSuccess) {
    ddm_plan_destroy(p);
    return hip_fail(e, "copy stream setup");
  }
  if (log_on()) {
    size_t mn = 0, full = 0;
    ddm_plan_workspace_size(p, &mn, &full);
    ddm_log("plan %p: %dx%d %s x %d frames, %lld q, %d lags, %s spectra, step two %s%s (L %d), step one %s, "
            "workspace min %.1f MB full %.1f MB",
            (void*)p, W, H, desc->pixel == DDM_PIX_U8 ? "u8" : "u16", N, (long long)p->nq, p->M,
            p->f16 ? "FP16" : "FP32", p->method == DDM_METHOD_DIRECT ? "direct" : "fourier",
            desc->method == DDM_METHOD_AUTO ? " (auto: cost model)" : "", p->L,
            p->fused ? "single launch" : "row + column kernels", mn / 1e6, full / 1e6);
  }
  *out = p;
  g_err.clear();
  return DDM_OK;
}

ddm_status ddm_plan_destroy(ddm_plan_t p) {
  if (p == nullptr) return DDM_OK;
  if (p->magic != kPlanMagic) return fail(DDM_ERR_STATE, "plan handle is not a live plan");
  hipStreamSynchronize(p->stream);
  if (p->s_copy) hipStreamSynchronize(p->s_copy);
  prof_drain(p);
  for (int i = 0; i < 2; ++i) {
    if (p->ev_h2d[i]) hipEventDestroy(p->ev_h2d[i]);
    if (p->ev_used[i]) hipEventDestroy(p->ev_used[i]);
  }
  if (p->ev_start) hipEventDestroy(p->ev_start);
  if (p->s_copy) hipStreamDestroy(p->s_copy);
  for (int i = 0; i < kReadback; ++i)
    if (p->rb_ev[i]) hipEventDestroy(p->rb_ev[i]);
  if (p->rb_host) hipHostFree(p->rb_host);
  p->magic = 0;
  if (p->dev_tables) hipFree(p->dev_tables);
  if (p->thr_d) hipFree(p->thr_d);
  if (p->thr_pin) hipHostFree(p->thr_pin);
  if (p->thr_ev) hipEventDestroy(p->thr_ev);
  delete p;
  return DDM_OK;
}

ddm_status ddm_plan_method(ddm_plan_t p, int32_t* method) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (method == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "method is NULL");
  *method = p->method;
  return DDM_OK;
}

ddm_status ddm_plan_query(ddm_plan_t p, int64_t* n_q, int32_t* max_lag, int32_t* n2) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (n_q) *n_q = p->nq;
  if (max_lag) *max_lag = p->M;
  if (n2) *n2 = p->n2_paper;
  return DDM_OK;
}

ddm_status ddm_plan_q_index(ddm_plan_t p, int32_t* kx_host, int32_t* ky_signed_host) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (kx_host == nullptr || ky_signed_host == nullptr)
    return fail(DDM_ERR_INVALID_ARGUMENT, "output arrays must be non-NULL");
  for (int ky = 0; ky < p->H; ++ky) {
    const int kys = ky <= p->H / 2 ? ky : ky - p->H;
    for (int kx = 0; kx < p->kxcnt[ky]; ++kx) {
      kx_host[p->qoff[ky] + kx] = kx;
      ky_signed_host[p->qoff[ky] + kx] = kys;
    }
  }
  return DDM_OK;
}

static size_t spec_elem_bytes(const ddm_plan_s* p) { return p->f16 ? 4 : sizeof(float2); }
static size_t spec_block_bytes(const ddm_plan_s* p) { return (size_t)p->N * kSpecQB * spec_elem_bytes(p); }
static int64_t n_spec_blocks(const ddm_plan_s* p) { return p->nslots / kSpecQB; }
// FP16 store only: pilot spectra [nq][np], per-q exponents, saturation
// counter, the exponents on the (ky, kx) grid [H][W/2 + 1] (int8)
static size_t aux_bytes(const ddm_plan_s* p) {
  if (!p->f16) return 0;
  return align256((size_t)p->nq * p->pilot.size() * sizeof(float2)) + align256((size_t)p->nq * 4) + 256 +
         align256((size_t)p->H * (p->W / 2 + 1));
}

ddm_status ddm_plan_workspace_size(ddm_plan_t p, size_t* min_bytes, size_t* full_bytes) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  const size_t fib = align256(p->frame_inter_bytes);
  if (full_bytes) *full_bytes = aux_bytes(p) + align256((size_t)p->fb_target * p->frame_inter_bytes) +
                                (size_t)n_spec_blocks(p) * spec_block_bytes(p);
  if (min_bytes) *min_bytes = aux_bytes(p) + fib + spec_block_bytes(p);
  return DDM_OK;
}

static void partition(const ddm_plan_s* p, int* fb, int64_t* gblocks);

ddm_status ddm_plan_set_workspace(ddm_plan_t p, void* ws, size_t bytes) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  size_t mn = 0;
  ddm_plan_workspace_size(p, &mn, nullptr);
  if (ws == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  if (bytes < mn) return fail(DDM_ERR_OUT_OF_MEMORY, "workspace %zu bytes < minimum %zu", bytes, mn);
  p->ws = ws;
  p->ws_bytes = bytes;
  if (log_on()) {
    int fb;
    int64_t gblocks;
    partition(p, &fb, &gblocks);
    const int64_t groups = (n_spec_blocks(p) + gblocks - 1) / gblocks;
    ddm_log("plan %p: workspace %.1f MB: %d frames of row intermediate, %lld group(s) of wave vectors%s",
            (void*)p, bytes / 1e6, fb, (long long)groups, groups > 1 ? " (every frame transformed per group)" : "");
  }
  return DDM_OK;
}

// Step two over slots [0, nslots) of a spectra store (layout qb: 16 blocked,
// 1 plain) with the plan's method.
static hipError_t launch_step_two(ddm_plan_s* p, const void* spec, int qb, int64_t nslots, const int32_t* qmap,
                                  const int32_t* qexp, float* D) {
  if (p->method == DDM_METHOD_DIRECT) return launch_direct(p->stream, spec, qb, nslots, p->N, p->M, qmap, qexp, D);
  return launch_time(p->stream, p->L, spec, qb, nslots, p->N, p->M, p->twT, p->ramp, qmap, qexp, D, p->tshape);
}

// Split the workspace (after the FP16 auxiliaries) into the row intermediate
// (fb frames) and the spectra store of one group (gblocks q-blocks).
static void partition(const ddm_plan_s* p, int* fb, int64_t* gblocks) {
  const size_t blk = spec_block_bytes(p);
  const int64_t nb = n_spec_blocks(p);
  const size_t fib = p->frame_inter_bytes;
  const size_t all_spec = (size_t)nb * blk;
  const size_t room_all = p->ws_bytes - aux_bytes(p);
  int f;
  int64_t g;
  if (room_all >= all_spec + align256(fib)) {
    g = nb;
    size_t room = room_all - all_spec;
    f = (int)std::min<size_t>(p->fb_target, std::max<size_t>(1, room / fib));
    while (f > 1 && align256((size_t)f * fib) > room) --f;
  } else {
    f = (int)std::min<size_t>(p->fb_target, std::max<size_t>(1, (room_all / 8) / fib));
    g = (int64_t)((room_all - align256((size_t)f * fib)) / blk);
    if (g < 1) {
      f = 1;
      g = (int64_t)((room_all - align256(fib)) / blk);
    }
  }
  *fb = f;
  *gblocks = g;
}

// Step one in one launch: the plan is fused and the workspace holds its frame
// buffers and control words (blocked store only).
static bool step_one_fused(const ddm_plan_s* p, int fb, int qb) {
  return p->fused && qb == kSpecQB && fb >= p->s1_frames;
}

// Control words of the fused step one, after its frame buffers; the last word
// is its error flag.
static int* step_one_ctl(const ddm_plan_s* p, float2* inter) {
  return (int*)(inter + (size_t)8 * step1_bufs() * ((size_t)p->H * p->kxw));
}

// Step one for frames 0..N-1 into slots [s_lo, s_hi): the blocked store
// (qb = 16, the plan's slot tables) or the plain [q][N] layout (qb = 1, slot = q).
// first: the first group of a call (the fused form clears its error flag;
// later groups keep it, so the flag covers the whole call).
static ddm_status run_step_one(ddm_plan_s* p, const void* frames, float2* inter, int fb, int64_t s_lo,
                               int64_t s_hi, int qb, SpecOut out, bool first) {
  QTable qt{p->qoff_d, p->kxcnt_d};
  const SlotMap sm = (qb == 1) ? SlotMap{p->qoff_d, -1} : SlotMap{p->sbase_d, p->sN};
  if (step_one_fused(p, fb, qb)) {
    hipError_t e;
    {
      ProfScope ps(p, DDM_KERNEL_STEP1);
      e = launch_step1(p->stream, p->d.pixel, frames, p->W, p->N, p->d.precondition, inter, p->kxw, p->ncol_tiles,
                       p->kxnyq, qt, sm, s_lo, s_hi, out, p->twW, p->twH, step_one_ctl(p, inter),
                       p->s1_maxslots, p->s1_nwg, step1_bufs(), first ? (p->s1_force_err ? 1 : 0) : -1);
    }
    if (e != hipSuccess) return hip_fail(e, "step one launch");
    return DDM_OK;
  }
  for (int t0 = 0; t0 < p->N; t0 += fb) {
    const int nf = std::min(fb, p->N - t0);
    hipError_t e;
    {
      ProfScope ps(p, DDM_KERNEL_ROW);
      e = launch_row(p->stream, p->d.pixel, frames, p->W, p->H, t0, nullptr, nf, p->d.precondition,
                     inter, p->kxw, p->kxnyq > 0, p->twW, 1);
    }
    if (e != hipSuccess) return hip_fail(e, "row transform launch");
    {
      ProfScope ps(p, DDM_KERNEL_COL);
      e = launch_col(p->stream, inter, p->H, p->kxw, p->ncol_tiles, t0, nf, p->N, qt, sm, s_lo, s_hi, qb,
                     p->kxnyq, out, p->twH, 1);
    }
    if (e != hipSuccess) return hip_fail(e, "column transform launch");
  }
  return DDM_OK;
}

// FP16 store: transform the pilot frames (FP32, [nq][np]) as many at a time as
// the intermediate holds, derive the per-q exponents, clear the saturation
// counter.
static ddm_status run_pilot(ddm_plan_s* p, const void* frames, float2* inter, int fb, float2* pilot,
                            int32_t* qexp, int32_t* sat, int8_t* qgrid) {
  QTable qt{p->qoff_d, p->kxcnt_d};
  const int np = (int)p->pilot.size();
  for (int i0 = 0; i0 < np; i0 += fb) {
    const int nf = std::min(fb, np - i0);
    hipError_t e = launch_row(p->stream, p->d.pixel, frames, p->W, p->H, 0, p->pilot_d + i0, nf,
                              p->d.precondition, inter, p->kxw, p->kxnyq > 0, p->twW, 1);
    if (e == hipSuccess)
      e = launch_col(p->stream, inter, p->H, p->kxw, p->ncol_tiles, i0, nf, np, qt, SlotMap{p->qoff_d, -1}, 0,
                     p->nq, 1, p->kxnyq, SpecOut{pilot, nullptr, nullptr}, p->twH, 1);
    if (e != hipSuccess) return hip_fail(e, "pilot transform launch");
  }
  hipError_t e = launch_qexp(p->stream, pilot, np, p->nq, qexp);
  if (e == hipSuccess) e = launch_qgrid(p->stream, qexp, qt, p->H, p->W / 2 + 1, qgrid);
  if (e == hipSuccess) e = launch_fill_i32(p->stream, sat, 1, 0);
  if (e != hipSuccess) return hip_fail(e, "FP16 scale launch");
  return DDM_OK;
}

// Fold readback slot i (its copies have completed).
static void rb_fold(ddm_plan_s* p, int i) {
  const int32_t* v = p->rb_host + 2 * i;
  if (v[0] != 0) p->s1_failed = true;
  p->sat_total += v[1];
  p->sat_unreported += v[1];
  p->rb_pending[i] = false;
}

// Fold every slot whose copies have completed; wait for them all when `wait`.
static hipError_t rb_collect(ddm_plan_s* p, bool wait) {
  for (int k = 0; k < kReadback; ++k) {
    const int i = (p->rb_next + k) % kReadback;  // oldest first
    if (!p->rb_pending[i]) continue;
    hipError_t e = wait ? hipEventSynchronize(p->rb_ev[i]) : hipEventQuery(p->rb_ev[i]);
    if (e == hipErrorNotReady) return hipSuccess;  // later slots are later still
    if (e != hipSuccess) return e;
    rb_fold(p, i);
  }
  return hipSuccess;
}

// Enqueue the copies of this call's error flag (err_dev, or 0 if NULL) and
// saturation count (sat_dev, or 0) into the next slot.
static hipError_t rb_push(ddm_plan_s* p, const int32_t* err_dev, const int32_t* sat_dev) {
  const int i = p->rb_next;
  if (p->rb_pending[i]) {
    hipError_t e = hipEventSynchronize(p->rb_ev[i]);
    if (e != hipSuccess) return e;
    rb_fold(p, i);
  }
  int32_t* v = p->rb_host + 2 * i;
  v[0] = v[1] = 0;
  hipError_t e = hipSuccess;
  if (err_dev != nullptr) e = hipMemcpyAsync(v, err_dev, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess && sat_dev != nullptr)
    e = hipMemcpyAsync(v + 1, sat_dev, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipEventRecord(p->rb_ev[i], p->stream);
  if (e != hipSuccess) return e;
  p->rb_pending[i] = true;
  p->rb_next = (i + 1) % kReadback;
  return hipSuccess;
}

static bool capturing(const ddm_plan_s* p) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  return hipStreamIsCapturing(p->stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone;
}

// The whole path on the workspace p->ws (p->ws_bytes); arguments checked.
static ddm_status structure_function_run(ddm_plan_s* p, const void* frames, float* D) {
  ddm_status st;
  // nothing comes back from a call made inside a graph capture
  const bool readback = p->rb_host != nullptr && !capturing(p);
  hipError_t e;
  if (readback && (e = rb_collect(p, false)) != hipSuccess) return hip_fail(e, "readback");
  if (p->s1_failed) {
    p->s1_failed = false;
    return fail(DDM_ERR_HIP, "step one: a wait between its row and column work ran out in an earlier call; "
                             "that call's result is not valid");
  }
  int fb;
  int64_t gblocks;
  partition(p, &fb, &gblocks);
  char* base = (char*)p->ws;
  float2* pilot = nullptr;
  int32_t *qexp = nullptr, *sat = nullptr;
  int8_t* qgrid = nullptr;
  if (p->f16) {
    pilot = (float2*)base;
    qexp = (int32_t*)(base + align256((size_t)p->nq * p->pilot.size() * sizeof(float2)));
    sat = (int32_t*)((char*)qexp + align256((size_t)p->nq * 4));
    qgrid = (int8_t*)sat + 256;
    base += aux_bytes(p);
  }
  float2* inter = (float2*)base;
  void* spec = base + align256((size_t)fb * p->frame_inter_bytes);
  if (p->f16) {
    st = run_pilot(p, frames, inter, fb, pilot, qexp, sat, qgrid);
    if (st != DDM_OK) return st;
  }
  const int64_t gs = gblocks * kSpecQB;
  for (int64_t s_lo = 0; s_lo < p->nslots; s_lo += gs) {
    const int64_t s_hi = std::min(p->nslots, s_lo + gs);
    st = run_step_one(p, frames, inter, fb, s_lo, s_hi, kSpecQB, SpecOut{spec, qgrid, sat, p->W / 2 + 1},
                      s_lo == 0);
    if (st != DDM_OK) return st;
    {
      ProfScope ps(p, DDM_KERNEL_TIME);
      e = launch_step_two(p, spec, kSpecQB, s_hi - s_lo, p->qmap_d + s_lo, qexp, D);
    }
    if (e != hipSuccess) return hip_fail(e, "time transform launch");
  }
  const int32_t* err = step_one_fused(p, fb, kSpecQB) ? step_one_ctl(p, inter) + step1_ctl_words(p->s1_maxslots) - 1
                                                      : nullptr;
  if (p->outcome_dev != nullptr) {
    e = err != nullptr ? launch_copy_i32(p->stream, err, p->outcome_dev, 1) : launch_fill_i32(p->stream, p->outcome_dev, 1, 0);
    if (e != hipSuccess) return hip_fail(e, "outcome copy");
  }
  if (readback && (err != nullptr || sat != nullptr)) {
    e = rb_push(p, err, sat);
    if (e != hipSuccess) return hip_fail(e, "readback copy");
  }
  if (p->sat_unreported > 0) {
    p->sat_unreported = 0;
    return DDM_WARN_FP16_SATURATED;
  }
  return DDM_OK;
}

static ddm_status check_sf_args(ddm_plan_t p, const void* frames, float* D) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (frames == nullptr || D == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "frames/D is NULL");
  if (((uintptr_t)frames & 15) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "frames must be 16-byte aligned");
  return DDM_OK;
}

ddm_status ddm_structure_function(ddm_plan_t p, const void* frames, float* D) {
  ddm_status st = check_sf_args(p, frames, D);
  if (st != DDM_OK) return st;
  if (p->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "no workspace attached (ddm_plan_set_workspace)");
  return structure_function_run(p, frames, D);
}

// ---------------------------------------------------------------------------
// The structure function on a workspace that the library holds in a static
// device array, for callers that cannot allocate device memory.  Each device
// holds its own copy of the array (from module load to process end); its
// address on a device is looked up once, with that device current, and kept.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[DDM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch` per device, or NULL before the lookup
}  // namespace

static ddm_status scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(DDM_ERR_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (ptr == nullptr || ((uintptr_t)ptr & 255) != 0)
      return fail(DDM_ERR_HIP, "static scratch has no usable device address");
    g_scratch_ptr[dev] = ptr;
    ddm_log("device %d: static scratch of %u bytes at %p", dev, (unsigned)DDM_NOALLOC_SCRATCH_BYTES, ptr);
  }
  *out = g_scratch_ptr[dev];
  return DDM_OK;
}

ddm_status ddm_structure_function_noalloc(ddm_plan_t p, const void* frames, float* D) {
  ddm_status st = check_sf_args(p, frames, D);
  if (st != DDM_OK) return st;
  size_t mn = 0;
  ddm_plan_workspace_size(p, &mn, nullptr);
  if (mn > (size_t)DDM_NOALLOC_SCRATCH_BYTES)
    return fail(DDM_ERR_UNSUPPORTED, "this plan needs at least %zu bytes of workspace; the static scratch holds %zu",
                mn, (size_t)DDM_NOALLOC_SCRATCH_BYTES);
  void* ptr = nullptr;
  if ((st = scratch_address(&ptr)) != DDM_OK) return st;
  // the call runs on the scratch in place of the attached workspace, which is
  // left as it was
  void* ws = p->ws;
  const size_t ws_bytes = p->ws_bytes;
  p->ws = ptr;
  p->ws_bytes = DDM_NOALLOC_SCRATCH_BYTES;
  st = structure_function_run(p, frames, D);
  p->ws = ws;
  p->ws_bytes = ws_bytes;
  return st;
}

// ---------------------------------------------------------------------------
// Frames resident in host memory: batches of frames go to the device through
// two staging halves on a copy stream while the row and column transforms of
// the previous batch run; frame 0 (the preconditioning reference) has a slot
// of its own.  Every group of wave vectors streams the frames again (the
// paper's group execution, Appendix C, with the frames re-read from the host).
// ---------------------------------------------------------------------------
ddm_status ddm_structure_function_host(ddm_plan_t p, const void* frames_host, void* staging, size_t staging_bytes,
                                       float* D) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (frames_host == nullptr || staging == nullptr || D == nullptr)
    return fail(DDM_ERR_INVALID_ARGUMENT, "frames_host/staging/D is NULL");
  if (((uintptr_t)staging & 255) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "staging must be 256-byte aligned");
  if (p->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "no workspace attached (ddm_plan_set_workspace)");
  if (p->f16) return fail(DDM_ERR_UNSUPPORTED, "host-resident frames take the FP32 spectrum store");
  if (capturing(p)) return fail(DDM_ERR_UNSUPPORTED, "host-resident frames: not inside a graph capture");
  const size_t fbytes = (size_t)p->W * p->H * (p->d.pixel == DDM_PIX_U8 ? 1 : 2);
  const size_t slot0 = align256(fbytes);
  if (staging_bytes < slot0 + 2 * fbytes)
    return fail(DDM_ERR_OUT_OF_MEMORY, "staging %zu bytes < %zu (frame 0 and two frames)", staging_bytes,
                slot0 + 2 * fbytes);
  int fb;
  int64_t gblocks;
  partition(p, &fb, &gblocks);
  const int per_half = (int)std::min<size_t>((size_t)fb, (staging_bytes - slot0) / 2 / fbytes);
  const size_t half_bytes = align256((size_t)per_half * fbytes);
  const int nf_batch = (slot0 + 2 * half_bytes <= staging_bytes) ? per_half : std::max(1, per_half - 1);
  char* stage0 = (char*)staging;
  char* half[2] = {stage0 + slot0, stage0 + slot0 + align256((size_t)nf_batch * fbytes)};
  char* base = (char*)p->ws;
  float2* inter = (float2*)base;
  void* spec = base + align256((size_t)fb * p->frame_inter_bytes);
  QTable qt{p->qoff_d, p->kxcnt_d};
  const SlotMap sm{p->sbase_d, p->sN};
  const char* host = (const char*)frames_host;
  // the copies start once the plan's stream has reached this call (earlier
  // calls may still read the staging memory)
  hipError_t e = hipEventRecord(p->ev_start, p->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->s_copy, p->ev_start, 0);
  if (e == hipSuccess) e = hipMemcpyAsync(stage0, host, fbytes, hipMemcpyHostToDevice, p->s_copy);
  if (e != hipSuccess) return hip_fail(e, "frame 0 copy");
  const int64_t gs = gblocks * kSpecQB;
  int bi = 0;
  for (int64_t s_lo = 0; s_lo < p->nslots; s_lo += gs) {
    const int64_t s_hi = std::min(p->nslots, s_lo + gs);
    for (int t0 = 0; t0 < p->N; t0 += nf_batch, ++bi) {
      const int nf = std::min(nf_batch, p->N - t0);
      const int k = bi % 2;
      if (bi >= 2 && (e = hipStreamWaitEvent(p->s_copy, p->ev_used[k], 0)) != hipSuccess)
        return hip_fail(e, "staging order");
      e = hipMemcpyAsync(half[k], host + (size_t)t0 * fbytes, (size_t)nf * fbytes, hipMemcpyHostToDevice,
                         p->s_copy);
      if (e == hipSuccess) e = hipEventRecord(p->ev_h2d[k], p->s_copy);
      if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_h2d[k], 0);
      if (e != hipSuccess) return hip_fail(e, "frame batch copy");
      {
        ProfScope ps(p, DDM_KERNEL_ROW);
        // the batch's frames are frames 0.. of the staging half; frame 0 of the stack is the reference
        e = launch_row(p->stream, p->d.pixel, half[k], p->W, p->H, 0, nullptr, nf, p->d.precondition, inter, p->kxw,
                       p->kxnyq > 0, p->twW, 1, stage0);
      }
      if (e == hipSuccess) e = hipEventRecord(p->ev_used[k], p->stream);
      if (e != hipSuccess) return hip_fail(e, "row transform launch");
      {
        ProfScope ps(p, DDM_KERNEL_COL);
        e = launch_col(p->stream, inter, p->H, p->kxw, p->ncol_tiles, t0, nf, p->N, qt, sm, s_lo, s_hi, kSpecQB,
                       p->kxnyq, SpecOut{spec, nullptr, nullptr}, p->twH, 1);
      }
      if (e != hipSuccess) return hip_fail(e, "column transform launch");
    }
    {
      ProfScope ps(p, DDM_KERNEL_TIME);
      e = launch_step_two(p, spec, kSpecQB, s_hi - s_lo, p->qmap_d + s_lo, nullptr, D);
    }
    if (e != hipSuccess) return hip_fail(e, "time transform launch");
  }
  // the copy stream's last work (frame 0 only, for N = 1 batch) is ordered before
  // the plan's stream continues
  e = hipEventRecord(p->ev_start, p->s_copy);
  if (e == hipSuccess) e = hipStreamWaitEvent(p->stream, p->ev_start, 0);
  if (e != hipSuccess) return hip_fail(e, "copy join");
  return DDM_OK;
}

ddm_status ddm_plan_status(ddm_plan_t p) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (capturing(p)) return fail(DDM_ERR_STATE, "ddm_plan_status waits for the stream; not allowed during a graph capture");
  hipError_t e = hipStreamSynchronize(p->stream);
  if (e == hipSuccess && p->rb_host != nullptr) e = rb_collect(p, true);
  if (e != hipSuccess) return hip_fail(e, "plan status");
  if (p->s1_failed) {
    p->s1_failed = false;
    p->sat_unreported = 0;
    return fail(DDM_ERR_HIP, "step one: a wait between its row and column work ran out; that call's result is not valid");
  }
  if (p->sat_unreported > 0) {
    p->sat_unreported = 0;
    return DDM_WARN_FP16_SATURATED;
  }
  return DDM_OK;
}

ddm_status ddm_plan_fp16_saturations(ddm_plan_t p, int64_t* count) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (count == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "count is NULL");
  if (p->rb_host != nullptr && !capturing(p)) {
    hipError_t e = rb_collect(p, true);
    if (e != hipSuccess) return hip_fail(e, "saturation count");
  }
  *count = p->sat_total;
  return DDM_OK;
}

ddm_status ddm_image_spectra(ddm_plan_t p, const void* frames, float* spectra) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (frames == nullptr || spectra == nullptr)
    return fail(DDM_ERR_INVALID_ARGUMENT, "frames/spectra is NULL");
  if (((uintptr_t)frames & 15) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "frames must be 16-byte aligned");
  if (p->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "no workspace attached (ddm_plan_set_workspace)");
  const size_t fib = p->frame_inter_bytes;
  int fb = (int)std::min<size_t>(p->fb_target, std::max<size_t>(1, p->ws_bytes / fib));
  while (fb > 1 && (size_t)fb * fib > p->ws_bytes) --fb;
  return run_step_one(p, frames, (float2*)p->ws, fb, 0, p->nq, 1, SpecOut{spectra, nullptr, nullptr}, true);
}

ddm_status ddm_structure_from_spectra(ddm_plan_t p, const float* spectra, float* D) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (spectra == nullptr || D == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "spectra/D is NULL");
  hipError_t e;
  {
    ProfScope ps(p, DDM_KERNEL_TIME);
    e = launch_step_two(p, spectra, 1, p->nq, nullptr, nullptr, D);
  }
  if (e != hipSuccess) return hip_fail(e, "time transform launch");
  return DDM_OK;
}

static ddm_status check_thresholds(const int64_t* thr, int32_t n_bins) {
  if (n_bins < 0) return fail(DDM_ERR_INVALID_ARGUMENT, "n_bins must be >= 0");
  if (thr == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "thresholds is NULL");
  if (thr[0] < 0) return fail(DDM_ERR_INVALID_ARGUMENT, "thresholds must be >= 0");
  for (int b = 0; b < n_bins; ++b)
    if (thr[b + 1] < thr[b])
      return fail(DDM_ERR_INVALID_ARGUMENT, "thresholds must be non-decreasing (at %d)", b);
  return DDM_OK;
}

// The plan's device copy of the bin thresholds (checked), sent on its stream
// through the pinned buffer once the previous launch that read the device copy
// has finished; unchanged thresholds are not sent again.
static ddm_status upload_thresholds(ddm_plan_s* p, const int64_t* thr, int32_t n_bins) {
  const size_t nthr = (size_t)n_bins + 1;
  const size_t need = nthr * sizeof(int64_t);
  hipError_t e = hipSuccess;
  if (p->thr_ev == nullptr && (e = hipEventCreateWithFlags(&p->thr_ev, hipEventDisableTiming)) != hipSuccess) {
    p->thr_ev = nullptr;
    return hip_fail(e, "hipEventCreate(thresholds)");
  }
  if (p->thr_last.size() != nthr || std::memcmp(p->thr_last.data(), thr, need) != 0) {
    p->thr_last.clear();
    if ((e = hipEventSynchronize(p->thr_ev)) != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    if (need > p->thr_cap) {
      if (p->thr_d) hipFree(p->thr_d);
      if (p->thr_pin) hipHostFree(p->thr_pin);
      p->thr_d = nullptr;
      p->thr_pin = nullptr;
      p->thr_cap = 0;
      if ((e = hipMalloc(&p->thr_d, need)) != hipSuccess) return hip_fail(e, "hipMalloc(thresholds)");
      if ((e = hipHostMalloc((void**)&p->thr_pin, need, hipHostMallocDefault)) != hipSuccess) {
        hipFree(p->thr_d);
        p->thr_d = nullptr;
        return hip_fail(e, "hipHostMalloc(thresholds)");
      }
      p->thr_cap = need;
    }
    std::memcpy(p->thr_pin, thr, need);
    e = hipMemcpyAsync(p->thr_d, p->thr_pin, need, hipMemcpyHostToDevice, p->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(thresholds)");
    p->thr_last.assign(thr, thr + nthr);
  }
  return DDM_OK;
}

ddm_status ddm_radial_average(ddm_plan_t p, const float* D, const int64_t* thr, int32_t n_bins,
                              double* Dbar, int64_t* counts, int32_t* bin_of_q) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (D == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "D is NULL");
  if ((st = check_thresholds(thr, n_bins)) != DDM_OK) return st;
  if (n_bins > 0 && (Dbar == nullptr || counts == nullptr))
    return fail(DDM_ERR_INVALID_ARGUMENT, "Dbar/counts is NULL");
  if ((st = upload_thresholds(p, thr, n_bins)) != DDM_OK) return st;
  hipError_t e;
  QTable qt{p->qoff_d, p->kxcnt_d};
  ProfScope ps(p, DDM_KERNEL_RADIAL);
  e = launch_radial(p->stream, D, p->nq, p->M, p->W, p->H, p->ca, p->cc, qt, p->thr_d, n_bins, Dbar,
                    counts, bin_of_q);
  if (e == hipSuccess) e = hipEventRecord(p->thr_ev, p->stream);
  if (e != hipSuccess) return hip_fail(e, "radial average launch");
  return DDM_OK;
}

ddm_status ddm_plan_set_profiling(ddm_plan_t p, uint32_t mask) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (mask & ~31u) return fail(DDM_ERR_INVALID_ARGUMENT, "unknown kernel kind bits in mask 0x%x", mask);
  hipError_t e = prof_drain(p);
  p->prof_mask = mask;
  for (int i = 0; i < 5; ++i) {
    p->prof_ms[i] = 0.0;
    p->prof_n[i] = 0;
  }
  if (e != hipSuccess) return hip_fail(e, "profiling events");
  return DDM_OK;
}

ddm_status ddm_plan_get_profile(ddm_plan_t p, uint32_t kind, double* total_ms, int64_t* launches) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  const int s = kind_slot(kind);
  if (s < 0) return fail(DDM_ERR_INVALID_ARGUMENT, "kernel_kind must be a single ddm_kernel_kind");
  hipError_t e = prof_drain(p);
  if (e != hipSuccess) return hip_fail(e, "profiling events");
  if (total_ms) *total_ms = p->prof_ms[s];
  if (launches) *launches = p->prof_n[s];
  return DDM_OK;
}

static ddm_status fill_lags(const float* lags, int32_t K, float lo, float hi, LagSet* out) {
  if (lags == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "lags is NULL");
  if (K < 1 || K > DDM_FIT_MAX_K) return fail(DDM_ERR_INVALID_ARGUMENT, "K must be in [1, 64]");
  out->K = K;
  for (int j = 0; j < DDM_FIT_MAX_K; ++j) out->m[j] = 0.f;
  for (int j = 0; j < K; ++j) {
    const float m = lags[j];
    if (!std::isfinite(m) || m < lo || m > hi)
      return fail(DDM_ERR_INVALID_ARGUMENT, "lag %d = %g outside [%g, %g]", j, (double)m, (double)lo, (double)hi);
    out->m[j] = m;
  }
  return DDM_OK;
}

ddm_status ddm_sample_curves(const float* D, int64_t n_rows, int32_t M, const float* lags, int32_t K,
                             float* curves, float* scale, void* stream) {
  if (D == nullptr || curves == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "D/curves is NULL");
  if (n_rows < 0) return fail(DDM_ERR_INVALID_ARGUMENT, "n_rows must be >= 0");
  if (M < 2) return fail(DDM_ERR_INVALID_ARGUMENT, "M must be >= 2");
  LagSet ls;
  ddm_status st = fill_lags(lags, K, 0.f, (float)(M - 1), &ls);
  if (st != DDM_OK) return st;
  hipError_t e = launch_sample((hipStream_t)stream, D, n_rows, M, ls, curves, scale);
  if (e != hipSuccess) return hip_fail(e, "curve sampling launch");
  return DDM_OK;
}

void ddm_fit_desc_init(ddm_fit_desc* d) {
  if (d == nullptr) return;
  std::memset(d, 0, sizeof(*d));
  d->struct_size = sizeof(ddm_fit_desc);
  d->K = 64;
  d->max_iter = 200;
  d->fallback = 1;
  d->lambda0 = 1e-3;
  d->ftol = 1e-7;
  d->xtol = 1e-7;
  d->gtol = 1e-3;
  d->stream = nullptr;
}

ddm_status ddm_fit(const ddm_fit_desc* f, const float* curves, const float* lags, int64_t n, const float* init,
                   float* params, int32_t* iters, int32_t* flags) {
  if (f == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "desc is NULL");
  if (f->struct_size != sizeof(ddm_fit_desc))
    return fail(DDM_ERR_INVALID_ARGUMENT, "desc.struct_size %u != %zu", f->struct_size, sizeof(ddm_fit_desc));
  if (curves == nullptr || params == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "curves/params is NULL");
  if (n < 0) return fail(DDM_ERR_INVALID_ARGUMENT, "n must be >= 0");
  if (f->max_iter < 1) return fail(DDM_ERR_INVALID_ARGUMENT, "max_iter must be >= 1");
  if (!(f->lambda0 > 0) || !(f->ftol >= 0) || !(f->xtol >= 0) || !(f->gtol >= 0))
    return fail(DDM_ERR_INVALID_ARGUMENT, "lambda0 must be > 0 and tolerances >= 0");
  if (f->fallback < 0 || f->fallback > 3) return fail(DDM_ERR_INVALID_ARGUMENT, "fallback must be 0, 1, 2 or 3");
  const bool fb = init != nullptr && f->fallback == 1;
  const int start_mode = init == nullptr ? 0 : (f->fallback == 2 ? 1 : (f->fallback == 3 ? 2 : 0));
  if (fb && flags == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "fallback needs flags_dev");
  LagSet ls;
  ddm_status st = fill_lags(lags, f->K, 1e-30f, 3.0e38f, &ls);
  if (st != DDM_OK) return st;
  LmParams prm;
  prm.lambda0 = f->lambda0;
  prm.lambda_max = 1e16;
  prm.ftol = f->ftol;
  prm.xtol = f->xtol;
  prm.gtol = f->gtol;
  prm.exact_fit = 1e-12;  // relative cost floor of FP32 residuals
  prm.max_iter = f->max_iter;
  hipStream_t s = (hipStream_t)f->stream;
  hipError_t e = launch_lm(s, curves, n, ls, init, prm, nullptr, params, iters, flags, start_mode);
  if (e == hipSuccess && fb) e = launch_lm(s, curves, n, ls, nullptr, prm, flags, params, iters, flags);
  if (e != hipSuccess) return hip_fail(e, "fit launch");
  return DDM_OK;
}


// ---------------------------------------------------------------------------
// Autotuner of the time-kernel launch shape.  Candidates (E in {16, 8} x wave
// vectors per workgroup in {1, 2, 4, 8, 16}, those that fit) are timed with
// HIP events on zero-filled spectra in the plan's workspace; the fastest is
// kept per (L, N, M, storage) for the process.  DDM_AUTOTUNE=off keeps the
// built-in choice.
// ---------------------------------------------------------------------------
static std::mutex g_tune_mu;
static std::map<std::tuple<int, int, int, int>, std::tuple<int, int, double>> g_tune;
static std::map<std::tuple<int, int, int, int>, double> g_tune_direct;  // direct-method ms

// DDM_TUNE_CACHE (environment): a text file that keeps autotune results across
// processes, one line per result, keyed by device architecture, HIP runtime
// version, time length, N, max_lag and storage:
//   <arch> <runtime> <L> <N> <M> <f16> fourier <E> <qpw> <ms>
//   <arch> <runtime> <L> <N> <M> <f16> direct <ms>
// Lines of other devices or runtimes are ignored; later lines win.  Read once
// per process (under g_tune_mu), appended to after each timing.
static bool g_tune_file_read = false;

static std::string tune_device_tag() {
  int dev = 0, rt = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "";
  if (hipRuntimeGetVersion(&rt) != hipSuccess) rt = 0;
  std::string arch = prop.gcnArchName;
  for (char& c : arch)
    if (c == ' ') c = '_';
  return arch + " " + std::to_string(rt);
}

static void tune_file_read(const std::string& tag) {
  const char* path = std::getenv("DDM_TUNE_CACHE");
  if (g_tune_file_read || path == nullptr || tag.empty()) return;
  g_tune_file_read = true;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return;
  char arch[128], kind[16];
  int rt, L, N, M, f16;
  char line[512];
  int n = 0;
  while (std::fgets(line, sizeof(line), f)) {
    if (std::sscanf(line, "%127s %d %d %d %d %d %15s", arch, &rt, &L, &N, &M, &f16, kind) != 7) continue;
    if (tag != std::string(arch) + " " + std::to_string(rt)) continue;
    const auto key = std::make_tuple(L, N, M, f16);
    int E, qpw;
    double ms;
    const char* rest = std::strstr(line, kind) + std::strlen(kind);
    if (std::strcmp(kind, "fourier") == 0 && std::sscanf(rest, "%d %d %lf", &E, &qpw, &ms) == 3) {
      g_tune[key] = std::make_tuple(E, qpw, ms);
      ++n;
    } else if (std::strcmp(kind, "direct") == 0 && std::sscanf(rest, "%lf", &ms) == 1) {
      g_tune_direct[key] = ms;
      ++n;
    }
  }
  std::fclose(f);
  ddm_log("autotune cache %s: %d result(s) for %s", path, n, tag.c_str());
}

static void tune_file_append(const std::string& tag, const std::string& line) {
  const char* path = std::getenv("DDM_TUNE_CACHE");
  if (path == nullptr || tag.empty()) return;
  FILE* f = std::fopen(path, "a");
  if (f == nullptr) {
    ddm_log("autotune cache %s: cannot append", path);
    return;
  }
  std::fprintf(f, "%s %s\n", tag.c_str(), line.c_str());
  std::fclose(f);
}

ddm_status ddm_plan_autotune(ddm_plan_t p, int32_t* E_out, int32_t* qpw_out, double* ms_out) {
  ddm_status st = check_plan(p);
  if (st != DDM_OK) return st;
  if (p->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "autotune needs the workspace (ddm_plan_set_workspace)");
  const char* env = std::getenv("DDM_AUTOTUNE");
  const bool off = env && std::strcmp(env, "off") == 0;
  const bool want_fourier = p->d.method != DDM_METHOD_DIRECT && p->N <= 16384;
  const bool want_direct = p->d.method != DDM_METHOD_FOURIER;
  const auto key = std::make_tuple(p->L, p->N, p->M, (int)p->f16);
  double best_ms = -1.0, direct_ms = -1.0;
  TimeShape best = p->tshape;
  bool have = !want_fourier, have_d = !want_direct;
  const std::string tag = std::getenv("DDM_TUNE_CACHE") ? tune_device_tag() : std::string();
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    tune_file_read(tag);
    auto it = g_tune.find(key);
    if (want_fourier && it != g_tune.end()) {
      best.E = std::get<0>(it->second);
      best.qpw = std::get<1>(it->second);
      best_ms = std::get<2>(it->second);
      have = true;
    }
    auto id = g_tune_direct.find(key);
    if (want_direct && id != g_tune_direct.end()) {
      direct_ms = id->second;
      have_d = true;
    }
  }
  if ((!have || !have_d) && !off) {
    // zero-filled spectra of nq_t slots in the workspace, D into the
    // row-intermediate region
    int fb;
    int64_t gblocks;
    partition(p, &fb, &gblocks);
    char* base = (char*)p->ws + aux_bytes(p);
    float* dout = (float*)base;
    void* spec = base + align256((size_t)fb * p->frame_inter_bytes);
    int64_t nq_t = std::min<int64_t>(gblocks * kSpecQB, 65536);
    nq_t = std::min<int64_t>(nq_t, (int64_t)(((size_t)fb * p->frame_inter_bytes) / ((size_t)p->M * 4)));
    nq_t = std::min<int64_t>(nq_t, p->nq);
    if (nq_t < 1) return fail(DDM_ERR_OUT_OF_MEMORY, "workspace too small to autotune");
    const int64_t words = ((size_t)((nq_t + kSpecQB - 1) / kSpecQB) * spec_block_bytes(p)) / 4;
    hipError_t e = launch_fill_i32(p->stream, (int32_t*)spec, words, 0);
    int32_t* qexp = nullptr;
    if (p->f16 && e == hipSuccess) {
      qexp = (int32_t*)((char*)p->ws + align256((size_t)p->nq * p->pilot.size() * sizeof(float2)));
      e = launch_fill_i32(p->stream, qexp, nq_t, 0);
    }
    hipEvent_t a = nullptr, b = nullptr;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    // one untimed launch, then two timed: ms per launch over all slots
    auto time_it = [&](auto&& launch, double* ms_all) {
      e = launch();
      if (e == hipSuccess) e = hipEventRecord(a, p->stream);
      for (int r = 0; r < 2 && e == hipSuccess; ++r) e = launch();
      if (e == hipSuccess) e = hipEventRecord(b, p->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      *ms_all = ms / 2.0 * ((double)p->nslots / (double)nq_t);
    };
    if (!have && p->L == 16384) {
      // the length-16384 kernel has one launch shape (16 values per thread,
      // one wave vector per workgroup): timed for the method choice only
      const TimeShape sh{16, 1};
      time_it([&] {
        return launch_time(p->stream, p->L, spec, kSpecQB, nq_t, p->N, p->M, p->twT, p->ramp, nullptr, qexp, dout, sh);
      }, &best_ms);
      best = sh;
    } else if (!have) {
      for (int E : {16, 8, 12}) {
        for (int qpw : {1, 2, 4, 8, 16}) {
          if (e != hipSuccess) break;
          // 2^k lengths take E = 16 or 8 (8 from L = 512 on); 3 * 2^k lengths E = 12
          if ((p->L % 3 == 0) != (E == 12)) continue;
          if (p->L / E < 1 || p->L % E != 0 || (E == 8 && p->L < 512)) continue;
          if (qpw * (p->L / E) > 1024 || time_lds_bytes(p->L, qpw) > 160 * 1024) continue;
          const TimeShape sh{E, qpw};
          double ms = 0.0;
          time_it([&] {
            return launch_time(p->stream, p->L, spec, kSpecQB, nq_t, p->N, p->M, p->twT, p->ramp, nullptr, qexp, dout,
                               sh);
          }, &ms);
          if (e == hipSuccess && (best_ms < 0 || ms < best_ms)) {
            best_ms = ms;
            best = sh;
          }
        }
      }
    }
    if (!have_d && e == hipSuccess)
      time_it([&] { return launch_direct(p->stream, spec, kSpecQB, nq_t, p->N, p->M, nullptr, qexp, dout); },
              &direct_ms);
    if (a) hipEventDestroy(a);
    if (b) hipEventDestroy(b);
    if (e != hipSuccess) return hip_fail(e, "autotune");
    std::lock_guard<std::mutex> g(g_tune_mu);
    const std::string k = std::to_string(p->L) + " " + std::to_string(p->N) + " " + std::to_string(p->M) + " " +
                          std::to_string((int)p->f16);
    char v[96];
    if (!have) {
      g_tune[key] = std::make_tuple(best.E, best.qpw, best_ms);
      std::snprintf(v, sizeof(v), " fourier %d %d %.6f", best.E, best.qpw, best_ms);
      tune_file_append(tag, k + v);
    }
    if (!have_d) {
      g_tune_direct[key] = direct_ms;
      std::snprintf(v, sizeof(v), " direct %.6f", direct_ms);
      tune_file_append(tag, k + v);
    }
  }
  p->tshape = best;
  if (p->d.method == DDM_METHOD_AUTO && best_ms > 0 && direct_ms > 0)
    p->method = direct_ms < best_ms ? DDM_METHOD_DIRECT : DDM_METHOD_FOURIER;
  ddm_log("autotune plan %p (L %d, N %d, M %d, %s): transform E %d, %d per workgroup, %.3f ms%s; direct %.3f ms%s; "
          "step two %s",
          (void*)p, p->L, p->N, p->M, p->f16 ? "FP16" : "FP32", best.E, best.qpw, best_ms,
          have ? " (cached)" : "", direct_ms, have_d ? " (cached)" : "",
          p->method == DDM_METHOD_DIRECT ? "direct" : "fourier");
  if (E_out) *E_out = best.E;
  if (qpw_out) *qpw_out = best.qpw;
  if (ms_out) *ms_out = p->method == DDM_METHOD_DIRECT ? direct_ms : best_ms;
  return DDM_OK;
}

// ---------------------------------------------------------------------------
// Batches of independent stacks of uneven sizes.  Each stack has its own plan;
// stacks are spread over `lanes` streams (largest first onto the least loaded
// lane); each lane owns one slice of the workspace, reused by its stacks in
// turn.  The whole fork / join sequence is captured once into a HIP graph and
// replayed with one hipGraphLaunch per call.
// ---------------------------------------------------------------------------
struct ddm_batch_s {
  uint32_t magic;
  hipStream_t stream;  // caller's stream
  hipStream_t root;    // internal stream the graph is captured on and launched on
  hipEvent_t in_ev, out_ev;
  std::vector<ddm_plan_t> plans;
  std::vector<int> lane_of;
  std::vector<hipStream_t> lanes;
  std::vector<size_t> lane_bytes, lane_off;
  hipEvent_t fork;
  std::vector<hipEvent_t> join;
  // captured graphs, one per set of caller pointers (a caller that alternates
  // output buffers replays instead of capturing again); the least recently
  // launched is replaced when a new set arrives and the cache is full
  struct Graph {
    hipGraphExec_t exec;
    std::vector<const void*> frames;
    std::vector<float*> D;
    std::vector<double*> Dbar;
    std::vector<int64_t*> counts;
    uint64_t used;  // the call that last launched it
  };
  static constexpr size_t kGraphs = 4;
  std::vector<Graph> graphs;
  uint64_t calls;
  void* ws;
  size_t ws_bytes;
  // per-stack step-one error flags: written by the graph into flags_d, copied
  // after each launch into a ring of pinned slots (like a plan's readback), and
  // folded into `failed` once a slot's event has completed
  int32_t* flags_d;
  int32_t* flags_h;  // pinned [kReadback][n]
  hipEvent_t fl_ev[kReadback];
  bool fl_pending[kReadback];
  int fl_next;
  std::vector<int32_t> failed;
};
static constexpr uint32_t kBatchMagic = 0x44444d42u;

static ddm_status check_batch(ddm_batch_t b) {
  if (b == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "batch is NULL");
  if (b->magic != kBatchMagic) return fail(DDM_ERR_STATE, "batch handle is not live");
  return DDM_OK;
}

// Destroy every captured graph (pointers, workspace or bins changed).
static void batch_drop_graphs(ddm_batch_s* b) {
  for (auto& g : b->graphs) hipGraphExecDestroy(g.exec);
  b->graphs.clear();
}

static void batch_free(ddm_batch_s* b) {
  batch_drop_graphs(b);
  for (int i = 0; i < kReadback; ++i)
    if (b->fl_ev[i]) hipEventDestroy(b->fl_ev[i]);
  if (b->flags_h) hipHostFree(b->flags_h);
  if (b->flags_d) hipFree(b->flags_d);
  if (b->root) hipStreamDestroy(b->root);
  if (b->in_ev) hipEventDestroy(b->in_ev);
  if (b->out_ev) hipEventDestroy(b->out_ev);
  for (auto* p : b->plans) ddm_plan_destroy(p);
  for (auto s : b->lanes) hipStreamDestroy(s);
  if (b->fork) hipEventDestroy(b->fork);
  for (auto e : b->join) hipEventDestroy(e);
  b->magic = 0;
  delete b;
}

ddm_status ddm_batch_create(const ddm_plan_desc* descs, int32_t n, int32_t lanes, void* stream, ddm_batch_t* out) {
  if (out == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (descs == nullptr || n < 1) return fail(DDM_ERR_INVALID_ARGUMENT, "need at least one descriptor");
  if (lanes < 1 || lanes > 16) return fail(DDM_ERR_INVALID_ARGUMENT, "lanes must be in [1, 16]");
  for (int i = 0; i < n; ++i) {
    const ddm_status st = check_desc(&descs[i]);
    if (st != DDM_OK) {
      const std::string why = g_err;
      return fail(st, "stack %d: %s", i, why.c_str());
    }
    if (descs[i].spectrum != DDM_SPEC_F32)
      return fail(DDM_ERR_UNSUPPORTED, "batched stacks use FP32 spectra (stack %d)", i);
  }
  ddm_batch_s* b = new (std::nothrow) ddm_batch_s();
  if (b == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "host allocation failed");
  b->magic = kBatchMagic;
  b->stream = (hipStream_t)stream;
  b->fork = nullptr;
  b->calls = 0;
  b->ws = nullptr;
  b->ws_bytes = 0;
  b->root = nullptr;
  b->in_ev = b->out_ev = nullptr;
  b->flags_d = nullptr;
  b->flags_h = nullptr;
  b->fl_next = 0;
  for (int i = 0; i < kReadback; ++i) {
    b->fl_ev[i] = nullptr;
    b->fl_pending[i] = false;
  }
  b->failed.assign(n, 0);
  {
    hipError_t e0 = hipStreamCreateWithFlags(&b->root, hipStreamNonBlocking);
    if (e0 == hipSuccess) e0 = hipEventCreateWithFlags(&b->in_ev, hipEventDisableTiming);
    if (e0 == hipSuccess) e0 = hipEventCreateWithFlags(&b->out_ev, hipEventDisableTiming);
    if (e0 == hipSuccess) e0 = hipMalloc((void**)&b->flags_d, (size_t)n * sizeof(int32_t));
    if (e0 == hipSuccess)
      e0 = hipHostMalloc((void**)&b->flags_h, (size_t)kReadback * n * sizeof(int32_t), hipHostMallocDefault);
    for (int i = 0; i < kReadback && e0 == hipSuccess; ++i)
      e0 = hipEventCreateWithFlags(&b->fl_ev[i], hipEventDisableTiming);
    if (e0 != hipSuccess) {
      batch_free(b);
      return hip_fail(e0, "batch stream setup");
    }
  }
  lanes = std::min(lanes, n);
  for (int l = 0; l < lanes; ++l) {
    hipStream_t s;
    hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "hipStreamCreate");
    }
    b->lanes.push_back(s);
    hipEvent_t ev;
    if ((e = hipEventCreateWithFlags(&ev, hipEventDisableTiming)) != hipSuccess) {
      batch_free(b);
      return hip_fail(e, "hipEventCreate");
    }
    b->join.push_back(ev);
  }
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  if (e != hipSuccess) {
    batch_free(b);
    return hip_fail(e, "hipEventCreate");
  }
  // plans, then lanes: largest stacks first onto the least loaded lane
  std::vector<size_t> full(n);
  std::vector<double> work(n);
  for (int i = 0; i < n; ++i) {
    ddm_plan_desc d = descs[i];
    ddm_plan_t p = nullptr;
    ddm_status st = ddm_plan_create(&d, &p);
    if (st != DDM_OK) {
      std::string msg = g_err;
      batch_free(b);
      return fail(st, "stack %d: %s", i, msg.c_str());
    }
    b->plans.push_back(p);
    p->outcome_dev = b->flags_d + i;
    size_t mn;
    ddm_plan_workspace_size(p, &mn, &full[i]);
    work[i] = (double)d.n_frames * d.width * d.height;
  }
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
  std::vector<double> load(lanes, 0.0);
  b->lane_of.assign(n, 0);
  b->lane_bytes.assign(lanes, 0);
  for (int i : order) {
    int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->lane_of[i] = l;
    load[l] += work[i];
    b->lane_bytes[l] = std::max(b->lane_bytes[l], align256(full[i]));
    b->plans[i]->stream = b->lanes[l];
  }
  size_t off = 0;
  for (int l = 0; l < lanes; ++l) {
    b->lane_off.push_back(off);
    off += b->lane_bytes[l];
    ddm_log("batch %p: lane %d holds %.1f MB of workspace", (void*)b, l, b->lane_bytes[l] / 1e6);
  }
  for (int i = 0; i < n; ++i) ddm_log("batch %p: stack %d -> plan %p, lane %d", (void*)b, i, (void*)b->plans[i],
                                      b->lane_of[i]);
  *out = b;
  g_err.clear();
  return DDM_OK;
}

ddm_status ddm_batch_destroy(ddm_batch_t b) {
  if (b == nullptr) return DDM_OK;
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  hipStreamSynchronize(b->stream);
  hipStreamSynchronize(b->root);
  for (auto s : b->lanes) hipStreamSynchronize(s);
  batch_free(b);
  return DDM_OK;
}

ddm_status ddm_batch_query(ddm_batch_t b, int32_t stack, int64_t* n_q, int32_t* max_lag, int32_t* lane) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (stack < 0 || stack >= (int)b->plans.size()) return fail(DDM_ERR_INVALID_ARGUMENT, "stack out of range");
  if (lane) *lane = b->lane_of[stack];
  return ddm_plan_query(b->plans[stack], n_q, max_lag, nullptr);
}

ddm_status ddm_batch_workspace_size(ddm_batch_t b, size_t* bytes) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (bytes == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "bytes is NULL");
  size_t t = 0;
  for (size_t x : b->lane_bytes) t += x;
  *bytes = t;
  return DDM_OK;
}

ddm_status ddm_batch_set_workspace(ddm_batch_t b, void* ws, size_t bytes) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  size_t need;
  ddm_batch_workspace_size(b, &need);
  if (ws == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "workspace is NULL");
  if (((uintptr_t)ws & 255) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "workspace must be 256-byte aligned");
  if (bytes < need) return fail(DDM_ERR_OUT_OF_MEMORY, "workspace %zu bytes < %zu", bytes, need);
  for (size_t i = 0; i < b->plans.size(); ++i) {
    const int l = b->lane_of[i];
    st = ddm_plan_set_workspace(b->plans[i], (char*)ws + b->lane_off[l], b->lane_bytes[l]);
    if (st != DDM_OK) return st;
  }
  b->ws = ws;
  b->ws_bytes = bytes;
  batch_drop_graphs(b);  // the captured graphs refer to the old workspace
  return DDM_OK;
}

ddm_status ddm_batch_autotune(ddm_batch_t b) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (b->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "no workspace attached");
  for (auto* p : b->plans) {
    st = ddm_plan_autotune(p, nullptr, nullptr, nullptr);
    if (st != DDM_OK) return st;
  }
  batch_drop_graphs(b);  // the captured graphs hold the old launch shapes
  return DDM_OK;
}

// Fold flag slot i (its copy has completed) into the per-stack failures.
static void batch_fold(ddm_batch_s* b, int i) {
  const size_t n = b->plans.size();
  const int32_t* v = b->flags_h + (size_t)i * n;
  for (size_t k = 0; k < n; ++k)
    if (v[k] != 0) b->failed[k] = 1;
  b->fl_pending[i] = false;
}

// Fold every completed slot, oldest first; wait for all of them when `wait`.
static hipError_t batch_collect(ddm_batch_s* b, bool wait) {
  for (int k = 0; k < kReadback; ++k) {
    const int i = (b->fl_next + k) % kReadback;
    if (!b->fl_pending[i]) continue;
    hipError_t e = wait ? hipEventSynchronize(b->fl_ev[i]) : hipEventQuery(b->fl_ev[i]);
    if (e == hipErrorNotReady) return hipSuccess;
    if (e != hipSuccess) return e;
    batch_fold(b, i);
  }
  return hipSuccess;
}

// Report (and clear) the failed stacks folded so far.
static ddm_status batch_report(ddm_batch_s* b, int32_t* stack_status) {
  const size_t n = b->plans.size();
  std::string bad;
  for (size_t k = 0; k < n; ++k) {
    if (stack_status) stack_status[k] = b->failed[k] ? DDM_ERR_HIP : DDM_OK;
    if (b->failed[k] && bad.size() < 200) bad += (bad.empty() ? "" : ", ") + std::to_string(k);
    b->failed[k] = 0;
  }
  if (!bad.empty())
    return fail(DDM_ERR_HIP, "stack(s) %s: step one's wait between its row and column work ran out; "
                             "their D is not valid", bad.c_str());
  return DDM_OK;
}

static ddm_status batch_enqueue(ddm_batch_s* b, const void* const* frames, float* const* D, double* const* Dbar,
                                int64_t* const* counts) {
  hipError_t e = hipEventRecord(b->fork, b->root);
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l) e = hipStreamWaitEvent(b->lanes[l], b->fork, 0);
  if (e != hipSuccess) return hip_fail(e, "batch fork");
  for (size_t i = 0; i < b->plans.size(); ++i) {
    ddm_plan_s* p = b->plans[i];
    ddm_status st = ddm_structure_function(p, frames[i], D[i]);
    if (st != DDM_OK) return st;
    if (Dbar != nullptr && p->batch_nbins > 0) {
      // the stack's |q| bins right after its D, on its lane
      QTable qt{p->qoff_d, p->kxcnt_d};
      e = launch_radial(p->stream, D[i], p->nq, p->M, p->W, p->H, p->ca, p->cc, qt, p->thr_d, p->batch_nbins,
                        Dbar[i], counts[i], nullptr);
      if (e != hipSuccess) return hip_fail(e, "batch radial average launch");
    }
  }
  for (size_t l = 0; l < b->lanes.size() && e == hipSuccess; ++l) {
    e = hipEventRecord(b->join[l], b->lanes[l]);
    if (e == hipSuccess) e = hipStreamWaitEvent(b->root, b->join[l], 0);
  }
  if (e != hipSuccess) return hip_fail(e, "batch join");
  return DDM_OK;
}

ddm_status ddm_batch_set_bins(ddm_batch_t b, int32_t stack, const int64_t* thr, int32_t n_bins) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (stack < 0 || stack >= (int)b->plans.size()) return fail(DDM_ERR_INVALID_ARGUMENT, "stack out of range");
  if ((st = check_thresholds(thr, n_bins)) != DDM_OK) return st;
  ddm_plan_s* p = b->plans[stack];
  // the plan's stream is a lane: wait for work in flight before replacing the thresholds
  hipError_t e = hipStreamSynchronize(b->root);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return hip_fail(e, "batch bins");
  if ((st = upload_thresholds(p, thr, n_bins)) != DDM_OK) return st;
  if ((e = hipStreamSynchronize(p->stream)) != hipSuccess) return hip_fail(e, "batch bins");
  p->batch_nbins = n_bins;
  batch_drop_graphs(b);  // the captured graphs refer to the old bins
  return DDM_OK;
}

static ddm_status batch_run(ddm_batch_t b, const void* const* frames, float* const* D, double* const* Dbar,
                            int64_t* const* counts);

ddm_status ddm_batch_structure_function(ddm_batch_t b, const void* const* frames, float* const* D) {
  return batch_run(b, frames, D, nullptr, nullptr);
}

ddm_status ddm_batch_structure_function_binned(ddm_batch_t b, const void* const* frames, float* const* D,
                                               double* const* Dbar, int64_t* const* counts) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (Dbar == nullptr || counts == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "Dbar/counts arrays are NULL");
  for (size_t i = 0; i < b->plans.size(); ++i)
    if (b->plans[i]->batch_nbins > 0 && (Dbar[i] == nullptr || counts[i] == nullptr))
      return fail(DDM_ERR_INVALID_ARGUMENT, "stack %zu has bins but a NULL Dbar/counts pointer", i);
  return batch_run(b, frames, D, Dbar, counts);
}

static ddm_status batch_run(ddm_batch_t b, const void* const* frames, float* const* D, double* const* Dbar,
                            int64_t* const* counts) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  if (frames == nullptr || D == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "pointer arrays are NULL");
  if (b->ws == nullptr) return fail(DDM_ERR_OUT_OF_MEMORY, "no workspace attached");
  const size_t n = b->plans.size();
  {
    // outcomes of earlier calls that have come back (checked without waiting)
    hipError_t e0 = batch_collect(b, false);
    if (e0 != hipSuccess) return hip_fail(e0, "batch readback");
    st = batch_report(b, nullptr);
    if (st != DDM_OK) return st;
  }
  for (size_t i = 0; i < n; ++i) {
    if (frames[i] == nullptr || D[i] == nullptr) return fail(DDM_ERR_INVALID_ARGUMENT, "stack %zu: NULL pointer", i);
    if (((uintptr_t)frames[i] & 15) != 0) return fail(DDM_ERR_INVALID_ARGUMENT, "stack %zu: frames not 16-byte aligned", i);
  }
  ddm_batch_s::Graph* gr = nullptr;
  for (auto& g : b->graphs) {
    bool same = true;
    for (size_t i = 0; same && i < n; ++i)
      same = g.frames[i] == frames[i] && g.D[i] == D[i] && g.Dbar[i] == (Dbar ? Dbar[i] : nullptr) &&
             g.counts[i] == (counts ? counts[i] : nullptr);
    if (same) {
      gr = &g;
      break;
    }
  }
  if (gr == nullptr) {
    if (b->graphs.size() >= ddm_batch_s::kGraphs) {  // replace the least recently launched
      size_t lru = 0;
      for (size_t k = 1; k < b->graphs.size(); ++k)
        if (b->graphs[k].used < b->graphs[lru].used) lru = k;
      hipGraphExecDestroy(b->graphs[lru].exec);
      b->graphs.erase(b->graphs.begin() + (std::ptrdiff_t)lru);
    }
    hipError_t e = hipStreamBeginCapture(b->root, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    st = batch_enqueue(b, frames, D, Dbar, counts);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(b->root, &g);
    if (st != DDM_OK) {
      if (g) hipGraphDestroy(g);
      return st;
    }
    if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
    ddm_batch_s::Graph ng;
    ng.exec = nullptr;
    e = hipGraphInstantiate(&ng.exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    ng.frames.assign(frames, frames + n);
    ng.D.assign(D, D + n);
    ng.Dbar.assign(n, nullptr);
    ng.counts.assign(n, nullptr);
    for (size_t i = 0; i < n; ++i) {
      if (Dbar) ng.Dbar[i] = Dbar[i];
      if (counts) ng.counts[i] = counts[i];
    }
    b->graphs.push_back(std::move(ng));
    gr = &b->graphs.back();
    ddm_log("batch %p: captured graph %zu of %zu for a new set of pointers", (void*)b, b->graphs.size(),
            ddm_batch_s::kGraphs);
  }
  gr->used = ++b->calls;
  // order after the caller's stream, launch, and order the caller's stream after it
  hipError_t e = hipEventRecord(b->in_ev, b->stream);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->root, b->in_ev, 0);
  if (e == hipSuccess) e = hipGraphLaunch(gr->exec, b->root);
  if (e == hipSuccess) e = hipEventRecord(b->out_ev, b->root);
  if (e == hipSuccess) e = hipStreamWaitEvent(b->stream, b->out_ev, 0);
  if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  // the per-stack flags go back through the next ring slot (waiting only when
  // that slot is still in flight, kReadback calls back)
  const int i = b->fl_next;
  if (b->fl_pending[i]) {
    if ((e = hipEventSynchronize(b->fl_ev[i])) != hipSuccess) return hip_fail(e, "batch readback");
    batch_fold(b, i);
  }
  e = hipMemcpyAsync(b->flags_h + (size_t)i * n, b->flags_d, n * sizeof(int32_t), hipMemcpyDeviceToHost, b->root);
  if (e == hipSuccess) e = hipEventRecord(b->fl_ev[i], b->root);
  if (e != hipSuccess) return hip_fail(e, "batch readback copy");
  b->fl_pending[i] = true;
  b->fl_next = (i + 1) % kReadback;
  return DDM_OK;
}

ddm_status ddm_batch_status(ddm_batch_t b, int32_t* stack_status_host) {
  ddm_status st = check_batch(b);
  if (st != DDM_OK) return st;
  hipError_t e = hipStreamSynchronize(b->root);
  if (e == hipSuccess) e = batch_collect(b, true);
  if (e != hipSuccess) return hip_fail(e, "batch status");
  return batch_report(b, stack_status_host);
}

}  // extern "C"
