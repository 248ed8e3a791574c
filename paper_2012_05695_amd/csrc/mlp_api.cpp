// C ABI of the fit-initialisation MLP: parameters, optimiser state and the
// forward / backward / Adam launch sequences.  All arithmetic runs in the
// kernels of k_mlp.hip; this file only lays out device buffers and orders
// the launches on the network's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

using namespace ddm;

namespace ddm {
hipError_t launch_gemm(hipStream_t s, int epi, int M, int N, int K, const void* A, int64_t sam, int64_t sak,
                       const void* B, int64_t sbk, int64_t sbn, const float* bias, float* C, int64_t ldc,
                       void* H, int64_t ldh, const float* Zin, int64_t ldz);
hipError_t launch_to_bf16(hipStream_t s, const float* x, void* y, int64_t n);
hipError_t launch_mlp_infer(hipStream_t s, const float* x, int64_t rows, const void* const* w,
                            const float* const* b, float* y);
hipError_t launch_mse(hipStream_t s, const float* Y, const float* T, int64_t n, void* dY, float* partial,
                      float* loss);
hipError_t launch_colsum(hipStream_t s, const void* dZ, int64_t B, int N, float* db);
hipError_t launch_adam(hipStream_t s, float* p, const float* g, float* m, float* v, void* pb, int64_t n, float lr,
                       float b1, float b2, float eps, float bc1, float bc2);
ddm_status api_fail(ddm_status st, const char* fmt, ...);
}  // namespace ddm

namespace {
enum { EPI_STORE = 0, EPI_BIAS = 1, EPI_BIAS_GELU = 2, EPI_GELU_BWD = 3 };
constexpr int NIN = DDM_MLP_IN, NH = DDM_MLP_HIDDEN, NOUT = DDM_MLP_OUT;
constexpr int64_t NP = DDM_MLP_NPARAMS;
// offsets of W_l and b_l in the flat parameter vector
constexpr int64_t OW1 = 0, OB1 = OW1 + (int64_t)NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + (int64_t)NH * NH,
                  OW3 = OB2 + NH, OB3 = OW3 + (int64_t)NH * NH, OW4 = OB3 + NH, OB4 = OW4 + (int64_t)NOUT * NH;
static_assert(OB4 + NOUT == NP, "parameter layout");

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

ddm_status hipf(hipError_t e, const char* what) {
  return api_fail(DDM_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}
}  // namespace

struct ddm_mlp_s {
  uint32_t magic;
  int64_t max_batch;
  hipStream_t stream;
  void* mem;
  float *p, *g, *m, *v;   // FP32 master parameters, gradient, Adam moments
  __bf16* pb;             // BF16 copy of the parameters
  // activations for one batch of max_batch rows
  __bf16* xb;             // [B][64]
  float* z[3];            // pre-activations [B][256]
  __bf16* h[3];           // GELU outputs [B][256]
  float* y;               // [B][3]
  __bf16* dy;             // [B][3]
  __bf16* dz[2];          // [B][256] ping-pong
  float* partial;         // loss partial sums
  float* loss;            // device scalar
  int64_t step;
  float beta1, beta2, eps;
};

static constexpr uint32_t kMlpMagic = 0x4d4c5031u;

static ddm_status check_mlp(ddm_mlp_t n) {
  if (n == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "mlp is NULL");
  if (n->magic != kMlpMagic) return api_fail(DDM_ERR_STATE, "mlp handle is not live");
  return DDM_OK;
}

// Forward over B rows already converted into n->xb; fills h and y (= out when
// given), and the pre-activations z when keep_z (the backward pass needs them).
static hipError_t forward_rows(ddm_mlp_s* n, int64_t B, bool keep_z = true, float* out = nullptr) {
  hipStream_t s = n->stream;
  const __bf16* in = n->xb;
  int64_t kin = NIN;
  const int64_t ow[3] = {OW1, OW2, OW3}, ob[3] = {OB1, OB2, OB3};
  for (int l = 0; l < 3; ++l) {
    // Z = H_in W^T + b : A = H_in [B][kin], B(k, j) = W[j][k]
    hipError_t e = launch_gemm(s, EPI_BIAS_GELU, (int)B, NH, (int)kin, in, kin, 1, n->pb + ow[l], 1, kin,
                               n->p + ob[l], keep_z ? n->z[l] : nullptr, NH, n->h[l], NH, nullptr, 0);
    if (e != hipSuccess) return e;
    in = n->h[l];
    kin = NH;
  }
  return launch_gemm(s, EPI_BIAS, (int)B, NOUT, NH, in, NH, 1, n->pb + OW4, 1, NH, n->p + OB4, out ? out : n->y,
                     NOUT, nullptr, 0, nullptr, 0);
}

// Gradient of the mean squared error of the last forward against T [B][3].
static hipError_t backward_rows(ddm_mlp_s* n, const float* T, int64_t B) {
  hipStream_t s = n->stream;
  hipError_t e = launch_mse(s, n->y, T, B * NOUT, n->dy, n->partial, n->loss);
  if (e != hipSuccess) return e;
  // layer 4: dW4 = dY^T H3, db4 = colsum dY, dZ3 = (dY W4) * gelu'(Z3)
  if ((e = launch_gemm(s, EPI_STORE, NOUT, NH, (int)B, n->dy, 1, NOUT, n->h[2], NH, 1, nullptr, n->g + OW4, NH,
                       nullptr, 0, nullptr, 0)) != hipSuccess)
    return e;
  if ((e = launch_colsum(s, n->dy, B, NOUT, n->g + OB4)) != hipSuccess) return e;
  if ((e = launch_gemm(s, EPI_GELU_BWD, (int)B, NH, NOUT, n->dy, NOUT, 1, n->pb + OW4, NH, 1, nullptr, nullptr, 0,
                       n->dz[0], NH, n->z[2], NH)) != hipSuccess)
    return e;
  const int64_t ow[3] = {OW1, OW2, OW3}, ob[3] = {OB1, OB2, OB3};
  int cur = 0;
  for (int l = 2; l >= 0; --l) {
    const __bf16* hin = (l == 0) ? n->xb : n->h[l - 1];
    const int64_t kin = (l == 0) ? NIN : NH;
    // dW_l = dZ_l^T H_{l-1}, db_l = colsum dZ_l
    if ((e = launch_gemm(s, EPI_STORE, NH, (int)kin, (int)B, n->dz[cur], 1, NH, hin, kin, 1, nullptr, n->g + ow[l],
                         kin, nullptr, 0, nullptr, 0)) != hipSuccess)
      return e;
    if ((e = launch_colsum(s, n->dz[cur], B, NH, n->g + ob[l])) != hipSuccess) return e;
    if (l > 0) {
      // dZ_{l-1} = (dZ_l W_l) * gelu'(Z_{l-1})
      if ((e = launch_gemm(s, EPI_GELU_BWD, (int)B, NH, NH, n->dz[cur], NH, 1, n->pb + ow[l], NH, 1, nullptr,
                           nullptr, 0, n->dz[cur ^ 1], NH, n->z[l - 1], NH)) != hipSuccess)
        return e;
      cur ^= 1;
    }
  }
  return hipSuccess;
}

extern "C" {

ddm_status ddm_mlp_create(uint64_t seed, int64_t max_batch, void* stream, ddm_mlp_t* out) {
  if (out == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  if (max_batch < 1 || max_batch > (1 << 22)) return api_fail(DDM_ERR_INVALID_ARGUMENT, "max_batch must be in [1, 2^22]");
  ddm_mlp_s* n = new (std::nothrow) ddm_mlp_s();
  if (n == nullptr) return api_fail(DDM_ERR_OUT_OF_MEMORY, "host allocation failed");
  n->max_batch = max_batch;
  n->stream = (hipStream_t)stream;
  const int64_t B = max_batch;
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off += a256(bytes); return o; };
  const size_t op = take(NP * 4), og = take(NP * 4), om = take(NP * 4), ov = take(NP * 4), opb = take(NP * 2);
  const size_t oxb = take(B * NIN * 2);
  size_t oz[3], oh[3], odz[2];
  for (int l = 0; l < 3; ++l) { oz[l] = take(B * NH * 4); oh[l] = take(B * NH * 2); }
  const size_t oy = take(B * NOUT * 4), ody = take(B * NOUT * 2);
  odz[0] = take(B * NH * 2);
  odz[1] = take(B * NH * 2);
  const size_t opart = take(((B * NOUT + 255) / 256) * 4), oloss = take(4);
  hipError_t e = hipMalloc(&n->mem, off);
  if (e != hipSuccess) {
    delete n;
    return hipf(e, "hipMalloc(mlp)");
  }
  char* b = (char*)n->mem;
  n->p = (float*)(b + op); n->g = (float*)(b + og); n->m = (float*)(b + om); n->v = (float*)(b + ov);
  n->pb = (__bf16*)(b + opb); n->xb = (__bf16*)(b + oxb);
  for (int l = 0; l < 3; ++l) { n->z[l] = (float*)(b + oz[l]); n->h[l] = (__bf16*)(b + oh[l]); }
  n->y = (float*)(b + oy); n->dy = (__bf16*)(b + ody);
  n->dz[0] = (__bf16*)(b + odz[0]); n->dz[1] = (__bf16*)(b + odz[1]);
  n->partial = (float*)(b + opart); n->loss = (float*)(b + oloss);
  n->step = 0;
  n->beta1 = 0.9f; n->beta2 = 0.999f; n->eps = 1e-8f;
  n->magic = kMlpMagic;
  // uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a splitmix64 stream
  std::vector<float> h(NP);
  uint64_t st = seed;
  auto next = [&]() {
    uint64_t z = (st += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  };
  const int64_t lo[8] = {OW1, OB1, OW2, OB2, OW3, OB3, OW4, OB4};
  const int64_t hi[8] = {OB1, OW2, OB2, OW3, OB3, OW4, OB4, NP};
  const int fan[8] = {NIN, NIN, NH, NH, NH, NH, NH, NH};
  for (int s = 0; s < 8; ++s) {
    const double sc = 1.0 / std::sqrt((double)fan[s]);
    for (int64_t i = lo[s]; i < hi[s]; ++i) h[i] = (float)(((next() >> 11) * 0x1.0p-53 * 2.0 - 1.0) * sc);
  }
  ddm_status rs = DDM_OK;
  *out = n;
  if ((rs = ddm_mlp_set_params(n, h.data())) != DDM_OK) {
    ddm_mlp_destroy(n);
    *out = nullptr;
  }
  return rs;
}

ddm_status ddm_mlp_destroy(ddm_mlp_t n) {
  if (n == nullptr) return DDM_OK;
  if (n->magic != kMlpMagic) return api_fail(DDM_ERR_STATE, "mlp handle is not live");
  hipStreamSynchronize(n->stream);
  n->magic = 0;
  hipFree(n->mem);
  delete n;
  return DDM_OK;
}

ddm_status ddm_mlp_set_params(ddm_mlp_t n, const float* host) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (host == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "params is NULL");
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess) e = hipMemcpy(n->p, host, NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemset(n->m, 0, NP * 4);
  if (e == hipSuccess) e = hipMemset(n->v, 0, NP * 4);
  if (e == hipSuccess) e = launch_to_bf16(n->stream, n->p, n->pb, NP);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return hipf(e, "mlp set params");
  n->step = 0;
  return DDM_OK;
}

ddm_status ddm_mlp_get_params(ddm_mlp_t n, float* host) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (host == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "params is NULL");
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess) e = hipMemcpy(host, n->p, NP * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipf(e, "mlp get params");
  return DDM_OK;
}

ddm_status ddm_mlp_get_state(ddm_mlp_t n, float* params, float* adam_m, float* adam_v, int64_t* step) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (!params || !adam_m || !adam_v || !step) return api_fail(DDM_ERR_INVALID_ARGUMENT, "NULL output");
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess) e = hipMemcpy(params, n->p, NP * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(adam_m, n->m, NP * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(adam_v, n->v, NP * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipf(e, "mlp get state");
  *step = n->step;
  return DDM_OK;
}

ddm_status ddm_mlp_set_state(ddm_mlp_t n, const float* params, const float* adam_m, const float* adam_v,
                             int64_t step) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (!params || !adam_m || !adam_v || step < 0) return api_fail(DDM_ERR_INVALID_ARGUMENT, "bad state");
  hipError_t e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess) e = hipMemcpy(n->p, params, NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->m, adam_m, NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(n->v, adam_v, NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_to_bf16(n->stream, n->p, n->pb, NP);
  if (e == hipSuccess) e = hipStreamSynchronize(n->stream);
  if (e != hipSuccess) return hipf(e, "mlp set state");
  n->step = step;
  return DDM_OK;
}

ddm_status ddm_mlp_forward(ddm_mlp_t n, const float* x, int64_t rows, float* y) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (x == nullptr || y == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "x/y is NULL");
  if (rows < 0) return api_fail(DDM_ERR_INVALID_ARGUMENT, "rows must be >= 0");
  if (rows == 0) return DDM_OK;
  // one fused launch over every row (activations kept in LDS) when the BF16
  // weights allow its 16-byte loads, else the layers one by one in batches
  const void* w[4] = {n->pb + OW1, n->pb + OW2, n->pb + OW3, n->pb + OW4};
  const float* b[4] = {n->p + OB1, n->p + OB2, n->p + OB3, n->p + OB4};
  bool aligned = true;
  for (const void* wl : w) aligned = aligned && ((uintptr_t)wl & 15) == 0;
  if (aligned) {
    hipError_t e = launch_mlp_infer(n->stream, x, rows, w, b, y);
    if (e != hipSuccess) return hipf(e, "mlp forward");
    return DDM_OK;
  }
  for (int64_t r0 = 0; r0 < rows; r0 += n->max_batch) {
    const int64_t B = std::min<int64_t>(n->max_batch, rows - r0);
    hipError_t e = launch_to_bf16(n->stream, x + r0 * NIN, n->xb, B * NIN);
    if (e == hipSuccess) e = forward_rows(n, B, false, y + r0 * NOUT);
    if (e != hipSuccess) return hipf(e, "mlp forward");
  }
  return DDM_OK;
}

ddm_status ddm_mlp_gradient(ddm_mlp_t n, const float* x, const float* t, int64_t B, float* grad_host,
                            float* loss_host) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (x == nullptr || t == nullptr) return api_fail(DDM_ERR_INVALID_ARGUMENT, "x/t is NULL");
  if (B < 1 || B > n->max_batch) return api_fail(DDM_ERR_INVALID_ARGUMENT, "batch must be in [1, max_batch]");
  hipError_t e = launch_to_bf16(n->stream, x, n->xb, B * NIN);
  if (e == hipSuccess) e = forward_rows(n, B);
  if (e == hipSuccess) e = backward_rows(n, t, B);
  if (e == hipSuccess && (grad_host || loss_host)) e = hipStreamSynchronize(n->stream);
  if (e == hipSuccess && grad_host) e = hipMemcpy(grad_host, n->g, NP * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess && loss_host) e = hipMemcpy(loss_host, n->loss, 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hipf(e, "mlp gradient");
  return DDM_OK;
}

ddm_status ddm_mlp_adam_step(ddm_mlp_t n, float lr) {
  ddm_status st = check_mlp(n);
  if (st != DDM_OK) return st;
  if (!(lr > 0.0f) || !std::isfinite(lr)) return api_fail(DDM_ERR_INVALID_ARGUMENT, "lr must be > 0");
  n->step += 1;
  const float bc1 = 1.0f - std::pow(n->beta1, (float)n->step);
  const float bc2 = 1.0f - std::pow(n->beta2, (float)n->step);
  hipError_t e = launch_adam(n->stream, n->p, n->g, n->m, n->v, n->pb, NP, lr, n->beta1, n->beta2, n->eps, bc1, bc2);
  if (e != hipSuccess) return hipf(e, "mlp adam");
  return DDM_OK;
}

ddm_status ddm_mlp_train_step(ddm_mlp_t n, const float* x, const float* t, int64_t B, float lr, float* loss_dev) {
  ddm_status st = ddm_mlp_gradient(n, x, t, B, nullptr, nullptr);
  if (st != DDM_OK) return st;
  st = ddm_mlp_adam_step(n, lr);
  if (st != DDM_OK) return st;
  if (loss_dev != nullptr) {
    hipError_t e = hipMemcpyAsync(loss_dev, n->loss, 4, hipMemcpyDeviceToDevice, n->stream);
    if (e != hipSuccess) return hipf(e, "mlp loss copy");
  }
  return DDM_OK;
}

}  // extern "C"
