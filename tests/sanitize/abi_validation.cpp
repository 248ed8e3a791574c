// Host-side validation paths of the C ABI, run under AddressSanitizer and
// UndefinedBehaviorSanitizer without a GPU: every call below must be refused
// before any HIP call, with a status other than DDM_OK and a message.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "ddm.h"

static int g_fail = 0;

static void expect(ddm_status got, ddm_status want, const char* what) {
  const char* msg = ddm_last_error();
  const bool ok = (want == DDM_OK) ? got == DDM_OK : (got == want && msg != nullptr && std::strlen(msg) > 0);
  if (!ok) {
    std::fprintf(stderr, "FAIL %s: status %d (want %d), message '%s'\n", what, (int)got, (int)want,
                 msg ? msg : "(null)");
    ++g_fail;
  }
}

int main() {
  const ddm_status INV = DDM_ERR_INVALID_ARGUMENT, UNS = DDM_ERR_UNSUPPORTED, STATE = DDM_ERR_STATE;
  ddm_plan_desc d;
  ddm_plan_desc_init(nullptr);
  ddm_plan_desc_init(&d);
  ddm_plan_t plan = reinterpret_cast<ddm_plan_t>(0x1);
  expect(ddm_plan_create(nullptr, &plan), INV, "create: NULL desc");
  expect(ddm_plan_create(&d, nullptr), INV, "create: NULL out");
  struct Case { void (*edit)(ddm_plan_desc&); ddm_status want; const char* what; };
  const Case cases[] = {
      {[](ddm_plan_desc& x) { x.struct_size = 7; }, INV, "struct_size"},
      {[](ddm_plan_desc& x) { x.width = 0; x.height = 64; x.n_frames = 8; }, INV, "width 0"},
      {[](ddm_plan_desc& x) { x.width = 100; x.height = 64; x.n_frames = 8; }, UNS, "width 100"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 8192; x.n_frames = 8; }, UNS, "height 8192"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 1; }, INV, "n_frames 1"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 17000; }, UNS, "n_frames 17000 fourier"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 70000; x.method = DDM_METHOD_DIRECT; },
       UNS, "n_frames 70000 direct"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.max_lag = 9; }, INV, "max_lag > N"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.max_lag = -1; }, INV, "max_lag < 0"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.pixel = 9; }, INV, "pixel"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.spectrum = 9; }, INV, "spectrum"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.precondition = 2; }, INV,
       "precondition"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.k2_max = -2; }, INV, "k2_max"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.padding = 5; }, INV, "padding"},
      {[](ddm_plan_desc& x) { x.width = 64; x.height = 64; x.n_frames = 8; x.method = -1; }, INV, "method"},
  };
  for (const Case& c : cases) {
    ddm_plan_desc_init(&d);
    c.edit(d);
    plan = reinterpret_cast<ddm_plan_t>(0x1);
    expect(ddm_plan_create(&d, &plan), c.want, c.what);
    if (plan != nullptr) {
      std::fprintf(stderr, "FAIL %s: *out not cleared\n", c.what);
      ++g_fail;
    }
  }

  // NULL handles, and a handle that is not a live plan (zeroed memory: the
  // magic word does not match)
  std::vector<unsigned char> fake(4096, 0);
  ddm_plan_t dead = reinterpret_cast<ddm_plan_t>(fake.data());
  float f = 0.f;
  int64_t i64 = 0;
  int32_t i32 = 0;
  size_t z = 0;
  double dbl = 0.0;
  const int64_t thr[2] = {0, 1};
  for (ddm_plan_t h : {static_cast<ddm_plan_t>(nullptr), dead}) {
    const ddm_status w = h ? STATE : INV;
    expect(ddm_plan_query(h, &i64, &i32, &i32), w, "query");
    expect(ddm_plan_q_index(h, &i32, &i32), w, "q_index");
    expect(ddm_plan_workspace_size(h, &z, &z), w, "workspace_size");
    expect(ddm_plan_set_workspace(h, &f, 4), w, "set_workspace");
    expect(ddm_structure_function(h, &f, &f), w, "structure_function");
    expect(ddm_plan_status(h), w, "status");
    expect(ddm_structure_function_host(h, &f, &f, 1024, &f), w, "structure_function_host");
    expect(ddm_structure_function_noalloc(h, &f, &f), w, "structure_function_noalloc");
    expect(ddm_image_spectra(h, &f, &f), w, "image_spectra");
    expect(ddm_structure_from_spectra(h, &f, &f), w, "structure_from_spectra");
    expect(ddm_plan_autotune(h, &i32, &i32, &dbl), w, "autotune");
    expect(ddm_plan_method(h, &i32), w, "method");
    expect(ddm_radial_average(h, &f, thr, 1, &dbl, &i64, &i32), w, "radial_average");
    expect(ddm_plan_fp16_saturations(h, &i64), w, "fp16_saturations");
    expect(ddm_plan_set_profiling(h, 1u), w, "set_profiling");
    expect(ddm_plan_get_profile(h, 1u, &dbl, &i64), w, "get_profile");
  }
  expect(ddm_plan_destroy(nullptr), DDM_OK, "destroy NULL");

  // batches
  ddm_batch_t b = reinterpret_cast<ddm_batch_t>(0x1);
  ddm_plan_desc_init(&d);
  d.width = d.height = 64;
  d.n_frames = 8;
  ddm_plan_desc bad[2] = {d, d};
  bad[1].width = 100;
  expect(ddm_batch_create(nullptr, 1, 1, nullptr, &b), INV, "batch: NULL descs");
  expect(ddm_batch_create(&d, 0, 1, nullptr, &b), INV, "batch: no stacks");
  expect(ddm_batch_create(&d, 1, 0, nullptr, &b), INV, "batch: no lanes");
  expect(ddm_batch_create(&d, 1, 1, nullptr, nullptr), INV, "batch: NULL out");
  expect(ddm_batch_create(bad, 2, 1, nullptr, &b), UNS, "batch: bad stack");
  expect(ddm_batch_destroy(nullptr), DDM_OK, "batch destroy NULL");
  expect(ddm_batch_query(nullptr, 0, &i64, &i32, &i32), INV, "batch query NULL");
  expect(ddm_batch_workspace_size(nullptr, &z), INV, "batch workspace_size NULL");
  expect(ddm_batch_structure_function(nullptr, nullptr, nullptr), INV, "batch run NULL");
  expect(ddm_batch_status(nullptr, &i32), INV, "batch status NULL");

  // curve sampling and the fit
  float lags[65];
  for (int k = 0; k < 65; ++k) lags[k] = (float)k;
  expect(ddm_sample_curves(&f, 1, 8, lags, 0, &f, &f, nullptr), INV, "sample: K 0");
  expect(ddm_sample_curves(&f, 1, 8, lags, 65, &f, &f, nullptr), INV, "sample: K 65");
  expect(ddm_sample_curves(nullptr, 1, 8, lags, 4, &f, &f, nullptr), INV, "sample: NULL D");
  ddm_fit_desc fd;
  ddm_fit_desc_init(&fd);
  fd.K = 4;
  float out[4];
  int32_t iters = 0, flags = 0;
  fd.struct_size = 3;
  expect(ddm_fit(&fd, &f, lags, 1, nullptr, out, &iters, &flags), INV, "fit: struct_size");
  ddm_fit_desc_init(&fd);
  fd.K = 65;
  expect(ddm_fit(&fd, &f, lags, 1, nullptr, out, &iters, &flags), INV, "fit: K 65");
  ddm_fit_desc_init(&fd);
  fd.K = 4;
  fd.fallback = 9;
  expect(ddm_fit(&fd, &f, lags, 1, nullptr, out, &iters, &flags), INV, "fit: fallback");
  expect(ddm_fit(nullptr, &f, lags, 1, nullptr, out, &iters, &flags), INV, "fit: NULL desc");

  // the network
  ddm_mlp_t m = reinterpret_cast<ddm_mlp_t>(0x1);
  expect(ddm_mlp_create(1, 0, nullptr, &m), INV, "mlp: max_batch 0");
  expect(ddm_mlp_create(1, 16, nullptr, nullptr), INV, "mlp: NULL out");
  expect(ddm_mlp_destroy(nullptr), DDM_OK, "mlp destroy NULL");
  expect(ddm_mlp_forward(nullptr, &f, 1, &f), INV, "mlp forward NULL");
  expect(ddm_mlp_get_params(nullptr, &f), INV, "mlp get_params NULL");
  expect(ddm_mlp_adam_step(nullptr, 1e-3f), INV, "mlp adam NULL");

  if (g_fail == 0) std::printf("abi validation: all refusals as expected\n");
  return g_fail == 0 ? 0 : 1;
}
