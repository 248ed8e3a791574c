/*
 * ddm.h -- C ABI of libddm: the DDM image structure function computed with a
 * Fourier transform in time (Norouzisadeh, Cerchiari, Croccolo,
 * arXiv 2012.05695), for AMD Instinct MI355X (gfx950).
 *
 * Problem statement (paper, section "The algorithm", Eq. (1)): N images I_n
 * taken at regular time intervals; for every wave vector q of their 2-D
 * Fourier transforms F(q, n) and every lag m (in frames),
 *
 *     D(q, m) = 1/(N-m) * sum_{n=m}^{N-1} |F(q, n) - F(q, n-m)|^2 .
 *
 * The library reaches this result without image differences: a 2-D FFT of each
 * frame (the paper's "step one"), then per wave vector a zero-padded FFT in time,
 * squared modulus, inverse FFT, and the squared-modulus prefix sums (Eq. (2) and
 * Appendix B, Eqs. (B1)-(B4), the "step two").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every call returns a ddm_status and never throws or aborts across the ABI.
 *  - Arguments are validated before anything is enqueued.  On any DDM_ERR_*
 *    status no output buffer has been written and no work is pending;
 *    ddm_last_error() then describes the failure (thread-local string).
 *  - "device" pointers are HIP device memory owned by the caller (PyTorch
 *    tensors in the Python binding).  "host" pointers are ordinary host memory,
 *    read or written before the call returns.
 *  - Work is enqueued asynchronously on the plan's stream; the caller
 *    synchronises.  A plan is not thread-safe; distinct plans are independent.
 *  - Wave-vector order ("q order"): the non-redundant half plane
 *    kx = 0..W/2, ky = 0..H-1 (unsigned DFT index; signed frequency ky for
 *    ky <= H/2 and ky-H above), ky-major then kx, restricted to the kept set
 *    k2 <= k2_max where k2 = kx^2 (H/g)^2 + ky_s^2 (W/g)^2, g = gcd(W, H)
 *    (k2 = kx^2 + ky^2 for square frames).  Real frames make F(-q) = conj F(q),
 *    so the half plane carries every distinct D.
 *  - Transform conventions: forward 2-D DFT with exp(-2 pi i (kx x/W + ky y/H))
 *    and no normalisation, so D is in (pixel value)^2 * pixels^2 units.
 */
#ifndef DDM_H
#define DDM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DDM_ABI_VERSION 1

typedef enum ddm_status {
  DDM_OK = 0,
  DDM_ERR_INVALID_ARGUMENT = 1, /* bad pointer, size or descriptor field */
  DDM_ERR_UNSUPPORTED = 2,      /* valid request outside what this build implements */
  DDM_ERR_OUT_OF_MEMORY = 3,    /* workspace missing or too small; host allocation failed */
  DDM_ERR_HIP = 4,              /* a HIP runtime call failed (message has the HIP error) */
  DDM_ERR_STATE = 5,            /* call on a destroyed / incomplete object */
  DDM_WARN_FP16_SATURATED = 100 /* result written; some FP16 spectrum values saturated */
} ddm_status;

typedef enum ddm_pixel { DDM_PIX_U8 = 1, DDM_PIX_U16 = 2 } ddm_pixel;

/* Storage of the per-wave-vector time series between step one and step two.
 * F32: complex FP32.  F16_QSCALED: complex FP16, each wave vector scaled by a
 * power of two 2^e(q) (exact) chosen so that the largest component over the
 * pilot frames {floor(jN/8), j = 1..7} and N-1 falls in (2^10, 2^11] (a factor
 * 32 below the FP16 maximum); components beyond 65504 are clipped and counted.
 * Halves the spectrum traffic; D within 5e-3 of the FP32 result's accuracy. */
typedef enum ddm_spectrum { DDM_SPEC_F32 = 0, DDM_SPEC_F16_QSCALED = 1 } ddm_spectrum;

/* Zero padding of the time sequences (Eq. (B4) and the exactness statement
 * after it: any N2 >= 2N - 1 gives D exactly).  POW2: N2 = 2L, L the smallest
 * power of two >= N (as Eq. (B4) prints it).  MINIMAL: L the smallest of
 * 2^k and 3 * 2^k >= N (3 * 2^k from 192 on), up to 1.5x less transform work;
 * the 3 * 2^k transforms take radix-4/2 passes and a radix-3 pass, more LDS
 * round trips per point, and are faster than POW2 only where N = L. */
typedef enum ddm_padding { DDM_PAD_POW2 = 0, DDM_PAD_MINIMAL = 1 } ddm_padding;

/* How step two computes D from the image spectra.
 * FOURIER: the time transform of Appendix B (Eq. (B3), (B4)): O(N log N) per
 *   wave vector, whatever max_lag is; N up to 16384 (N2 up to 32768).
 * DIRECT: Eq. (1) term by term, |F_{n+m}(q) - F_n(q)|^2 averaged over the
 *   N - m pairs of each lag (the direct scheme of section "The algorithm",
 *   applied to the stored spectra: the spectrum of a difference image is the
 *   difference of the spectra): O(N M) per wave vector.  FP32 differences,
 *   FP32 sums over 64 time points added into FP64 totals.  Cheaper than
 *   FOURIER when few lags are wanted (at 512 x 512 x 1024 below about 52); the
 *   only method for N above 16384 (up to 65536).
 * AUTO: DIRECT where a cost model (N M - M (M - 1) / 2 difference pairs
 *   against c L log2 L for the transform of length L, c = 5.2 up to L = 8192
 *   and 16 at L = 16384, the constants from the measured crossovers) expects
 *   it to be faster, else FOURIER;
 *   ddm_plan_autotune replaces the model's choice by a timing of both.
 *   ddm_plan_method reports the choice. */
typedef enum ddm_method { DDM_METHOD_FOURIER = 0, DDM_METHOD_DIRECT = 1, DDM_METHOD_AUTO = 2 } ddm_method;

typedef struct ddm_plan_s* ddm_plan_t;

typedef struct ddm_plan_desc {
  uint32_t struct_size;  /* = sizeof(ddm_plan_desc); guards ABI drift */
  int32_t width;         /* W: even, 8..4096, a power of two or 3 * a power of two */
  int32_t height;        /* H: same rules as W */
  int32_t n_frames;      /* N >= 2 (up to 16384: time FFT length N2 <= 32768; up to
                            65536 with DDM_METHOD_DIRECT) */
  int32_t max_lag;       /* M in [1, N]: lags 0..M-1 are produced; 0 means N */
  int32_t pixel;         /* ddm_pixel of the frames */
  int32_t spectrum;      /* ddm_spectrum */
  int32_t precondition;  /* 1: transform I_t - I_0 instead of I_t (D is unchanged
                            because D depends on frame differences only; it
                            shrinks the dynamic range of the FP32 transforms) */
  int32_t padding;       /* ddm_padding of the time transform (default POW2) */
  int32_t method;        /* ddm_method of step two (default FOURIER) */
  int64_t k2_max;        /* keep q with k2 <= k2_max (the paper's low-frequency
                            restriction, section "Conclusion"); -1 keeps all */
  void* stream;          /* hipStream_t for all work of this plan; NULL = default */
} ddm_plan_desc;

/* Fill a descriptor with defaults: struct_size set, max_lag 0, U16, F32,
 * precondition 1, padding POW2, method FOURIER, k2_max -1, stream NULL.  Size
 * fields are set to 0. */
void ddm_plan_desc_init(ddm_plan_desc* desc);

/* Create a plan.  Allocates only small device tables (twiddles, row offsets;
 * O(W + H + N) bytes).  The large buffers are the caller's: a workspace (see
 * ddm_plan_workspace_size) and the input / output arrays.  *out is NULL on error. */
ddm_status ddm_plan_create(const ddm_plan_desc* desc, ddm_plan_t* out);

/* Release the plan and its small tables.  NULL is accepted.  Synchronises the
 * plan's stream first so that no enqueued kernel still reads the tables. */
ddm_status ddm_plan_destroy(ddm_plan_t plan);

/* n_q: number of kept wave vectors (rows of D).  max_lag: M.  n2: the
 * zero-padded time-FFT length that Eq. (B4) prints, log2 N2 = ceil(log2 N) + 1
 * (whatever the plan's padding and method; the minimal padding's length is
 * 2 L with L the smallest 2^k or 3 * 2^k >= N).  Any output pointer may be
 * NULL. */
ddm_status ddm_plan_query(ddm_plan_t plan, int64_t* n_q, int32_t* max_lag, int32_t* n2);

/* Host arrays of n_q entries: kx and signed ky of every row of D, in q order. */
ddm_status ddm_plan_q_index(ddm_plan_t plan, int32_t* kx_host, int32_t* ky_signed_host);

/* Workspace needed by ddm_structure_function: *full_bytes processes all wave
 * vectors in one group; *min_bytes is the smallest workspace accepted, with
 * which the wave vectors are processed in several groups and every frame is
 * transformed once per group (the paper's group execution, Appendix C).
 * Results are bit-identical for every accepted workspace size. */
ddm_status ddm_plan_workspace_size(ddm_plan_t plan, size_t* min_bytes, size_t* full_bytes);

/* Attach caller-owned device memory (at least min_bytes, 256-byte aligned).
 * The plan keeps the pointer; the caller keeps ownership and must keep it alive
 * while work that uses it is pending. */
ddm_status ddm_plan_set_workspace(ddm_plan_t plan, void* workspace_dev, size_t bytes);

/* The full path: frames_dev [N][H][W] (uint8 or uint16 per the plan, row-major,
 * device, 16-byte aligned) -> D_dev [n_q][M] float32 (device), D(q, m) of Eq. (1).
 * Requires a workspace.
 * Device-side outcomes come back without stalling the host: each call enqueues
 * a copy of them, and each later call takes in those that have completed,
 * checked without waiting (the host waits only when it is 4 calls ahead of the
 * device).  The call returns DDM_WARN_FP16_SATURATED (result written) when
 * FP16 spectrum values clipped by earlier calls have come back since the last
 * report, and returns DDM_ERR_HIP (enqueuing nothing) once for an earlier
 * call whose single-launch step one ran out of time in a wait (that call's D
 * is not valid).  ddm_plan_status reports the outcome of every call made so
 * far, its last call included.  Calls made inside a HIP graph capture hand
 * nothing back to the plan (a batch collects them per stack). */
ddm_status ddm_structure_function(ddm_plan_t plan, const void* frames_dev, float* D_dev);

/* Synchronise the plan's stream and report the device-side outcomes of every
 * call since the last report, then clear them: DDM_ERR_HIP if a single-launch
 * step one ran out of time in a wait (that call's D is not valid; the message
 * says so), else DDM_WARN_FP16_SATURATED if FP16 spectrum values were clipped,
 * else DDM_OK.  DDM_ERR_STATE inside a graph capture.  Setting DDM_STEP1_FAIL=1
 * in the environment before a plan is created makes that plan's single-launch
 * step one start with its error flag raised: every wait gives up at once and
 * the kernel exits normally with an invalid result, which this call reports
 * (for testing the reporting path). */
ddm_status ddm_plan_status(ddm_plan_t plan);

/* Frames resident in host memory (a camera or file reader's buffers; the
 * paper's memory-IO share of step one): frames_host [N][H][W] as in
 * ddm_structure_function but in host memory, pinned (hipHostMalloc or a pinned
 * torch tensor) for the copies to overlap the transforms (pageable memory
 * works, without overlap).  staging_dev: caller-owned device memory of
 * staging_bytes (256-byte aligned, at least frame 0 plus two frames,
 * align256(H W b) + 2 H W b): frame 0 is copied once, then batches of frames
 * alternate between two halves of the rest on a copy stream while the
 * previous batch is transformed (two-kernel step one).  Requires the plan's
 * workspace; each group of wave vectors (Appendix C) copies the frames again.
 * D_dev as ddm_structure_function, bit-identical to it.  FP32 spectrum store
 * only (DDM_ERR_UNSUPPORTED otherwise, and inside a graph capture).  The host
 * memory must stay valid until the call's work has completed. */
ddm_status ddm_structure_function_host(ddm_plan_t plan, const void* frames_host, void* staging_dev,
                                       size_t staging_bytes, float* D_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * result as ddm_structure_function, bit for bit, with the library's own
 * static device scratch of DDM_NOALLOC_SCRATCH_BYTES (256 MiB, held by each
 * device the library runs on from module load to process end) as the
 * workspace instead of the attached one (which is neither needed nor
 * touched).  The caller passes frames and D as for ddm_structure_function.
 * Plans whose minimum workspace (ddm_plan_workspace_size) exceeds the scratch
 * return DDM_ERR_UNSUPPORTED; a plan whose full workspace exceeds it runs in
 * groups (every frame transformed once per group).  The call allocates no
 * device or host memory (the scratch address is looked up once per device,
 * on that device's first call).  Every call on a device uses the same
 * scratch, which keeps the last call's contents: calls that overlap on one
 * device (different streams, or different threads) race and give invalid
 * results; calls on one stream are ordered and safe. */
#define DDM_NOALLOC_SCRATCH_BYTES (256u << 20)
ddm_status ddm_structure_function_noalloc(ddm_plan_t plan, const void* frames_dev, float* D_dev);

/* FP16 spectrum store: total number of spectrum components clipped to
 * +-65504 since the plan was created (waits for every call enqueued so far). */
ddm_status ddm_plan_fp16_saturations(ddm_plan_t plan, int64_t* count);

/* Step one only: frames_dev [N][H][W] -> spectra_dev [n_q][N] complex float32
 * (interleaved re, im; q order, time contiguous), the 2-D transforms F(q, t)
 * of the frames, or of I_t - I_0 when the plan preconditions.  Requires a
 * workspace.  Used to check step one on its own. */
ddm_status ddm_image_spectra(ddm_plan_t plan, const void* frames_dev, float* spectra_dev);

/* Step two only, with the plan's method (the time transform of Appendix B, or
 * Eq. (1) directly): spectra_dev [n_q][N] complex float32 (as written by
 * ddm_image_spectra, or any time series) -> D_dev [n_q][M] float32.  Needs no
 * workspace. */
ddm_status ddm_structure_from_spectra(ddm_plan_t plan, const float* spectra_dev, float* D_dev);

/* Pick the time-kernel launch shape (values per thread, wave vectors per
 * workgroup) for this plan by timing the candidates on zero-filled spectra in
 * the plan's workspace (required); the choice is cached per (time length, N,
 * max_lag, storage) for the process and used by later calls.  Synchronises
 * the stream.  DDM_AUTOTUNE=off (environment) keeps the built-in shape.
 * DDM_TUNE_CACHE=<file> (environment) keeps the results across processes: the
 * file's lines for this device architecture and HIP runtime version are read
 * at the first autotune, and every new timing is appended as a line
 * "<arch> <runtime> <L> <N> <M> <f16> fourier <E> <qpw> <ms>" or
 * "... direct <ms>".  DDM_LOG=1 (environment) prints one line per plan, batch,
 * workspace and autotune decision on stderr.
 * Outputs (may be NULL): E, wave vectors per workgroup, estimated ms per call
 * of step two.  DDM_METHOD_AUTO plans also time the direct kernel on the same
 * spectra and keep the faster method (the ms is that method's); DDM_METHOD_DIRECT
 * plans time only the direct kernel. */
ddm_status ddm_plan_autotune(ddm_plan_t plan, int32_t* E, int32_t* qpw, double* ms);

/* The method step two uses (DDM_METHOD_FOURIER or DDM_METHOD_DIRECT): the
 * descriptor's, or for DDM_METHOD_AUTO the cost model's choice, replaced by
 * ddm_plan_autotune's timing once that has run. */
ddm_status ddm_plan_method(ddm_plan_t plan, int32_t* method);

/* ---------------------------------------------------------------------------
 * Batches of independent stacks of uneven sizes (many regions of interest or
 * stacks at once).  One plan per stack (FP32 spectra); stacks are spread over
 * `lanes` internal streams, largest first onto the least loaded one; each
 * lane owns a slice of the caller's workspace, reused by its stacks in turn.
 * A call with a new set of frame / output pointers captures the whole
 * fork/join sequence into a HIP graph; the batch keeps the graphs of up to 4
 * pointer sets (a caller alternating output buffers replays them; the least
 * recently launched is replaced), and every call is one graph launch on
 * `stream`.  Changing the workspace, the bins or the launch shapes (autotune)
 * drops the graphs.  Results per stack equal ddm_structure_function bit for
 * bit.
 * ------------------------------------------------------------------------- */
typedef struct ddm_batch_s* ddm_batch_t;

ddm_status ddm_batch_create(const ddm_plan_desc* descs, int32_t n_stacks, int32_t lanes, void* stream,
                            ddm_batch_t* out);
ddm_status ddm_batch_destroy(ddm_batch_t batch);
/* rows of D (n_q) and lags (max_lag) of one stack, and the lane it runs on */
ddm_status ddm_batch_query(ddm_batch_t batch, int32_t stack, int64_t* n_q, int32_t* max_lag, int32_t* lane);
ddm_status ddm_batch_workspace_size(ddm_batch_t batch, size_t* bytes);
ddm_status ddm_batch_set_workspace(ddm_batch_t batch, void* workspace_dev, size_t bytes);
/* ddm_plan_autotune for every stack (needs the workspace). */
ddm_status ddm_batch_autotune(ddm_batch_t batch);
/* frames_dev[i] [N_i][H_i][W_i] -> D_dev[i] [n_q_i][M_i]; both arrays are host
 * arrays of n_stacks device pointers.  Each stack's step-one outcome is
 * copied back after the graph through a ring of pinned slots (the host waits
 * only when it is 4 calls ahead); the call returns DDM_ERR_HIP (enqueuing
 * nothing) once when an earlier call's outcomes that have come back name a
 * stack whose step one ran out of time in a wait. */
ddm_status ddm_batch_structure_function(ddm_batch_t batch, const void* const* frames_dev,
                                        float* const* D_dev);
/* Azimuthal |q| bins of one stack computed inside the batch (as
 * ddm_radial_average: T[b] <= k2 < T[b+1], weights 2 for 0 < kx < W/2, FP64
 * fixed-order sums; bit-identical to ddm_radial_average on the stack's D).
 * thresholds_host [n_bins + 1] is copied before the call returns; n_bins = 0
 * removes the stack's bins.  Synchronises the batch's streams; the next call
 * captures a new graph. */
ddm_status ddm_batch_set_bins(ddm_batch_t batch, int32_t stack, const int64_t* thresholds_host, int32_t n_bins);
/* ddm_batch_structure_function plus the bins of every stack that has them:
 * Dbar_dev[i] [n_bins_i][M_i] float64 and counts_dev[i] [n_bins_i] int64
 * (host arrays of n_stacks device pointers; entries of stacks without bins are
 * ignored and may be NULL).  Each stack's radial kernel runs on its lane right
 * after its D, inside the same graph. */
ddm_status ddm_batch_structure_function_binned(ddm_batch_t batch, const void* const* frames_dev, float* const* D_dev,
                                               double* const* Dbar_dev, int64_t* const* counts_dev);
/* Synchronise and report every call since the last report: DDM_ERR_HIP if any
 * stack's step one ran out of time in a wait (its D not valid), else DDM_OK;
 * stack_status_host [n_stacks] (may be NULL) receives each stack's status.
 * Clears what it reports. */
ddm_status ddm_batch_status(ddm_batch_t batch, int32_t* stack_status_host);

/* Azimuthal average of D over |q| bins (standard DDM reduction; not in the
 * paper).  Bin b holds the kept q with T[b] <= k2 < T[b+1], T =
 * k2_thresholds_host[0..n_bins] (non-decreasing int64 >= 0, host; equal
 * neighbours make an empty bin); other q are unbinned.
 * Weight w(q) = 2 for 0 < kx < W/2 (q stands for q and -q), else 1.
 *   Dbar_dev [n_bins][M] float64: sum w D / sum w   (0 for an empty bin)
 *   counts_dev [n_bins] int64:     sum w            (full-plane lattice points)
 *   bin_of_q_dev [n_q] int32:      bin of each row of D, -1 if unbinned (may be NULL)
 * D_dev is [n_q][M] float32 as produced by ddm_structure_function.  Each bin is
 * summed in FP64 in a fixed order (its members in q order, dealt round-robin to
 * four partial sums that are added in order), so results are deterministic.
 * The thresholds are read before the call returns (the host array may be
 * released then); the call waits only when they differ from the last call's
 * and the previous radial launch of the plan is still running. */
ddm_status ddm_radial_average(ddm_plan_t plan, const float* D_dev, const int64_t* k2_thresholds_host,
                              int32_t n_bins, double* Dbar_dev, int64_t* counts_dev,
                              int32_t* bin_of_q_dev);

/* ---------------------------------------------------------------------------
 * Fit of D(q, m) = A (1 - exp(-m / tau)) + B per wave vector (the standard DDM
 * model; the paper computes D and leaves the fit to the analysis).
 * ------------------------------------------------------------------------- */

#define DDM_FIT_MAX_K 64

/* Per-curve result flags. */
enum {
  DDM_FIT_CONVERGED = 1,  /* stopping test met (or stationary to precision) */
  DDM_FIT_MAXITER = 2,    /* iteration limit reached */
  DDM_FIT_NONFINITE = 4,  /* non-finite data or parameters */
  DDM_FIT_STALLED = 8,    /* no decreasing step found, not stationary */
  DDM_FIT_FALLBACK = 16,  /* refitted from the default start after failing from the given one */
  DDM_FIT_DEFAULT_START = 32 /* fallback 2 or 3: the default start was used */
};

/* Sample rows of D at K fractional lags: linear interpolation between the two
 * integer lags around each m_j, then division by the row maximum c.
 *   D_dev [n_rows][M] float32 (device), lags_host [K] float32 in [0, M-1] (host),
 *   1 <= K <= 64; curves_dev [n_rows][K] float32 out; scale_dev [n_rows] out
 *   (c, or 1 when the row maximum is not positive; may be NULL).
 * Asynchronous on `stream` (hipStream_t, NULL = default). */
ddm_status ddm_sample_curves(const float* D_dev, int64_t n_rows, int32_t M, const float* lags_host,
                             int32_t K, float* curves_dev, float* scale_dev, void* stream);

typedef struct ddm_fit_desc {
  uint32_t struct_size; /* = sizeof(ddm_fit_desc) */
  int32_t K;            /* samples per curve, 1..64 */
  int32_t max_iter;     /* Jacobian evaluations per curve (default 200) */
  int32_t fallback;     /* with init_dev: 0 fit from it; 1 curves not converged from it are refitted
                           from the default start; 2 each curve starts from whichever of init_dev and
                           the default start has the lower cost (one fit, no refit); 3 each curve
                           starts from init_dev when its tau lies within [m_1 / 4, 4 m_K] and its A
                           is at least 5% of |A| + |B| (a decay the sampled lags resolve), else from
                           the default start (one fit) */
  double lambda0;       /* initial Marquardt damping (default 1e-3) */
  double ftol;          /* stop when an accepted step lowers the cost by <= ftol * cost (1e-7) */
  double xtol;          /* stop when |step| <= xtol (|p| + xtol), p = (A, B, log tau) (1e-7) */
  double gtol;          /* at a stall: converged if |J_i . r| <= gtol |J_i| |r| for all i (1e-3) */
  void* stream;         /* hipStream_t */
} ddm_fit_desc;

void ddm_fit_desc_init(ddm_fit_desc* desc);

/* Levenberg-Marquardt fit of every curve (one per row): minimise
 * sum_j (A (1 - exp(-m_j / tau)) + B - y_j)^2 over (A, B, log tau) with
 * Marquardt damping lambda diag(J^T J) (x10 on a rejected step, /10 on an
 * accepted one); FP32 residuals, FP64 normal equations.
 *   curves_dev [n][K] float32 (device); lags_host [K] float32 m_j > 0 (host);
 *   init_dev [n][3] (A, B, log tau) float32 start, or NULL for the default start
 *   (on the curve normalised by c = max_j y_j: B0 = y_1/c, A0 = 1 - B0,
 *   tau0 = sqrt(m_1 m_K), scaled back by c);
 *   params_dev [n][3] out (A, B, tau); iters_dev [n] (may be NULL);
 *   flags_dev [n] DDM_FIT_* bits (required when fallback is set, else may be NULL). */
ddm_status ddm_fit(const ddm_fit_desc* desc, const float* curves_dev, const float* lags_host, int64_t n,
                   const float* init_dev, float* params_dev, int32_t* iters_dev, int32_t* flags_dev);

/* ---------------------------------------------------------------------------
 * Fit-initialisation network (not in the paper): a normalised curve of
 * DDM_MLP_IN samples (ddm_sample_curves at log-spaced lags) -> 3 x
 * [Linear(256), GELU] -> Linear(3) = a start (A, B, log tau) for ddm_fit, in
 * the units of the normalised curve (targets are standardised by the caller).
 * BF16 matrix-core products with FP32 accumulation; FP32 master parameters
 * and Adam state.  Parameter vector layout (DDM_MLP_NPARAMS floats, row-major,
 * W[o][i] maps input i to output o): W1[256][64] b1[256] W2[256][256] b2[256]
 * W3[256][256] b3[256] W4[3][256] b4[3].  GELU is exact: z Phi(z).
 * Loss: mean squared error over the batch and the 3 outputs.
 * ------------------------------------------------------------------------- */

#define DDM_MLP_IN 64
#define DDM_MLP_HIDDEN 256
#define DDM_MLP_OUT 3
#define DDM_MLP_NPARAMS 148995

typedef struct ddm_mlp_s* ddm_mlp_t;

/* Create a network with parameters uniform in +-1/sqrt(fan_in) from `seed`
 * and device buffers for training batches of up to max_batch rows (about
 * max_batch * 5.6 KB plus 2.7 MB; inference needs none of them).  All work
 * runs on `stream` (hipStream_t). */
ddm_status ddm_mlp_create(uint64_t seed, int64_t max_batch, void* stream, ddm_mlp_t* out);
ddm_status ddm_mlp_destroy(ddm_mlp_t mlp);

/* Host copies of the FP32 parameters (DDM_MLP_NPARAMS floats).  set_params
 * also clears the Adam state (step 0).  Both synchronise the stream. */
ddm_status ddm_mlp_set_params(ddm_mlp_t mlp, const float* params_host);
ddm_status ddm_mlp_get_params(ddm_mlp_t mlp, float* params_host);

/* Full training state (parameters, Adam moments, step count) for checkpoints:
 * three host arrays of DDM_MLP_NPARAMS floats.  Synchronises the stream. */
ddm_status ddm_mlp_get_state(ddm_mlp_t mlp, float* params_host, float* adam_m_host, float* adam_v_host,
                             int64_t* step);
ddm_status ddm_mlp_set_state(ddm_mlp_t mlp, const float* params_host, const float* adam_m_host,
                             const float* adam_v_host, int64_t step);

/* Inference: x_dev [rows][64] float32 -> y_dev [rows][3] float32 (any rows).
 * One launch over all rows whose workgroups keep 64 rows' activations in LDS
 * (the same BF16 roundings, MFMA products and sums as the training forward,
 * so the same results); uses no batch buffer.  Asynchronous. */
ddm_status ddm_mlp_forward(ddm_mlp_t mlp, const float* x_dev, int64_t rows, float* y_dev);

/* Forward + backward on one batch (1 <= B <= max_batch): keeps the gradient
 * on the device for ddm_mlp_adam_step; if grad_host / loss_host are non-NULL
 * the call synchronises and copies the gradient (DDM_MLP_NPARAMS floats) and
 * the loss out. */
ddm_status ddm_mlp_gradient(ddm_mlp_t mlp, const float* x_dev, const float* target_dev, int64_t B,
                            float* grad_host, float* loss_host);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) with the
 * last gradient. */
ddm_status ddm_mlp_adam_step(ddm_mlp_t mlp, float lr);

/* ddm_mlp_gradient + ddm_mlp_adam_step without host synchronisation; the
 * batch loss is written to loss_dev (device float, may be NULL). */
ddm_status ddm_mlp_train_step(ddm_mlp_t mlp, const float* x_dev, const float* target_dev, int64_t B, float lr,
                              float* loss_dev);

/* Kernel kinds for profiling masks. */
typedef enum ddm_kernel_kind {
  DDM_KERNEL_ROW = 1,    /* row transforms of step one */
  DDM_KERNEL_COL = 2,    /* column transforms + spectra write of step one */
  DDM_KERNEL_TIME = 4,   /* per-wave-vector time transform of step two */
  DDM_KERNEL_RADIAL = 8, /* radial average */
  DDM_KERNEL_STEP1 = 16  /* step one in one launch (rows and columns; square frames up to 512) */
} ddm_kernel_kind;

/* Bracket every launch of the kernel kinds in kernel_mask with a pair of HIP
 * events on the plan's stream (the paper's step-one / step-two time breakdown,
 * its Fig. 2).  0 disables.  Resets the accumulated totals.  Host-side only. */
ddm_status ddm_plan_set_profiling(ddm_plan_t plan, uint32_t kernel_mask);

/* Total device time (ms) and launch count of one kernel kind since the last
 * ddm_plan_set_profiling; waits for the recorded events (host sync).  One kind
 * per call (a single ddm_kernel_kind bit). */
ddm_status ddm_plan_get_profile(ddm_plan_t plan, uint32_t kernel_kind, double* total_ms,
                                int64_t* launches);

/* Thread-local description of the last error on this thread ("" if none). */
const char* ddm_last_error(void);

/* Library ABI version (DDM_ABI_VERSION of the build). */
int32_t ddm_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* DDM_H */
