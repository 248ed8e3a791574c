#!/usr/bin/env python3
"""Throughput of the DDM structure function D(q, m) on one MI355X.

One step = the whole hot path on one stack already resident in HBM:
2-D transform of every frame, transpose to per-q time series, time-FFT
autocorrelation + FP64 prefix sums -> D(q, m) for every kept q and every lag,
then the azimuthal |q| average.  Default workload: 512x512 uint16 (12-bit)
frames, N = 1024, synthetic Brownian spots (the paper-shaped case).

Prints one JSON line with frames/s, the whole-path algorithmic HBM fraction, a
roofline entry for the dominant kernel (timed live with HIP events on the
plan's stream) and the CPU oracle timed on a bounded sample.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
# FP32 vector FMA peak: 256 CUs x 4 SIMDs x 32 FP32 lanes per cycle x 2 flops x
# 2.4 GHz = 157.3 TFLOP/s.  The SIMDs retire FP32 adds and FMAs of a 64-wide wave
# in two cycles also without packed instructions (which this library never
# emits): the counters of the direct-difference kernel show more FP32 VALU
# instructions per cycle than one wave per four cycles per SIMD could issue.
ALU_PEAK_TFLOPS = 256 * 4 * 32 * 2 * 2.4e9 / 1e12
FP32_LANE_OPS = 256 * 4 * 32 * 2.4e9  # FP32 vector lane-instructions per second


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="paper", choices=["paper", "plain", "large"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-columns", type=int, default=None,
                    help="kx columns of the oracle sample (0: all, i.e. the whole workload; "
                         "default all for the 512x512 workload, 2 for 2048x2048)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the tau-fit leg (network training + LM vs MLP+LM on 1024x1024x2048)")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the batched-stacks leg (graph launch vs a loop of single plans)")
    ap.add_argument("--batched-stacks", type=int, default=64)
    ap.add_argument("--no-direct", action="store_true",
                    help="skip the direct-difference leg (step two by Eq. (1) against the time transform)")
    ap.add_argument("--no-long", action="store_true",
                    help="skip the long-stack leg (the bench frames' recipe at 16384 frames, direct differences)")
    ap.add_argument("--long-lags", type=int, default=64)
    ap.add_argument("--learned-curves", type=int, default=1_000_000)
    ap.add_argument("--learned-epochs", type=int, default=30)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy a 1 GiB buffer 3 times (HBM byte-counter calibration)")
    ap.add_argument("--kernel-only", default=None,
                    help="run only this many steps and nothing else (for profilers)")
    ap.add_argument("--f16", action="store_true",
                    help="with --kernel-only: the FP16 per-q-scaled spectra store (profiles; never a bench line)")
    ap.add_argument("--frames", type=int, default=0,
                    help="with --kernel-only: this many frames of the workload's recipe (profiles of "
                         "the long-stack kernels; never a bench line)")
    ap.add_argument("--direct-lags", type=int, default=0,
                    help="with --kernel-only: step two by direct differences for this many lags "
                         "(profiles of the direct kernel; never a bench line)")
    return ap.parse_args()


def algorithmic_bytes(W, H, N, M, nq, pix_bytes):
    """Bytes each kernel must move once, per unit (frame or wave vector)."""
    kx = W // 2  # the row intermediate holds W/2 values per row (kx = 0 carries W/2 too)
    per = {
        # per frame: read the frame, write its half spectrum along x
        "row": H * W * pix_bytes + H * kx * 8,
        # per frame: read the x-spectra, write the kept spectra to the q-major store
        "col": H * kx * 8 + nq * 8,
        # per frame, step one in one launch: read the frame, write its kept spectra
        # (the row intermediate stays in the XCD's L2)
        "step1": H * W * pix_bytes + nq * 8,
        # per wave vector: read its time series, write its D row
        "time": N * 8 + M * 4,
    }
    whole = N * H * W * pix_bytes + 2 * nq * N * 8 + nq * M * 4
    return per, whole


def time_flops(N, M):
    """Algorithmic flops of the time kernel per wave vector (L = 2^ceil(log2 N)):
    three L-point complex FFTs at 5 L log2 L, the half-angle pre-twiddle (6 L),
    the power spectra of both halves (6 L), offset removal (4 L), |x'|^2 and the
    FP64 prefix sums (4 L), and the per-lag combination (13 M)."""
    import math
    L = 16
    while L < N:
        L *= 2
    return 15 * L * math.log2(L) + 20 * L + 13 * M


# sources each profiled kernel is built from (a summary is valid while they hash the same)
PROFILED_SOURCES = {"k_time": ("time_kernel.hpp", "fft.hpp", "internal.hpp"),
                    "k_step1": ("k_spatial.hip", "fft.hpp", "internal.hpp")}


def recorded_traffic(kernel, config):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summary, or
    None when there is none or the kernel sources changed since it was taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", "%s_%s_f32.md" % (kernel, config))
    if kernel not in PROFILED_SOURCES or not os.path.exists(path):
        return None
    text = open(path).read()
    m_t = re.search(r"^traffic_bytes_per_launch: (\d+)", text, re.M)
    m_h = re.search(r"^source_sha256: ([0-9a-f]+)", text, re.M)
    if not (m_t and m_h):
        return None
    src = "".join(open(os.path.join(ROOT, "paper_2012_05695_amd", "csrc", f)).read()
                  for f in PROFILED_SOURCES[kernel])
    if hashlib.sha256(src.encode()).hexdigest() != m_h.group(1):
        return None
    return int(m_t.group(1))


def cpu_baseline(frames_cpu, ncols, nq_total):
    import numpy as np
    from oracle import dft, structure
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fr = frames_cpu.numpy()
    N, H, W = fr.shape
    if ncols <= 0:
        ncols = W // 2 + 1
    cols = list(range(ncols))
    t0 = time.perf_counter()
    F = dft.dft_columns(fr, cols, np.arange(H))              # [N, H, ncols]
    Fq = F.reshape(N, -1).T.copy()                           # [H*ncols, N]
    structure.structure_function_direct(Fq, impl="c", threads=threads)
    dt = time.perf_counter() - t0
    nq_s = H * ncols
    full_s = dt * nq_total / nq_s
    if nq_s >= nq_total:
        sample = "whole workload: all %d q, all %d frames and lags (%.1f s)" % (nq_total, N, dt)
    else:
        sample = ("kx columns 0..%d x all %d ky (%d of %d q), all %d frames and lags; "
                  "%.2f s measured, extrapolated linearly in q to %.0f s" %
                  (ncols - 1, H, nq_s, nq_total, N, dt, full_s))
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": N / full_s, "unit": "frames/s", "cores": threads, "kind": "oracle", "sample": sample,
            "cpu": cpu, "host_cpus": os.cpu_count()}


def cpu_fourier(frames, max_lag=0, workers=None, chunk=256):
    """The paper's Fourier method on the host (its CPU WITH_FT mode; section
    "The algorithm" and Appendix B), as a second host baseline beside the
    O(N^2) oracle: pocketfft (scipy.fft) in single precision, like the device
    path, on `workers` threads; not part of the library, which has no CPU path.

    Step one: the 2-D real transform of every frame minus frame 0 (D depends on
    differences only), batches of frames on all threads.  Step two: chunks of
    `chunk` wave vectors, one chunk per thread at a time: the temporal mean
    removed (D is unchanged), the zero-padded transform of length 2L >= 2N - 1
    (Eq. (B4)), the inverse of its squared modulus (the autocorrelation; only
    its real part is needed, the inverse of the even part of the squared
    modulus, a half-length real transform), and Eq. (B3) with FP64 prefix sums
    of |F_n|^2.  frames: array [N, H, W] (integers); returns D [H (W/2 + 1), M]
    float64 in the library's q order (ky-major, then kx)."""
    import numpy as np
    import scipy.fft as sfft
    from concurrent.futures import ThreadPoolExecutor
    fr = np.asarray(frames)
    N, H, W = fr.shape
    M = N if not max_lag else int(max_lag)
    if workers is None:
        workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    f0 = fr[0].astype(np.float32)
    F = np.empty((N, H, W // 2 + 1), dtype=np.complex64)
    for t0 in range(0, N, 64):
        F[t0:t0 + 64] = sfft.rfft2(fr[t0:t0 + 64].astype(np.float32) - f0, workers=workers)
    Fq = F.reshape(N, -1).T                                   # [Q, N] (a strided view)
    Q = Fq.shape[0]
    L2 = 1
    while L2 < 2 * N - 1:
        L2 <<= 1
    D = np.empty((Q, M), dtype=np.float64)
    ramp = 1.0 / (N - np.arange(1, M, dtype=np.float64))
    neg = (-np.arange(L2 // 2 + 1)) % L2
    m = np.arange(1, M)

    def run(q0):
        x = np.ascontiguousarray(Fq[q0:q0 + chunk])
        x -= x.mean(axis=1, keepdims=True)
        X = sfft.fft(x, n=L2, axis=1)
        P = X.real ** 2 + X.imag ** 2
        s = sfft.irfft(0.5 * (P[:, :L2 // 2 + 1] + P[:, neg]), n=L2, axis=1)
        c = np.zeros((x.shape[0], N + 1))
        np.cumsum(x.real.astype(np.float64) ** 2 + x.imag.astype(np.float64) ** 2, axis=1, out=c[:, 1:])
        # sum_{n<N-m} |F_n|^2 + sum_{n>=m} |F_n|^2 - 2 Re sum_n F_{n+m} F_n^*, over N - m
        out = D[q0:q0 + chunk]
        out[:, 0] = 0.0
        out[:, 1:] = c[:, N - m] + (c[:, N:N + 1] - c[:, m]) - 2.0 * s[:, 1:M]
        out[:, 1:] *= ramp

    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(run, range(0, Q, chunk)))
    return D


def cpu_fourier_leg(frames_cpu, thresholds, nbins):
    """The host Fourier method on the whole bench workload, binned: frames/s."""
    import numpy as np
    import scipy.sparse
    workers = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    fr = frames_cpu.numpy()
    N, H, W = fr.shape
    t0 = time.perf_counter()
    D = cpu_fourier(fr, workers=workers)
    # bins as ddm_radial_average: T[b] <= k2 < T[b+1], k2 = kx^2 ca + ky^2 cc,
    # weight 2 for 0 < kx < W/2 (the other half plane), weighted means
    g = math.gcd(W, H)
    ca, cc = (H // g) ** 2, (W // g) ** 2
    ky = np.repeat(np.arange(H), W // 2 + 1)
    kx = np.tile(np.arange(W // 2 + 1), H)
    kys = np.where(ky <= H // 2, ky, ky - H).astype(np.int64)
    k2 = kx.astype(np.int64) ** 2 * ca + kys ** 2 * cc
    b = np.searchsorted(np.asarray(thresholds, dtype=np.int64), k2, side="right") - 1
    w = np.where((kx > 0) & (kx < W // 2), 2.0, 1.0)
    ok = np.nonzero((b >= 0) & (b < nbins))[0]
    S = scipy.sparse.csr_matrix((w[ok], (b[ok], ok)), shape=(nbins, D.shape[0]))
    cnt = np.asarray(S.sum(axis=1)).ravel()
    Dbar = (S @ D) / np.maximum(cnt, 1.0)[:, None]
    dt = time.perf_counter() - t0
    return {"value": N / dt, "unit": "frames/s", "cores": workers, "kind": "host Fourier method (scipy.fft)",
            "sample": "whole workload: all %d q, all %d lags, %d bins (%.2f s)" % (D.shape[0], N, nbins, dt)}


def learned_leg(log):
    """tau-fit time of MLP+LM against LM from the default start, on every q of a
    1024x1024x2048 stack; the network is trained first on curves computed by
    the pipeline from 128x128x2048 stacks (D0 and SNR log-uniform)."""
    import numpy as np
    import torch
    from paper_2012_05695_amd import learn

    args = parse()
    t0 = time.perf_counter()
    X, T, lags = learn.make_training_set(args.learned_curves, W=128, H=128, N=2048, seed0=1000)
    t1 = time.perf_counter()
    init, losses = learn.train(X, T, epochs=args.learned_epochs, batch=4096, lr=2e-3)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    del X, T
    rng = np.random.default_rng(7)
    D0, snr, n_spots, a = learn.draw_stack_params(rng, 1024, 1024)
    curves, scale, (A, B, tau) = learn.stack_curves(1024, 1024, 2048, D0, n_spots, a, 7, lags)
    learn.compare(curves[:4096].contiguous(), lags, init)  # warm-up
    res = learn.compare(curves, lags, init, truth_tau=tau, tau_window=(2.0, 512.0))
    log("learned leg: data %.1f s, training %.1f s (loss %.3f -> %.3f)" %
        (t1 - t0, t2 - t1, losses[0], losses[-1]))
    return {"stack": "1024x1024 uint16 x 2048 frames, D0 %.3g px^2/frame, SNR %.3g, seed 7" % (D0, snr),
            "n_curves": res["n"], "K": 64,
            "lm_default_ms": res["default_ms"], "mlp_ms": res["mlp_ms"], "mlp_plus_lm_ms": res["learned_ms"],
            "mlp_plus_lm_refit_ms": res["learned_refit_ms"], "mlp_plus_lm_gated_ms": res["learned_gated_ms"],
            "learned": "start from the lower-cost of the network's and the default start, one fit; "
                       "learned_refit: network start, refit from the default start if not converged; "
                       "learned_gated: network start where its tau is within [m_1/4, 4 m_K], else the "
                       "default start, one fit",
            "all": res["all"], "measurable_tau_2_to_512": res.get("measurable"),
            "training": {"curves": args.learned_curves, "epochs": args.learned_epochs,
                         "final_loss": losses[-1], "data_s": t1 - t0, "train_s": t2 - t1}}


def kernel_roof(kind, ms_per_launch, launches_per_step, W, H, N, M, nq, pix_bytes):
    """Roofline entry of one kernel from its average launch time: achieved HBM
    rate on its algorithmic bytes, and for the time kernel also its FP32 rate;
    "bound" is the roof that needs the longer time at peak."""
    per, _ = algorithmic_bytes(W, H, N, M, nq, pix_bytes)
    if kind in ("row", "col", "step1"):
        nbytes = per[kind] * N / launches_per_step
    elif kind == "time":
        nbytes = per["time"] * nq / launches_per_step
    else:
        nbytes = nq * M * 4 / launches_per_step
    gbs = nbytes / (ms_per_launch * 1e-3) / 1e9
    roof = {"kernel": kind, "bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": nbytes,
            "avg_launch_ms": ms_per_launch}
    if kind == "time":
        flops = time_flops(N, M) * nq / launches_per_step
        tf = flops / (ms_per_launch * 1e-3) / 1e12
        if flops / (ALU_PEAK_TFLOPS * 1e12) > nbytes / (HBM_PEAK_GBS * 1e9):
            roof.update({"bound": "alu", "achieved": tf, "peak": ALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tf / ALU_PEAK_TFLOPS, "algorithmic_flops_per_launch": flops,
                         "hbm_achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS})
        else:
            roof.update({"algorithmic_flops_per_launch": flops, "alu_achieved_TFLOPs": tf,
                         "alu_frac": tf / ALU_PEAK_TFLOPS})
    return roof


def copy_bandwidth():
    """GB/s (bytes read + written) of a 1 GiB device-to-device torch copy: what
    a plain streaming kernel reaches on this machine."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(5):
        dst.copy_(src)
    ev[1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / 5
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def batched_leg(n_stacks, log, lanes=4):
    """a7: stacks of mixed shapes (W = H in {128, 256, 384, 512, 1024}, N log-uniform in
    [256, 4096], D0 log-uniform in [0.01, 10], 2000 spots per 512x512, uint16) in one graph
    launch, against the same stacks as a loop of single-plan calls on one stream."""
    import math
    import numpy as np
    import torch
    from paper_2012_05695_amd import api, synth
    rng = np.random.default_rng(64)
    shapes, frames = [], []
    for i in range(n_stacks):
        w = int(rng.choice([128, 256, 384, 512, 1024]))
        n = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
        d0 = math.exp(rng.uniform(math.log(0.01), math.log(10.0)))
        nsp = max(1, int(round(2000 * w * w / (512 * 512))))
        frames.append(synth.brownian_stack(w, w, n, nsp, 1.5, 40.0, 800.0, d0, seed=5000 + i, pixel="u16",
                                           device="cuda"))
        shapes.append((w, w, n))
    torch.cuda.synchronize()
    total = sum(n for _, _, n in shapes)
    log("batched leg: %d stacks, %d frames, %.1f GB of frames" %
        (n_stacks, total, sum(f.numel() * 2 for f in frames) / 1e9))
    batch = api.Batch(shapes, lanes=lanes)
    batch.allocate_workspace()
    # integer |q| bins (b = round |k|) of every stack, computed inside the graph
    thr = [api.integer_bin_thresholds(int(w * 0.7072) + 2) for (w, _, _) in shapes]
    for i, t in enumerate(thr):
        batch.set_bins(i, t)
    outs, dbar, cnt = batch.structure_function_binned(frames)
    # the loop's plans run one after another on one stream, after the batch: they
    # share the batch's workspace (it holds the largest stack's full workspace)
    plans = [api.Plan(w, h, n) for (w, h, n) in shapes]
    shared = batch._ws
    assert shared.numel() >= max(p.workspace_size()[1] for p in plans)
    for p in plans:
        p.set_workspace(shared)

    def loop():
        for p, f, o, t in zip(plans, frames, outs, thr):
            p.structure_function(f, out=o)
            p.radial_average(o, t, bin_of_q=False)

    loop()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    reps = 3
    ev[0].record()
    for _ in range(reps):
        batch.structure_function_binned(frames, outs, dbar, cnt)
    ev[1].record()
    for _ in range(reps):
        loop()
    ev[2].record()
    torch.cuda.synchronize()
    t_b = ev[0].elapsed_time(ev[1]) / reps
    t_l = ev[1].elapsed_time(ev[2]) / reps
    stack_status = batch.status()
    if any(st != 0 for st in stack_status):
        raise RuntimeError("batched leg: stacks reported errors: %s" % stack_status)
    for p in plans:
        p.status()
        p.close()
    batch.close()
    del shared
    torch.cuda.empty_cache()
    # the same batch with minimal padding (time transforms of the smallest 2^k
    # or 3 * 2^k >= N) instead of powers of two (the length Eq. (B4) prints)
    b2 = api.Batch(shapes, lanes=lanes, padding="minimal")
    b2.allocate_workspace()
    for i, t in enumerate(thr):
        b2.set_bins(i, t)
    b2.structure_function_binned(frames, outs, dbar, cnt)
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        b2.structure_function_binned(frames, outs, dbar, cnt)
    ev[1].record()
    torch.cuda.synchronize()
    t_p2 = ev[0].elapsed_time(ev[1]) / reps
    if any(st != 0 for st in b2.status()):
        raise RuntimeError("batched leg (minimal padding): stacks reported errors")
    b2.close()
    del frames, outs, dbar, cnt
    torch.cuda.empty_cache()
    return {"stacks": n_stacks, "shapes": ["%dx%dx%d" % s for s in shapes], "frames": total,
            "batched_ms": t_b, "loop_ms": t_l, "batched_frames_per_s": total / (t_b * 1e-3),
            "loop_frames_per_s": total / (t_l * 1e-3),
            "batched_minimal_padding_ms": t_p2,
            "work": "D of every stack and its integer |q| bins; graph launch (4 lanes) vs the same "
                    "calls one after another on one stream",
            "recipe": "%d stacks of the batched workload's recipe, seeds 5000+i" % n_stacks}


def main():
    args = parse()
    if (args.direct_lags or args.f16 or args.frames) and args.kernel_only is None:
        print("bench.py: --direct-lags, --f16 and --frames are for --kernel-only profiling runs", file=sys.stderr)
        sys.exit(2)
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU only (the path shards over q across GPUs "
              "but no multi-GPU run exists); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2012_05695_amd import api, synth

    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 3 x 1 GiB", file=sys.stderr)
        return

    recipe = {"paper": synth.PAPER, "plain": synth.PLAIN, "large": synth.LARGE}[args.config]
    W, H, N = recipe["W"], recipe["H"], args.frames or recipe["N"]
    print("bench: generating %dx%dx%d %s stack on GPU" % (W, H, N, recipe["pixel"]), file=sys.stderr,
          flush=True)
    frames = synth.make(recipe, device="cuda", N=N)
    torch.cuda.synchronize()
    spectrum = "f16" if args.f16 else "f32"
    if args.direct_lags:
        plan = api.Plan(W, H, N, pixel=recipe["pixel"], spectrum=spectrum, max_lag=args.direct_lags,
                        method="direct")
    else:
        plan = api.Plan(W, H, N, pixel=recipe["pixel"], spectrum=spectrum)
    plan.allocate_workspace()
    M, nq = plan.max_lag, plan.n_q
    D = torch.empty((nq, M), dtype=torch.float32, device="cuda")
    kx, ky = plan.q_index()
    nbins = int((kx.astype("int64") ** 2 + ky.astype("int64") ** 2).max() ** 0.5) + 2
    thr = api.integer_bin_thresholds(nbins)

    def step():
        plan.structure_function(frames, out=D)
        plan.radial_average(D, thr, bin_of_q=False)

    if args.kernel_only is not None:
        for _ in range(int(args.kernel_only)):
            step()
        torch.cuda.synchronize()
        print("kernel-only steps done", file=sys.stderr)
        return

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # untimed profiling pass over a few steps: which kernel dominates?
    kinds = ["row", "col", "step1", "time", "radial"]
    plan.set_profiling(kinds)
    nprof = 5
    for _ in range(nprof):
        step()
    torch.cuda.synchronize()
    prof = {k: plan.profile(k) for k in kinds}
    prof = {k: (v[0] / nprof, v[1] / nprof) for k, v in prof.items() if v[1] > 0}  # per step, kinds that launched
    dominant = max(prof, key=lambda k: prof[k][0])
    print("bench: per-kernel ms in one step: %s" % {k: round(v[0], 4) for k, v in prof.items()},
          file=sys.stderr, flush=True)

    # timed region: whole steps; only the dominant kernel is bracketed by events
    plan.set_profiling([dominant])
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    ms_step = ev0.elapsed_time(ev1) / args.steps
    k_ms, k_n = plan.profile(dominant)
    plan.set_profiling([])
    plan.status()  # raises if any timed call's step one reported an error

    pix_bytes = 1 if recipe["pixel"] == "u8" else 2
    per, whole = algorithmic_bytes(W, H, N, M, nq, pix_bytes)
    # launches per step of row/col split the frames into batches
    launches_per_step = k_n / args.steps
    if dominant in ("row", "col", "step1"):
        bytes_per_launch = per[dominant] * N / launches_per_step
    elif dominant == "time":
        bytes_per_launch = per["time"] * nq / launches_per_step
    else:
        bytes_per_launch = nq * M * 4 / launches_per_step
    avg_launch_ms = k_ms / k_n
    achieved = bytes_per_launch / (avg_launch_ms * 1e-3) / 1e9
    # the binding roof: the larger of the time its bytes need at HBM peak and
    # the time its flops need at the FP32 vector peak
    roof = {"kernel": dominant, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS}
    if dominant == "time":
        flops_per_launch = time_flops(N, M) * nq / launches_per_step
        t_alu = flops_per_launch / (ALU_PEAK_TFLOPS * 1e12)
        t_hbm = bytes_per_launch / (HBM_PEAK_GBS * 1e9)
        tf = flops_per_launch / (avg_launch_ms * 1e-3) / 1e12
        if t_alu > t_hbm:
            roof = {"kernel": dominant, "bound": "alu", "achieved": tf, "peak": ALU_PEAK_TFLOPS,
                    "unit": "TFLOP/s", "frac": tf / ALU_PEAK_TFLOPS,
                    "algorithmic_flops_per_launch": flops_per_launch,
                    "hbm_achieved_GBs": achieved, "hbm_frac": achieved / HBM_PEAK_GBS}
        else:
            roof.update({"algorithmic_flops_per_launch": flops_per_launch, "alu_achieved_TFLOPs": tf,
                         "alu_frac": tf / ALU_PEAK_TFLOPS})

    out = {
        "metric": "frames/s & % HBM peak for D(q,dt) at 512x512x1024; tau-fit time MLP+LM vs LM",
        "value": N / (ms_step * 1e-3),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%dx%d uint16 (12-bit) x %d frames, Brownian spots, FP32 spectra, "
                               "all %d half-plane q, all %d lags, %d integer |q| bins" %
                               (W, H, N, nq, M, nbins),
                   "n_q": nq, "max_lag": M},
        "hbm_frac_whole_path": (whole / (ms_step * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "algorithmic_bytes_whole_path": whole,
        "kernel_ms_per_step": {k: v[0] for k, v in prof.items()},
        "roofline": dict(roof, **{
            "traffic": recorded_traffic("k_" + dominant, "%dx%dx%d" % (W, H, N)),
            "avg_launch_ms": avg_launch_ms, "launches": k_n,
            "algorithmic_bytes_per_launch": bytes_per_launch}),
    }
    # every kernel of the step against its roof (from the profiling pass)
    out["kernel_rooflines"] = {k: kernel_roof(k, v[0] / v[1], v[1], W, H, N, M, nq, pix_bytes)
                               for k, v in prof.items()}
    out["copy_GBs"] = copy_bandwidth()
    if args.config == "large":
        args.no_batched = args.no_learned = True  # legs of the other workloads
    frames_cpu = None
    if not args.no_cpu_baseline:
        frames_cpu = frames.cpu()
    if args.config != "paper":
        del frames, D
        plan.close()
        torch.cuda.empty_cache()
        finish(args, out, frames_cpu, nq)
        return
    # the same workload with the FP16 per-q-scaled spectra store
    plan16 = api.Plan(W, H, N, pixel=recipe["pixel"], spectrum="f16")
    plan16.allocate_workspace()
    for _ in range(2):
        plan16.structure_function(frames, out=D)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(args.steps):
        plan16.structure_function(frames, out=D)
        plan16.radial_average(D, thr, bin_of_q=False)
    ev1.record()
    torch.cuda.synchronize()
    ms16 = ev0.elapsed_time(ev1) / args.steps
    out["f16_store"] = {"ms_per_step": ms16, "frames_per_s": N / (ms16 * 1e-3),
                        "saturated_values": int(plan16.fp16_saturations())}
    plan16.status()
    plan16.close()
    out["host_frames"] = host_frames_leg(plan, frames, D, args.steps)
    if frames_cpu is not None:
        print("bench: host Fourier method (scipy.fft) on the whole workload", file=sys.stderr, flush=True)
        out["cpu_fourier"] = cpu_fourier_leg(frames_cpu, thr, nbins)
    if not args.no_direct:
        print("bench: direct-difference leg (max_lag and N sweeps against the time transform)", file=sys.stderr,
              flush=True)
        out["direct"] = direct_leg(frames, recipe["pixel"])
    if not args.no_long:
        print("bench: long-stack leg (16384 frames, direct differences)", file=sys.stderr, flush=True)
        out["long_stack"] = long_stack_leg(recipe, args.long_lags)
    del frames, D
    plan.close()
    torch.cuda.empty_cache()
    finish(args, out, frames_cpu, nq)


def host_frames_leg(plan, frames, D, steps):
    """The same workload with the frames in pinned host memory
    (ddm_structure_function_host): the PCIe-inclusive rate, beside a plain
    host-to-device copy of the frames."""
    import torch
    N, H, W = frames.shape
    pinned = frames.cpu().pin_memory()
    fb = H * W * pinned.element_size()
    staging = torch.empty(((fb + 255) // 256) * 256 + 2 * 64 * fb + 512, dtype=torch.uint8, device="cuda")
    plan.structure_function_host(pinned, staging, out=D)
    dev = torch.empty_like(frames)
    dev.copy_(pinned, non_blocking=True)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    reps = max(3, steps // 4)
    ev[0].record()
    for _ in range(reps):
        plan.structure_function_host(pinned, staging, out=D)
    ev[1].record()
    for _ in range(reps):
        dev.copy_(pinned, non_blocking=True)
    ev[2].record()
    torch.cuda.synchronize()
    plan.status()
    t_h = ev[0].elapsed_time(ev[1]) / reps
    t_c = ev[1].elapsed_time(ev[2]) / reps
    del dev, staging
    return {"ms_per_stack": t_h, "frames_per_s": N / (t_h * 1e-3), "h2d_copy_ms": t_c,
            "h2d_GBs": pinned.numel() * pinned.element_size() / (t_c * 1e-3) / 1e9,
            "work": "structure function only (no bins), frames in pinned host memory, 2 x 64-frame staging"}


def direct_leg(frames, pixel, reps=3):
    """Step two by direct differences (method "direct") against the time
    transform on the bench frames: a max_lag sweep at N = 1024 and an all-lags
    sweep over N (the first N frames), step-two device ms per call from the
    plan's event pairs; the direct kernel against the FP32 vector roof (four
    FP32 vector instructions per difference pair: two subtractions, two FMAs) and,
    where few lags make it memory-bound, against HBM (the spectra read once, D
    written once)."""
    import torch
    from paper_2012_05695_amd import api
    N, H, W = frames.shape
    lane_ops = FP32_LANE_OPS

    def step_two_ms(n, M, method, fr):
        p = api.Plan(W, H, n, pixel=pixel, max_lag=M, method=method)
        p.allocate_workspace()
        D = p.structure_function(fr)
        p.set_profiling(["time"])
        for _ in range(reps):
            p.structure_function(fr, out=D)
        torch.cuda.synchronize()
        ms, k = p.profile("time")
        p.status()
        nq = p.n_q
        p.close()
        return ms / k, nq

    lags = []
    for M in (8, 16, 32, 48, 64, 128, 1024):
        md, nq = step_two_ms(N, M, "direct", frames)
        mf, _ = step_two_ms(N, M, "fourier", frames)
        pairs = nq * (N * M - M * (M - 1) // 2)
        byts = nq * (N * 8 + M * 4)
        auto = api.Plan(W, H, N, pixel=pixel, max_lag=M, method="auto")
        lags.append({"max_lag": M, "direct_ms": md, "fourier_ms": mf, "direct_over_fourier": md / mf,
                     "direct_valu_frac": 4.0 * pairs / (md * 1e-3) / lane_ops,
                     "direct_hbm_frac": byts / (md * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "auto_model_choice": auto.method})
        auto.close()
    sweep = []
    for n in (16, 32, 64, 128, 256, 512, 1024):
        fr = frames[:n].contiguous() if n < N else frames
        md, _ = step_two_ms(n, n, "direct", fr)
        mf, _ = step_two_ms(n, n, "fourier", fr)
        sweep.append({"n_frames": n, "direct_ms": md, "fourier_ms": mf, "direct_over_fourier": md / mf})
    torch.cuda.empty_cache()
    return {"workload": "%dx%d frames of the bench stack, FP32 spectra store; step two only" % (W, H),
            "max_lag_sweep_at_N%d" % N: lags, "all_lags_sweep": sweep}


def long_stack_leg(recipe, M, N=16384, steps=3):
    """The bench frames' recipe at N = 16384 frames (the paper's longest stacks):
    step one, then step two by direct differences for M lags, timed over whole
    steps (the frames resident in HBM); then all N lags by both methods."""
    import torch
    from paper_2012_05695_amd import api, synth
    W, H = recipe["W"], recipe["H"]
    frames = synth.make(recipe, device="cuda", N=N)
    plan = api.Plan(W, H, N, pixel=recipe["pixel"], max_lag=M, method="direct")
    plan.allocate_workspace()
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    plan.set_profiling(["step1", "row", "col", "time"])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(steps):
        plan.structure_function(frames, out=D)
    ev[1].record()
    torch.cuda.synchronize()
    plan.status()
    ms = ev[0].elapsed_time(ev[1]) / steps
    prof = {k: plan.profile(k) for k in ("step1", "row", "col", "time")}
    per = {("direct" if k == "time" else k): v[0] / steps for k, v in prof.items() if v[1] > 0}
    nq = plan.n_q
    plan.close()
    del D
    torch.cuda.empty_cache()
    out = {"workload": "%dx%d %s x %d frames, %d lags, step two by direct differences" % (W, H, recipe["pixel"], N, M),
           "ms_per_stack": ms, "frames_per_s": N / (ms * 1e-3), "kernel_ms": per,
           "algorithmic_bytes": N * H * W * (2 if recipe["pixel"] == "u16" else 1) + 2 * nq * N * 8 + nq * M * 4}
    out["all_lags"] = long_stack_all_lags(recipe, frames, N)
    del frames
    torch.cuda.empty_cache()
    return out


def long_stack_all_lags(recipe, frames, N, steps=3):
    """All N lags of the same stack by the time transform of length 16384 (FP32
    and FP16 spectra stores) and, once, by direct differences (the comparison
    the paper draws between the two schemes at its longest stacks); the largest
    per-q relative differences of the D."""
    import torch
    from paper_2012_05695_amd import api
    W, H = recipe["W"], recipe["H"]
    res, Ds = {}, {}
    for method, reps in (("fourier", steps), ("fourier_f16", steps), ("direct", 1)):
        print("bench: long stack, all %d lags, %s" % (N, method), file=sys.stderr, flush=True)
        spectrum = "f16" if method.endswith("f16") else "f32"
        plan = api.Plan(W, H, N, pixel=recipe["pixel"], spectrum=spectrum, method=method.split("_")[0])
        plan.allocate_workspace()
        D = plan.structure_function(frames)
        torch.cuda.synchronize()
        plan.set_profiling(["step1", "row", "col", "time"])
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            plan.structure_function(frames, out=D)
        ev[1].record()
        torch.cuda.synchronize()
        plan.status()
        ms = ev[0].elapsed_time(ev[1]) / reps
        prof = {k: plan.profile(k) for k in ("step1", "row", "col", "time")}
        name = "direct" if method == "direct" else "time"
        per = {(name if k == "time" else k): v[0] / reps for k, v in prof.items() if v[1] > 0}
        res[method] = {"ms_per_stack": ms, "frames_per_s": N / (ms * 1e-3), "kernel_ms": per}
        plan.close()
        Ds[method] = D
    num = (Ds["fourier"].double() - Ds["direct"].double()).abs().amax(dim=1)
    den = Ds["direct"].double().amax(dim=1).clamp_min(1e-300)
    res["max_rel_diff_fourier_vs_direct"] = float((num / den).max())
    num = (Ds["fourier_f16"].double() - Ds["fourier"].double()).abs().amax(dim=1)
    res["max_rel_diff_fourier_f16_vs_f32"] = float((num / den).max())
    res["direct_over_fourier"] = res["direct"]["ms_per_stack"] / res["fourier"]["ms_per_stack"]
    del Ds, D
    torch.cuda.empty_cache()
    return res


def finish(args, out, frames_cpu, nq):
    if not args.no_batched:
        print("bench: batched leg (graph launch vs loop)", file=sys.stderr, flush=True)
        out["batched"] = batched_leg(args.batched_stacks,
                                     lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if not args.no_learned:
        print("bench: tau-fit leg (training the start network, then LM vs MLP+LM)", file=sys.stderr,
              flush=True)
        out["tau_fit"] = learned_leg(lambda m: print("bench: " + m, file=sys.stderr, flush=True))
    if frames_cpu is not None:
        print("bench: timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cols = args.cpu_columns
        if cols is None:
            cols = 2 if args.config == "large" else 0
        out["cpu_baseline"] = cpu_baseline(frames_cpu, cols, nq)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
