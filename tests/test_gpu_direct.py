"""Step two by direct differences (method "direct": Eq. (1) term by term on
the stored spectra) against the FP64 oracle, on the paths that reach it: the
blocked FP32 and FP16 stores, holes of a low-q cut, several groups, ragged
last lag tiles, the plain layout of ddm_structure_from_spectra, long stacks
(N = 9000 and 16384), and the automatic choice."""

import sys

import numpy as np
import pytest
import torch

from oracle import structure
from paper_2012_05695_amd import _lib as L
from paper_2012_05695_amd import synth

from helpers import TOL_F32, describe, oracle_D, per_q_error

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("W,H,N,pixel,kw", [
    (32, 32, 300, "u8", {}),                                    # every lag
    (64, 48, 1000, "u16", {"max_lag": 37}),                     # ragged last lag tile
    (16, 16, 2, "u8", {}),                                      # the smallest stack
    (16, 16, 3, "u16", {"max_lag": 1}),                         # lag 0 only
    (48, 32, 129, "u16", {"k2_max": 300}),                      # low-q cut: holes in the store
    (64, 64, 700, "u16", {"spectrum": "f16", "max_lag": 100}),  # FP16 store
    (96, 64, 517, "u8", {"max_lag": 200, "ws": "min"}),         # several groups
    (128, 128, 200, "u16", {"max_lag": 64, "ws": "min"}),       # single-launch step one, groups
])
def test_direct_matches_oracle(gpu, W, H, N, pixel, kw):
    kw = dict(kw)
    ws = kw.pop("ws", "full")
    say("case: direct", W, H, N, pixel, kw, ws)
    frames = synth.brownian_stack(W, H, N, max(4, W * H // 30), 1.5, 40.0, 200.0, 0.3, seed=N + W, pixel=pixel)
    plan = gpu.Plan(W, H, N, pixel=pixel, method="direct", **kw)
    assert plan.method == "direct"
    mn, full = plan.workspace_size()
    plan.allocate_workspace(mn if ws == "min" else full)
    D = plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    assert plan.status() == L.DDM_OK
    Do, _ = oracle_D(frames.numpy(), k2_max=kw.get("k2_max", -1), max_lag=kw.get("max_lag"))
    e = per_q_error(D.cpu().numpy(), Do)
    say("direct", W, H, N, kw, describe(e))
    assert e.max() <= (5e-3 if kw.get("spectrum") == "f16" else TOL_F32)
    assert np.all(D[:, 0].cpu().numpy() == 0.0)
    # the same bits on a second call
    assert torch.equal(D, plan.structure_function(frames.cuda()))


@pytest.mark.parametrize("N,M", [(2, 2), (97, 97), (1000, 300), (4096, 24)])
def test_direct_from_spectra_plain_layout(gpu, N, M):
    """ddm_structure_from_spectra with the direct method: time series [n_q][N]
    in the plain layout (one slot per lane reads its own row)."""
    say("case: direct from spectra", N, M)
    plan = gpu.Plan(16, 16, N, max_lag=M, method="direct")
    g = torch.Generator().manual_seed(N)
    F = torch.complex(torch.randn(plan.n_q, N, generator=g), torch.randn(plan.n_q, N, generator=g)) * 50.0
    F = F + (3.0 + 1.0j) * 100.0  # a static part, removed by the differences
    F = F.to(torch.complex64)
    D = plan.structure_from_spectra(F.cuda())
    torch.cuda.synchronize()
    Do = structure.structure_function_direct(F.numpy().astype(np.complex128), M)
    e = per_q_error(D.cpu().numpy(), Do)
    say("from spectra", N, M, describe(e))
    assert e.max() <= TOL_F32


def test_direct_long_stack_256x256x16384(gpu):
    """N = 16384, beyond the time transform's lengths: the single-launch step
    one over 16384 frames, then direct differences for 128 lags; every ky, kx
    columns {0, 3, 128} against the oracle."""
    say("case: direct 256x256x16384 u16, max_lag 128")
    frames = synth.brownian_stack(256, 256, 16384, 300, 1.5, 40.0, 800.0, 0.1, seed=16384, pixel="u16",
                                  device="cuda")
    plan = gpu.Plan(256, 256, 16384, max_lag=128, method="direct")
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    assert plan.status() == L.DDM_OK
    Dg = D.cpu().numpy()
    Do, rows = oracle_D(frames.cpu().numpy(), max_lag=128, kx_subset=[0, 3, 128])
    e = per_q_error(Dg[rows], Do)
    say("256x256x16384 direct (%d q):" % len(rows), describe(e))
    assert e.max() <= TOL_F32


def test_direct_long_stack_nonsquare_split_step_one(gpu):
    """N = 9000 on 64 x 32 frames (the two-kernel step one), all 40 lags."""
    say("case: direct 64x32x9000 u8, max_lag 40")
    frames = synth.brownian_stack(64, 32, 9000, 60, 1.5, 40.0, 200.0, 0.5, seed=9000, pixel="u8")
    plan = gpu.Plan(64, 32, 9000, pixel="u8", max_lag=40, method="auto")
    assert plan.method == "direct"  # the cost model's choice for 40 of 9000 lags
    D = plan.structure_function(frames.cuda())
    torch.cuda.synchronize()
    Do, _ = oracle_D(frames.numpy(), max_lag=40)
    e = per_q_error(D.cpu().numpy(), Do)
    say("64x32x9000 direct", describe(e))
    assert e.max() <= TOL_F32


def test_auto_method_choice_and_autotune(gpu):
    """AUTO takes the cost model's choice at creation (direct for few lags,
    the transform for all), and the faster timed one after autotune; D stays
    within the bar either way."""
    say("case: auto method 128x128x1024")
    frames = synth.brownian_stack(128, 128, 1024, 500, 1.5, 40.0, 300.0, 0.3, seed=5, pixel="u16")
    few = gpu.Plan(128, 128, 1024, max_lag=16, method="auto")
    every = gpu.Plan(128, 128, 1024, method="auto")
    assert few.method == "direct" and every.method == "fourier"
    cols = [0, 1, 40]
    Do, rows = oracle_D(frames.numpy(), kx_subset=cols)
    for plan in (few, every):
        E, qpw, ms = plan.autotune()
        say("autotuned: M", plan.max_lag, "->", plan.method, "%.3f ms" % ms)
        D = plan.structure_function(frames.cuda())
        torch.cuda.synchronize()
        e = per_q_error(D.cpu().numpy()[rows], Do[:, :plan.max_lag])
        assert e.max() <= TOL_F32
    # with all 1024 lags the transform is an order of magnitude cheaper
    assert every.method == "fourier"


def test_direct_in_batch_and_noalloc(gpu):
    """A batch mixing the two methods, and the no-allocation entry point with
    the direct method, equal the single plans bit for bit."""
    say("case: direct in a batch and without allocation")
    shapes = [dict(width=64, height=64, n_frames=300, max_lag=20, method="direct"),
              dict(width=96, height=48, n_frames=200),
              dict(width=128, height=128, n_frames=9000, max_lag=8, method="direct")]
    fr = [synth.uniform_stack(s["width"], s["height"], s["n_frames"], seed=i).cuda() for i, s in enumerate(shapes)]
    batch = gpu.Batch(shapes, lanes=2)
    Db = batch.structure_function(fr)
    torch.cuda.synchronize()
    for i, s in enumerate(shapes):
        p = gpu.Plan(s["width"], s["height"], s["n_frames"], max_lag=s.get("max_lag", 0),
                     method=s.get("method", "fourier"))
        assert torch.equal(Db[i], p.structure_function(fr[i])), i
        if i == 0:
            assert torch.equal(Db[i], p.structure_function_noalloc(fr[i]))
    assert batch.status() == [L.DDM_OK] * 3


def test_direct_paper_shape_sampled(gpu):
    """The bench workload (512 x 512 u16 x 1024 frames) with 16 lags by direct
    differences, the launch shape the bench times: kx columns {0, 1, 255, 256}
    (the packed column pair and the Nyquist column included), every ky."""
    say("case: direct 512x512x1024 u16, 16 lags, kx columns {0, 1, 255, 256}")
    frames = synth.make(synth.PAPER, device="cuda")
    plan = gpu.Plan(512, 512, 1024, max_lag=16, method="direct")
    D = plan.structure_function(frames)
    torch.cuda.synchronize()
    Dg = D.cpu().numpy()
    Do, rows = oracle_D(frames.cpu().numpy(), max_lag=16, kx_subset=[0, 1, 255, 256])
    e = per_q_error(Dg[rows], Do)
    say("512x512x1024 direct (%d q):" % len(rows), describe(e))
    assert e.max() <= TOL_F32


def test_direct_lags_per_lane_same_bits(gpu, tmp_path):
    """8 and 16 lags per lane (DDM_DIRECT_LAGS, read once per process, so the
    other setting runs in a child process) sum each lag's pairs in the same
    time order: the same bits."""
    import os
    import subprocess
    say("case: direct, 8 vs 16 lags per lane, 128x128x300, 64 and 200 lags")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    frames = synth.brownian_stack(128, 128, 300, 400, 1.5, 40.0, 300.0, 0.3, seed=77)
    ref = {M: gpu.Plan(128, 128, 300, max_lag=M, method="direct").structure_function(frames.cuda()).cpu()
           for M in (64, 200)}
    src, dst = str(tmp_path / "f.pt"), str(tmp_path / "d.pt")
    torch.save(frames, src)
    child = ("import sys; sys.path.insert(0, %r)\n"
             "import torch\nfrom paper_2012_05695_amd import api\n"
             "f = torch.load(sys.argv[1], weights_only=True).cuda()\n"
             "torch.save({M: api.Plan(128, 128, 300, max_lag=M, method='direct').structure_function(f).cpu()"
             " for M in (64, 200)}, sys.argv[2])\n" % root)
    r = subprocess.run([sys.executable, "-c", child, src, dst], capture_output=True, text=True,
                       env=dict(os.environ, DDM_DIRECT_LAGS="8"), timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    got = torch.load(dst, weights_only=True)
    for M in (64, 200):
        assert torch.equal(got[M], ref[M]), M


def test_direct_time_ranges_match_oracle(gpu, tmp_path):
    """The split of the base points into 2 or 4 ranges of 64-point chunks
    (ranges past N - m left empty for the high lag tiles) against a single
    range (DDM_DIRECT_PARTS=1, read once per process, so in a child process)
    and against the oracle: 32 x 32 x 300 (4 ranges, every lag), 64 x 48 x 1000
    (4 ranges, 37 lags), 96 x 96 x 700 FP16 (4 ranges, 100 lags), 48 x 32 x 150
    (2 ranges: three chunks, every lag)."""
    import os
    import subprocess
    cases = [(32, 32, 300, 300, "f32"), (64, 48, 1000, 37, "f32"), (96, 96, 700, 100, "f16"),
             (48, 32, 150, 150, "f32")]
    say("case: direct time ranges vs one range", cases)
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    frames = [synth.brownian_stack(W, H, N, max(4, W * H // 30), 1.5, 40.0, 200.0, 0.3, seed=N + 7, pixel="u16")
              for (W, H, N, M, sp) in cases]
    src, dst = str(tmp_path / "f.pt"), str(tmp_path / "d.pt")
    torch.save(frames, src)
    child = ("import sys; sys.path.insert(0, %r)\n"
             "import torch\nfrom paper_2012_05695_amd import api\n"
             "fr = torch.load(sys.argv[1], weights_only=True)\n"
             "cases = %r\n"
             "torch.save([api.Plan(W, H, N, max_lag=M, method='direct', spectrum=sp).structure_function(f.cuda()).cpu()"
             " for (W, H, N, M, sp), f in zip(cases, fr)], sys.argv[2])\n" % (root, cases))
    r = subprocess.run([sys.executable, "-c", child, src, dst], capture_output=True, text=True,
                       env=dict(os.environ, DDM_DIRECT_PARTS="1"), timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    one = torch.load(dst, weights_only=True)
    for (W, H, N, M, sp), f, D1 in zip(cases, frames, one):
        D = gpu.Plan(W, H, N, max_lag=M, method="direct", spectrum=sp).structure_function(f.cuda()).cpu()
        Do, _ = oracle_D(f.numpy(), max_lag=M)
        tol = 5e-3 if sp == "f16" else TOL_F32
        e, e1 = per_q_error(D.numpy(), Do), per_q_error(D1.numpy(), Do)
        say("ranges", (W, H, N, M, sp), "default", describe(e), "one range", describe(e1))
        assert e.max() <= tol and e1.max() <= tol
        # the FP64 totals of FP32 chunk sums: the two orders agree to FP64 rounding
        assert per_q_error(D.numpy(), D1.numpy().astype(np.float64)).max() <= 1e-6
