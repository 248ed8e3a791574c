"""Every output element is written: D (and the bins) start as NaN sentinels and
must come back finite, for every path that writes D: one group, several
groups, a low-q cut (padding slots in the spectra store), minimal padding,
the FP16 store, host-resident frames, the no-allocation entry point and a
batch.  Rows of D are also checked against a second run to catch stale
values."""

import pytest
import torch

from paper_2012_05695_amd import synth

pytestmark = pytest.mark.gpu


def sentinel(plan):
    return torch.full((plan.n_q, plan.max_lag), float("nan"), device="cuda")


@pytest.mark.parametrize("W,H,N,kw,ws", [(96, 64, 90, {}, "full"), (96, 64, 90, {}, "min"),
                                         (128, 128, 77, {"k2_max": 700, "max_lag": 50}, "full"),
                                         (64, 48, 300, {"padding": "minimal"}, "third"),
                                         (64, 64, 200, {"spectrum": "f16"}, "min"),
                                         (256, 256, 40, {}, "full")])
def test_every_element_of_D_is_written(gpu, W, H, N, kw, ws):
    print("case: coverage", W, H, N, kw, ws, flush=True)
    frames = synth.brownian_stack(W, H, N, max(4, W * H // 60), 1.5, 40.0, 300.0, 0.3, seed=W + N).cuda()
    plan = gpu.Plan(W, H, N, **kw)
    mn, full = plan.workspace_size()
    plan.allocate_workspace({"full": full, "min": mn, "third": mn + (full - mn) // 3}[ws])
    D = plan.structure_function(frames, out=sentinel(plan))
    torch.cuda.synchronize()
    assert torch.isfinite(D).all()
    D2 = plan.structure_function(frames, out=sentinel(plan))
    torch.cuda.synchronize()
    assert torch.equal(D, D2)
    if kw.get("spectrum") != "f16":
        staging = torch.empty(1 << 22, dtype=torch.uint8, device="cuda")
        Dh = plan.structure_function_host(frames.cpu().pin_memory(), staging, out=sentinel(plan))
        Dn = plan.structure_function_noalloc(frames, out=sentinel(plan))
        torch.cuda.synchronize()
        assert torch.equal(Dh, D) and torch.equal(Dn, D)
    T = gpu.integer_bin_thresholds(30)
    Dbar, counts, boq = plan.radial_average(D, T)
    torch.cuda.synchronize()
    assert torch.isfinite(Dbar).all() and (boq >= -1).all()


def test_batch_writes_every_element(gpu):
    print("case: coverage, batch", flush=True)
    shapes = [(64, 64, 50), (96, 48, 33), (128, 128, 20)]
    fr = [synth.uniform_stack(w, h, n, seed=i).cuda() for i, (w, h, n) in enumerate(shapes)]
    batch = gpu.Batch(shapes, lanes=2)
    outs = [torch.full((batch.n_q[i], batch.max_lag[i]), float("nan"), device="cuda") for i in range(3)]
    batch.set_bins(1, gpu.integer_bin_thresholds(20))
    D, Dbar, cnt = batch.structure_function_binned(fr, outs)
    torch.cuda.synchronize()
    assert all(torch.isfinite(d).all() for d in D)
    assert torch.isfinite(Dbar[1]).all() and Dbar[0] is None
