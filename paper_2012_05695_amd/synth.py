"""Seeded synthetic image stacks (inputs only; none of the method's arithmetic).

The paper measures on recorded 16-bit image sets that are not available here.
These generators stand in for them with the same shapes and value ranges:
Gaussian spots undergoing Brownian motion in a periodic box, over a uniform
background, with Poisson (shot) noise, quantised to uint8 or 12-bit uint16.

Recipe (one stack):
  * n_spots centres uniform in [0, W) x [0, H) at t = 0;
  * every frame each centre moves by a N(0, 2 D0) step per axis (so the mean
    squared displacement is 4 D0 per frame), wrapped periodically;
  * mean image bg + a * sum_i g(x - x_i) g(y - y_i) with
    g(d) = exp(-d^2 / (2 sigma^2)) on the minimum-image distance, cut to 0 for
    |d| > 5 sigma (a separable, square-truncated Gaussian spot);
  * frame = Poisson(mean image), clipped to [0, max_value].

Random numbers come from ``torch.Generator`` seeded with ``seed`` on the chosen
device; CPU generation is bit-reproducible.  Stacks made on a GPU are handed
unchanged to the GPU path and, copied to the host, to the oracle, so both
sides always see the same bytes.
"""

import math

import torch


def _profiles(pos, L, sigma, dtype):
    # pos: [c, n] positions along one axis -> [c, n, L] truncated Gaussian profiles
    x = torch.arange(L, dtype=dtype, device=pos.device)
    d = torch.remainder(x[None, None, :] - pos[:, :, None] + L / 2.0, float(L)) - L / 2.0
    g = torch.exp(-(d * d) / (2.0 * sigma * sigma))
    return torch.where(d.abs() <= 5.0 * sigma, g, torch.zeros_like(g))


def trajectories(n_frames, n_spots, W, H, D0, generator, device):
    """Spot centres [N, n_spots, 2] (x, y) in float64."""
    pos0 = torch.rand((n_spots, 2), generator=generator, dtype=torch.float64, device=device)
    pos0 = pos0 * torch.tensor([float(W), float(H)], dtype=torch.float64, device=device)
    steps = torch.randn((max(n_frames - 1, 0), n_spots, 2), generator=generator,
                        dtype=torch.float64, device=device) * math.sqrt(2.0 * D0)
    traj = torch.cat([pos0[None], pos0[None] + torch.cumsum(steps, dim=0)], dim=0)
    box = torch.tensor([float(W), float(H)], dtype=torch.float64, device=device)
    return torch.remainder(traj, box)


def brownian_stack(W, H, N, n_spots, sigma, amplitude, background, D0, seed=0,
                   pixel="u16", max_value=None, device="cpu", chunk=None):
    """Frames [N, H, W] as torch.uint8 or torch.uint16 on `device`."""
    device = torch.device(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    traj = trajectories(N, n_spots, W, H, D0, g, device)
    if max_value is None:
        max_value = 255 if pixel == "u8" else 4095
    out_dtype = torch.uint8 if pixel == "u8" else torch.uint16
    frames = torch.empty((N, H, W), dtype=out_dtype, device=device)
    work = torch.float64 if device.type == "cpu" else torch.float32
    if chunk is None:
        per_frame = 4 * n_spots * (W + H) + 8 * W * H
        chunk = max(1, min(N, (256 << 20) // max(per_frame, 1)))
    for t0 in range(0, N, chunk):
        t1 = min(N, t0 + chunk)
        gx = _profiles(traj[t0:t1, :, 0].to(work), W, sigma, work)   # [c, n, W]
        gy = _profiles(traj[t0:t1, :, 1].to(work), H, sigma, work)   # [c, n, H]
        mean = background + amplitude * torch.bmm(gy.transpose(1, 2).contiguous(), gx)
        sample = torch.poisson(mean, generator=g)
        frames[t0:t1] = sample.clamp_(0, max_value).to(torch.int32).to(out_dtype)
    return frames


def uniform_stack(W, H, N, seed=0, pixel="u16", max_value=None, device="cpu"):
    """Independent uniform integer pixels in [0, max_value] (white-noise frames)."""
    device = torch.device(device)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    if max_value is None:
        max_value = 255 if pixel == "u8" else 4095
    x = torch.randint(0, int(max_value) + 1, (N, H, W), generator=g, dtype=torch.int32, device=device)
    return x.to(torch.uint8 if pixel == "u8" else torch.uint16)


# Workload recipes with the shapes and parameters of the measured cases.
PLAIN = dict(W=64, H=64, N=128, n_spots=200, sigma=1.5, amplitude=40.0, background=100.0,
             D0=0.5, seed=0, pixel="u8")
PAPER = dict(W=512, H=512, N=1024, n_spots=2000, sigma=1.5, amplitude=40.0, background=800.0,
             D0=0.2, seed=0, pixel="u16")
LARGE = dict(W=2048, H=2048, N=4096, n_spots=30000, sigma=1.5, amplitude=40.0, background=800.0,
             D0=0.05, seed=0, pixel="u16")


def make(recipe, device="cpu", **over):
    r = dict(recipe)
    r.update(over)
    return brownian_stack(r["W"], r["H"], r["N"], r["n_spots"], r["sigma"], r["amplitude"],
                          r["background"], r["D0"], seed=r["seed"], pixel=r["pixel"], device=device)
