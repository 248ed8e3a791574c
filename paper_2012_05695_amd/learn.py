"""Training and use of the fit-initialisation network.

The network maps a normalised structure-function curve (64 samples at
log-spaced lags, divided by its maximum) to a start (A, B, log tau) for the
least-squares fit of D(q, m) = A (1 - exp(-m / tau)) + B.  It is trained on
curves that this library computes (ddm_structure_function, ddm_sample_curves)
from synthetic Brownian-spot stacks, with labels from the generator's own
parameters; every arithmetic step runs in the library's kernels, this module
only orchestrates.

Labels of a stack with n_spots Gaussian spots (width sigma, amplitude a),
background bg, P = W H pixels, diffusion D0 (px^2 / frame) and wave vector
q = 2 pi (kx / W, ky / H) rad/px:
    tau = 1 / (D0 |q|^2)                       (mean squared step 2 D0 per axis)
    A   = 2 n_spots a^2 (2 pi sigma^2)^2 exp(-|q|^2 sigma^2)
    B   = 2 (P bg + n_spots a 2 pi sigma^2)     (Poisson noise: 2 sum of the mean image)
The signal-to-noise ratio of a stack is A(q -> 0) / B; the amplitude a that
gives a requested ratio solves a quadratic.
"""

import math
import time

import numpy as np
import torch

from . import api, synth

SIGMA = 1.5
BACKGROUND = 800.0


def amplitude_for_snr(snr, n_spots, W, H, sigma=SIGMA, bg=BACKGROUND):
    s = 2.0 * math.pi * sigma * sigma
    P = W * H
    b = snr * n_spots * s
    return (b + math.sqrt(b * b + 4.0 * n_spots * s * s * snr * P * bg)) / (2.0 * n_spots * s * s)


def labels(kx, ky_s, W, H, D0, n_spots, a, sigma=SIGMA, bg=BACKGROUND):
    """Ground-truth (A, B, tau) per wave vector."""
    q2 = (2 * np.pi * np.asarray(kx) / W) ** 2 + (2 * np.pi * np.asarray(ky_s) / H) ** 2
    s = 2.0 * math.pi * sigma * sigma
    A = 2.0 * n_spots * a * a * s * s * np.exp(-q2 * sigma * sigma)
    B = np.full_like(q2, 2.0 * (W * H * bg + n_spots * a * s))
    with np.errstate(divide="ignore"):
        tau = np.where(q2 > 0, 1.0 / (D0 * q2), np.inf)
    return A, B, tau


def draw_stack_params(rng, W, H):
    """D0 log-uniform in [0.01, 10] px^2/frame, SNR log-uniform in [1, 100]."""
    D0 = math.exp(rng.uniform(math.log(0.01), math.log(10.0)))
    snr = math.exp(rng.uniform(math.log(1.0), math.log(100.0)))
    n_spots = max(1, int(round(2000 * W * H / (512 * 512))))
    return D0, snr, n_spots, amplitude_for_snr(snr, n_spots, W, H)


def stack_curves(W, H, N, D0, n_spots, a, seed, lags, device="cuda"):
    """Curves, scales and labels of every q != 0 of one synthetic stack."""
    frames = synth.brownian_stack(W, H, N, n_spots, SIGMA, a, BACKGROUND, D0, seed=seed, pixel="u16",
                                  device=device)
    plan = api.Plan(W, H, N, pixel="u16")
    D = plan.structure_function(frames)
    kx, ky = plan.q_index()
    keep = ~((kx == 0) & (ky == 0))
    idx = torch.from_numpy(np.flatnonzero(keep)).to(D.device)
    curves, scale = api.sample_curves(D.index_select(0, idx).contiguous(), lags)
    A, B, tau = labels(kx[keep], ky[keep], W, H, D0, n_spots, a)
    plan.close()
    del frames, D
    return curves, scale, (A, B, tau)


def make_training_set(n_curves, W=128, H=128, N=2048, seed0=1000, K=64, device="cuda", log=None):
    """(X [n, 64] curves, T [n, 3] targets (A/c, B/c, log tau)) from enough stacks."""
    lags = api.log_lags(N, K)
    xs, ts = [], []
    got, i = 0, 0
    while got < n_curves:
        rng = np.random.default_rng(seed0 + i)
        D0, snr, n_spots, a = draw_stack_params(rng, W, H)
        curves, scale, (A, B, tau) = stack_curves(W, H, N, D0, n_spots, a, seed0 + i, lags, device)
        c = scale.cpu().numpy().astype(np.float64)
        T = np.stack([A / c, B / c, np.log(tau)], axis=1).astype(np.float32)
        # only curves whose relaxation time is measurable from the sampled lags
        # carry their labels (tau << 1 frame is flat, tau >> N is a straight line)
        keep = np.flatnonzero((tau > 0.5 * lags[0]) & (tau < 2.0 * lags[-1]))
        kt = torch.from_numpy(keep).to(curves.device)
        xs.append(curves.index_select(0, kt))
        ts.append(torch.from_numpy(T[keep]).to(curves.device))
        got += len(keep)
        i += 1
        if log:
            log("stack %d: D0 %.3g SNR %.3g, %d curves" % (i, D0, snr, got))
    X = torch.cat(xs)[:n_curves].contiguous()
    T = torch.cat(ts)[:n_curves].contiguous()
    return X, T, lags


# offsets of the last layer in the flat parameter vector (see include/ddm.h)
_OW4 = 256 * 64 + 256 + 2 * (256 * 256 + 256)
_OB4 = _OW4 + 3 * 256


class Initialiser:
    """A trained network whose last layer also undoes the target
    standardisation (W4 <- diag(std) W4, b4 <- std b4 + mean), so that its
    outputs are the start (A/c, B/c, log tau) itself."""

    def __init__(self, net, mean, std):
        p = net.get_params().astype(np.float64)
        m = mean.detach().cpu().numpy().astype(np.float64)
        s = std.detach().cpu().numpy().astype(np.float64)
        p[_OW4:_OB4] = (p[_OW4:_OB4].reshape(3, 256) * s[:, None]).ravel()
        p[_OB4:_OB4 + 3] = p[_OB4:_OB4 + 3] * s + m
        # inference over a whole stack is one launch whatever max_batch is (it
        # sizes only the training buffers)
        self.net = api.Mlp(seed=0, max_batch=net.max_batch, device=net.device)
        self.net.set_params(p.astype(np.float32))

    def init(self, curves):
        """Start (A/c, B/c, log tau) for every curve [n, 64] (device)."""
        return self.net.forward(curves)


def train(X, T, epochs=40, batch=4096, lr=1e-3, seed=0, log=None):
    mean = T.mean(dim=0)
    std = T.std(dim=0).clamp_min(1e-6)
    Ts = ((T - mean) / std).contiguous()
    net = api.Mlp(seed=seed, max_batch=batch)
    n = X.shape[0]
    g = torch.Generator(device="cpu")
    g.manual_seed(seed)
    losses = []
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(X.device)
        Xp, Tp = X.index_select(0, perm).contiguous(), Ts.index_select(0, perm).contiguous()
        tot = torch.zeros((), device=X.device)
        nb = 0
        for b0 in range(0, n - batch + 1, batch):
            net.train_step(Xp[b0:b0 + batch], Tp[b0:b0 + batch], lr)
            tot += net.loss_dev[0]
            nb += 1
        losses.append(float(tot) / max(nb, 1))
        if log:
            log("epoch %d loss %.4f" % (ep, losses[-1]))
    return Initialiser(net, mean, std), losses


def compare(curves, lags, init, truth_tau=None, tau_window=None):
    """Fit every curve from the default start and from the learned one.

    Three ways to use the learned start: "learned" starts each curve from
    whichever of the network's start and the default start has the lower cost
    (one fit); "learned_refit" starts from the network's start and refits from
    the default start the curves that do not converge; "learned_gated" starts
    from the network's start where its tau lies within [m_1 / 4, 4 m_K] and its
    A is at least 5% of |A| + |B|, from the default start elsewhere (one fit).  Returns device times (the
    learned times include the network; "mlp_ms" is the network alone) and, per
    subset ("all", and with ground truth "measurable" = true tau inside
    tau_window), the mean iterations, converged fraction, median
    |log tau - log tau_true| and the fraction of curves whose final cost is not
    worse than from the default start."""
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(7)]
    ev[0].record()
    p0, i0, f0 = api.fit(curves, lags)
    ev[1].record()
    y = init.init(curves)
    ev[2].record()
    p1, i1, f1 = api.fit(curves, lags, init=y, fallback="best")
    ev[3].record()
    y = init.init(curves)
    p2, i2, f2 = api.fit(curves, lags, init=y, fallback=True)
    ev[4].record()
    y = init.init(curves)
    p3, i3, f3 = api.fit(curves, lags, init=y, fallback="gate")
    ev[5].record()
    torch.cuda.synchronize()
    lags64 = torch.from_numpy(lags.astype(np.float64)).to(curves.device)

    def cost(p):
        A, B, tau = p[:, 0:1].double(), p[:, 1:2].double(), p[:, 2:3].double()
        r = A * (1 - torch.exp(-lags64[None, :] / tau)) + B - curves.double()
        return (r * r).sum(dim=1)

    c0 = cost(p0)
    costs = {"learned": cost(p1), "learned_refit": cost(p2), "learned_gated": cost(p3)}
    subsets = {"all": torch.ones(curves.shape[0], dtype=torch.bool, device=curves.device)}
    t = None
    if truth_tau is not None:
        t = torch.from_numpy(np.asarray(truth_tau, dtype=np.float64)).to(curves.device)
        subsets["measurable"] = (t > tau_window[0]) & (t < tau_window[1])
    out = {"n": int(curves.shape[0]), "default_ms": ev[0].elapsed_time(ev[1]),
           "mlp_ms": ev[1].elapsed_time(ev[2]), "learned_ms": ev[1].elapsed_time(ev[3]),
           "learned_refit_ms": ev[3].elapsed_time(ev[4]), "learned_gated_ms": ev[4].elapsed_time(ev[5])}
    for name, sel in subsets.items():
        if not bool(sel.any()):
            continue
        rec = {"n": int(sel.sum())}
        for key, p, it, fl in (("default", p0, i0, f0), ("learned", p1, i1, f1), ("learned_refit", p2, i2, f2),
                               ("learned_gated", p3, i3, f3)):
            r = {"mean_iters": float(it[sel].float().mean()),
                 "converged": float(((fl[sel] & 1) != 0).float().mean())}
            if key in ("learned", "learned_gated"):
                r["default_start_chosen"] = float(((fl[sel] & 32) != 0).float().mean())
            if key == "learned_refit":
                r["refitted"] = float(((fl[sel] & 16) != 0).float().mean())
            if t is not None:
                e = torch.abs(torch.log(p[sel, 2].double()) - torch.log(t[sel]))
                r["median_abs_log_tau_err"] = float(e.median())
            if key != "default":
                c = costs[key]
                r["cost_not_worse"] = float((c[sel] <= c0[sel] * (1 + 1e-4) + 1e-12).float().mean())
            rec[key] = r
        out[name] = rec
    return out
