"""One-time fit of a velocity network by conditional flow matching (paper section "Conditional
Flow Matching", eq. 9; training data as in "Network Architecture and Inputs": pure-scattering
Monte Carlo exits over a range of optical dimensions and entry states).  Four models: the
boundary model (condition: ln tau, c, entry height, sin of the entry angle), the boundary model
of rectangular cells (the same plus ln A, A = width over entry-face length, ln A ~ U[ln 1/4,
ln 4]), the boundary model in XY geometry (entry direction a projection of a direction on the
sphere: its in-plane components omega_y, omega_x; exit directions inside the unit disk) and the
internal model for particles born inside a cell (condition: ln tau, c, birth point, birth
direction).  A fifth, the collided boundary model (blob flag bit 1), is the boundary model fitted
only on walks with at least one collision (and likewise the rectangular-cell and XY ones): the
transport places the uncollided crossings exactly (first-flight split) and leaves the rest to it.

Data come from this library's own analog walk (`mc_transmit` / `mc_transmit_internal`,
continuous-absorption mode: the exit law of a walk whose flights are drawn from
sigma_s = c tau), on the GPU.  Targets are the
5-dim exit encoding the sampler decodes:
  a0 = 2 pos - 1, (a1, a2) = exit direction, a3 = ln(path / L), a4 = face - 1.5 + u,
  u ~ U(-1/2, 1/2) (dequantisation: the face is recovered exactly by the decoder's thresholds
  -1, 0, 1).
Loss (eq. 9, sigma_min = 0): E || v(x_t, t | c) - (x1 - x0) ||^2, x_t = (1 - t) x0 + t x1,
x0 ~ N(0, I), t ~ U[0, 1].  The fit itself is offline PyTorch (autograd), not the hot path.

Usage: python -m paper_2512_13965_amd.train --hidden 512 --out paper_2512_13965_amd/weights/gmc_h512.bin
       python -m paper_2512_13965_amd.train --hidden 128 --steps 150000 --data 8000000 \
           --tau-max 1000 --out paper_2512_13965_amd/weights/gmc_h128.bin
       (width 128 likewise, --steps 150000 --data 8000000: --model collided ->
        gmc_h128_collided.bin; --model internal --tau-max 1000 -> gmc_h128_internal.bin)
       python -m paper_2512_13965_amd.train --model internal --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_internal.bin
       python -m paper_2512_13965_amd.train --model rect --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_rect.bin
       python -m paper_2512_13965_amd.train --model xy --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_xy.bin
       python -m paper_2512_13965_amd.train --model collided --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_collided.bin
       python -m paper_2512_13965_amd.train --model rect_collided --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_rect_collided.bin
       python -m paper_2512_13965_amd.train --model xy_collided --hidden 512 \
           --out paper_2512_13965_amd/weights/gmc_h512_xy_collided.bin
       python -m paper_2512_13965_amd.train --net film --hidden 512 --steps 150000 --data 8000000 \
           --batch 16384 --out paper_2512_13965_amd/weights/gmc_film_h512.bin
The residual network with adaptive modulation (--net film; section "Network Architecture and
Inputs") is fitted with the same loss and data.
"""
from __future__ import annotations

import argparse
import math
import time

import numpy as np
import torch

from . import binding, inputs

LOG_TAU_TRAIN = (math.log(0.05), math.log(300.0))
LOG_ASPECT_TRAIN = (math.log(0.25), math.log(4.0))


def make_dataset(n: int, seed: int, device="cuda", kind: str = "boundary", log_tau_range=LOG_TAU_TRAIN):
    """(conditions [n, 4] (boundary), [n, 5] (rect, xy) or [n, 6] (internal), targets [n, 5]) on
    `device`, from the GPU analog walk.  For the collided models (kinds "collided",
    "rect_collided", "xy_collided") twice the walks are run and the first n with a collision
    kept."""
    if kind == "internal":
        cond = inputs.internal_conditions(n, seed, log_tau_range=log_tau_range)
        dc = binding.DeviceCondInternal.from_host(cond, device)
        ex = binding.mc_transmit_internal(dc, binding.MODE_CONTINUOUS, seed=seed + 7919)
        feats = torch.stack([dc.log_tau, dc.c, 2.0 * dc.x - 1.0, 2.0 * dc.y - 1.0,
                             dc.cos_phi, dc.sin_phi], dim=1)
    else:
        collided = kind.endswith("collided")
        nw = 2 * n if collided else n
        if kind in ("xy", "xy_collided"):
            cond = inputs.xy_conditions(nw, seed, log_tau_range=log_tau_range)
        else:
            la = LOG_ASPECT_TRAIN if kind in ("rect", "rect_collided") else None
            cond = inputs.transmission_conditions(nw, seed, log_tau_range=log_tau_range, log_aspect_range=la)
        dc = binding.DeviceCond.from_host(cond, device)
        nc = torch.empty(nw, dtype=torch.int32, device=device) if collided else None
        ex = binding.mc_transmit(dc, binding.MODE_CONTINUOUS, seed=seed + 7919, ncoll=nc)
        cols = [dc.log_tau, dc.c, 2.0 * dc.y_in - 1.0, dc.sin_th]
        if kind in ("rect", "rect_collided"):
            cols.append(dc.log_aspect)
        if kind in ("xy", "xy_collided"):
            cols.append(dc.omega_x)
        feats = torch.stack(cols, dim=1)
        if collided:
            keep = torch.nonzero(nc > 0).squeeze(1)[:n]
            ex = binding.DeviceExit(*(t[keep] for t in (ex.face, ex.pos, ex.dir_cos, ex.dir_sin, ex.path)))
            feats = feats[keep]
    torch.cuda.synchronize()
    g = torch.Generator(device=device).manual_seed(seed + 1)
    u = torch.rand(n, device=device, generator=g) - 0.5
    tgt = torch.stack([2.0 * ex.pos - 1.0, ex.dir_cos, ex.dir_sin,
                       torch.log(torch.clamp(ex.path, min=1e-6)),
                       ex.face.float() - 1.5 + u], dim=1)
    return feats, tgt


class VelocityMLP(torch.nn.Module):
    """Same network as the sampler kernels: n_in -> H (SiLU) x4 -> 5, input [x, t, condition]
    (n_in = 10 boundary, 12 internal)."""

    def __init__(self, hidden: int, n_in: int = inputs.N_IN):
        super().__init__()
        dims = inputs.layer_dims(hidden, n_in)
        self.layers = torch.nn.ModuleList([torch.nn.Linear(i, o) for (o, i) in dims])

    def forward(self, x, t, c):
        h = torch.cat([x, t[:, None], c], dim=1)
        for i, lin in enumerate(self.layers):
            h = lin(h)
            if i < len(self.layers) - 1:
                h = torch.nn.functional.silu(h)
        return h

    def to_weights(self, seed: int, act_scale, flags: int = 0) -> inputs.Weights:
        W = [l.weight.detach().float().cpu().numpy().astype(np.float32) for l in self.layers]
        b = [l.bias.detach().float().cpu().numpy().astype(np.float32) for l in self.layers]
        w_scale = np.array([inputs.pow2_ceil_scale(float(np.abs(x).max())) for x in W], np.float32)
        return inputs.Weights(W[0].shape[0], W, b, np.asarray(act_scale, np.float32), w_scale, seed,
                              n_in=W[0].shape[1], flags=flags)


class VelocityFiLM(torch.nn.Module):
    """The residual network with adaptive modulation of the sampler kernel for such models
    (blob flag bit 2): u = [x, phi(t), c], phi = sin and cos of pi 2^j t (j = 0..3);
    h = W_in u + b_in; e = SiLU(W_e [phi, c] + b_e); per block
    h <- h + SiLU((1 + G e + g) * (A h + a) + (S e + s)); v = W_o h + b_o.  The scale and shift
    maps start at zero, so training starts from unmodulated residual blocks."""

    def __init__(self, hidden: int, n_in: int = inputs.N_IN, emb: int = inputs.FILM_EMB,
                 blocks: int = inputs.FILM_BLOCKS):
        super().__init__()
        dims = inputs.film_layer_dims(hidden, emb, n_in, blocks)
        self.layers = torch.nn.ModuleList([torch.nn.Linear(i, o) for (o, i) in dims])
        self.blocks = blocks
        with torch.no_grad():
            for j in range(blocks):
                for l in (3 + 3 * j, 4 + 3 * j):
                    self.layers[l].weight.zero_()
                    self.layers[l].bias.zero_()

    def forward(self, x, t, c):
        silu = torch.nn.functional.silu
        ang = math.pi * t[:, None] * torch.tensor([1.0, 2.0, 4.0, 8.0], device=t.device)
        phi = torch.stack([torch.sin(ang), torch.cos(ang)], dim=2).reshape(-1, 8)
        L = self.layers
        h = L[0](torch.cat([x, phi, c], dim=1))
        e = silu(L[1](torch.cat([phi, c], dim=1)))
        for j in range(self.blocks):
            h = h + silu((1.0 + L[3 + 3 * j](e)) * L[2 + 3 * j](h) + L[4 + 3 * j](e))
        return L[-1](h)

    def to_weights(self, seed: int, flags: int = 0) -> inputs.FilmWeights:
        W = [l.weight.detach().float().cpu().numpy().astype(np.float32) for l in self.layers]
        b = [l.bias.detach().float().cpu().numpy().astype(np.float32) for l in self.layers]
        n_in = W[0].shape[1] - 7          # input layer over [x (5), time features (8), condition]
        return inputs.FilmWeights(W[0].shape[0], W[1].shape[0], W, b, seed, n_in, flags | inputs.FILM_FLAG)


@torch.no_grad()
def activation_scales(model: VelocityMLP, feats, tgt, n=65536, seed=0):
    """Static per-layer FP8 activation scales: the power of two bringing the largest input of
    each layer (over a calibration batch at every t) under 448."""
    g = torch.Generator(device=feats.device).manual_seed(seed)
    idx = torch.randint(0, feats.shape[0], (n,), device=feats.device, generator=g)
    c, x1 = feats[idx], tgt[idx]
    amax = np.zeros(len(model.layers))
    for t0 in np.linspace(0.0, 1.0, 17):
        t = torch.full((n,), float(t0), device=feats.device)
        x0 = torch.randn(n, 5, device=feats.device, generator=g)
        h = torch.cat([(1 - t[:, None]) * x0 + t[:, None] * x1, t[:, None], c], dim=1)
        for i, lin in enumerate(model.layers):
            amax[i] = max(amax[i], float(h.abs().max()))
            h = lin(h)
            if i < len(model.layers) - 1:
                h = torch.nn.functional.silu(h)
    return [inputs.pow2_ceil_scale(a) for a in amax]


def train(hidden=512, n_data=4_000_000, steps=40_000, batch=8192, lr=1e-3, seed=20251213,
          log_every=1000, device="cuda", kind="boundary", log_tau_range=LOG_TAU_TRAIN, net="mlp"):
    torch.manual_seed(seed)
    t0 = time.time()
    feats, tgt = make_dataset(n_data, seed, device, kind, log_tau_range)
    n_data = feats.shape[0]
    print(f"data: {n_data} {kind} exits in {time.time() - t0:.1f}s", flush=True)
    n_in = 5 + 1 + feats.shape[1]
    model = (VelocityFiLM(hidden, n_in) if net == "film" else VelocityMLP(hidden, n_in)).to(device)
    opt = torch.optim.AdamW(model.parameters(), lr=lr, weight_decay=1e-4)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps, pct_start=0.05)
    g = torch.Generator(device=device).manual_seed(seed + 2)
    run = 0.0
    for it in range(1, steps + 1):
        idx = torch.randint(0, n_data, (batch,), device=device, generator=g)
        c, x1 = feats[idx], tgt[idx]
        x0 = torch.randn(batch, 5, device=device, generator=g)
        t = torch.rand(batch, device=device, generator=g)
        xt = (1 - t[:, None]) * x0 + t[:, None] * x1
        loss = torch.mean((model(xt, t, c) - (x1 - x0)) ** 2)
        opt.zero_grad(set_to_none=True)
        loss.backward()
        opt.step()
        sched.step()
        run += float(loss) if it % 50 == 0 else 0.0
        if it % log_every == 0:
            print(f"step {it}/{steps} loss {run / (log_every / 50):.4f} ({time.time() - t0:.0f}s)", flush=True)
            run = 0.0
    flags = {"xy": 1, "collided": 2, "rect_collided": 2, "xy_collided": 3}.get(kind, 0)
    if net == "film":
        return model.to_weights(seed & 0xFFFFFFFF, flags=flags)
    scales = activation_scales(model, feats, tgt)
    return model.to_weights(seed & 0xFFFFFFFF, scales, flags=flags)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--hidden", type=int, default=512)
    ap.add_argument("--steps", type=int, default=40_000)
    ap.add_argument("--data", type=int, default=4_000_000)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--model", choices=("boundary", "rect", "xy", "internal", "collided", "rect_collided",
                                                "xy_collided"), default="boundary")
    ap.add_argument("--tau-max", type=float, default=math.exp(LOG_TAU_TRAIN[1]),
                    help="largest optical thickness of the training cells (ln tau uniform)")
    ap.add_argument("--net", choices=("mlp", "film"), default="mlp",
                    help="plain MLP, or the residual network with adaptive modulation")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    w = train(a.hidden, a.data, a.steps, a.batch, a.lr, kind=a.model,
              log_tau_range=(LOG_TAU_TRAIN[0], math.log(a.tau_max)), net=a.net)
    inputs.save_blob(w, a.out)
    if a.net == "film":
        print("saved", a.out, "residual network", w.hidden, "x", w.blocks, "blocks", flush=True)
    else:
        print("saved", a.out, "act scales", list(w.act_scale), "w scales", list(w.w_scale), flush=True)


if __name__ == "__main__":
    main()
