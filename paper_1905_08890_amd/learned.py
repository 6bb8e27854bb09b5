"""Learned initial guess for the constraint solve.

The network (gr_unet_*) sees, at multigrid level `level` (the fields
restricted by averaging), the new matter sources and the previous step's ten
solved fields, and predicts each field's increment.  The prediction is
prolonged back to the finest level and added to the previous-step field;
solving with GR_GUESS_CHECKED then keeps, per field, whichever of the learned
and the previous-step guess has the smaller FP64 residual (the fallback).

Training data come from the solver itself: for each seed, a Zel'dovich
displacement pattern at amplitudes growing 25 % per step stands in for
consecutive time steps; each step is solved to 1e-10 from the previous one.
Every step after the first gives one (input, increment) pair.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

from . import grmg, synth

SOURCES = (grmg.S0, grmg.SX, grmg.SY, grmg.SZ)
SOLVED = tuple(range(10))
IN_FIELDS = SOURCES + SOLVED
OUT_FIELDS = SOLVED
CHANNELS = (16, 32, 64, 64)


def log(msg):
    print(f"[learned] {msg}", file=sys.stderr, flush=True)


def trajectory_amplitudes(r0: float, steps: int):
    return [r0 * (1.0 + 0.25 * s) for s in range(steps)]


class Normaliser:
    """Per-channel affine maps: inputs (x - mean)/std, outputs y * std."""

    def __init__(self, in_mean, in_std, out_std):
        self.in_mean = np.asarray(in_mean, dtype=np.float64)
        self.in_std = np.asarray(in_std, dtype=np.float64)
        self.out_std = np.asarray(out_std, dtype=np.float64)

    def as_dict(self):
        return dict(in_mean=self.in_mean.tolist(), in_std=self.in_std.tolist(), out_std=self.out_std.tolist())


def raw_features(grid, level, torch):
    """Unnormalised inputs and previous-field features at `level`: [14][m^3]."""
    m = grid.n >> level
    out = torch.empty((len(IN_FIELDS), m, m, m), dtype=torch.float32, device=grid.device)
    k = len(IN_FIELDS)
    grmg.features(grid.handle, level, IN_FIELDS, [0.0] * k, [1.0] * k, out)
    return out


def generate(n, seeds, steps, r0, level, torch, device="cuda", precision="mixed"):
    """Solve trajectories; returns lists of raw inputs [14][m^3] and increments [10][m^3] (device FP32)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    xs, ys = [], []
    for seed in seeds:
        t0 = time.time()
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            grid.deposit_sources(pos, u, mass)
            guess = "zero" if s == 0 else "current"
            if s > 0:
                x = raw_features(grid, level, torch)
            rep = grid.solve_constraints(rtol=1e-10, precision=precision, guess=guess)
            if s > 0:
                new = raw_features(grid, level, torch)[len(SOURCES):]
                xs.append(x)
                ys.append((new - x[len(SOURCES):]).contiguous())
        log(f"seed {seed}: {steps} steps in {time.time() - t0:.1f} s (last cycles {rep['cycles']})")
    grid.close()
    return xs, ys


def fit_normaliser(xs, ys):
    """Per-channel mean / std over all samples (FP64 sums on the device)."""
    def stats(ts):
        s1 = sum(t.double().flatten(1).sum(1) for t in ts)
        s2 = sum((t.double().flatten(1) ** 2).sum(1) for t in ts)
        cnt = len(ts) * ts[0][0].numel()
        mean = (s1 / cnt).cpu().numpy()
        var = np.maximum((s2 / cnt).cpu().numpy() - mean ** 2, 0.0)
        return mean, np.sqrt(var)

    in_mean, in_std = stats(xs)
    _, out_std = stats(ys)
    in_std[in_std == 0] = 1.0
    out_std[out_std == 0] = 1.0
    return Normaliser(in_mean, in_std, out_std)


def normalise(xs, ys, norm, torch):
    dev = xs[0].device
    im = torch.tensor(norm.in_mean, dtype=torch.float32, device=dev).view(-1, 1, 1, 1)
    isd = torch.tensor(norm.in_std, dtype=torch.float32, device=dev).view(-1, 1, 1, 1)
    osd = torch.tensor(norm.out_std, dtype=torch.float32, device=dev).view(-1, 1, 1, 1)
    return [((x - im) / isd).contiguous() for x in xs], [(y / osd).contiguous() for y in ys]


def train(xs, ys, m, epochs, lr, seed, torch, device="cuda", channels=CHANNELS):
    net = grmg.UNet(len(IN_FIELDS), len(OUT_FIELDS), channels, max_n=m, device=device)
    net.init(seed)
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        order = rng.permutation(len(xs))
        ep_loss = [net.train_step(xs[i], ys[i], lr * (0.5 ** (ep // max(1, epochs // 3)))) for i in order]
        losses.append(float(np.mean(ep_loss)))
        log(f"epoch {ep}: loss {losses[-1]:.4e}")
    return net, losses


def save(path, net, norm, level, meta):
    p = net.get_params().cpu().numpy()
    np.savez_compressed(path, params=p, in_mean=norm.in_mean, in_std=norm.in_std, out_std=norm.out_std,
                        level=np.int64(level), channels=np.asarray(net.channels, dtype=np.int64),
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


class LearnedGuess:
    """A trained network bound to grids of one size; `apply` sets the guesses."""

    def __init__(self, path, n, torch, device="cuda"):
        z = np.load(path, allow_pickle=False)
        self.level = int(z["level"])
        self.norm = Normaliser(z["in_mean"], z["in_std"], z["out_std"])
        self.m = n >> self.level
        self.torch = torch
        self.net = grmg.UNet(len(IN_FIELDS), len(OUT_FIELDS), tuple(int(c) for c in z["channels"]), max_n=self.m,
                             device=device)
        self.net.set_params(z["params"])
        self.buf = torch.empty((len(IN_FIELDS), self.m, self.m, self.m), dtype=torch.float32, device=device)
        self.meta = json.loads(bytes(z["meta"]).decode())

    def apply(self, grid):
        """Network guess for every solved field (previous-step values kept as the alternative)."""
        grmg.features(grid.handle, self.level, IN_FIELDS, self.norm.in_mean, 1.0 / self.norm.in_std, self.buf)
        pred = self.net.forward(self.buf)
        grmg.set_guess(grid.handle, self.level, OUT_FIELDS, self.norm.out_std, pred, 1)


def _timed_solve(grid, torch, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = grid.solve_constraints(**kw)
    torch.cuda.synchronize()
    rep["ms"] = (time.perf_counter() - t0) * 1e3
    return rep


def evaluate(guess, n, seeds, steps, r0, torch, device="cuda", rtol=1e-10, control=None):
    """Per step after the first, solve the same sources to `rtol` from
      zero_fp64     : zero guess, FP64 cycles
      prev_fp64     : previous-step fields, FP64
      prev_mixed    : previous-step fields, mixed precision
      learned_mixed : previous step + network increment (checked), mixed; the
                      network's own time is included
      control_mixed : as learned_mixed with `control` (e.g. an untrained net)
    and return per-variant lists of (ms, total cycles, guess fallbacks)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    res = {k: [] for k in ("zero_fp64", "prev_fp64", "prev_mixed", "learned_mixed", "control_mixed")}

    def load(vals):
        for f, v in enumerate(vals):
            grid.set_field(f, v)

    for seed in seeds:
        prev = None
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            grid.deposit_sources(pos, u, mass)
            if prev is None:
                grid.solve_constraints(rtol=rtol)
                prev = [grid.get_field(f).clone() for f in SOLVED]
                continue
            variants = [("zero_fp64", dict(precision="fp64", guess="zero"), None),
                        ("prev_fp64", dict(precision="fp64", guess="current"), None),
                        ("prev_mixed", dict(precision="mixed", guess="current"), None),
                        ("learned_mixed", dict(precision="mixed", guess="checked"), guess)]
            if control is not None:
                variants.append(("control_mixed", dict(precision="mixed", guess="checked"), control))
            for name, kw, net in variants:
                load(prev)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if net is not None:
                    net.apply(grid)
                rep = _timed_solve(grid, torch, rtol=rtol, **kw)
                ms = (time.perf_counter() - t0) * 1e3
                res[name].append(dict(ms=ms, solve_ms=rep["ms"], cycles=sum(rep["cycles"]),
                                      fallback=rep["guess_fallback"], status=rep["status"]))
            # the trajectory continues from this step's own solution
            prev = [grid.get_field(f).clone() for f in SOLVED]
    grid.close()
    return {k: v for k, v in res.items() if v}


def summarise(res):
    out = {}
    for k, rows in res.items():
        out[k] = dict(ms=float(np.median([r["ms"] for r in rows])),
                      cycles=float(np.mean([r["cycles"] for r in rows])),
                      fallback=float(np.mean([r["fallback"] for r in rows])),
                      all_ok=all(r["status"] == grmg.OK for r in rows), samples=len(rows))
    return out


def main(argv=None):
    import argparse

    import torch

    ap = argparse.ArgumentParser(description="train the learned-guess network on solver trajectories")
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--level", type=int, default=1)
    ap.add_argument("--seeds", type=int, default=16)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--r0", type=float, default=1.0)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", required=True)
    ap.add_argument("--eval-seeds", type=int, default=2)
    ap.add_argument("--eval-seed0", type=int, default=9000)
    a = ap.parse_args(argv)
    t0 = time.time()
    xs, ys = generate(a.n, range(a.seed0, a.seed0 + a.seeds), a.steps, a.r0, a.level, torch)
    norm = fit_normaliser(xs, ys)
    xs, ys = normalise(xs, ys, norm, torch)
    log(f"{len(xs)} samples in {time.time() - t0:.0f} s; training")
    net, losses = train(xs, ys, a.n >> a.level, a.epochs, a.lr, a.seed0, torch)
    meta = dict(n=a.n, level=a.level, seeds=[a.seed0, a.seed0 + a.seeds], steps=a.steps, r0=a.r0,
                epochs=a.epochs, lr=a.lr, samples=len(xs), losses=losses)
    save(a.out, net, norm, a.level, meta)
    log(f"saved {a.out} after {time.time() - t0:.0f} s")
    if a.eval_seeds > 0:
        g = LearnedGuess(a.out, a.n, torch)
        ctl = LearnedGuess(a.out, a.n, torch)
        ctl.net.init(a.seed0 + 777)  # same normaliser, untrained weights
        res = evaluate(g, a.n, range(a.eval_seed0, a.eval_seed0 + a.eval_seeds), a.steps, a.r0, torch, control=ctl)
        print(json.dumps(summarise(res)), flush=True)


if __name__ == "__main__":
    main()
