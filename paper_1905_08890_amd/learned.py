"""Learned initial guess for the constraint solve.

The network (gr_unet_*) sees, at multigrid level `level` (the fields
restricted by averaging), the change of the matter sources s0, s_i over the
step, the new s0, and the previous step's ten solved fields, and predicts
each field's increment.  The prediction is interpolated back to the finest
level and added to the previous-step field; solving with GR_GUESS_CHECKED
then keeps, per field, whichever of the learned and the previous-step guess
has the smaller FP64 residual (the fallback).

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
# input channels: [change of s0, s_x, s_y, s_z] + [new s0] + previous solved fields
NOW_FIELDS = (grmg.S0,) + SOLVED
IN_CH = len(SOURCES) + len(NOW_FIELDS)
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


class Features:
    """Network inputs at one level, built by the library's restriction kernels:
    `before_deposit` snapshots the old sources, `after_deposit` completes the
    inputs from the new sources and the held (previous-step) fields (it may be
    called again for the same step)."""

    def __init__(self, level, m, torch, device, norm=None):
        self.level = level
        self.k = len(SOURCES)
        self.snap = torch.empty((self.k, m, m, m), dtype=torch.float32, device=device)
        self.buf = torch.empty((IN_CH, m, m, m), dtype=torch.float32, device=device)
        if norm is None:
            self.mean, self.inv = np.zeros(IN_CH), np.ones(IN_CH)
        else:
            self.mean, self.inv = norm.in_mean, 1.0 / norm.in_std

    def before_deposit(self, grid):
        k = self.k
        grmg.features(grid.handle, self.level, SOURCES, [0.0] * k, list(-self.inv[:k]), self.snap)

    def after_deposit(self, grid):
        k = self.k
        self.buf[:k].copy_(self.snap)
        # adds (new - mean) * inv to -old * inv: (new - old - mean) * inv
        grmg.features(grid.handle, self.level, SOURCES, list(self.mean[:k]), list(self.inv[:k]), self.buf,
                      grmg.FEAT_ACCUMULATE)
        grmg.features(grid.handle, self.level, NOW_FIELDS, list(self.mean[k:]), list(self.inv[k:]), self.buf[k:])
        return self.buf


def generate(n, seeds, steps, r0, level, torch, device="cuda", precision="mixed"):
    """Solve trajectories; returns lists of raw inputs [IN_CH][m^3] and increments [10][m^3] (device FP32)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    m = n >> level
    feats = Features(level, m, torch, device)
    new = torch.empty((len(SOLVED), m, m, m), dtype=torch.float32, device=device)
    xs, ys = [], []
    for seed in seeds:
        t0 = time.time()
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            if s > 0:
                feats.before_deposit(grid)
            grid.deposit_sources(pos, u, mass)
            if s > 0:
                x = feats.after_deposit(grid).clone()
            rep = grid.solve_constraints(rtol=1e-10, precision=precision, guess="zero" if s == 0 else "current")
            if s > 0:
                grmg.features(grid.handle, level, SOLVED, [0.0] * 10, [1.0] * 10, new)
                xs.append(x)
                ys.append((new - x[IN_CH - len(SOLVED):]).contiguous())
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


def train(xs, ys, m, epochs, lr, seed, torch, device="cuda", channels=CHANNELS, lap_weight=0.0):
    net = grmg.UNet(IN_CH, len(OUT_FIELDS), channels, max_n=m, device=device, lap_weight=lap_weight)
    net.init(seed)
    rng = np.random.default_rng(seed)
    losses = []
    for ep in range(epochs):
        t0 = time.time()
        order = rng.permutation(len(xs))
        ep_loss = [net.train_step(xs[i], ys[i], lr * (0.5 ** (ep // max(1, epochs // 3)))) for i in order]
        losses.append(float(np.mean(ep_loss)))
        log(f"epoch {ep}: loss {losses[-1]:.4e} ({time.time() - t0:.1f} s)")
    return net, losses


def save(path, net, norm, level, meta):
    p = net.get_params().cpu().numpy()
    np.savez_compressed(path, params=p, in_mean=norm.in_mean, in_std=norm.in_std, out_std=norm.out_std,
                        level=np.int64(level), channels=np.asarray(net.channels, dtype=np.int64),
                        meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


class LearnedGuess:
    """A trained network bound to grids of one size.  Per step:
    `before_deposit(grid)`, deposit the new sources, then `apply(grid)`."""

    def __init__(self, path, n, torch, device="cuda"):
        z = np.load(path, allow_pickle=False)
        self.level = int(z["level"])
        self.norm = Normaliser(z["in_mean"], z["in_std"], z["out_std"])
        self.m = n >> self.level
        self.torch = torch
        self.net = grmg.UNet(IN_CH, len(OUT_FIELDS), tuple(int(c) for c in z["channels"]), max_n=self.m,
                             device=device)
        self.net.set_params(z["params"])
        self.features = Features(self.level, self.m, torch, device, self.norm)
        self.meta = json.loads(bytes(z["meta"]).decode())

    def before_deposit(self, grid):
        self.features.before_deposit(grid)

    def apply(self, grid, cubic=True):
        """Network guess for every solved field (previous-step values kept as the alternative)."""
        pred = self.net.forward(self.features.after_deposit(grid))
        flags = grmg.SET_ADD | (grmg.SET_CUBIC if cubic else 0)
        grmg.set_guess(grid.handle, self.level, OUT_FIELDS, self.norm.out_std, pred, flags)


class ExactIncrement:
    """Diagnostic stand-in for the network: the true increment (from a solve
    of the same step) restricted to the network's level."""

    def __init__(self, level, pred):
        self.level, self.pred = level, pred

    def apply(self, grid, cubic=True):
        flags = grmg.SET_ADD | (grmg.SET_CUBIC if cubic else 0)
        grmg.set_guess(grid.handle, self.level, OUT_FIELDS, [1.0] * len(OUT_FIELDS), self.pred, flags)


def _timed_solve(grid, torch, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = grid.solve_constraints(**kw)
    torch.cuda.synchronize()
    rep["ms"] = (time.perf_counter() - t0) * 1e3
    return rep


def evaluate(guess, n, seeds, steps, r0, torch, device="cuda", rtol=1e-10, control=None, cubic=True,
             exact=True):
    """Per step after the first, solve the same sources to `rtol` from
      zero_fp64     : zero guess, FP64 cycles
      prev_fp64     : previous-step fields, FP64
      prev_mixed    : previous-step fields, mixed precision
      learned_mixed : previous step + network increment (checked), mixed; the
                      network's own time is included
      control_mixed : as learned_mixed with `control` (e.g. an untrained net)
      exact_mixed   : as learned_mixed with the true increment restricted to
                      the network's level (the best a level guess can do)
    and return per-variant rows (ms, cycles, guess fallbacks, per-field
    stopping quantities of both guesses)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    names = ("zero_fp64", "prev_fp64", "prev_mixed", "learned_mixed", "control_mixed", "exact_mixed")
    res = {k: [] for k in names}
    level = guess.level
    m = n >> level
    fa = torch.empty((len(OUT_FIELDS), m, m, m), dtype=torch.float32, device=device)
    fb = torch.empty_like(fa)

    def load(vals):
        for f, v in enumerate(vals):
            grid.set_field(f, v)

    for seed in seeds:
        prev = None
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            if prev is not None:
                for gs in (guess, control):
                    if gs is not None:
                        gs.before_deposit(grid)
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
            if exact:
                variants.append(("exact_mixed", dict(precision="mixed", guess="checked"), "exact"))
            sol = None
            for name, kw, net in variants:
                load(prev)
                if net == "exact":
                    grmg.features(grid.handle, level, OUT_FIELDS, [0.0] * 10, [1.0] * 10, fa)
                    load(sol)
                    grmg.features(grid.handle, level, OUT_FIELDS, [0.0] * 10, [1.0] * 10, fb)
                    load(prev)
                    net = ExactIncrement(level, (fb - fa).contiguous())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if net is not None:
                    net.apply(grid, cubic=cubic)
                rep = _timed_solve(grid, torch, rtol=rtol, **kw)
                ms = (time.perf_counter() - t0) * 1e3
                res[name].append(dict(ms=ms, solve_ms=rep["ms"], cycles=sum(rep["cycles"]),
                                      field_cycles=rep["cycles"], fallback=rep["guess_fallback"],
                                      status=rep["status"], guess_rel=rep["guess_rel"], alt_rel=rep["alt_rel"]))
                if name == "prev_fp64":
                    sol = [grid.get_field(f).clone() for f in SOLVED]
            # the trajectory continues from this step's own solution
            prev = sol
    grid.close()
    return {k: v for k, v in res.items() if v}


def summarise(res):
    out = {}
    for k, rows in res.items():
        d = dict(ms=float(np.median([r["ms"] for r in rows])),
                 cycles=float(np.mean([r["cycles"] for r in rows])),
                 fallback=float(np.mean([r["fallback"] for r in rows])),
                 all_ok=all(r["status"] == grmg.OK for r in rows), samples=len(rows))
        if any(r["alt_rel"][0] > 0 for r in rows):
            # per field: median of (held guess / previous step) stopping quantities
            d["rel_ratio"] = [float(np.median([r["guess_rel"][f] / max(r["alt_rel"][f], 1e-300) for r in rows]))
                              for f in range(10)]
            d["field_cycles"] = [float(np.mean([r["field_cycles"][f] for r in rows])) for f in range(10)]
        out[k] = d
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
    ap.add_argument("--lap-weight", type=float, default=1.0,
                    help="weight of mean (Lap error)^2 in the loss (the residual judge weights errors by Lap)")
    ap.add_argument("--out", required=True)
    ap.add_argument("--eval-seeds", type=int, default=2)
    ap.add_argument("--eval-seed0", type=int, default=2000)
    ap.add_argument("--eval-json", default="")
    ap.add_argument("--trilinear", action="store_true", help="spread the guess with the multigrid prolongation")
    a = ap.parse_args(argv)
    t0 = time.time()
    xs, ys = generate(a.n, range(a.seed0, a.seed0 + a.seeds), a.steps, a.r0, a.level, torch)
    norm = fit_normaliser(xs, ys)
    xs, ys = normalise(xs, ys, norm, torch)
    log(f"{len(xs)} samples in {time.time() - t0:.0f} s; training")
    net, losses = train(xs, ys, a.n >> a.level, a.epochs, a.lr, a.seed0, torch, lap_weight=a.lap_weight)
    meta = dict(n=a.n, level=a.level, seeds=[a.seed0, a.seed0 + a.seeds], steps=a.steps, r0=a.r0,
                epochs=a.epochs, lr=a.lr, lap_weight=a.lap_weight, samples=len(xs), losses=losses)
    save(a.out, net, norm, a.level, meta)
    log(f"saved {a.out} after {time.time() - t0:.0f} s")
    if a.eval_seeds > 0:
        g = LearnedGuess(a.out, a.n, torch)
        ctl = LearnedGuess(a.out, a.n, torch)
        ctl.net.init(a.seed0 + 777)  # same normaliser, untrained weights
        res = evaluate(g, a.n, range(a.eval_seed0, a.eval_seed0 + a.eval_seeds), a.steps, a.r0, torch, control=ctl,
                       cubic=not a.trilinear)
        print(json.dumps(summarise(res)), flush=True)
        if a.eval_json:
            with open(a.eval_json, "w") as fh:
                json.dump(dict(summary=summarise(res), rows=res), fh, indent=1)


if __name__ == "__main__":
    main()
