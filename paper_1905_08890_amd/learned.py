"""Learned initial guess for the constraint solve.

Along a trajectory of time steps the fields change smoothly, so the guess for
step s starts from the linear extrapolation 2 f_{s-1} - f_{s-2} of the two
previous solutions (the library keeps f_{s-2} as each field's history) and the
network predicts the correction to it.  The network (gr_unet_*) sees, at
multigrid level `level` (fields restricted by averaging): the change of the
matter sources s0, s_i over the step, the new s0, and each solved field's
previous increment f_{s-1} - f_{s-2}; it predicts, per field, the restricted
difference between the step's solution and the extrapolation.  The
prediction is interpolated to the finest level (4-point cubic per axis) and
added to the extrapolation (GR_SET_EXTRAP).  Solving with GR_GUESS_CHECKED
then keeps, per field, whichever of this guess and the previous-step field
has the smaller FP64 stopping quantity (the fallback).  With a zero
prediction the same path gives the plain extrapolation, the control that
separates what the network adds.

Training data come from the solver itself: for each seed, a Zel'dovich
displacement pattern at amplitudes growing 25 % per step stands in for
consecutive time steps; each step is solved to 1e-10 from the previous one.
Every step from the third on gives one (input, correction) pair.
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
HIST = tuple(grmg.HIST + f for f in SOLVED)
# input channels: [change of s0, s_x, s_y, s_z] + [new s0] + previous increment of each solved field
IN_CH = len(SOURCES) + 1 + len(SOLVED)
OUT_FIELDS = SOLVED
CHANNELS = (16, 32, 64, 64)
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "unet_extrap_level1_zeldovich256.npz")


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


class Features:
    """Network inputs at one level, built by the library's restriction kernels:
    `before_deposit` snapshots the old sources, `after_deposit` completes the
    inputs from the new sources, the held (previous-step) fields and their
    history (it may be called again for the same step)."""

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
        grmg.features(grid.handle, self.level, (grmg.S0,), [self.mean[k]], [self.inv[k]], self.buf[k:k + 1])
        # previous increments: (f - h - mean) * inv
        q = k + 1
        grmg.features(grid.handle, self.level, HIST, [0.0] * 10, list(-self.inv[q:]), self.buf[q:])
        grmg.features(grid.handle, self.level, SOLVED, list(self.mean[q:]), list(self.inv[q:]), self.buf[q:],
                      grmg.FEAT_ACCUMULATE)
        return self.buf


def extrapolate(grid, level, m, torch, device, pred=None, scale=None):
    """The step's guess: linear extrapolation from the history plus the
    (scaled) prediction at `level`, cubic interpolation; zero prediction: the
    plain extrapolation."""
    if pred is None:
        pred = torch.zeros((len(OUT_FIELDS), m, m, m), dtype=torch.float32, device=device)
        scale = [0.0] * len(OUT_FIELDS)
    grmg.set_guess(grid.handle, level, OUT_FIELDS, list(scale), pred, grmg.SET_EXTRAP | grmg.SET_CUBIC)


def generate(n, seeds, steps, r0, level, torch, device="cuda", precision="mixed"):
    """Solve trajectories; returns lists of raw inputs [IN_CH][m^3] and
    corrections [10][m^3] (restricted solution minus restricted extrapolation)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    m = n >> level
    feats = Features(level, m, torch, device)
    ext = torch.empty((len(SOLVED), m, m, m), dtype=torch.float32, device=device)
    new = torch.empty_like(ext)
    xs, ys = [], []
    for seed in seeds:
        t0 = time.time()
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            if s > 0:
                feats.before_deposit(grid)
            grid.deposit_sources(pos, u, mass)
            x = feats.after_deposit(grid).clone() if s > 1 else None
            if s > 0:
                extrapolate(grid, level, m, torch, device)   # s = 1: no history yet, the previous step
            if s > 1:
                grmg.features(grid.handle, level, SOLVED, [0.0] * 10, [1.0] * 10, ext)
            rep = grid.solve_constraints(rtol=1e-10, precision=precision, guess="zero" if s == 0 else "current")
            if s > 1:
                grmg.features(grid.handle, level, SOLVED, [0.0] * 10, [1.0] * 10, new)
                xs.append(x)
                ys.append((new - ext).contiguous())
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


def lr_at(step, total, lr, warmup):
    """Linear warm-up over `warmup` steps, then cosine decay to lr/20."""
    if step < warmup:
        return lr * (step + 1) / warmup
    t = (step - warmup) / max(1, total - warmup)
    return lr * (0.05 + 0.95 * 0.5 * (1.0 + np.cos(np.pi * t)))


def train(xs, ys, m, epochs, lr, seed, torch, device="cuda", channels=CHANNELS, lap_weight=0.0, clip=1.0,
          warmup=None):
    """Adam with gradient-norm clipping and learning-rate warm-up; returns the
    network and per-epoch mean losses."""
    net = grmg.UNet(IN_CH, len(OUT_FIELDS), channels, max_n=m, device=device, lap_weight=lap_weight,
                    clip_norm=clip)
    net.init(seed)
    rng = np.random.default_rng(seed)
    total = epochs * len(xs)
    warmup = warmup if warmup is not None else max(1, total // 20)
    losses, step = [], 0
    for ep in range(epochs):
        t0 = time.time()
        ep_loss = []
        for i in rng.permutation(len(xs)):
            ep_loss.append(net.train_step(xs[i], ys[i], float(lr_at(step, total, lr, warmup))))
            step += 1
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
        self.device = device
        self.net = grmg.UNet(IN_CH, len(OUT_FIELDS), tuple(int(c) for c in z["channels"]), max_n=self.m,
                             device=device)
        self.net.set_params(z["params"])
        self.features = Features(self.level, self.m, torch, device, self.norm)
        self.meta = json.loads(bytes(z["meta"]).decode())

    def before_deposit(self, grid):
        self.features.before_deposit(grid)

    def apply(self, grid):
        """Extrapolation + network correction for every solved field (the
        previous-step values kept as the alternative)."""
        pred = self.net.forward(self.features.after_deposit(grid))
        extrapolate(grid, self.level, self.m, self.torch, self.device, pred, self.norm.out_std)


class Extrapolation:
    """The same path with a zero prediction (no network)."""

    def __init__(self, level, m, torch, device):
        self.level, self.m, self.torch, self.device = level, m, torch, device

    def before_deposit(self, grid):
        pass

    def apply(self, grid):
        extrapolate(grid, self.level, self.m, self.torch, self.device)


class ExactCorrection:
    """Diagnostic stand-in for the network: the true correction (from a solve
    of the same step) restricted to the network's level, the best any
    prediction at that level can do."""

    def __init__(self, level, m, torch, device, pred):
        self.level, self.m, self.torch, self.device, self.pred = level, m, torch, device, pred

    def before_deposit(self, grid):
        pass

    def apply(self, grid):
        extrapolate(grid, self.level, self.m, self.torch, self.device, self.pred, [1.0] * len(OUT_FIELDS))


def _timed_solve(grid, torch, **kw):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = grid.solve_constraints(**kw)
    torch.cuda.synchronize()
    rep["ms"] = (time.perf_counter() - t0) * 1e3
    return rep


def evaluate(guess, n, seeds, steps, r0, torch, device="cuda", rtol=1e-10, control=None, exact=True):
    """Per step from the third on (two previous solutions exist), solve the
    same sources to `rtol` from
      zero_fp64     : zero guess, FP64 cycles
      prev_fp64     : previous-step fields, FP64
      prev_mixed    : previous-step fields, mixed precision
      extrap_mixed  : linear extrapolation of the two previous steps (no
                      network), checked against the previous step, mixed
      learned_mixed : extrapolation + network correction (checked), mixed;
                      the network's own time is included
      control_mixed : as learned_mixed with `control` (e.g. an untrained net)
      exact_mixed   : extrapolation + the true correction restricted to the
                      network's level (the best a prediction there can do)
    and return per-variant rows (ms, cycles, guess fallbacks, per-field
    stopping quantities of both guesses)."""
    grid = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=device)
    level = guess.level
    m = n >> level
    names = ("zero_fp64", "prev_fp64", "prev_mixed", "extrap_mixed", "learned_mixed", "control_mixed", "exact_mixed")
    res = {k: [] for k in names}
    fa = torch.empty((len(OUT_FIELDS), m, m, m), dtype=torch.float32, device=device)
    fb = torch.empty_like(fa)

    def load(vals, hist=None):
        for f, v in enumerate(vals):
            grid.set_field(f, v)
        if hist is not None:
            for f, v in enumerate(hist):
                grid.set_field(grmg.HIST + f, v)

    for seed in seeds:
        log(f"evaluating held-out seed {seed}")
        prev2 = prev = None
        for s, (pos, u, mass) in enumerate(synth.zeldovich_trajectory(n, seed, trajectory_amplitudes(r0, steps))):
            if prev2 is not None:
                load(prev, prev2)
                for gs in (guess, control):
                    if gs is not None:
                        gs.before_deposit(grid)
            grid.deposit_sources(pos, u, mass)
            if prev2 is None:   # the first two steps only build the history
                grid.solve_constraints(rtol=rtol, guess="zero" if prev is None else "current")
                prev2, prev = prev, [grid.get_field(f).clone() for f in SOLVED]
                continue
            variants = [("zero_fp64", dict(precision="fp64", guess="zero"), None),
                        ("prev_fp64", dict(precision="fp64", guess="current"), None),
                        ("prev_mixed", dict(precision="mixed", guess="current"), None),
                        ("extrap_mixed", dict(precision="mixed", guess="checked"), Extrapolation(level, m, torch,
                                                                                                  device)),
                        ("learned_mixed", dict(precision="mixed", guess="checked"), guess)]
            if control is not None:
                variants.append(("control_mixed", dict(precision="mixed", guess="checked"), control))
            if exact:
                variants.append(("exact_mixed", dict(precision="mixed", guess="checked"), "exact"))
            sol = None
            for name, kw, net in variants:
                load(prev, prev2)
                if net == "exact":
                    extrapolate(grid, level, m, torch, device)
                    grmg.features(grid.handle, level, OUT_FIELDS, [0.0] * 10, [1.0] * 10, fa)
                    load(sol)
                    grmg.features(grid.handle, level, OUT_FIELDS, [0.0] * 10, [1.0] * 10, fb)
                    load(prev, prev2)
                    net = ExactCorrection(level, m, torch, device, (fb - fa).contiguous())
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if net is not None:
                    net.apply(grid)
                rep = _timed_solve(grid, torch, rtol=rtol, **kw)
                ms = (time.perf_counter() - t0) * 1e3
                res[name].append(dict(ms=ms, solve_ms=rep["ms"], cycles=sum(rep["cycles"]),
                                      field_cycles=rep["cycles"], fallback=rep["guess_fallback"],
                                      status=rep["status"], guess_rel=rep["guess_rel"], alt_rel=rep["alt_rel"]))
                if name == "prev_fp64":
                    sol = [grid.get_field(f).clone() for f in SOLVED]
            # the trajectory continues from this step's own solution
            prev2, prev = prev, sol
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
    ap.add_argument("--seeds", type=int, default=64)
    ap.add_argument("--seed0", type=int, default=1000)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--r0", type=float, default=1.0)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--clip", type=float, default=1.0, help="gradient-norm clip of each Adam step")
    ap.add_argument("--lap-weight", type=float, default=0.3,
                    help="weight of mean (Lap error)^2 in the loss (the residual judge weights errors by Lap)")
    ap.add_argument("--out", default=WEIGHTS)
    ap.add_argument("--eval-seeds", type=int, default=2)
    ap.add_argument("--eval-seed0", type=int, default=2000)
    ap.add_argument("--eval-steps", type=int, default=4)
    ap.add_argument("--eval-json", default="")
    ap.add_argument("--eval-only", action="store_true", help="evaluate the weights at --out without training")
    a = ap.parse_args(argv)
    if a.eval_only:
        evaluate_saved(a, torch)
        return
    t0 = time.time()
    xs, ys = generate(a.n, range(a.seed0, a.seed0 + a.seeds), a.steps, a.r0, a.level, torch)
    norm = fit_normaliser(xs, ys)
    xs, ys = normalise(xs, ys, norm, torch)
    log(f"{len(xs)} samples in {time.time() - t0:.0f} s; training")
    net, losses = train(xs, ys, a.n >> a.level, a.epochs, a.lr, a.seed0, torch, lap_weight=a.lap_weight,
                        clip=a.clip)
    meta = dict(n=a.n, level=a.level, seeds=[a.seed0, a.seed0 + a.seeds], steps=a.steps, r0=a.r0,
                epochs=a.epochs, lr=a.lr, clip=a.clip, lap_weight=a.lap_weight, samples=len(xs), losses=losses,
                inputs="d s0, d sx, d sy, d sz, s0, previous increment of the 10 fields",
                target="restricted solution minus restricted linear extrapolation")
    del xs, ys
    save(a.out, net, norm, a.level, meta)
    log(f"saved {a.out} after {time.time() - t0:.0f} s")
    if a.eval_seeds > 0:
        evaluate_saved(a, torch)


def evaluate_saved(a, torch):
    """Held-out evaluation of the weights at `a.out` (see `evaluate`)."""
    g = LearnedGuess(a.out, a.n, torch)
    ctl = LearnedGuess(a.out, a.n, torch)
    ctl.net.init(a.seed0 + 777)  # same normaliser, untrained weights
    seeds = range(a.eval_seed0, a.eval_seed0 + a.eval_seeds)
    res = evaluate(g, a.n, seeds, a.eval_steps, a.r0, torch, control=ctl)
    summary = summarise(res)
    summary["eval"] = dict(seeds=[seeds[0], seeds[-1]], steps=a.eval_steps, weights=os.path.basename(a.out))
    print(json.dumps(summary), flush=True)
    if a.eval_json:
        with open(a.eval_json, "w") as fh:
            json.dump(dict(summary=summary, rows=res), fh, indent=1)


if __name__ == "__main__":
    main()
