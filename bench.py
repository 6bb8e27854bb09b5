#!/usr/bin/env python3
"""Benchmark of the constraint solve on one MI355X.

One step = CIC deposit of 256^3 Zel'dovich particles (seed 2, rms displacement
1 cell) + the ten field equations solved to rms(eps)/rms(f) <= 1e-10 from
zero guesses, through the C ABI of libgrmg.so.  Inputs are resident in HBM
before the timed region.  Prints one JSON line.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 256]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
# algorithmic bytes per grid point of one red-black sweep (both colours):
# phi read + write, source read, coefficient read (none for Poisson)
SWEEP_BYTES = {"hamiltonian": 32.0, "poisson": 24.0}
SWEEP_BYTES_KIND = {0: 24.0, 1: 32.0, 2: 32.0, 3: 12.0, 4: 20.0, 5: 16.0}
KIND_NAMES = {0: "poisson_fp64", 1: "hamiltonian_fp64", 2: "cmc_fp64", 3: "poisson_fp32", 4: "hamiltonian_fp32",
              5: "cmc_fp32"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_sweeps(torch, grmg, g, kind, nsweeps, reps):
    """Average duration of one red-black sweep of the finest level (HIP events
    on the grid's stream)."""
    st = g.stream
    grmg.debug_sweep(g.handle, kind, grmg.PSI, 0.0, 0.0, 2)  # warm
    best = None
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        grmg.debug_sweep(g.handle, kind, grmg.PSI, 0.0, 0.0, nsweeps)
        e1.record(st)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / nsweeps)
    times.sort()
    best = times[len(times) // 2]
    return best * 1e-3  # seconds per sweep


def copy_probe(torch, grmg, g, n, reps=7):
    """A plain device copy of n^3 doubles through the library (gr_set_field:
    reads and writes 8 n^3 bytes), timed with HIP events on the grid's
    stream: the practical HBM rate beside the 8 TB/s peak."""
    src = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda:0")
    torch.cuda.synchronize()
    fid = grmg.FIELD_IDS["rhs"]
    grmg.set_field(g.handle, fid, src, grmg.F64)
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(g.stream)
        for _ in range(4):
            grmg.set_field(g.handle, fid, src, grmg.F64)
        e1.record(g.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 4)
    times.sort()
    return 16.0 * n ** 3 / (times[len(times) // 2] * 1e-3) / 1e9


def pmc_traffic(n):
    """HBM bytes per launch of the FP64 Hamiltonian sweep at 256^3 from the
    committed counter summary, scaled by its copy-kernel calibration; None if
    the smoother sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "rb_fused_hamiltonian_fp64_256_pmc.md")
    if n != 256 or not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            v = v.strip()
            vals[k.strip()] = v[1:v.index("`", 1)] if v.startswith("`") else v
    if vals.get("kernel sources sha256") != kernel_sources_sha():
        return None
    return int(vals["traffic bytes per launch"])


SWEEP_SOURCES = ("stencil.hip", "fused_sweep.h", "stencil_ops.h", "gr_internal.h")


def kernel_sources_sha():
    """sha256 over the sources that define the fused sweep and its launch
    configuration, in a fixed order."""
    import hashlib

    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1905_08890_amd", "csrc", name), "rb").read())
    return h.hexdigest()


def cpu_baseline(n, pos, u, mass, cycles):
    """Oracle timed on the host on a bounded sample: two V(2,2) cycles of each
    equation kind at n^3 plus the CIC deposit (10-15 s of CPU work at 256^3),
    scaled by the GPU run's per-field cycle counts to the whole job."""
    import numpy as np

    import oracle as O
    from paper_1905_08890_amd import synth

    prm = O.params(1.0, synth.OMEGA_M, synth.C_TILDE)
    t0 = time.perf_counter()
    s0, sx, sy, sz, sm = O.cic_deposit(n, pos, u, mass, prm=prm)
    t_cic = time.perf_counter() - t0
    per_kind = {}
    f_p = 3 * prm.omega_m * prm.a * (sx - sx.mean())
    f_h = 1.5 * prm.a * prm.omega_m * (s0 - 1.0)
    z = np.zeros_like(s0)
    m2, f_c = O.build_cmc(z, s0, sm, z, prm=prm)
    for kind, f, coef in ((O.POISSON, f_p, None), (O.HAMILTONIAN, f_h, z), (O.CMC, f_c, m2)):
        t0 = time.perf_counter()
        O.solve_equation(kind, z, f, coef, prm=prm, rtol=0, max_cycles=2)
        per_kind[kind] = (time.perf_counter() - t0) / 2.0
    sample_s = t_cic + 2.0 * sum(per_kind.values())
    kinds = [O.POISSON] * 4 + [O.HAMILTONIAN, O.CMC] + [O.POISSON] * 4
    est = t_cic + sum(c * per_kind[k] for c, k in zip(cycles, kinds))
    return est, sample_s


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_sample_worker(args):
    """One process: the bounded oracle sample (as cpu_baseline) on its own
    copy of the inputs; returns its wall time."""
    n, pos, u, mass = args
    import oracle as O
    from paper_1905_08890_amd import synth
    import numpy as np

    prm = O.params(1.0, synth.OMEGA_M, synth.C_TILDE)
    t0 = time.perf_counter()
    s0, sx, sy, sz, sm = O.cic_deposit(n, pos, u, mass, prm=prm)
    z = np.zeros_like(s0)
    m2, f_c = O.build_cmc(z, s0, sm, z, prm=prm)
    for kind, f, coef in ((O.POISSON, 3 * prm.omega_m * (sx - sx.mean()), None),
                          (O.HAMILTONIAN, 1.5 * prm.omega_m * (s0 - 1.0), z), (O.CMC, f_c, m2)):
        O.solve_equation(kind, z, f, coef, prm=prm, rtol=0, max_cycles=2)
    return time.perf_counter() - t0


def cpu_all_cores(n, pos, u, mass, sample_1core):
    """The same bounded sample run as independent copies in P processes at
    once (P = the host threads available to this process, at most 16): the
    oracle is serial, so all cores serve independent work; the ratio of P
    samples to the wall time is the throughput gain over one core."""
    import multiprocessing as mp

    import numpy as np

    P = max(1, min(16, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("fork")
    t0 = time.perf_counter()
    with ctx.Pool(P) as pool:
        per = pool.map(_oracle_sample_worker, [(n, pos, u, mass)] * P)
    wall = time.perf_counter() - t0
    return P, wall, P * sample_1core / wall, float(np.median(per))


def smoother_only(torch, grmg, n):
    """Finest-level sweeps on seeded smooth data plus one plain copy of n^3
    doubles (gr_set_field: reads 8 n^3 and writes 8 n^3 bytes), whose counter
    readings calibrate the hardware byte counters."""
    from paper_1905_08890_amd import synth

    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0")
    gen = torch.Generator(device="cuda:0").manual_seed(0)
    g.set_field("Psi", 1e-3 * torch.randn((n,) * 3, device="cuda:0", dtype=torch.float64, generator=gen))
    g.set_field("rhs", torch.randn((n,) * 3, device="cuda:0", dtype=torch.float64, generator=gen))
    g.set_field("coef", torch.rand((n,) * 3, device="cuda:0", dtype=torch.float64, generator=gen))
    src = torch.zeros((n,) * 3, device="cuda:0", dtype=torch.float64)
    torch.cuda.synchronize()
    g.set_field("s0", src)                      # the calibration copy
    torch.cuda.synchronize()
    t_ham = time_sweeps(torch, grmg, g, grmg.HAMILTONIAN, 4, 3)
    t_poi = time_sweeps(torch, grmg, g, grmg.POISSON, 4, 3)
    N = n ** 3
    print(json.dumps({"n": n, "copy_bytes": 16 * N,
                      "hamiltonian_us_per_sweep": round(t_ham * 1e6, 2),
                      "hamiltonian_GBps": round(SWEEP_BYTES["hamiltonian"] * N / t_ham / 1e9, 1),
                      "poisson_us_per_sweep": round(t_poi * 1e6, 2),
                      "poisson_GBps": round(SWEEP_BYTES["poisson"] * N / t_poi / 1e9, 1)}), flush=True)


C12_FIELDS = ("Vx", "Vy", "Vz", "U", "Psi", "xi", "Phi", "Bx", "By", "Bz", "b", "beta_x", "beta_y", "beta_z")


def c3_errors(torch, grmg, g, d_pos, d_u, mass):
    """Per-field error of the mixed-precision solve refined to rms(eps)/rms(f)
    <= 1e-12 against the FP64 path run to its floor (rtol 1e-14, at most 30
    cycles per field): max|x - x_ref| / max|x_ref| per deviation field."""
    g.deposit_sources(d_pos, d_u, mass)
    r64 = g.solve_constraints(allow=(grmg.OK, grmg.ENOTCONV), rtol=1e-14, max_cycles=30)
    ref = {name: g.get_field(name) for name in C12_FIELDS}
    g.deposit_sources(d_pos, d_u, mass)
    rm = g.solve_constraints(rtol=1e-12, precision="mixed")
    errs = {}
    for name in C12_FIELDS:
        x = g.get_field(name)
        errs[name] = float(((x - ref[name]).abs().max() / ref[name].abs().max()).item())
    del ref
    return {"workload": "same particles; mixed refined to 1e-12 vs FP64 at its floor (rtol 1e-14, <= 30 cycles)",
            "max_rel_err": {k: float(f"{v:.3e}") for k, v in errs.items()},
            "worst": float(f"{max(errs.values()):.3e}"), "bar": 1e-9,
            "fp64_floor_rel_res_max": float(f"{max(r64['rel_res']):.3e}"), "mixed_status": rm["status"],
            "mixed_fallback_fields": rm["fallback"]}


def unet_only(torch, grmg, m, reps):
    """The shipped network (15 -> 10 channels, 16/32/64/64) on an m^3 grid:
    `reps` forward passes and `reps` loss-gradient passes on seeded inputs, each
    kind timed with HIP events; FLOP counts of the 3^3 convolutions (2 x 27 x
    cin x cout per voxel, backward 2x forward) give the MFMA rate."""
    net = grmg.UNet(15, 10, (16, 32, 64, 64), max_n=m, device="cuda:0")
    net.init(7)
    gen = torch.Generator(device="cuda:0").manual_seed(3)
    x = torch.randn((15, m, m, m), device="cuda:0", dtype=torch.float32, generator=gen)
    t = torch.randn((10, m, m, m), device="cuda:0", dtype=torch.float32, generator=gen)
    c = (16, 32, 64, 64)
    convs = [(15, c[0]), (c[0], c[0])]
    for l in range(1, 4):
        convs += [(c[l - 1], c[l]), (c[l], c[l])]
    for l in (2, 1, 0):
        convs += [(c[l + 1] + c[l], c[l]), (c[l], c[l])]
    levels = [0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0]
    fwd_flop = sum(2.0 * 27 * ci * co * (m >> lv) ** 3 for (ci, co), lv in zip(convs, levels))
    net.forward(x)
    net.loss_grad(x, t)
    torch.cuda.synchronize()
    out = {}
    for name, fn, flop in (("forward", lambda: net.forward(x), fwd_flop),
                           ("loss_grad", lambda: net.loss_grad(x, t), 3.0 * fwd_flop)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(reps):
            fn()
        e1.record(net.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        out[name] = {"ms": round(ms, 3), "conv_TFLOPs": round(flop / (ms * 1e-3) / 1e12, 1)}
    print(json.dumps({"unet_only": m, "in_ch": 15, "out_ch": 10, "channels": c, "conv_GFLOP_forward": round(fwd_flop / 1e9, 1),
                      **out}), flush=True)


def vector_modes(torch, grmg, g, n, reps=5):
    """Vector-mode extraction (curl, divergence, FFTs, shell spectra up to a
    quarter of Nyquist) of the solved shift beta^i and of the momentum density
    s_i on the bench grid; the FFT's per-pass rate from one 3-D transform of a
    complex n^3 array (each pass reads and writes 16 B per point)."""
    S = grmg.Spectra(n, n // 8, stream=g.stream)
    res = {"workload": f"beta^i and s_i of the {n}^3 step, {n // 8} shells (a quarter of Nyquist), FP64"}
    for name, ids in (("beta", (grmg.BETAX, grmg.BETAY, grmg.BETAZ)), ("s", (grmg.SX, grmg.SY, grmg.SZ))):
        f = [g.get_field(i) for i in ids]
        spec = S.vector(*f)
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            spec = S.vector(*f)
            ts.append(time.perf_counter() - t0)
        res[f"{name}_ms"] = round(sorted(ts)[len(ts) // 2] * 1e3, 3)
        res[f"{name}_shell0"] = {"k": round(float(spec[0, 0]), 4), "modes": int(spec[1, 0]),
                                 "p_vector": float(f"{spec[4, 0]:.4e}"), "p_scalar": float(f"{spec[5, 0]:.4e}")}
        del f
    buf = torch.zeros((n, n, n), dtype=torch.complex128, device=g.device)
    S.fft(buf)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lib = grmg.load_library()
    e0.record(g.stream)
    for _ in range(reps):
        assert lib.gr_spectra_fft(S.handle, buf.data_ptr()) == grmg.OK
    e1.record(g.stream)
    e1.synchronize()
    t_pass = e0.elapsed_time(e1) * 1e-3 / (3 * reps)
    res["fft_pass_us"] = round(t_pass * 1e6, 1)
    res["fft_pass_GBps"] = round(32.0 * n ** 3 / t_pass / 1e9, 1)
    del buf
    S.close()
    return res


def c1_workload(torch, grmg, synth):
    """The 32^3 Hamiltonian-only solve (s0 = 1 + k^-2 GRF, sigma 0.1, seed 0;
    V(2,2) from Psi = 0 to 1e-10): launch-latency bound on the GPU."""
    n = 32
    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0")
    src = synth.hamiltonian_only_sources(n, 0, 0.1)
    for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
        g.set_field(name, x)
    times = []
    for _ in range(6):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = g.solve_constraints(field_mask=1 << grmg.PSI, rtol=1e-10)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    cyc = rep["cycles"][grmg.PSI]
    g.close()
    return {"workload": "32^3 Hamiltonian only, s0 = 1 + GRF(k^-2, sigma 0.1, seed 0), FP64, rtol 1e-10",
            "ms": round(sorted(times[1:])[len(times[1:]) // 2] * 1e3, 3), "cycles": cyc,
            "factor_per_cycle": round(rep["rel_res"][grmg.PSI] ** (1.0 / max(cyc, 1)), 4)}, src


def c2_workload(torch, grmg, synth):
    """The 128^3 all-field FP64 solve: 128^3 Zel'dovich particles (seed 1, rms
    displacement 0.3 cells), CIC, the ten fields from zero guesses to 1e-10."""
    n = 128
    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0")
    pos, u, mass = synth.zeldovich(n, 1, 0.3)
    pos_d = torch.as_tensor(pos, device="cuda:0")
    u_d = torch.as_tensor(u, device="cuda:0")
    grmg.autotune(g.handle)
    times = []
    for _ in range(4):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.deposit_sources(pos_d, u_d, mass)
        rep = g.solve_constraints(rtol=1e-10)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    g.close()
    dt = sorted(times[1:])[len(times[1:]) // 2]
    return {"workload": "128^3 Zel'dovich particles seed 1 rms 0.3 cells, CIC + 10 fields FP64 from zero guess, "
                        "rtol 1e-10", "ms": round(dt * 1e3, 3), "cycles": rep["cycles"],
            "points_cycles_per_s": round(n ** 3 * sum(rep["cycles"]) / dt, 1)}


def c1_oracle_seconds(src, cycles):
    import numpy as np

    import oracle as O
    from paper_1905_08890_amd import synth

    f = 1.5 * synth.OMEGA_M * (src[0] - 1.0)
    t0 = time.perf_counter()
    O.solve_equation(O.HAMILTONIAN, np.zeros_like(f), f, np.zeros_like(f),
                     prm=O.params(1.0, synth.OMEGA_M, synth.C_TILDE), rtol=0, max_cycles=cycles)
    return time.perf_counter() - t0


def bench_learned(torch, grmg, synth, n):
    """Held-out trajectory (seed 2000, amplitudes 1.0, 1.25, 1.5, 1.75 cells):
    the first two steps build the history; for the next two, time to 1e-10
    from (i) zero guess FP64, (ii) previous step FP64, (iii) previous step
    mixed, (iv) linear extrapolation of the two previous steps, mixed (no
    network), (v) extrapolation + network correction, mixed (network time
    included), each guess judged per field against the previous step by the
    FP64 stopping quantity; the same with untrained weights (control); and
    (vi) extrapolation + the true correction restricted to the network's level
    (the ceiling of any prediction there).  rel_ratio: per field, the held
    guess's stopping quantity over the previous step's (below 1: kept)."""
    from paper_1905_08890_amd import learned

    path = learned.WEIGHTS
    gs = learned.LearnedGuess(path, n, torch)
    ctl = learned.LearnedGuess(path, n, torch)
    ctl.net.init(4242)
    res = learned.evaluate(gs, n, [2000], 4, 1.0, torch, control=ctl, exact=True)
    summ = learned.summarise(res)
    out = {"workload": f"{n}^3 Zel'dovich trajectory, held-out seed 2000, steps 3 and 4 (after two steps of "
                       f"history); network on level 1 ({n // 2}^3), weights {os.path.basename(path)} "
                       f"({gs.meta.get('samples')} training pairs from seeds {gs.meta.get('seeds')})"}
    for k, v in summ.items():
        out[k] = {"ms": round(v["ms"], 3), "cycles": v["cycles"], "fallback_fields": v["fallback"]}
        if "rel_ratio" in v:
            out[k]["rel_ratio"] = [float(f"{x:.3g}") for x in v["rel_ratio"]]
            out[k]["field_cycles"] = v["field_cycles"]
    z, l = summ["zero_fp64"]["ms"], summ["learned_mixed"]["ms"]
    out["speedup_learned_mixed_vs_zero_fp64"] = round(z / l, 3)
    out["speedup_learned_mixed_vs_prev_fp64"] = round(summ["prev_fp64"]["ms"] / l, 3)
    out["speedup_learned_mixed_vs_prev_mixed"] = round(summ["prev_mixed"]["ms"] / l, 3)
    out["speedup_learned_mixed_vs_extrap_mixed"] = round(summ["extrap_mixed"]["ms"] / l, 3)
    out["speedup_prev_mixed_vs_zero_fp64"] = round(z / summ["prev_mixed"]["ms"], 3)
    out["speedup_exact_mixed_vs_zero_fp64"] = round(z / summ["exact_mixed"]["ms"], 3)
    out["cycles_saved_by_network_vs_extrapolation"] = round(summ["extrap_mixed"]["cycles"] - summ["learned_mixed"]["cycles"], 2)
    out["cycles_saved_vs_previous_step"] = round(summ["prev_mixed"]["cycles"] - summ["learned_mixed"]["cycles"], 2)
    return out


def bench_batch(torch, grmg, synth, steps):
    """96 periodic boxes with sides drawn from {32,48,64,96,128} (seeds
    100..195), s0 = 1 + delta with sigma log-uniform in [0.05, 1], longitudinal
    momentum, and 32 Dirichlet refinement patches (seeds 196..227: sides
    24..80 in steps of 8 at half their parent's spacing, own sources, boundary
    values from the parent); all ten fields of every item to rtol 1e-10 in one
    batched solve."""
    import numpy as np

    log("batch: generating 96 boxes + 32 patches")
    items = [synth.batch_item(100 + b) for b in range(96)]
    sides = [n for n, _ in items]
    pitems = [synth.patch_item(j, sides) for j in range(32)]
    B = grmg.Batch(sides, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0",
                   patches=[d for d, _ in pitems])
    for i, src in enumerate([src for _, src in items] + [src for _, src in pitems]):
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            B.set_field(i, name, x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tune = B.autotune()
    tune_s = time.perf_counter() - t0
    log(f"batch autotune ({tune_s:.2f} s):\n{tune}")
    rep = B.solve(rtol=1e-10)  # warm-up (also captures the per-cycle graphs)
    times = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rep = B.solve(rtol=1e-10)
        times.append(time.perf_counter() - t0)
    dt = min(times)
    rep_m = B.solve(rtol=1e-10, precision="mixed")  # warm-up of the mixed-precision graphs
    mtimes = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rep_m = B.solve(rtol=1e-10, precision="mixed")
        mtimes.append(time.perf_counter() - t0)
    dtm = min(mtimes)
    # a sub-step of the refined levels: the 32 patches alone, from the boxes'
    # kept fields (as between two coarse time steps)
    rep_p = B.solve(rtol=1e-10, patches_only=True)
    ptimes = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rep_p = B.solve(rtol=1e-10, patches_only=True)
        ptimes.append(time.perf_counter() - t0)
    B.close()
    # the same solve with the device task queue (levels of at most 32^3 points and
    # each box's coarse cycle in one persistent launch per cycle)
    os.environ["GRMG_BATCH_QUEUE"] = "1"
    try:
        Q = grmg.Batch(sides, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0",
                       patches=[d for d, _ in pitems])
    finally:
        del os.environ["GRMG_BATCH_QUEUE"]
    for i, src in enumerate([src for _, src in items] + [src for _, src in pitems]):
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            Q.set_field(i, name, x)
    Q.autotune()
    rep_q = Q.solve(rtol=1e-10)
    qtimes = []
    for _ in range(steps):
        t0 = time.perf_counter()
        rep_q = Q.solve(rtol=1e-10)
        qtimes.append(time.perf_counter() - t0)
    Q.close()
    pts = np.array([n ** 3 for n in sides] + [d[0] ** 3 for d, _ in pitems], dtype=np.float64)
    cyc = np.array(rep["cycles"], dtype=np.float64)
    secs = np.array(rep["item_seconds"]) * 1e3
    npb = len(sides)
    out = {"workload": "96 periodic boxes (sides {32,48,64,96,128}, seeds 100-195) + 32 Dirichlet patches (sides "
                       "24-80, seeds 196-227, half the parent's spacing), all ten fields to rtol 1e-10, FP64, autotuned "
                       "smoothing forms, one grouped launch per phase, hipGraph per cycle",
           "status": rep["status"], "points": int(pts.sum()), "patch_points": int(pts[npb:].sum()),
           "seconds": round(dt, 4),
           "points_cycles_per_s": round(float((pts[:, None] * cyc).sum() / dt), 1),
           "item_ms_p50": round(float(np.percentile(secs, 50)), 3),
           "item_ms_p99": round(float(np.percentile(secs, 99)), 3),
           "patch_item_ms_p50": round(float(np.percentile(secs[npb:], 50)), 3),
           "cycles_min_max": [int(cyc.sum(1).min()), int(cyc.sum(1).max())],
           "patch_cycles_min_max": [int(cyc[npb:].sum(1).min()), int(cyc[npb:].sum(1).max())],
           "autotune": {"seconds": round(tune_s, 3), "choices": tune.strip().splitlines()},
           "mixed": {"status": rep_m["status"], "seconds": round(dtm, 4),
                     "note": "boxes by FP64/FP32 iterative refinement, patches in FP64"},
           "patch_substep": {"status": rep_p["status"], "seconds": round(min(ptimes), 4),
                             "note": "the 32 patches solved again from the boxes' kept fields (gr_batch_solve_patches)"},
           "queue": {"status": rep_q["status"], "seconds": round(min(qtimes), 4),
                     "same_cycles": rep_q["cycles"] == rep["cycles"],
                     "note": "FP64 with the device task queue for every box's levels of at most 32^3 points and "
                             "its coarse cycle (one persistent launch per cycle), grouped launches above"}}
    log(f"batch: {out}")
    return out


def substep_only(torch, grmg, synth, steps):
    """The batched workload's 32 patches solved again from the kept fields of
    their boxes (gr_batch_solve_patches), after one full solve; ends with a
    plain copy of 256^3 doubles (the counters' calibration)."""
    items = [synth.batch_item(100 + b) for b in range(96)]
    sides = [n for n, _ in items]
    pitems = [synth.patch_item(j, sides) for j in range(32)]
    B = grmg.Batch(sides, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0",
                   patches=[d for d, _ in pitems])
    for i, src in enumerate([src for _, src in items] + [src for _, src in pitems]):
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            B.set_field(i, name, x)
    B.autotune()
    B.solve(rtol=1e-10)
    times = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rep = B.solve(rtol=1e-10, patches_only=True)
        times.append(time.perf_counter() - t0)
    B.close()
    g = grmg.Grid(256, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0")
    copy_probe(torch, grmg, g, 256, reps=1)
    g.close()
    print(json.dumps({"substep_s": round(min(times), 4), "status": rep["status"]}), flush=True)


def spectra_only(torch, grmg, synth, n):
    """The vector-mode extraction of the bench workload's solved shift and
    momentum density (one mixed solve first), then a plain copy of n^3
    doubles (the counters' calibration)."""
    pos, u, mass = synth.zeldovich(n, 2, 1.0)
    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device="cuda:0")
    g.deposit_sources(pos, u, mass)
    g.solve_constraints(rtol=1e-10, precision="mixed")
    res = vector_modes(torch, grmg, g, n, reps=2)
    copy_probe(torch, grmg, g, n, reps=1)
    g.close()
    print(json.dumps({"vector_modes": res}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-all-cores", action="store_true", help="skip the all-cores oracle timing")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched workload (96 boxes + 32 patches)")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-guess trajectory")
    ap.add_argument("--batch-only", action="store_true", help="only the batched workload (96 boxes + 32 patches)")
    ap.add_argument("--step-only", choices=("fp64", "mixed", "both"),
                    help="only the 256^3 step(s) of that precision: autotune, warm-up, --steps timed steps "
                         "(for kernel traces and counters)")
    ap.add_argument("--unet-only", action="store_true",
                    help="only the learned-guess network at its shipped shape (level 1 of 256^3: 128^3, 15 -> 10 "
                         "channels): --steps forward passes and loss-gradient passes (for MFMA counters)")
    ap.add_argument("--smoother-only", action="store_true",
                    help="only the finest-level sweeps and a copy of known size (for hardware counters)")
    ap.add_argument("--substep-only", action="store_true",
                    help="only the refined levels: the 32 patches of the batched workload solved again from their "
                         "boxes' kept fields, --steps times, then a copy of known size (for traces and counters)")
    ap.add_argument("--spectra-only", action="store_true",
                    help="only the vector-mode extraction of the solved 256^3 step's shift and momentum density, "
                         "then a copy of known size (for traces and counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_08890_amd import grmg, synth

    n = args.n
    if args.unet_only:
        unet_only(torch, grmg, n // 2, max(1, args.steps))
        return
    if args.smoother_only:
        smoother_only(torch, grmg, n)
        return
    if args.batch_only:
        print(json.dumps(bench_batch(torch, grmg, synth, max(1, args.steps))), flush=True)
        return
    if args.substep_only:
        substep_only(torch, grmg, synth, max(1, args.steps))
        return
    if args.spectra_only:
        spectra_only(torch, grmg, synth, n)
        return
    seed, rms = (2, 1.0) if n == 256 else (1, 0.3)
    log(f"generating Zel'dovich particles n={n} seed={seed} rms={rms}")
    pos, u, mass = synth.zeldovich(n, seed, rms)
    dev = torch.device("cuda:0")
    g = grmg.Grid(n, a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE, device=dev)
    d_pos = torch.as_tensor(pos, device=dev)
    d_u = torch.as_tensor(u, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tune_report = grmg.autotune(g.handle)
    tune_s = time.perf_counter() - t0
    log(f"autotune ({tune_s:.2f} s):\n{tune_report}")

    def step(precision):
        grmg.deposit_sources(g.handle, d_pos, d_u, mass)
        return grmg.solve_constraints(g.handle, grmg.default_opts(rtol=1e-10, precision=precision)).as_dict()

    def timed(precision):
        for _ in range(args.warmup):
            rep = step(precision)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            rep = step(precision)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / args.steps, rep

    if args.step_only:
        for prec in (("fp64", "mixed") if args.step_only == "both" else (args.step_only,)):
            dt_, rep_ = timed(prec)
            log(f"{prec}: cycles {rep_['cycles']}, fallback {rep_['fallback']}, {dt_ * 1e3:.3f} ms/step")
            print(json.dumps({"step_only": prec, "n": n, "ms_per_step": round(dt_ * 1e3, 3),
                              "cycles": rep_["cycles"], "status": rep_["status"]}), flush=True)
        # one plain copy of n^3 doubles (reads and writes 8 n^3 bytes): the
        # calibration of the hardware byte counters in the same run
        src = torch.zeros((n,) * 3, device=dev, dtype=torch.float64)
        torch.cuda.synchronize()
        g.set_field("rhs", src)
        torch.cuda.synchronize()
        g.close()
        return

    log(f"plain FP64: warmup {args.warmup}, timing {args.steps} steps")
    dt64, rep64 = timed("fp64")
    log(f"  cycles per field {rep64['cycles']}, {dt64 * 1e3:.2f} ms/step")
    log(f"mixed FP32/FP64: warmup {args.warmup}, timing {args.steps} steps")
    dt, rep = timed("mixed")
    log(f"  refinement steps per field {rep['cycles']}, fallback {rep['fallback']}, {dt * 1e3:.2f} ms/step")
    cycles = rep64["cycles"]
    log("c3: per-field error of mixed (1e-12) against FP64 at its floor")
    c3 = c3_errors(torch, grmg, g, d_pos, d_u, mass)
    log(f"  {c3['max_rel_err']}")

    # the dominant kernel inside the solves: every finest-level fused sweep of one
    # FP64 and one mixed step, bracketed by HIP events on the solve's stream
    grmg.sweep_timing(g.handle, True)
    step("fp64")
    step("mixed")
    in_solve = grmg.sweep_timing(g.handle, False)
    log(f"in-solve sweep launches (kind: count, mean ms): {in_solve}")

    # dominant kernel: the finest-level red-black smoother
    g.set_field("rhs", g.get_field("s0"))
    g.set_field("coef", g.get_field("AA"))
    N = n ** 3
    t_ham = time_sweeps(torch, grmg, g, grmg.HAMILTONIAN, 20, 5)
    t_poi = time_sweeps(torch, grmg, g, grmg.POISSON, 20, 5)
    gbps_ham = SWEEP_BYTES["hamiltonian"] * N / t_ham / 1e9
    gbps_poi = SWEEP_BYTES["poisson"] * N / t_poi / 1e9
    log(f"smoother sweep: hamiltonian {t_ham * 1e6:.1f} us ({gbps_ham:.0f} GB/s), "
        f"poisson {t_poi * 1e6:.1f} us ({gbps_poi:.0f} GB/s)")

    copy_gbps = copy_probe(torch, grmg, g, n)
    log(f"copy probe: {copy_gbps:.0f} GB/s")

    ham_in_solve = SWEEP_BYTES["hamiltonian"] * N / (in_solve[1][1] * 1e-3) / 1e9
    out = {
        "metric": "time-to-residual 1e-10 and smoother GB/s at 256^3; learned+mixed vs plain FP64",
        "value": round(dt * 1e3, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"zeldovich{n}: {n}^3 particles seed {seed} rms {rms} cells, CIC + 10 fields "
                               f"to rtol 1e-10 from zero guess, V(2,2); value = mixed precision (FP32 inner "
                               f"cycles, FP64 residual/update)",
                   "n": n, "rtol": 1e-10, "precision": "mixed", "guess": "zero"},
        "fp64_ms_per_step": round(dt64 * 1e3, 3),
        "speedup_mixed_vs_fp64": round(dt64 / dt, 3),
        "cycles_fp64": rep64["cycles"],
        "refinement_steps_mixed": rep["cycles"],
        "mixed_fallback_fields": rep["fallback"],
        "c3_mixed_vs_fp64_floor": c3,
        "points_cycles_per_s_fp64": round(N * sum(rep64["cycles"]) / dt64, 1),
        "autotune": {"seconds": round(tune_s, 3), "choices": tune_report.strip().splitlines()},
        "smoother_back_to_back": {"hamiltonian_us_per_sweep": round(t_ham * 1e6, 2), "hamiltonian_GBps": round(gbps_ham, 1),
                     "poisson_us_per_sweep": round(t_poi * 1e6, 2), "poisson_GBps": round(gbps_poi, 1)},
        "roofline": {"bound": "hbm", "achieved": round(ham_in_solve, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(ham_in_solve / HBM_PEAK_GBPS, 4), "traffic": None,
                     "copy_probe_GBps": round(copy_gbps, 1),
                     "kernel": f"fused red-black Newton sweep, Hamiltonian, FP64, finest level: 32 B/point/sweep x "
                               f"{n}^3 points per launch, mean of {in_solve[1][0]} launches in one FP64 solve step "
                               f"({in_solve[1][1] * 1e3:.2f} us)"},
        "in_solve_sweeps_us": {KIND_NAMES[k]: round(v[1] * 1e3, 2) for k, v in in_solve.items()},
        # algorithmic GB/s of the in-solve sweeps: FP64 phi r+w, f, coefficient; FP32 e r+w, b, c (and a)
        "in_solve_sweeps_GBps": {KIND_NAMES[k]: round(SWEEP_BYTES_KIND[k] * N / (v[1] * 1e-3) / 1e9, 1)
                                 for k, v in in_solve.items() if v[1] > 0},
    }
    traffic = pmc_traffic(n)
    if traffic is not None:
        out["roofline"]["traffic"] = traffic
    log("vector modes of the solved shift and momentum density")
    out["vector_modes"] = vector_modes(torch, grmg, g, n)
    g.close()
    del d_pos, d_u
    c1, c1_src = c1_workload(torch, grmg, synth)
    out["c1"] = c1
    log("c2: 128^3 all fields")
    out["c2"] = c2_workload(torch, grmg, synth)
    if not args.no_learned and n == 256:
        log("learned guess: held-out trajectory")
        out["learned"] = bench_learned(torch, grmg, synth, n)
    if not args.no_batch:
        out["batch"] = bench_batch(torch, grmg, synth, max(1, min(args.steps, 2)))
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 thread)")
        est, sample_s = cpu_baseline(n, pos, u, mass, cycles)
        out["cpu_baseline"] = {"value": round(est * 1e3, 1), "unit": "ms", "cores": 1, "kind": "oracle",
                               "sample": f"CIC + two V(2,2) cycles of each equation kind at {n}^3 "
                                         f"({sample_s:.1f} s measured), scaled by the GPU per-field cycle counts",
                               "cpu_model": cpu_model(),
                               "c1_oracle_ms": round(c1_oracle_seconds(c1_src, c1["cycles"]) * 1e3, 1)}
        if not args.no_cpu_all_cores:
            log("cpu baseline, all cores (independent copies of the sample)")
            P, wall, gain, per = cpu_all_cores(n, pos, u, mass, sample_s)
            out["cpu_baseline"]["all_cores"] = {
                "cores": P, "wall_s": round(wall, 2), "median_sample_s": round(per, 2),
                "throughput_gain": round(gain, 2), "value": round(est * 1e3 / gain, 1), "unit": "ms",
                "note": f"{P} copies of the bounded sample in {P} processes at once; value = the one-core step "
                        f"estimate divided by the measured throughput gain (the oracle is serial)"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
