"""GPU checks of the learned-guess plumbing: level features (restriction),
guess prolongation, and the residual-checked choice between a supplied guess
and the previous-step fields.

Restriction and prolongation are compared with the oracle's (FP32 output:
relative 2e-6 of the largest value; FP64 prolongation and cubic guess
interpolation: 1e-13).  The checked
choice is compared with the plain previous-step solve, which it must
reproduce (up to the rounding of one more mean removal) whenever it falls
back.
"""
import numpy as np
import pytest

import oracle as O
from paper_1905_08890_amd import grmg, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRM = dict(a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE)


def maxrel(x, ref):
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.mark.parametrize("n,level", [(32, 0), (32, 1), (32, 2), (48, 1), (64, 3)])
def test_features_match_oracle_restriction(n, level):
    print(f"[gpu] features n={n} level={level}", flush=True)
    g = grmg.Grid(n, **PRM)
    rng = np.random.default_rng(n + level)
    fields = [grmg.VX, grmg.PSI, grmg.S0, grmg.AA]
    vals = [rng.standard_normal((n, n, n)) * (1 + i) + i for i in range(len(fields))]
    for f, v in zip(fields, vals):
        g.set_field(f, v)
    off = [0.5, -1.0, 2.0, 0.0]
    sc = [2.0, 0.25, -1.0, 3.0]
    m = n >> level
    out = torch.empty((len(fields), m, m, m), dtype=torch.float32, device="cuda")
    grmg.features(g.handle, level, fields, off, sc, out)
    got = out.cpu().numpy().astype(np.float64)
    refs = []
    for c, v in enumerate(vals):
        r = v
        for _ in range(level):
            r = O.restrict(r)
        refs.append(r)
        ref = (r - off[c]) * sc[c]
        assert maxrel(got[c], ref) < 2e-6, c
    # accumulate: adds (value - offset) * scale to what the buffer holds
    grmg.features(g.handle, level, fields, [1.0] * 4, [-0.5] * 4, out, grmg.FEAT_ACCUMULATE)
    got = out.cpu().numpy().astype(np.float64)
    for c, r in enumerate(refs):
        ref = (r - off[c]) * sc[c] + (r - 1.0) * -0.5
        assert maxrel(got[c], ref) < 4e-6, c


@pytest.mark.parametrize("n,level", [(32, 0), (32, 1), (32, 2), (48, 1), (64, 3)])
@pytest.mark.parametrize("add", [0, 1])
@pytest.mark.parametrize("cubic", [0, 1])
def test_set_guess_matches_oracle_prolongation(n, level, add, cubic):
    print(f"[gpu] set_guess n={n} level={level} add={add} cubic={cubic}", flush=True)
    g = grmg.Grid(n, **PRM)
    rng = np.random.default_rng(7 * n + level)
    m = n >> level
    fields = [grmg.VY, grmg.XI, grmg.BB]
    base = [rng.standard_normal((n, n, n)) for _ in fields]
    for f, b in zip(fields, base):
        g.set_field(f, b)
    src = rng.standard_normal((len(fields), m, m, m)).astype(np.float32)
    sc = [1.5, -0.5, 4.0]
    flags = (grmg.SET_ADD if add else 0) | (grmg.SET_CUBIC if cubic else 0)
    grmg.set_guess(g.handle, level, fields, sc, torch.tensor(src, device="cuda"), flags)
    for c, f in enumerate(fields):
        e = src[c].astype(np.float64) * sc[c]
        for _ in range(level):
            e = O.interp_cubic(e) if cubic else O.prolong_add(e, np.zeros((2 * e.shape[0],) * 3))
        ref = e + (base[c] if add else 0.0)
        got = g.get_field(f).cpu().numpy()
        assert maxrel(got, ref) < 1e-13, f


def test_features_and_set_guess_reject_bad_arguments():
    g = grmg.Grid(16, **PRM)
    out = torch.empty(16 ** 3, dtype=torch.float32, device="cuda")
    lib = grmg.load_library()
    for level in (-1, 9):
        with pytest.raises(grmg.GrError):
            grmg.features(g.handle, level, [0], [0.0], [1.0], out)
        with pytest.raises(grmg.GrError):
            grmg.set_guess(g.handle, level, [0], [1.0], out, 1)
    for bad in ([grmg.FIELD_IDS["rhs"]], [99]):
        with pytest.raises(grmg.GrError):
            grmg.features(g.handle, 0, bad, [0.0], [1.0], out)
    with pytest.raises(grmg.GrError):
        grmg.set_guess(g.handle, 0, [grmg.S0], [1.0], out, 1)
    with pytest.raises(grmg.GrError):
        grmg.set_guess(g.handle, 0, [0], [1.0], out, 8)   # no such flag
    assert lib.gr_features(g.handle, 0, 1, None, None, None, None, 0) == grmg.EINVAL


# ------------------------------------------------ checked guess vs fallback

N = 32


def _state(g):
    return [g.get_field(f).clone() for f in range(10)]


def _load(g, fields):
    for f, v in enumerate(fields):
        g.set_field(f, v)


@pytest.fixture(scope="module")
def trajectory():
    """Step A solved from zero, step B's sources, and step B solved from A."""
    print("[gpu] checked-guess trajectory n=32", flush=True)
    g = grmg.Grid(N, **PRM)
    steps = list(synth.zeldovich_trajectory(N, 21, [0.8, 1.0]))
    g.deposit_sources(*steps[0])
    rep = g.solve_constraints(rtol=1e-10)
    assert rep["status"] == grmg.OK
    prev = _state(g)
    g.deposit_sources(*steps[1])
    rep_cur = g.solve_constraints(rtol=1e-10, guess="current")
    assert rep_cur["status"] == grmg.OK
    return g, prev, rep_cur, _state(g)


def _checked_solve(g, prev, pred):
    _load(g, prev)
    grmg.set_guess(g.handle, 1, list(range(10)), [1.0] * 10, pred, 1)
    return g.solve_constraints(rtol=1e-10, guess="checked")


@pytest.mark.parametrize("pred", ["zero", "nan", "garbage"])
def test_checked_guess_falls_back_to_previous_step(trajectory, pred):
    g, prev, rep_cur, cur = trajectory
    m = N // 2
    p = torch.zeros((10, m, m, m), dtype=torch.float32, device="cuda")
    if pred == "nan":
        p[:, 3, 4, 5] = float("nan")
    elif pred == "garbage":
        p.normal_(generator=torch.Generator(device="cuda").manual_seed(3)).mul_(10.0)
    rep = _checked_solve(g, prev, p)
    assert rep["status"] == grmg.OK
    assert rep["guess_fallback"] == 10
    assert rep["cycles"] == rep_cur["cycles"]
    for f in range(10):
        # the residual check pins the mean of the alternative once more: rounding only
        assert maxrel(g.get_field(f).cpu().numpy(), cur[f].cpu().numpy()) < 1e-12, f


def test_checked_guess_keeps_a_better_prediction(trajectory):
    """The increment itself (restricted to level 1) as the prediction: kept for
    most fields, and the solve needs fewer cycles than from the previous step."""
    g, prev, rep_cur, cur = trajectory
    m = N // 2
    fa = torch.empty((10, m, m, m), dtype=torch.float32, device="cuda")
    fb = torch.empty_like(fa)
    _load(g, cur)
    grmg.features(g.handle, 1, list(range(10)), [0.0] * 10, [1.0] * 10, fb)
    _load(g, prev)
    grmg.features(g.handle, 1, list(range(10)), [0.0] * 10, [1.0] * 10, fa)
    rep = _checked_solve(g, prev, (fb - fa).contiguous())
    print("cycles checked", rep["cycles"], "previous-step", rep_cur["cycles"], "fallbacks", rep["guess_fallback"])
    assert rep["status"] == grmg.OK
    assert rep["guess_fallback"] <= 2
    assert sum(rep["cycles"]) < sum(rep_cur["cycles"])
    assert max(rep["rel_res"]) <= 1e-10
    # a second solve without a new prediction has no alternative left: plain CURRENT
    rep2 = g.solve_constraints(rtol=1e-10, guess="checked")
    assert rep2["guess_fallback"] == 0


@pytest.mark.parametrize("n,level", [(32, 1), (64, 1), (48, 2)])
def test_extrapolated_guess_and_history(n, level):
    """GR_SET_EXTRAP: without a history the field becomes f + P pred (the
    previous step); the history then holds f; the next call gives
    (2 f' - f) + P pred'.  P = the oracle's cubic interpolation (1e-13); the
    history is readable (GR_HIST), settable, and a zero-guess solve discards
    it (the next extrapolation is again f + P pred)."""
    print(f"[gpu] extrapolated guess n={n} level={level}", flush=True)
    g = grmg.Grid(n, **PRM)
    rng = np.random.default_rng(11 * n + level)
    m = n >> level
    fields = [grmg.VX, grmg.PSI, grmg.BB]
    f0 = [rng.standard_normal((n, n, n)) for _ in fields]
    f1 = [rng.standard_normal((n, n, n)) for _ in fields]
    p0 = rng.standard_normal((len(fields), m, m, m)).astype(np.float32)
    p1 = rng.standard_normal((len(fields), m, m, m)).astype(np.float32)
    sc = [0.5, -2.0, 3.0]
    flags = grmg.SET_EXTRAP | grmg.SET_CUBIC

    def prolonged(p, c):
        e = p[c].astype(np.float64) * sc[c]
        for _ in range(level):
            e = O.interp_cubic(e)
        return e

    for f, v in zip(fields, f0):
        g.set_field(f, v)
    grmg.set_guess(g.handle, level, fields, sc, torch.tensor(p0, device="cuda"), flags)
    for c, f in enumerate(fields):
        assert maxrel(g.get_field(f).cpu().numpy(), f0[c] + prolonged(p0, c)) < 1e-13
        assert np.array_equal(g.get_field(grmg.HIST + f).cpu().numpy(), f0[c])
    for f, v in zip(fields, f1):
        g.set_field(f, v)
    grmg.set_guess(g.handle, level, fields, sc, torch.tensor(p1, device="cuda"), flags)
    for c, f in enumerate(fields):
        ref = (2.0 * f1[c] - f0[c]) + prolonged(p1, c)
        assert maxrel(g.get_field(f).cpu().numpy(), ref) < 1e-13
        assert np.array_equal(g.get_field(grmg.HIST + f).cpu().numpy(), f1[c])
    # a history set from outside is used; a zero-guess solve discards it
    for c, f in enumerate(fields):
        g.set_field(grmg.HIST + f, f0[c])
        g.set_field(f, f1[c])
    grmg.set_guess(g.handle, level, fields, [0.0] * 3, torch.tensor(p1, device="cuda"), flags)
    for c, f in enumerate(fields):
        assert maxrel(g.get_field(f).cpu().numpy(), 2.0 * f1[c] - f0[c]) < 1e-13
    g.set_field("s0", np.ones((n, n, n)))
    g.solve_constraints(rtol=1e-10)          # zero guess: a new trajectory
    for c, f in enumerate(fields):
        g.set_field(f, f1[c])
    grmg.set_guess(g.handle, level, fields, sc, torch.tensor(p0, device="cuda"), flags)
    for c, f in enumerate(fields):
        assert maxrel(g.get_field(f).cpu().numpy(), f1[c] + prolonged(p0, c)) < 1e-13


def test_shipped_learned_guess_saves_cycles():
    """The shipped network on the 256^3 workload's held-out trajectory (seed
    2000, steps 3 and 4 after two steps of history): extrapolation + network
    needs fewer V-cycles than the previous-step guess, keeps its guess on
    every field (no fallback), and does not need more cycles than the plain
    extrapolation (what the network adds)."""
    from paper_1905_08890_amd import learned

    print("[gpu] shipped learned guess 256^3", flush=True)
    n = 256
    g = learned.LearnedGuess(learned.WEIGHTS, n, torch)
    res = learned.evaluate(g, n, [2000], 4, 1.0, torch, exact=False)
    summ = learned.summarise(res)
    print({k: (v["cycles"], v["fallback"], round(v["ms"], 1)) for k, v in summ.items()}, flush=True)
    assert all(v["all_ok"] for v in summ.values())
    assert summ["learned_mixed"]["cycles"] < summ["prev_mixed"]["cycles"]
    assert summ["learned_mixed"]["fallback"] < 10
    assert summ["learned_mixed"]["cycles"] <= summ["extrap_mixed"]["cycles"]
