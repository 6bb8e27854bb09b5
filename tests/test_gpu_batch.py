"""Batched solve of uneven periodic boxes: every box equals its single-grid
solve and the oracle at identical cycle counts; graph replays equal eager
launches."""
import numpy as np
import pytest

import oracle as O
from paper_1905_08890_amd import grmg, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

PRM = dict(a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE)
SIDES = (8, 12, 16, 24, 32, 48)


def maxrel(x, ref):
    x = x.cpu().numpy() if hasattr(x, "cpu") else x
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def make_items(count, seed0):
    return [synth.batch_item(seed0 + i, sides=SIDES, sigma_range=(0.05, 0.5)) for i in range(count)]


def load(batch, items):
    for i, (n, src) in enumerate(items):
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            batch.set_field(i, name, x)


def test_batch_matches_single_grid_and_oracle():
    items = make_items(7, 300)
    print("[gpu] batch sides", [n for n, _ in items], flush=True)
    B = grmg.Batch([n for n, _ in items], **PRM)
    load(B, items)
    rep = B.solve(rtol=1e-10)
    assert rep["status"] == 0
    p = O.params(**PRM)
    for i, (n, src) in enumerate(items):
        g = grmg.Grid(n, **PRM)
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            g.set_field(name, x)
        single = g.solve_constraints(rtol=1e-10)
        assert single["cycles"] == rep["cycles"][i], i
        fields, st, cyc, rel, AA = O.solve_all(*src, prm=p, rtol=0, max_cycles=rep["cycles"][i])
        for name in O.FIELDS:
            out = B.get_field(i, name)
            assert maxrel(out, g.get_field(name).cpu().numpy()) < 1e-13, (i, name)
            assert maxrel(out, fields[name]) < 1e-12, (i, name)
        assert max(rep["rel_res"][i]) <= 1e-10
        assert rep["item_seconds"][i] > 0


@pytest.mark.parametrize("fused", ["1", "0"])
def test_batch_fused_boxes_match_single_grids(fused, monkeypatch):
    """Boxes of 64^3 and 96^3 take the batched fused sweep (32x16 tiles), 48^3
    the colour kernels, in the same launches; every box equals its single-grid
    solve at identical cycle counts."""
    monkeypatch.setenv("GRMG_BATCH_FUSED", fused)
    items = [synth.batch_item(500 + i, sides=(side,), sigma_range=(0.05, 0.5)) for i, side in
             enumerate((64, 48, 96, 64))]
    print(f"[gpu] batch fused={fused} sides", [n for n, _ in items], flush=True)
    B = grmg.Batch([n for n, _ in items], **PRM)
    load(B, items)
    rep = B.solve(rtol=1e-10)
    assert rep["status"] == 0
    for i, (n, src) in enumerate(items):
        g = grmg.Grid(n, **PRM)
        for name, x in zip(("s0", "sx", "sy", "sz", "sm"), src):
            g.set_field(name, x)
        single = g.solve_constraints(rtol=1e-10)
        assert single["cycles"] == rep["cycles"][i], i
        for name in O.FIELDS:
            assert maxrel(B.get_field(i, name), g.get_field(name).cpu().numpy()) < 1e-12, (i, name)


def test_batch_graph_replays_equal_eager(monkeypatch):
    """The per-cycle graph, replayed 1..4 times (with the solver's own eager
    launches and synchronisations between replays), gives the same fields as
    launching the same sequence eagerly."""
    items = make_items(5, 400)
    results = {}
    for use_graph in ("1", "0"):
        monkeypatch.setenv("GRMG_BATCH_GRAPH", use_graph)
        B = grmg.Batch([n for n, _ in items], **PRM)
        load(B, items)
        per_k = []
        for k in (1, 2, 3, 4):
            rep = B.solve(rtol=0, max_cycles=k)
            per_k.append([[B.get_field(i, f).cpu().numpy() for f in ("Vx", "Psi", "xi", "b")]
                          for i in range(len(items))])
        results[use_graph] = per_k
    for k in range(4):
        for i in range(len(items)):
            for a, b in zip(results["1"][k][i], results["0"][k][i]):
                assert np.array_equal(a, b), (k, i)


def test_batch_rejects_bad_input():
    with pytest.raises(grmg.GrError):
        grmg.create_batch([16, 7], 1.0, 0.3, 11.7)
    B = grmg.Batch([8, 16], **PRM)
    with pytest.raises(grmg.GrError):
        grmg.batch_solve(B.handle, 2, grmg.default_opts(precision=7))
    x = torch.zeros((8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(grmg.GrError):
        grmg.batch_set_field(B.handle, 5, grmg.S0, x, grmg.F64)


def test_batch_autotune_keeps_the_solve_bit_identical():
    """The batch autotuner only changes which launch form smooths each
    (level, box side); the solve after tuning equals the untuned one exactly,
    and field b (its scratch while tuning) is restored."""
    sides = [64, 128, 96, 64, 32]
    print(f"[gpu] batch autotune {sides}", flush=True)
    A = grmg.Batch(sides, **PRM)
    T = grmg.Batch(sides, **PRM)
    srcs = [synth._matter_sources(n, 700 + i, 0.3) for i, n in enumerate(sides)]
    for B in (A, T):
        for i, src in enumerate(srcs):
            for name, v in zip(("s0", "sx", "sy", "sz", "sm"), src):
                B.set_field(i, name, v)
    # a mixed-precision solve before tuning captures the mixed cycle graphs,
    # which the tuner must drop together with the FP64 ones
    rm0 = T.solve(rtol=1e-10, precision=grmg.MIXED)
    assert rm0["status"] == grmg.OK
    b_before = [T.get_field(i, "b").clone() for i in range(len(sides))]
    rep = T.autotune()
    lines = [ln for ln in rep.splitlines() if ln.startswith("depth=")]
    assert lines and all("form=" in ln and "us=" in ln for ln in lines), rep
    for i in range(len(sides)):
        assert torch.equal(T.get_field(i, "b"), b_before[i])
    ra = A.solve(rtol=1e-10)
    rt = T.solve(rtol=1e-10)
    assert ra["status"] == rt["status"] == grmg.OK
    assert ra["cycles"] == rt["cycles"]
    for i in range(len(sides)):
        for f in range(10):
            assert torch.equal(A.get_field(i, f), T.get_field(i, f)), (i, f)
    ma = A.solve(rtol=1e-10, precision=grmg.MIXED)
    mt = T.solve(rtol=1e-10, precision=grmg.MIXED)
    assert ma["status"] == mt["status"] == grmg.OK
    assert ma["cycles"] == mt["cycles"]
    for i in range(len(sides)):
        for f in range(10):
            assert torch.equal(A.get_field(i, f), T.get_field(i, f)), ("mixed", i, f)


def test_batch_mixed_precision_matches_fp64():
    """Iterative refinement in the batch (FP64 residual and update, FP32
    correction cycles with FP64 coarse levels): every field of every box,
    refined to 1e-12, within 1e-9 of the FP64 solution converged to 1e-13;
    at 1e-10 the refinement steps stay within two of the FP64 cycles."""
    sides = [64, 32, 48, 96]
    print(f"[gpu] batch mixed {sides}", flush=True)
    A = grmg.Batch(sides, **PRM)
    M = grmg.Batch(sides, **PRM)
    srcs = [synth._matter_sources(n, 800 + i, 0.4) for i, n in enumerate(sides)]
    for B in (A, M):
        for i, src in enumerate(srcs):
            for name, v in zip(("s0", "sx", "sy", "sz", "sm"), src):
                B.set_field(i, name, v)
    ra = A.solve(rtol=1e-13, max_cycles=60)
    rm = M.solve(rtol=1e-12, max_cycles=60, precision="mixed")
    assert ra["status"] == rm["status"] == grmg.OK
    for i in range(len(sides)):
        for f in range(10):
            ref = A.get_field(i, f).cpu().numpy()
            got = M.get_field(i, f).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), (i, f)
    r64 = A.solve(rtol=1e-10)
    r32 = M.solve(rtol=1e-10, precision="mixed")
    assert r32["status"] == grmg.OK
    for i in range(len(sides)):
        assert all(x <= 1e-10 for x in r32["rel_res"][i])
        for f in range(10):
            assert abs(r32["cycles"][i][f] - r64["cycles"][i][f]) <= 2, (i, f, r32["cycles"][i], r64["cycles"][i])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_per_point_forms_match_marching(precision, monkeypatch):
    """With the plane-marching stopping norms, residual + restriction and
    refinement residual switched off (one thread per point everywhere), the
    batch gives the same cycle counts and fields within 1e-12 of the default
    forms (only the order of the norm sums differs)."""
    sides = [64, 48, 96]
    print(f"[gpu] batch per-point forms {sides} {precision}", flush=True)
    srcs = [synth._matter_sources(n, 850 + i, 0.3) for i, n in enumerate(sides)]
    monkeypatch.setenv("GRMG_MARCH", "0")
    P = grmg.Batch(sides, **PRM)
    monkeypatch.delenv("GRMG_MARCH")
    Q = grmg.Batch(sides, **PRM)
    for B in (P, Q):
        for i, src in enumerate(srcs):
            for name, v in zip(("s0", "sx", "sy", "sz", "sm"), src):
                B.set_field(i, name, v)
    rp = P.solve(rtol=1e-10, precision=precision)
    rq = Q.solve(rtol=1e-10, precision=precision)
    assert rp["status"] == rq["status"] == grmg.OK
    assert rp["cycles"] == rq["cycles"]
    for i in range(len(sides)):
        for f in range(10):
            assert maxrel(P.get_field(i, f), Q.get_field(i, f).cpu().numpy()) < 1e-12, (i, f)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_fused16_form_is_bit_identical(precision, monkeypatch):
    """The fused 16x16 form (forced where the 32x16 one does not apply: the
    48^3 and 32^3 boxes and the 48^3 and 32^3 levels of the larger ones) gives
    the per-colour launches' solve bit for bit, in FP64 and in the FP32
    correction cycles."""
    sides = [48, 96, 32, 64]
    print(f"[gpu] batch fused16 {sides} {precision}", flush=True)
    srcs = [synth._matter_sources(n, 900 + i, 0.3) for i, n in enumerate(sides)]
    A = grmg.Batch(sides, **PRM)
    monkeypatch.setenv("GRMG_BATCH_FORM", "3")
    F = grmg.Batch(sides, **PRM)
    monkeypatch.delenv("GRMG_BATCH_FORM")
    for B in (A, F):
        for i, src in enumerate(srcs):
            for name, v in zip(("s0", "sx", "sy", "sz", "sm"), src):
                B.set_field(i, name, v)
    ra = A.solve(rtol=1e-10, precision=precision)
    rf = F.solve(rtol=1e-10, precision=precision)
    assert ra["status"] == rf["status"] == grmg.OK
    assert ra["cycles"] == rf["cycles"]
    for i in range(len(sides)):
        for f in range(10):
            assert torch.equal(A.get_field(i, f), F.get_field(i, f)), (i, f)


@pytest.mark.parametrize("tuned", [False, True])
def test_batch_fused_boxes_match_oracle(tuned):
    """A 64^3 and a 96^3 box, which take the batched fused sweeps (the default
    32x16 form, or the forms the batch autotuner picks), beside a 32^3 box:
    every field equals the oracle's at the batch's own per-field cycle counts
    (1e-12)."""
    items = [synth.batch_item(700 + i, sides=(side,), sigma_range=(0.05, 0.5)) for i, side in
             enumerate((64, 96, 32))]
    print(f"[gpu] batch fused boxes vs oracle, tuned={tuned}", flush=True)
    B = grmg.Batch([n for n, _ in items], **PRM)
    load(B, items)
    if tuned:
        print(B.autotune(), flush=True)
    rep = B.solve(rtol=1e-10)
    assert rep["status"] == 0
    p = O.params(**PRM)
    for i, (n, src) in enumerate(items[:2]):
        fields, st, cyc, rel, AA = O.solve_all(*src, prm=p, rtol=0, max_cycles=rep["cycles"][i])
        assert list(cyc) == list(rep["cycles"][i])
        for name in O.FIELDS:
            assert maxrel(B.get_field(i, name), fields[name]) < 1e-12, (n, name)


def test_batch_mixed_stagnation_falls_back_to_fp64(monkeypatch):
    """Forced from the host: with a stagnation ratio of 0 every refinement step
    after the first counts as stalled, so each box's field finishes with FP64
    FAS cycles after its third measurement (the single grid's rule); the
    result meets the tolerance, equals the FP64 solution within 1e-9, and the
    fallback flags say so.  With the default ratio nothing falls back."""
    sides = [32, 48, 64]
    srcs = [synth._matter_sources(n, 820 + i, 0.4) for i, n in enumerate(sides)]

    def make():
        B = grmg.Batch(sides, **PRM)
        for i, src in enumerate(srcs):
            for name, v in zip(("s0", "sx", "sy", "sz", "sm"), src):
                B.set_field(i, name, v)
        return B

    A = make()
    ra = A.solve(rtol=1e-13, max_cycles=60)
    N = make()
    rn = N.solve(rtol=1e-12, max_cycles=60, precision="mixed")
    assert rn["status"] == grmg.OK and all(f == 0 for row in rn["fallback"] for f in row)
    monkeypatch.setenv("GRMG_MIXED_STALL", "0")
    print("[gpu] batch mixed forced stagnation", flush=True)
    M = make()
    rm = M.solve(rtol=1e-12, max_cycles=60, precision="mixed")
    assert ra["status"] == rm["status"] == grmg.OK
    for i in range(len(sides)):
        assert all(x <= 1e-12 for x in rm["rel_res"][i])
        for f in range(10):
            assert rm["fallback"][i][f] == 1, (i, f, rm["cycles"][i])
            ref = A.get_field(i, f).cpu().numpy()
            got = M.get_field(i, f).cpu().numpy()
            assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), (i, f)


QUEUE_SIDES = (8, 12, 16, 24, 32, 48, 64, 96, 128)


def _solve_sides(items, monkeypatch, queue, graph="1", tune=False, **kw):
    monkeypatch.setenv("GRMG_BATCH_QUEUE", "1" if queue else "0")
    monkeypatch.setenv("GRMG_BATCH_GRAPH", graph)
    B = grmg.Batch([n for n, _ in items], **PRM)
    load(B, items)
    if tune:
        B.autotune()
    rep = B.solve(**kw)
    return B, rep


def test_batch_queue_is_bit_identical_to_grouped_launches(monkeypatch):
    """The device task queue (levels of at most 32^3 points and the coarse
    cycle of every box in one persistent launch per cycle) runs each phase with
    the per-cell arithmetic of the grouped per-colour and per-cell launches, so
    with those forms (GRMG_MARCH=0) every field of every box is bit-identical
    and the cycle counts equal; the same with eager launches instead of the
    captured cycle."""
    monkeypatch.setenv("GRMG_MARCH", "0")
    items = [synth.batch_item(900 + i, sides=(side,), sigma_range=(0.05, 0.5)) for i, side in enumerate(QUEUE_SIDES)]
    print("[gpu] batch queue vs grouped, sides", QUEUE_SIDES, flush=True)
    A, ra = _solve_sides(items, monkeypatch, queue=False, rtol=1e-10)
    Q, rq = _solve_sides(items, monkeypatch, queue=True, rtol=1e-10)
    E, re_ = _solve_sides(items, monkeypatch, queue=True, graph="0", rtol=1e-10)
    assert ra["status"] == rq["status"] == re_["status"] == grmg.OK
    assert ra["cycles"] == rq["cycles"] == re_["cycles"]
    for i in range(len(items)):
        for f in range(10):
            a = A.get_field(i, f)
            assert torch.equal(a, Q.get_field(i, f)), (QUEUE_SIDES[i], f)
            assert torch.equal(a, E.get_field(i, f)), (QUEUE_SIDES[i], f)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_queue_with_tuned_forms(precision, monkeypatch):
    """Default (plane-marching) forms and autotuned sweeps: the queue gives the
    grouped launches' cycle counts and fields within 1e-12 (the marching
    restriction adds in another order than the queue's per-cell form), and a
    32^3 box equals the oracle at those cycle counts; V-cycles beyond the
    queue's task table (nu > 8) are rejected."""
    items = [synth.batch_item(950 + i, sides=(side,), sigma_range=(0.05, 0.5)) for i, side in
             enumerate((32, 64, 96, 48))]
    print(f"[gpu] batch queue tuned, {precision}", flush=True)
    A, ra = _solve_sides(items, monkeypatch, queue=False, tune=True, rtol=1e-10, precision=precision)
    Q, rq = _solve_sides(items, monkeypatch, queue=True, tune=True, rtol=1e-10, precision=precision)
    assert ra["status"] == rq["status"] == grmg.OK
    assert ra["cycles"] == rq["cycles"]
    for i in range(len(items)):
        for f in range(10):
            assert maxrel(Q.get_field(i, f), A.get_field(i, f).cpu().numpy()) < 1e-12, (i, f)
    if precision == "fp64":
        n, src = items[0]
        fields, *_ = O.solve_all(*src, prm=O.params(**PRM), rtol=0, max_cycles=rq["cycles"][0])
        for name in O.FIELDS:
            assert maxrel(Q.get_field(0, name), fields[name]) < 1e-12, name
        st = Q.solve(allow=(grmg.OK, grmg.EINVAL), rtol=1e-10, nu1=9, nu2=2)
        assert st["status"] == grmg.EINVAL
