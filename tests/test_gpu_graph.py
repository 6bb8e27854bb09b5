"""Captured-cycle replay (hipGraph) against launching every kernel eagerly.

Both grids get bit-identical sources (copied, since the cell-ordered deposit
may order particles of one cell differently from run to run); the cycle
kernels are deterministic, so replayed graphs must reproduce the eager solve
bit for bit, over many replays and with eager work between them.
"""
import pytest

from paper_1905_08890_amd import grmg, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRM = dict(a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE)
SOURCES = ("s0", "sx", "sy", "sz", "sm")


def _pair(n, monkeypatch):
    monkeypatch.setenv("GRMG_GRAPH", "0")
    eager = grmg.Grid(n, **PRM)
    monkeypatch.delenv("GRMG_GRAPH")
    graph = grmg.Grid(n, **PRM)
    return graph, eager


def _same_sources(dst, src):
    for name in SOURCES:
        dst.set_field(name, src.get_field(name))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_graph_replay_matches_eager(precision, monkeypatch):
    n = 64
    print(f"[gpu] graph vs eager n={n} {precision}", flush=True)
    graph, eager = _pair(n, monkeypatch)
    steps = list(synth.zeldovich_trajectory(n, 11, [0.8, 1.0, 1.2]))
    for k, (pos, u, mass) in enumerate(steps):
        graph.deposit_sources(pos, u, mass)
        _same_sources(eager, graph)
        guess = "zero" if k == 0 else "current"
        rg = graph.solve_constraints(rtol=1e-10, precision=precision, guess=guess)
        re = eager.solve_constraints(rtol=1e-10, precision=precision, guess=guess)
        assert rg["status"] == re["status"] == grmg.OK
        assert rg["cycles"] == re["cycles"]
        assert rg["rel_res"] == re["rel_res"]
        for f in range(10):
            # read on the caller's stream right after the solve: ordered by the join
            assert torch.equal(graph.get_field(f), eager.get_field(f)), (k, f)


def test_graph_cache_follows_options(monkeypatch):
    """A change of nu1/nu2 records a new graph instead of replaying the old one."""
    n = 32
    graph, eager = _pair(n, monkeypatch)
    pos, u, mass = synth.zeldovich(n, 4, 0.5)
    graph.deposit_sources(pos, u, mass)
    _same_sources(eager, graph)
    for nu in ((2, 2), (1, 3), (2, 2)):
        rg = graph.solve_constraints(rtol=1e-10, nu1=nu[0], nu2=nu[1])
        re = eager.solve_constraints(rtol=1e-10, nu1=nu[0], nu2=nu[1])
        assert rg["cycles"] == re["cycles"], nu
        for f in range(10):
            assert torch.equal(graph.get_field(f), eager.get_field(f)), (nu, f)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_autotuned_launch_shapes_give_the_same_solve(precision):
    """The autotuner changes only launch shapes of the fused sweep: the solve
    after tuning equals the untuned one bit for bit."""
    n = 128
    print(f"[gpu] autotune n={n} {precision}", flush=True)
    a = grmg.Grid(n, **PRM)
    b = grmg.Grid(n, **PRM)
    pos, u, mass = synth.zeldovich(n, 5, 0.5)
    a.deposit_sources(pos, u, mass)
    _same_sources(b, a)
    report = grmg.autotune(b.handle)
    lines = [ln for ln in report.splitlines() if ln.startswith("n=")]
    assert len(lines) == 18 and all("us=" in ln for ln in lines)   # levels 128^3, 64^3 and 32^3, six kinds each
    _same_sources(b, a)   # the tuner may use the deposit scratch, never the sources
    ra = a.solve_constraints(rtol=1e-10, precision=precision)
    rb = b.solve_constraints(rtol=1e-10, precision=precision)
    assert ra["cycles"] == rb["cycles"]
    for f in range(10):
        assert torch.equal(a.get_field(f), b.get_field(f)), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("tile,pf,remap", [("2", "3", "0"), ("2", "4", "2"), ("2", "1", "1"), ("3", "2", "2")])
def test_forced_launch_shapes_give_the_same_solve(precision, tile, pf, remap, monkeypatch):
    """Every prefetch depth and workgroup order of the 64x16 fused sweep, and
    the 128x8 tile (FP64 and FP32 kinds, fused from 64^3 down; 128x8 where the
    side allows it), give the default shapes' solve bit for bit."""
    n = 128
    print(f"[gpu] forced shapes n={n} {precision} tile={tile} pf={pf} remap={remap}", flush=True)
    a = grmg.Grid(n, **PRM)
    monkeypatch.setenv("GRMG_FUSED_MIN", "64")
    monkeypatch.setenv("GRMG_FUSED_TILE", tile)
    monkeypatch.setenv("GRMG_FUSED_PF", pf)
    monkeypatch.setenv("GRMG_XCD_REMAP", remap)
    b = grmg.Grid(n, **PRM)
    pos, u, mass = synth.zeldovich(n, 6, 0.5)
    a.deposit_sources(pos, u, mass)
    _same_sources(b, a)
    ra = a.solve_constraints(rtol=1e-10, precision=precision)
    rb = b.solve_constraints(rtol=1e-10, precision=precision)
    assert ra["cycles"] == rb["cycles"]
    for f in range(10):
        assert torch.equal(a.get_field(f), b.get_field(f)), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_poisson_single_workgroup_threshold_16_matches_8(precision, monkeypatch):
    """The Poisson V-cycles take the 16^3 level into the single-workgroup cycle
    by default; with that level on the multi-launch path instead the solve
    agrees to rounding (the two forms add the restriction's children in other
    orders): the same cycle counts, fields within 1e-12 (FP64) / 1e-10 (mixed)."""
    n = 64
    print(f"[gpu] single-workgroup threshold n={n} {precision}", flush=True)
    a = grmg.Grid(n, **PRM)
    monkeypatch.setenv("GRMG_COARSE_NP", "8")
    b = grmg.Grid(n, **PRM)
    pos, u, mass = synth.zeldovich(n, 8, 0.5)
    a.deposit_sources(pos, u, mass)
    _same_sources(b, a)
    ra = a.solve_constraints(rtol=1e-10, precision=precision)
    rb = b.solve_constraints(rtol=1e-10, precision=precision)
    assert ra["status"] == rb["status"] == grmg.OK
    assert ra["cycles"] == rb["cycles"]
    tol = 1e-12 if precision == "fp64" else 1e-10
    for f in range(10):
        x, y = a.get_field(f), b.get_field(f)
        assert float((x - y).abs().max()) <= tol * float(y.abs().max()), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_fused_sweep_on_sides_of_32_mod_64_matches_per_colour(precision, monkeypatch):
    """A level whose side is an odd multiple of 32 (96^3 here) takes the fused
    sweep in 32x16 tiles; its solve equals one launch per colour bit for bit."""
    n = 96
    print(f"[gpu] fused 32x16 on n={n} {precision}", flush=True)
    monkeypatch.setenv("GRMG_SMOOTHER", "split")
    a = grmg.Grid(n, **PRM)
    monkeypatch.setenv("GRMG_SMOOTHER", "fused")
    monkeypatch.setenv("GRMG_FUSED_MIN", "96")
    b = grmg.Grid(n, **PRM)
    pos, u, mass = synth.zeldovich(n, 7, 0.5)
    a.deposit_sources(pos, u, mass)
    _same_sources(b, a)
    ra = a.solve_constraints(rtol=1e-10, precision=precision)
    rb = b.solve_constraints(rtol=1e-10, precision=precision)
    assert ra["cycles"] == rb["cycles"]
    for f in range(10):
        assert torch.equal(a.get_field(f), b.get_field(f)), f


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_concurrent_vector_components_match_sequential(precision, monkeypatch):
    """The three components of the vector equations solved side by side, each on
    a helper hierarchy with its own stream, give the sequential solve bit for bit."""
    n = 64
    print(f"[gpu] concurrent components n={n} {precision}", flush=True)
    monkeypatch.setenv("GRMG_CONCURRENT", "0")
    seq = grmg.Grid(n, **PRM)
    monkeypatch.delenv("GRMG_CONCURRENT")
    conc = grmg.Grid(n, **PRM)
    steps = list(synth.zeldovich_trajectory(n, 12, [0.9, 1.1]))
    for k, (pos, u, mass) in enumerate(steps):
        conc.deposit_sources(pos, u, mass)
        _same_sources(seq, conc)
        guess = "zero" if k == 0 else "current"
        rc = conc.solve_constraints(rtol=1e-10, precision=precision, guess=guess)
        rs = seq.solve_constraints(rtol=1e-10, precision=precision, guess=guess)
        assert rc["status"] == rs["status"] == grmg.OK
        assert rc["cycles"] == rs["cycles"]
        assert rc["rel_res"] == rs["rel_res"]
        for f in range(10):
            assert torch.equal(conc.get_field(f), seq.get_field(f)), (k, f)
