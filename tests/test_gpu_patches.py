"""Dirichlet refinement patches in the batched solve, through the C ABI,
against the patch oracle (oracle/dirichlet.py) and the periodic oracle for
their parents.
"""
import numpy as np
import pytest

import oracle as O
from oracle import dirichlet as OD
from paper_1905_08890_amd import grmg, synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

PRM = dict(a=1.0, omega_m=synth.OMEGA_M, c_tilde=synth.C_TILDE)
SRC = ("s0", "sx", "sy", "sz", "sm")


def maxrel(x, ref):
    return float(np.max(np.abs(x - ref)) / np.max(np.abs(ref)))


def face_mask(m):
    f = np.zeros((m + 2,) * 3, dtype=bool)
    I = slice(1, m + 1)
    for sl in ((0, I, I), (m + 1, I, I), (I, 0, I), (I, m + 1, I), (I, I, 0), (I, I, m + 1)):
        f[sl] = True
    return f


def test_boundary_values_match_oracle():
    """Face values of every level, sampled from the parent's current field:
    patches inside, across the parent's periodic edge, at another spacing."""
    boxes = [16, 24]
    patches = [(12, 1 / 32, 0, (5 / 16, 13 / 16, 1 / 16)), (10, 1 / 48, 1, (0.9, 0.1, 0.5)),
               (6, 1 / 20, 0, (0.0, 0.0, 0.0)), (24, 1 / 48, 1, (23 / 24, 0.5, 0.25))]
    print("[gpu] patch boundary values", flush=True)
    B = grmg.Batch(boxes, **PRM, patches=patches)
    rng = np.random.default_rng(0)
    parents = [rng.standard_normal((n,) * 3) for n in boxes]
    for i, P in enumerate(parents):
        B.set_field(i, "U", P)
    for j, (n, h, par, o) in enumerate(patches):
        for l, m in enumerate(OD.levels(n)):
            got = B.debug_boundary(len(boxes) + j, "U", l).cpu().numpy()
            ref = OD.face_values(parents[par], 1.0 / boxes[par], m, h * 2 ** l, o)
            fm = face_mask(m)
            # O(1) random parent: the interpolation coordinate (o + u h)/H rounds
            # differently with FMA contraction, ~1e-15 of cell, times O(1) jumps
            assert np.max(np.abs(got[fm] - ref[fm])) < 1e-13, (j, l)


def _patch_case():
    boxes = [32, 24]
    patches = [(24, 1 / 64, 0, (5 / 32, 20 / 32, 30 / 32)),     # wraps in z
               (16, 1 / 64, 0, (10 / 32, 2 / 32, 12 / 32)),
               (12, 1 / 48, 1, (3 / 24, 15 / 24, 7 / 24)),
               (5, 1 / 48, 1, (0.5, 0.5, 0.5))]                  # odd: one level, 32 sweeps per cycle
    box_src = []
    for b, n in enumerate(boxes):
        box_src.append(synth._matter_sources(n, 300 + b, 0.2))
    patch_src = [synth._matter_sources(n, 400 + j, 0.1) for j, (n, _, _, _) in enumerate(patches)]
    return boxes, patches, box_src, patch_src


def _load(B, boxes, box_src, patch_src):
    for i, src in enumerate(box_src):
        for name, v in zip(SRC, src):
            B.set_field(i, name, v)
    for j, src in enumerate(patch_src):
        for name, v in zip(SRC, src):
            B.set_field(len(boxes) + j, name, v)


def test_patch_solve_matches_oracle_at_equal_cycles():
    """All ten fields of boxes and patches after exactly 12 cycles per field:
    boxes against the periodic oracle, patches against the patch oracle fed
    with the oracle's own parents (1e-12)."""
    K = 12
    boxes, patches, box_src, patch_src = _patch_case()
    print("[gpu] patch solve vs oracle", flush=True)
    B = grmg.Batch(boxes, **PRM, patches=patches)
    _load(B, boxes, box_src, patch_src)
    r = B.solve(rtol=0.0, max_cycles=K)
    assert r["status"] == grmg.OK
    assert all(c == [K] * 10 for c in r["cycles"])
    prm = O.params(a=PRM["a"], omega_m=PRM["omega_m"], c_tilde=PRM["c_tilde"])
    parents = []
    for i, n in enumerate(boxes):
        F, st, cyc, rel, AA = O.solve_all(*box_src[i], prm=prm, max_cycles=K, rtol=0.0)
        assert st == O.OK
        for k in O.FIELDS:
            assert maxrel(B.get_field(i, k).cpu().numpy(), F[k]) < 1e-12, (i, k)
        parents.append((F, O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])[0]))
    for j, (n, h, par, o) in enumerate(patches):
        F, A6 = parents[par]
        src = dict(zip(SRC, patch_src[j]))
        out, st, cyc, rel, AA = OD.solve_patch(F, A6, 1.0 / boxes[par], src, n, h, o, prm, max_cycles=K, rtol=0.0)
        assert st == OD.OK
        for k in OD.FIELDS:
            got = B.get_field(len(boxes) + j, k).cpu().numpy()
            assert maxrel(got, OD.interior(out[k])) < 1e-12, (j, k)


def test_patch_solve_converges_and_graphs_replay_eager(monkeypatch):
    """Default tolerance: every patch field meets 1e-10 in a few cycles; the
    captured cycle graphs give the eager launches' result bit for bit."""
    boxes, patches, box_src, patch_src = _patch_case()
    print("[gpu] patch convergence + graph replay", flush=True)
    monkeypatch.setenv("GRMG_BATCH_GRAPH", "0")
    E = grmg.Batch(boxes, **PRM, patches=patches)
    monkeypatch.delenv("GRMG_BATCH_GRAPH")
    G = grmg.Batch(boxes, **PRM, patches=patches)
    for B in (E, G):
        _load(B, boxes, box_src, patch_src)
    for rep in range(2):
        re = E.solve(rtol=1e-10)
        rg = G.solve(rtol=1e-10)
        assert re["status"] == rg["status"] == grmg.OK
        assert re["cycles"] == rg["cycles"]
        for j in range(len(patches)):
            item = len(boxes) + j
            assert all(c <= 14 for c in rg["cycles"][item]), rg["cycles"][item]
            assert all(x <= 1e-10 for x in rg["rel_res"][item])
            for f in range(10):
                assert torch.equal(E.get_field(item, f), G.get_field(item, f)), (rep, j, f)


def test_concurrent_patches_match_sequential(monkeypatch):
    """Patches on their own stream, each field started as soon as the boxes'
    solve of it is done, give the sequential order's result bit for bit."""
    boxes, patches, box_src, patch_src = _patch_case()
    print("[gpu] concurrent vs sequential patches", flush=True)
    monkeypatch.setenv("GRMG_BATCH_CONCURRENT", "0")
    S = grmg.Batch(boxes, **PRM, patches=patches)
    monkeypatch.delenv("GRMG_BATCH_CONCURRENT")
    Cc = grmg.Batch(boxes, **PRM, patches=patches)
    for B in (S, Cc):
        _load(B, boxes, box_src, patch_src)
    rs = S.solve(rtol=1e-10)
    rc = Cc.solve(rtol=1e-10)
    assert rs["status"] == rc["status"] == grmg.OK
    assert rs["cycles"] == rc["cycles"] and rs["rel_res"] == rc["rel_res"]
    for item in range(len(boxes) + len(patches)):
        for f in range(10):
            assert torch.equal(S.get_field(item, f), Cc.get_field(item, f)), (item, f)


def test_patches_with_odd_coarsest_levels_converge():
    """Sides whose hierarchies end at 7^3 and 9^3 (56, 72) and 5^3 (40) on a
    64^3 parent."""
    boxes = [64]
    patches = [(56, 1 / 128, 0, (10 / 64, 20 / 64, 30 / 64)), (72, 1 / 128, 0, (40 / 64, 2 / 64, 5 / 64)),
               (40, 1 / 128, 0, (0.5, 0.5, 0.5))]
    print("[gpu] patch odd coarsest", flush=True)
    B = grmg.Batch(boxes, **PRM, patches=patches)
    _load(B, boxes, [synth._matter_sources(64, 500, 0.3)],
          [synth._matter_sources(n, 510 + j, 0.3) for j, (n, _, _, _) in enumerate(patches)])
    r = B.solve(rtol=1e-10)
    assert r["status"] == grmg.OK
    for j in range(len(patches)):
        assert all(x <= 1e-10 for x in r["rel_res"][1 + j])
        assert max(r["cycles"][1 + j]) <= 14, r["cycles"][1 + j]


def test_patch_descriptors_rejected():
    with pytest.raises(grmg.GrError):
        grmg.Batch([16], **PRM, patches=[(2, 0.01, 0, (0, 0, 0))])
    with pytest.raises(grmg.GrError):
        grmg.Batch([16], **PRM, patches=[(8, 0.01, 1, (0, 0, 0))])      # no box 1
    with pytest.raises(grmg.GrError):
        grmg.Batch([16], **PRM, patches=[(8, 0.01, 0, (float("nan"), 0, 0))])
    B = grmg.Batch([16], **PRM, patches=[(8, 0.01, 0, (0, 0, 0))])
    with pytest.raises(grmg.GrError):
        B.debug_boundary(0, "U", 0)                                        # not a patch
    with pytest.raises(grmg.GrError):
        B.debug_boundary(1, "U", 3)                                        # 8 -> 4: two levels


def _nested_case():
    boxes = [32]
    nb = len(boxes)
    patches = [(24, 1 / 64, 0, (5 / 32, 6 / 32, 8 / 32)),              # depth 1
               (16, 1 / 128, nb + 0, (3 / 64, 5 / 64, 2 / 64)),       # depth 2, inside patch 0
               (8, 1 / 256, nb + 1, (2 / 128, 4 / 128, 3 / 128)),     # depth 3, inside patch 1
               (8, 1 / 128, nb + 0, (10 / 64, 12 / 64, 9 / 64))]      # depth 2, inside patch 0
    box_src = [synth._matter_sources(n, 600 + b, 0.2) for b, n in enumerate(boxes)]
    patch_src = [synth._matter_sources(n, 700 + j, 0.1) for j, (n, _, _, _) in enumerate(patches)]
    return boxes, patches, box_src, patch_src


def _oracle_patches(boxes, patches, parents_box, patch_src, prm, K):
    """Oracle solves of the patches in item order (parents first), each from
    its parent's oracle fields: (fields by name as interior arrays, A_ij)."""
    nb = len(boxes)
    res = []
    for j, (n, h, par, o) in enumerate(patches):
        src = dict(zip(SRC, patch_src[j]))
        if par < nb:
            F, A6 = parents_box[par]
            H, periodic = 1.0 / boxes[par], True
        else:
            F, A6 = res[par - nb]
            H, periodic = patches[par - nb][1], False
        out, st, cyc, rel, AA, pA6 = OD.solve_patch(F, A6, H, src, n, h, o, prm, max_cycles=K, rtol=0.0,
                                                   periodic=periodic, return_A6=True)
        assert st == OD.OK
        res.append(({k: OD.interior(out[k]) for k in OD.FIELDS}, pA6))
    return res


def test_nested_patches_match_oracle_at_equal_cycles():
    """Nested refinement (reading D6): patches inside patches, three deep,
    each depth solved from the finished field of the depth above; after
    exactly 12 cycles per field every patch equals the patch oracle fed with
    the oracle's own parents (1e-12)."""
    K = 12
    boxes, patches, box_src, patch_src = _nested_case()
    print("[gpu] nested patches vs oracle", flush=True)
    B = grmg.Batch(boxes, **PRM, patches=patches)
    _load(B, boxes, box_src, patch_src)
    r = B.solve(rtol=0.0, max_cycles=K)
    assert r["status"] == grmg.OK and all(c == [K] * 10 for c in r["cycles"])
    prm = O.params(a=PRM["a"], omega_m=PRM["omega_m"], c_tilde=PRM["c_tilde"])
    F, st, *_ = O.solve_all(*box_src[0], prm=prm, max_cycles=K, rtol=0.0)
    for k in O.FIELDS:
        assert maxrel(B.get_field(0, k).cpu().numpy(), F[k]) < 1e-12, k
    ref = _oracle_patches(boxes, patches, [(F, O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])[0])], patch_src,
                          prm, K)
    for j in range(len(patches)):
        for k in OD.FIELDS:
            got = B.get_field(len(boxes) + j, k).cpu().numpy()
            assert maxrel(got, ref[j][0][k]) < 1e-12, (j, k)


def test_patch_substep_keeps_the_coarse_fields():
    """A sub-step of the refined levels: after a full solve, new sources on
    the patches and gr_batch_solve_patches leave the box's fields bit for bit
    and give the patches the oracle's solution from those kept fields (12
    cycles per field, 1e-12)."""
    K = 12
    boxes, patches, box_src, patch_src = _nested_case()
    print("[gpu] patch sub-step", flush=True)
    B = grmg.Batch(boxes, **PRM, patches=patches)
    _load(B, boxes, box_src, patch_src)
    assert B.solve(rtol=1e-10)["status"] == grmg.OK
    kept = [B.get_field(0, f).clone() for f in range(10)]
    new_src = [synth._matter_sources(n, 800 + j, 0.1) for j, (n, _, _, _) in enumerate(patches)]
    for j, src in enumerate(new_src):
        for name, v in zip(SRC, src):
            B.set_field(len(boxes) + j, name, v)
    r = B.solve(patches_only=True, rtol=0.0, max_cycles=K)
    assert r["status"] == grmg.OK
    for j in range(len(patches)):
        assert r["cycles"][len(boxes) + j] == [K] * 10
    for f in range(10):
        assert torch.equal(B.get_field(0, f), kept[f]), f
    prm = O.params(a=PRM["a"], omega_m=PRM["omega_m"], c_tilde=PRM["c_tilde"])
    F = {k: kept[i].cpu().numpy() for i, k in enumerate(O.FIELDS)}
    ref = _oracle_patches(boxes, patches, [(F, O.build_Aij(F["Vx"], F["Vy"], F["Vz"], F["U"])[0])], new_src, prm, K)
    for j in range(len(patches)):
        for k in OD.FIELDS:
            got = B.get_field(len(boxes) + j, k).cpu().numpy()
            assert maxrel(got, ref[j][0][k]) < 1e-12, (j, k)

