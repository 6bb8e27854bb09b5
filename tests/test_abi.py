"""CPU-side checks of the C ABI: the built library loads, exports every
function declared in include/gr.h, and rejects bad host-side arguments
without touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1905_08890_amd import grmg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "gr.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gr_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = grmg.load_library()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(grmg.EXPORTS)


def test_create_grid_validation():
    lib = grmg.load_library()
    g = C.c_void_p()
    prm = grmg.GrParams(1.0, 0.3, 11.7)
    for n, h in [(7, 1 / 7), (0, 1.0), (2048, 1.0), (16, 0.0), (16, -1.0)]:
        assert lib.gr_create_grid(C.byref(grmg.GrGridDesc(n, h)), C.byref(prm), C.byref(g)) == grmg.EINVAL
    assert lib.gr_create_grid(C.byref(grmg.GrGridDesc(16, 1 / 16)), C.byref(grmg.GrParams(0.0, 0.3, 1.0)),
                              C.byref(g)) == grmg.EINVAL
    assert lib.gr_create_grid(None, C.byref(prm), C.byref(g)) == grmg.EINVAL


def test_workspace_size_and_unbound_errors():
    g = grmg.create_grid(32, 1.0, 0.3072, 11.7)
    try:
        nbytes = grmg.workspace_bytes(g)
        # 45 fine FP64 arrays (fields, sources, A_ij, AA, shift sources, alternative
        # guesses, guess history), the FP64 and FP32 level hierarchies, the guess
        # interpolation scratch and the cell-ordered deposit (64 B per particle slot
        # plus 3 ints per cell and slot): about 63 fine arrays
        assert nbytes >= 60 * 8 * 32 ** 3
        assert nbytes < 66 * 8 * 32 ** 3
        lib = grmg.load_library()
        rep = grmg.GrSolveReport()
        assert lib.gr_solve_constraints(g, C.byref(grmg.default_opts()), C.byref(rep)) == grmg.ESTATE
        assert lib.gr_deposit_sources(g, None, None, 1.0, 0) == grmg.ESTATE
    finally:
        grmg.destroy_grid(g)


def test_default_options():
    o = grmg.default_opts()
    assert (o.nu1, o.nu2, o.max_cycles, o.rtol, o.precision, o.guess, o.field_mask) == \
        (2, 2, 100, 1e-10, grmg.FP64, grmg.GUESS_ZERO, grmg.ALL_FIELDS)


def test_no_cpu_fallback(monkeypatch):
    """The binding refuses to run without a GPU device instead of falling back."""
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        grmg.Grid(8)


def test_batch_with_patches_host_side():
    """Patch descriptors are checked on the host; the workspace holds the
    patches' padded iterate arrays."""
    lib = grmg.load_library()
    prm = grmg.GrParams(1.0, 0.3072, 11.7)
    boxes = (grmg.GrGridDesc * 1)(grmg.GrGridDesc(16, 1 / 16))
    b = C.c_void_p()

    def make(n, h, parent, origin):
        pd = (grmg.GrPatchDesc * 1)(grmg.GrPatchDesc(n, h, parent, (C.c_double * 3)(*origin)))
        return lib.gr_create_batch_patches(boxes, 1, pd, 1, C.byref(prm), C.byref(b))

    for bad in [(2, 0.01, 0, (0, 0, 0)), (600, 0.01, 0, (0, 0, 0)), (8, 0.0, 0, (0, 0, 0)),
                (8, 0.01, 1, (0, 0, 0)), (8, 0.01, -1, (0, 0, 0)), (8, 0.01, 0, (float("nan"), 0, 0)),
                (8, 0.01, 0, (0, 2e6, 0))]:
        assert make(*bad) == grmg.EINVAL, bad
    assert lib.gr_create_batch_patches(boxes, 1, None, 1, C.byref(prm), C.byref(b)) == grmg.EINVAL
    sizes = {}
    for npatch in (0, 1):
        h = grmg.create_batch([16], 1.0, 0.3072, 11.7, [(24, 1 / 32, 0, (0.1, 0.2, 0.3))] * npatch)
        try:
            sizes[npatch] = grmg.batch_workspace_bytes(h)
        finally:
            grmg.destroy_batch(h)
    # ten padded 26^3 fields and level 0's padded scratch for the fused sweep,
    # sources/A_ij/AA/shift sources and level 0's four work arrays dense 24^3,
    # and the levels 12, 6, 3 (padded iterate + four dense arrays each)
    extra = sizes[1] - sizes[0]
    assert extra >= 8 * (11 * 26 ** 3 + 19 * 24 ** 3)
    assert extra < 8 * (11 * 26 ** 3 + 19 * 24 ** 3 + 5 * 14 ** 3 + 5 * 8 ** 3 + 5 * 5 ** 3) + 64 * 1024


def test_bench_runs_on_one_gpu_only():
    """The benchmark refuses a multi-GPU run before touching a device."""
    import subprocess
    import sys
    from pathlib import Path

    root = Path(__file__).resolve().parents[1]
    r = subprocess.run([sys.executable, str(root / "bench.py"), "--gpus", "2", "--steps", "1"], cwd=root,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in (r.stdout + r.stderr)


def test_spectra_handle_validation():
    lib = grmg.load_library()
    h = C.c_void_p()
    for n, nb in [(12, 1), (4, 1), (2048, 4), (32, 0), (32, 9), (64, -1)]:
        assert lib.gr_create_spectra(n, nb, C.byref(h)) == grmg.EINVAL, (n, nb)
    assert lib.gr_create_spectra(32, 4, None) == grmg.EINVAL
    assert lib.gr_create_spectra(32, 8, C.byref(h)) == grmg.OK
    try:
        nbytes = C.c_size_t()
        assert lib.gr_spectra_workspace_bytes(h, C.byref(nbytes)) == grmg.OK
        # two complex n^3 arrays plus the twiddles and the shell partials
        assert 2 * 16 * 32 ** 3 <= nbytes.value < 2 * 16 * 32 ** 3 + (1 << 20)
        out = (C.c_double * 48)()
        x = C.c_void_p(256)
        # not bound: rejected before any device work
        assert lib.gr_vector_spectra(h, x, x, x, out) == grmg.ESTATE
        assert lib.gr_spectra_fft(h, x) == grmg.ESTATE
        assert lib.gr_vector_spectra(h, None, x, x, out) == grmg.EINVAL
        assert lib.gr_spectra_bind(h, x, nbytes.value - 1, None) == grmg.EINVAL
        assert lib.gr_spectra_bind(h, C.c_void_p(257), nbytes.value, None) == grmg.EINVAL
    finally:
        assert lib.gr_destroy_spectra(h) == grmg.OK


def test_nested_patch_descriptors_rejected():
    """A nested patch needs an earlier parent and every interpolation sample
    strictly between its parent patch's cell centres (host-side checks)."""
    nb = 1
    good = (24, 1 / 64, 0, (5 / 32, 6 / 32, 8 / 32))
    for bad in [(8, 1 / 128, nb + 1, (0.05, 0.05, 0.05)),       # parent not earlier
                (8, 1 / 128, nb + 0, (0.005, 0.05, 0.05)),      # closer than (H + h)/2 to the low face
                (16, 1 / 128, nb + 0, (0.05, 0.3, 0.05))]:      # beyond the high face
        with pytest.raises(grmg.GrError):
            grmg.create_batch([32], 1.0, 0.3, 1.0, patches=[good, bad])
    grmg.destroy_batch(grmg.create_batch([32], 1.0, 0.3, 1.0, patches=[good, (8, 1 / 128, nb + 0, (0.05, 0.05, 0.05))]))


def test_multiply_high_division_is_exact_where_the_coarse_cycle_uses_it():
    """The single-workgroup coarse cycle divides cell indices t < 2^24 by level
    sides 1 < d < 256 as the high 32 bits of t * ceil(2^32 / d): checked here
    against integer division for every such d, on every t below 2^16, a stride
    through the rest of the range, and the values just below and at the largest
    multiples of d (where the rounding error of m is largest)."""
    import numpy as np

    small = np.arange(1 << 16, dtype=np.uint64)
    stride = np.arange(1 << 16, 1 << 24, 997, dtype=np.uint64)
    for d in range(2, 256):
        m = np.uint64(0xFFFFFFFF // d + 1)
        k = np.arange((1 << 24) // d - 64, (1 << 24) // d + 1, dtype=np.uint64)
        edges = np.concatenate([k * np.uint64(d) - np.uint64(1), k * np.uint64(d)])
        edges = edges[edges < (1 << 24)]
        t = np.concatenate([small, stride, edges])
        q = (t * m) >> np.uint64(32)
        assert np.array_equal(q, t // np.uint64(d)), d
