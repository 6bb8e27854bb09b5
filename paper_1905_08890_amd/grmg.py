"""ctypes binding of libgrmg.so (C ABI in include/gr.h).

Argument marshalling only: every step of the solve runs in the HIP library.
PyTorch supplies device memory (the workspace and the caller's tensors) and
the HIP stream.  Importing this module does not touch the GPU; the library
is loaded on first use and a missing library raises immediately - there is
no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgrmg.so")

# ---- constants mirrored from gr.h ----
OK, EINVAL, EDEVICE, ENOTCONV, ENAN, ESTATE = 0, -1, -2, -3, -4, -6
POISSON, HAMILTONIAN, CMC = 0, 1, 2
(VX, VY, VZ, U, PSI, XI, BX, BY, BZ, BB, S0, SX, SY, SZ, SM, AA, PHI, ALPHA, CONF, BETAX, BETAY, BETAZ,
 RHS, COEF) = range(24)
F64, F32 = 0, 1
FP64, MIXED = 0, 1
GUESS_ZERO, GUESS_CURRENT, GUESS_CHECKED = 0, 1, 2
SET_ADD, SET_CUBIC, SET_EXTRAP = 1, 2, 4
HIST = 24   # GR_HIST + f: history of solved field f (read only)
FEAT_ACCUMULATE = 1
ALL_FIELDS = 0x3FF
SOLVED = ("Vx", "Vy", "Vz", "U", "Psi", "xi", "Bx", "By", "Bz", "b")
FIELD_IDS = {name: i for i, name in enumerate(SOLVED)}
FIELD_IDS.update(dict(s0=S0, sx=SX, sy=SY, sz=SZ, sm=SM, AA=AA, Phi=PHI, alpha=ALPHA, psi_conf=CONF,
                      beta_x=BETAX, beta_y=BETAY, beta_z=BETAZ, rhs=RHS, coef=COEF))
FIELD_IDS.update({f"hist_{name}": HIST + i for i, name in enumerate(SOLVED)})

EXPORTS = ("gr_default_opts", "gr_create_grid", "gr_workspace_bytes", "gr_bind", "gr_deposit_sources",
           "gr_set_field", "gr_get_field", "gr_solve_constraints", "gr_solve_equation", "gr_solve_equation_static",
           "gr_debug_sweep", "gr_kick", "gr_drift", "gr_newtonian_kick",
           "gr_debug_residual", "gr_destroy_grid", "gr_last_error", "gr_features", "gr_set_guess", "gr_autotune", "gr_sweep_timing", "gr_create_batch", "gr_create_batch_patches",
           "gr_batch_debug_boundary", "gr_batch_autotune", "gr_batch_mixed_fallbacks", "gr_batch_workspace_bytes",
           "gr_batch_bind", "gr_batch_set_field", "gr_batch_get_field", "gr_batch_solve", "gr_batch_solve_patches",
           "gr_destroy_batch",
           "gr_batch_last_error", "gr_unet_create", "gr_unet_workspace_bytes", "gr_unet_param_count", "gr_unet_bind",
           "gr_unet_init", "gr_unet_set_params", "gr_unet_get_params", "gr_unet_forward", "gr_unet_loss_grad",
           "gr_unet_train_step", "gr_destroy_unet", "gr_unet_last_error", "gr_create_spectra",
           "gr_spectra_workspace_bytes", "gr_spectra_bind", "gr_vector_spectra", "gr_spectra_fft", "gr_destroy_spectra",
           "gr_spectra_last_error")


class GrParams(C.Structure):
    _fields_ = [("a", C.c_double), ("omega_m", C.c_double), ("c_tilde", C.c_double)]


class GrGridDesc(C.Structure):
    _fields_ = [("n", C.c_int), ("h", C.c_double)]


class GrPatchDesc(C.Structure):
    _fields_ = [("n", C.c_int), ("h", C.c_double), ("parent", C.c_int), ("origin", C.c_double * 3)]


class GrSolveOpts(C.Structure):
    _fields_ = [("nu1", C.c_int), ("nu2", C.c_int), ("max_cycles", C.c_int), ("rtol", C.c_double),
                ("precision", C.c_int), ("guess", C.c_int), ("field_mask", C.c_uint)]


class GrUnetDesc(C.Structure):
    _fields_ = [("in_ch", C.c_int), ("out_ch", C.c_int), ("c", C.c_int * 4), ("lap_weight", C.c_float),
                ("clip_norm", C.c_float)]


class GrSolveReport(C.Structure):
    _fields_ = [("status", C.c_int), ("cycles", C.c_int * 10), ("rel_res", C.c_double * 10),
                ("seconds", C.c_double), ("fallback", C.c_int), ("guess_fallback", C.c_int),
                ("guess_rel", C.c_double * 10), ("alt_rel", C.c_double * 10)]

    def as_dict(self):
        return dict(status=self.status, cycles=list(self.cycles), rel_res=list(self.rel_res),
                    seconds=self.seconds, fallback=self.fallback, guess_fallback=self.guess_fallback,
                    guess_rel=list(self.guess_rel), alt_rel=list(self.alt_rel))


class GrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gr error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libgrmg.so and declare its signatures (no GPU work)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run __graft_entry__.build() (no CPU fallback exists)")
    lib = C.CDLL(path)
    vp, i64 = C.c_void_p, C.c_int64
    sig = {
        "gr_default_opts": [C.POINTER(GrSolveOpts)],
        "gr_create_grid": [C.POINTER(GrGridDesc), C.POINTER(GrParams), C.POINTER(vp)],
        "gr_workspace_bytes": [vp, C.POINTER(C.c_size_t)],
        "gr_bind": [vp, vp, C.c_size_t, vp],
        "gr_deposit_sources": [vp, vp, vp, C.c_double, i64],
        "gr_set_field": [vp, C.c_int, vp, C.c_int],
        "gr_get_field": [vp, C.c_int, vp, C.c_int],
        "gr_solve_constraints": [vp, C.POINTER(GrSolveOpts), C.POINTER(GrSolveReport)],
        "gr_solve_equation": [vp, C.c_int, C.c_int, C.POINTER(GrSolveOpts), C.POINTER(GrSolveReport)],
        "gr_solve_equation_static": [C.c_int, C.POINTER(GrParams), C.c_int, vp, vp, vp, C.POINTER(GrSolveOpts), vp,
                                     C.POINTER(GrSolveReport)],
        "gr_debug_sweep": [vp, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int],
        "gr_kick": [vp, vp, vp, i64, C.c_double, C.c_int],
        "gr_drift": [vp, vp, vp, i64, C.c_double],
        "gr_newtonian_kick": [vp, vp, vp, i64, C.c_double, C.POINTER(GrSolveOpts), C.POINTER(GrSolveReport)],
        "gr_debug_residual": [vp, C.c_int, C.c_int, C.c_double, C.c_double, vp],
        "gr_destroy_grid": [vp],
        "gr_features": [vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), C.POINTER(C.c_double), vp,
                        C.c_int],
        "gr_autotune": [vp, C.c_char_p, C.c_size_t],
        "gr_sweep_timing": [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)],
        "gr_set_guess": [vp, C.c_int, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double), vp, C.c_int],
        "gr_create_batch": [C.POINTER(GrGridDesc), C.c_int, C.POINTER(GrParams), C.POINTER(vp)],
        "gr_create_batch_patches": [C.POINTER(GrGridDesc), C.c_int, C.POINTER(GrPatchDesc), C.c_int,
                                    C.POINTER(GrParams), C.POINTER(vp)],
        "gr_batch_debug_boundary": [vp, C.c_int, C.c_int, C.c_int, vp],
        "gr_batch_autotune": [vp, C.c_char_p, C.c_size_t],
        "gr_batch_mixed_fallbacks": [vp, C.POINTER(C.c_int)],
        "gr_batch_workspace_bytes": [vp, C.POINTER(C.c_size_t)],
        "gr_batch_bind": [vp, vp, C.c_size_t, vp],
        "gr_batch_set_field": [vp, C.c_int, C.c_int, vp, C.c_int],
        "gr_batch_get_field": [vp, C.c_int, C.c_int, vp, C.c_int],
        "gr_batch_solve": [vp, C.POINTER(GrSolveOpts), C.POINTER(C.c_int), C.POINTER(C.c_double),
                           C.POINTER(C.c_double)],
        "gr_batch_solve_patches": [vp, C.POINTER(GrSolveOpts), C.POINTER(C.c_int), C.POINTER(C.c_double),
                                   C.POINTER(C.c_double)],
        "gr_destroy_batch": [vp],
        "gr_unet_create": [C.POINTER(GrUnetDesc), C.c_int, C.POINTER(vp)],
        "gr_unet_workspace_bytes": [vp, C.POINTER(C.c_size_t)],
        "gr_unet_param_count": [vp, C.POINTER(C.c_int64)],
        "gr_unet_bind": [vp, vp, C.c_size_t, vp],
        "gr_unet_init": [vp, C.c_uint64],
        "gr_unet_set_params": [vp, vp],
        "gr_unet_get_params": [vp, vp],
        "gr_unet_forward": [vp, C.c_int, vp, vp],
        "gr_unet_loss_grad": [vp, C.c_int, vp, vp, vp, C.POINTER(C.c_double)],
        "gr_unet_train_step": [vp, C.c_int, vp, vp, C.c_float, C.POINTER(C.c_double)],
        "gr_destroy_unet": [vp],
        "gr_create_spectra": [C.c_int, C.c_int, C.POINTER(vp)],
        "gr_spectra_workspace_bytes": [vp, C.POINTER(C.c_size_t)],
        "gr_spectra_bind": [vp, vp, C.c_size_t, vp],
        "gr_vector_spectra": [vp, vp, vp, vp, C.POINTER(C.c_double)],
        "gr_spectra_fft": [vp, vp],
        "gr_destroy_spectra": [vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.gr_last_error.argtypes = []
    lib.gr_last_error.restype = C.c_char_p
    lib.gr_batch_last_error.argtypes = []
    lib.gr_batch_last_error.restype = C.c_char_p
    lib.gr_unet_last_error.argtypes = []
    lib.gr_unet_last_error.restype = C.c_char_p
    lib.gr_spectra_last_error.argtypes = []
    lib.gr_spectra_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().gr_last_error().decode()


def _check(code: int, allow=(OK,)):
    if code not in allow:
        raise GrError(code, last_error())
    return code


def batch_last_error() -> str:
    return load_library().gr_batch_last_error().decode()


def _bcheck(code: int, allow=(OK,)):
    if code not in allow:
        raise GrError(code, batch_last_error())
    return code


def _ptr(t) -> int:
    return t.data_ptr()


# ---- one function per ABI entry point ----

def default_opts(**kw) -> GrSolveOpts:
    o = GrSolveOpts()
    _check(load_library().gr_default_opts(C.byref(o)))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = {"fp64": FP64, "mixed": MIXED}[v]
        if k == "guess" and isinstance(v, str):
            v = {"zero": GUESS_ZERO, "current": GUESS_CURRENT, "checked": GUESS_CHECKED}[v]
        setattr(o, k, v)
    return o


def create_grid(n: int, a: float, omega_m: float, c_tilde: float, h: float | None = None) -> int:
    g = C.c_void_p()
    _check(load_library().gr_create_grid(C.byref(GrGridDesc(n, h if h is not None else 1.0 / n)),
                                         C.byref(GrParams(a, omega_m, c_tilde)), C.byref(g)))
    return g.value


def workspace_bytes(g: int) -> int:
    b = C.c_size_t()
    _check(load_library().gr_workspace_bytes(g, C.byref(b)))
    return b.value


def bind(g: int, workspace, stream: int) -> None:
    _check(load_library().gr_bind(g, _ptr(workspace), workspace.numel() * workspace.element_size(), stream))


def deposit_sources(g: int, pos, u, mass: float) -> None:
    _check(load_library().gr_deposit_sources(g, _ptr(pos), _ptr(u), float(mass), int(pos.shape[0])))


def set_field(g: int, field: int, src, dtype: int) -> None:
    _check(load_library().gr_set_field(g, field, _ptr(src), dtype))


def get_field(g: int, field: int, dst, dtype: int) -> None:
    _check(load_library().gr_get_field(g, field, _ptr(dst), dtype))


def solve_constraints(g: int, opts: GrSolveOpts, allow=(OK,)) -> GrSolveReport:
    r = GrSolveReport()
    _check(load_library().gr_solve_constraints(g, C.byref(opts), C.byref(r)), allow)
    return r


def solve_equation(g: int, kind: int, field: int, opts: GrSolveOpts, allow=(OK,)) -> GrSolveReport:
    r = GrSolveReport()
    _check(load_library().gr_solve_equation(g, kind, field, C.byref(opts), C.byref(r)), allow)
    return r


def solve_equation_static(n: int, a: float, omega_m: float, c_tilde: float, kind: int, f, coef, phi, stream: int,
                          opts: GrSolveOpts, allow=(OK,)) -> GrSolveReport:
    """Allocation-free solve of one equation: f, coef (may be None for
    Poisson) and phi are caller-owned float64 device tensors of n^3 values."""
    r = GrSolveReport()
    _check(load_library().gr_solve_equation_static(n, C.byref(GrParams(a, omega_m, c_tilde)), kind, _ptr(f),
                                                   _ptr(coef) if coef is not None else None, _ptr(phi),
                                                   C.byref(opts), stream, C.byref(r)), allow)
    return r


KICK_FORWARD, KICK_REVERSE = 0, 1


def kick(g: int, pos, u, dt: float, order: int) -> None:
    _check(load_library().gr_kick(g, _ptr(pos), _ptr(u), int(pos.shape[0]), float(dt), int(order)))


def drift(g: int, pos, u, dt: float) -> None:
    _check(load_library().gr_drift(g, _ptr(pos), _ptr(u), int(pos.shape[0]), float(dt)))


def newtonian_kick(g: int, pos, u, dt: float, opts: GrSolveOpts, allow=(OK,)) -> GrSolveReport:
    r = GrSolveReport()
    _check(load_library().gr_newtonian_kick(g, _ptr(pos), _ptr(u), int(pos.shape[0]), float(dt), C.byref(opts),
                                            C.byref(r)), allow)
    return r


def debug_sweep(g: int, kind: int, field: int, Fbar: float, fshift: float, nsweeps: int) -> None:
    _check(load_library().gr_debug_sweep(g, kind, field, Fbar, fshift, nsweeps))


def debug_residual(g: int, kind: int, field: int, Fbar: float, fshift: float, out) -> None:
    _check(load_library().gr_debug_residual(g, kind, field, Fbar, fshift, _ptr(out)))


def features(g: int, level: int, fields, offset, scale, out, flags: int = 0) -> None:
    k = len(fields)
    _check(load_library().gr_features(g, level, k, (C.c_int * k)(*fields), (C.c_double * k)(*offset),
                                      (C.c_double * k)(*scale), _ptr(out), flags))


def set_guess(g: int, level: int, fields, scale, src, flags: int) -> None:
    k = len(fields)
    _check(load_library().gr_set_guess(g, level, k, (C.c_int * k)(*fields), (C.c_double * k)(*scale), _ptr(src),
                                       flags))


def autotune(g: int) -> str:
    buf = C.create_string_buffer(8192)
    _check(load_library().gr_autotune(g, buf, len(buf)))
    return buf.value.decode()


def sweep_timing(g: int, enable: bool):
    """Start (enable=True) or stop timing of finest-level fused sweeps; on stop
    returns {kind: (launches, mean ms)}."""
    ms = (C.c_double * 6)()
    cnt = (C.c_int * 6)()
    _check(load_library().gr_sweep_timing(g, 1 if enable else 0, ms, cnt))
    if enable:
        return None
    return {k: (cnt[k], ms[k] / cnt[k]) for k in range(6) if cnt[k] > 0}


def destroy_grid(g: int) -> None:
    _check(load_library().gr_destroy_grid(g))


# ---- convenience owner of a grid + torch workspace ----

class Grid:
    """A periodic n^3 grid bound to a torch-allocated workspace on `device`."""

    def __init__(self, n: int, a: float = 1.0, omega_m: float = 0.3072, c_tilde: float = 2997.92458 / 256.0,
                 h: float | None = None, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.n = n
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU device (no CPU fallback)")
        self.handle = create_grid(n, a, omega_m, c_tilde, h)
        nbytes = workspace_bytes(self.handle)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        bind(self.handle, self.workspace, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "handle", None):
            destroy_grid(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, x, dtype):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(x)
        return x.to(device=self.device, dtype=dtype).contiguous()

    def deposit_sources(self, pos, u, mass):
        pos = self._dev(pos, self.torch.float64)
        u = self._dev(u, self.torch.float64)
        assert pos.shape == u.shape and pos.shape[-1] == 3
        deposit_sources(self.handle, pos, u, mass)

    def set_field(self, field, values):
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        v = values if isinstance(values, self.torch.Tensor) else self.torch.as_tensor(values)
        dt = F32 if v.dtype == self.torch.float32 else F64
        v = self._dev(v, self.torch.float32 if dt == F32 else self.torch.float64)
        assert v.numel() == self.n ** 3
        set_field(self.handle, fid, v, dt)
        self._keep = v  # keep alive until the stream has consumed it
        return v

    def get_field(self, field, dtype=None):
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        dtype = dtype or self.torch.float64
        out = self.torch.empty((self.n,) * 3, dtype=dtype, device=self.device)
        get_field(self.handle, fid, out, F32 if dtype == self.torch.float32 else F64)
        return out

    def solve_constraints(self, allow=(OK,), **kw):
        return solve_constraints(self.handle, default_opts(**kw), allow).as_dict()

    def solve_equation(self, kind, field, allow=(OK,), **kw):
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        return solve_equation(self.handle, kind, fid, default_opts(**kw), allow).as_dict()


# ---- batched solve ----

def create_batch(ns, a: float, omega_m: float, c_tilde: float, patches=()) -> int:
    """Periodic unit boxes of sides ns, then patches given as (n, h, parent, (ox, oy, oz))."""
    descs = (GrGridDesc * len(ns))(*[GrGridDesc(int(n), 1.0 / int(n)) for n in ns])
    g = C.c_void_p()
    prm = C.byref(GrParams(a, omega_m, c_tilde))
    if patches:
        pd = (GrPatchDesc * len(patches))(*[GrPatchDesc(int(n), float(h), int(par), (C.c_double * 3)(*map(float, o)))
                                            for n, h, par, o in patches])
        _bcheck(load_library().gr_create_batch_patches(descs, len(ns), pd, len(patches), prm, C.byref(g)))
    else:
        _bcheck(load_library().gr_create_batch(descs, len(ns), prm, C.byref(g)))
    return g.value


def batch_workspace_bytes(b: int) -> int:
    v = C.c_size_t()
    _bcheck(load_library().gr_batch_workspace_bytes(b, C.byref(v)))
    return v.value


def batch_bind(b: int, workspace, stream: int) -> None:
    _bcheck(load_library().gr_batch_bind(b, _ptr(workspace), workspace.numel() * workspace.element_size(), stream))


def batch_set_field(b: int, item: int, field: int, src, dtype: int) -> None:
    _bcheck(load_library().gr_batch_set_field(b, item, field, _ptr(src), dtype))


def batch_get_field(b: int, item: int, field: int, dst, dtype: int) -> None:
    _bcheck(load_library().gr_batch_get_field(b, item, field, _ptr(dst), dtype))


def batch_autotune(b: int) -> str:
    buf = C.create_string_buffer(8192)
    _bcheck(load_library().gr_batch_autotune(b, buf, len(buf)))
    return buf.value.decode()


def batch_debug_boundary(b: int, item: int, field: int, level: int, dst) -> None:
    _bcheck(load_library().gr_batch_debug_boundary(b, item, field, level, _ptr(dst)))


def batch_solve(b: int, count: int, opts: GrSolveOpts, allow=(OK,), patches_only: bool = False):
    cyc = (C.c_int * (10 * count))()
    rel = (C.c_double * (10 * count))()
    sec = (C.c_double * count)()
    lib = load_library()
    fn = lib.gr_batch_solve_patches if patches_only else lib.gr_batch_solve
    st = _bcheck(fn(b, C.byref(opts), cyc, rel, sec), allow)
    return st, [list(cyc[10 * i:10 * i + 10]) for i in range(count)], \
        [list(rel[10 * i:10 * i + 10]) for i in range(count)], list(sec)


def destroy_batch(b: int) -> None:
    _bcheck(load_library().gr_destroy_batch(b))


class Batch:
    """Many periodic boxes (sides ns) and Dirichlet refinement patches
    (n, h, parent, origin) solved together on `device`; items are the boxes,
    then the patches.  Uses its own non-default stream so that each cycle can
    be captured in a hipGraph."""

    def __init__(self, ns, a: float = 1.0, omega_m: float = 0.3072, c_tilde: float = 2997.92458 / 256.0,
                 device="cuda", patches=()):
        import torch

        self.torch = torch
        self.patches = [(int(n), float(h), int(p), tuple(map(float, o))) for n, h, p, o in patches]
        self.nbox = len(ns)
        self.ns = [int(n) for n in ns] + [q[0] for q in self.patches]
        self.device = torch.device(device)
        if self.device.type != "cuda" or not torch.cuda.is_available():
            raise RuntimeError("the HIP library needs a GPU device (no CPU fallback)")
        self.handle = create_batch(self.ns[:self.nbox], a, omega_m, c_tilde, self.patches)
        self.workspace = torch.empty(batch_workspace_bytes(self.handle), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.current_stream(self.device).synchronize()
        batch_bind(self.handle, self.workspace, self.stream.cuda_stream)
        self._keep = []

    def close(self):
        if getattr(self, "handle", None):
            destroy_batch(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_field(self, item, field, values):
        t = self.torch
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        v = values if isinstance(values, t.Tensor) else t.as_tensor(values)
        v = v.to(device=self.device, dtype=t.float64).contiguous()
        assert v.numel() == self.ns[item] ** 3
        t.cuda.current_stream(self.device).synchronize()
        batch_set_field(self.handle, item, fid, v, F64)
        self._keep.append(v)

    def get_field(self, item, field):
        t = self.torch
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        n = self.ns[item]
        out = t.empty((n, n, n), dtype=t.float64, device=self.device)
        batch_get_field(self.handle, item, fid, out, F64)
        self.stream.synchronize()
        return out

    def autotune(self) -> str:
        """Choose each (level, box side)'s smoothing form by timing them."""
        rep = batch_autotune(self.handle)
        self.stream.synchronize()
        return rep

    def debug_boundary(self, item, field, level):
        """Padded level `level` of patch `item` after writing its boundary values
        from the parent's current field."""
        t = self.torch
        fid = FIELD_IDS[field] if isinstance(field, str) else field
        m = self.ns[item] >> level
        out = t.empty((m + 2, m + 2, m + 2), dtype=t.float64, device=self.device)
        batch_debug_boundary(self.handle, item, fid, level, out)
        self.stream.synchronize()
        return out

    def solve(self, allow=(OK,), patches_only=False, **kw):
        """All items, or (patches_only) a sub-step of the patches from the kept
        fields of the boxes and of the patches above them."""
        st, cyc, rel, sec = batch_solve(self.handle, len(self.ns), default_opts(**kw), allow, patches_only)
        self._keep.clear()
        count = len(self.ns)
        fb = (C.c_int * (10 * count))()
        _bcheck(load_library().gr_batch_mixed_fallbacks(self.handle, fb))
        return dict(status=st, cycles=cyc, rel_res=rel, item_seconds=sec,
                    fallback=[list(fb[10 * i:10 * i + 10]) for i in range(count)])


# ---- learned initial guess network ----

def unet_last_error() -> str:
    return load_library().gr_unet_last_error().decode()


def _ucheck(code: int):
    if code != OK:
        raise GrError(code, unet_last_error())
    return code


class UNet:
    """The U-Net of the learned guess (see gr.h); device memory from torch."""

    def __init__(self, in_ch: int, out_ch: int, channels=(16, 32, 64, 64), max_n: int = 64, device="cuda",
                 stream=None, lap_weight: float = 0.0, clip_norm: float = 0.0):
        import torch

        self.torch = torch
        self.in_ch, self.out_ch, self.channels = in_ch, out_ch, tuple(channels)
        self.device = torch.device(device)
        lib = load_library()
        h = C.c_void_p()
        _ucheck(lib.gr_unet_create(C.byref(GrUnetDesc(in_ch, out_ch, (C.c_int * 4)(*channels), lap_weight,
                                                      clip_norm)), max_n, C.byref(h)))
        self.lap_weight = lap_weight
        self.handle = h.value
        nbytes, cnt = C.c_size_t(), C.c_int64()
        _ucheck(lib.gr_unet_workspace_bytes(self.handle, C.byref(nbytes)))
        _ucheck(lib.gr_unet_param_count(self.handle, C.byref(cnt)))
        self.nparam = cnt.value
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _ucheck(lib.gr_unet_bind(self.handle, self.workspace.data_ptr(), nbytes.value, self.stream.cuda_stream))

    def close(self):
        if getattr(self, "handle", None):
            load_library().gr_destroy_unet(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, x):
        t = self.torch
        x = x if isinstance(x, t.Tensor) else t.as_tensor(x)
        return x.to(device=self.device, dtype=t.float32).contiguous()

    def init(self, seed: int):
        _ucheck(load_library().gr_unet_init(self.handle, seed))

    def get_params(self):
        out = self.torch.empty(self.nparam, dtype=self.torch.float32, device=self.device)
        _ucheck(load_library().gr_unet_get_params(self.handle, out.data_ptr()))
        self.stream.synchronize()
        return out

    def set_params(self, p):
        p = self._f32(p)
        assert p.numel() == self.nparam
        _ucheck(load_library().gr_unet_set_params(self.handle, p.data_ptr()))
        self.stream.synchronize()

    def forward(self, x):
        x = self._f32(x)
        n = x.shape[-1]
        out = self.torch.empty((self.out_ch, n, n, n), dtype=self.torch.float32, device=self.device)
        _ucheck(load_library().gr_unet_forward(self.handle, n, x.data_ptr(), out.data_ptr()))
        self.stream.synchronize()
        return out

    def loss_grad(self, x, t):
        x, t = self._f32(x), self._f32(t)
        g = self.torch.empty(self.nparam, dtype=self.torch.float32, device=self.device)
        loss = C.c_double()
        _ucheck(load_library().gr_unet_loss_grad(self.handle, x.shape[-1], x.data_ptr(), t.data_ptr(), g.data_ptr(),
                                                 C.byref(loss)))
        self.stream.synchronize()
        return loss.value, g

    def train_step(self, x, t, lr: float) -> float:
        x, t = self._f32(x), self._f32(t)
        loss = C.c_double()
        _ucheck(load_library().gr_unet_train_step(self.handle, x.shape[-1], x.data_ptr(), t.data_ptr(), lr,
                                                  C.byref(loss)))
        return loss.value


# ---- vector-mode extraction ----

SPECTRA_ROWS = ("k", "count", "p_curl", "p_div", "p_vector", "p_scalar")


def spectra_last_error() -> str:
    return load_library().gr_spectra_last_error().decode()


def _scheck(code: int):
    if code != OK:
        raise GrError(code, spectra_last_error())
    return code


class Spectra:
    """Shell-binned curl / divergence power spectra of a 3-component field
    (see gr.h, gr_vector_spectra); workspace from torch."""

    def __init__(self, n: int, nbins: int | None = None, device="cuda", stream=None):
        import torch

        self.torch = torch
        self.n = n
        self.nbins = n // 8 if nbins is None else nbins
        self.device = torch.device(device)
        lib = load_library()
        h = C.c_void_p()
        _scheck(lib.gr_create_spectra(n, self.nbins, C.byref(h)))
        self.handle = h.value
        nbytes = C.c_size_t()
        _scheck(lib.gr_spectra_workspace_bytes(self.handle, C.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        _scheck(lib.gr_spectra_bind(self.handle, self.workspace.data_ptr(), nbytes.value, self.stream.cuda_stream))

    def _f64(self, x):
        t = self.torch
        x = x if isinstance(x, t.Tensor) else t.as_tensor(x)
        x = x.to(device=self.device, dtype=t.float64).contiguous()
        assert tuple(x.shape) == (self.n,) * 3
        return x

    def vector(self, vx, vy, vz):
        """[6][nbins] numpy array, rows SPECTRA_ROWS."""
        import numpy as np

        v = [self._f64(a) for a in (vx, vy, vz)]
        out = np.zeros(6 * self.nbins)
        _scheck(load_library().gr_vector_spectra(self.handle, v[0].data_ptr(), v[1].data_ptr(), v[2].data_ptr(),
                                                 out.ctypes.data_as(C.POINTER(C.c_double))))
        return out.reshape(6, self.nbins)

    def fft(self, data):
        """In-place forward 3-D FFT of a complex128 (n, n, n) device tensor."""
        assert data.dtype == self.torch.complex128 and data.is_contiguous() and tuple(data.shape) == (self.n,) * 3
        _scheck(load_library().gr_spectra_fft(self.handle, data.data_ptr()))
        self.stream.synchronize()
        return data

    def close(self):
        if getattr(self, "handle", None):
            load_library().gr_destroy_spectra(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
