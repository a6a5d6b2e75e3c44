"""Python binding of the C ABI in include/mg.h (ctypes; argument marshalling only).

Every numerical step runs in the HIP library libmg.so next to this file.  If
the library is missing the binding raises: there is no CPU fallback.  torch
supplies device memory (complex128 CUDA tensors) and the stream.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmg.so")

MG_OK, MG_EINVAL, MG_ENOMEM, MG_EDEVICE, MG_ENOTCONV, MG_EDIVERGED = 0, -1, -2, -3, -4, -5
VARIANTS = {"add": 0, "hb": 1, "bpx": 2}
OMEGA_SCHEMES = {"const": 0, "jacobi": 1, "lgrid": 2, "exp": 3, "transition": 4, "two_phase": 5}
PRECISIONS = {"fp64": 0, "fp32_refine": 1}
DRIVERS = {"stationary": 0, "bicgstab": 1}
RESTRICT_FORMS = {"auto": 0, "fas": 1, "galerkin": 2}
SWEEPS = {"auto": 0, "generic": 1, "fused": 2}
FIELDS = {"u": 0, "b": 1, "sc": 2, "sf": 3, "si": 4}

EXPORTED = [
    "mg_params_default", "mg_setup", "mg_destroy", "mg_last_error", "mg_level_size", "mg_apply",
    "mg_rhs_from_nodal", "mg_set_rhs", "mg_set_solution", "mg_cycle", "mg_flush", "mg_get_level",
    "mg_precondition", "mg_precondition_apply", "mg_solve", "mg_residual_norm", "mg_grad_potential", "mg_time_sweeps",
    "mg_sweep_time", "mg_tiles", "mg_set_tile", "mg_autotune", "mg_batch_setup", "mg_batch_destroy",
    "mg_batch_problem", "mg_batch_cycle", "mg_batch_autotune", "mg_batch_configs", "mg_batch_solve",
    "mg_batch_trace", "mg_batch_get_trace", "mg_prolong", "mg_solve_nested", "mg_batch_set_spin_limit",
    "mg_residual_norm_noalloc", "mg_batch_precondition_apply", "mg_mc_setup", "mg_mc_destroy", "mg_mc_apply",
    "mg_mc_set_rhs", "mg_mc_set_solution", "mg_mc_cycle", "mg_mc_flush", "mg_batch_set_config",
    "mg_amr_setup", "mg_amr_destroy", "mg_amr_mark", "mg_amr_adapt", "mg_amr_interpolate", "mg_amr_get",
    "mg_amr_set_cells",
]


class MGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mg error {code}: {msg}")
        self.code = code


class c128(ctypes.Structure):
    _fields_ = [("re", ctypes.c_double), ("im", ctypes.c_double)]


class Params(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("level_min", ctypes.c_int), ("level_max", ctypes.c_int),
        ("theta", ctypes.c_double), ("phi", c128), ("phi_field", ctypes.c_void_p),
        ("variant", ctypes.c_int), ("omega_scheme", ctypes.c_int), ("omega", c128),
        ("omega_L", ctypes.c_int), ("precision", ctypes.c_int), ("conjugate", ctypes.c_int),
        ("restrict_form", ctypes.c_int), ("sweep", ctypes.c_int), ("inner_rtol", ctypes.c_double),
        ("layer_theta", ctypes.c_double), ("layer_width", ctypes.c_double), ("layer_faces", ctypes.c_int),
    ]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Loads libmg.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: run `python -m paper_1508_03954_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I = ctypes.c_int
    D = ctypes.c_double
    lib.mg_params_default.argtypes = [ctypes.POINTER(Params)]
    lib.mg_params_default.restype = None
    lib.mg_setup.argtypes = [ctypes.POINTER(Params), P, ctypes.POINTER(P)]
    lib.mg_destroy.argtypes = [P]
    lib.mg_destroy.restype = None
    lib.mg_last_error.restype = ctypes.c_char_p
    lib.mg_level_size.argtypes = [P, I]
    lib.mg_apply.argtypes = [P, P, P]
    lib.mg_rhs_from_nodal.argtypes = [P, P, P]
    lib.mg_set_rhs.argtypes = [P, P]
    lib.mg_set_solution.argtypes = [P, P]
    lib.mg_cycle.argtypes = [P, I, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mg_flush.argtypes = [P, P]
    lib.mg_get_level.argtypes = [P, I, I, P]
    lib.mg_precondition.argtypes = [P, P, P]
    lib.mg_precondition_apply.argtypes = [P, P, P, P]
    lib.mg_solve.argtypes = [P, P, P, D, I, I, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.mg_residual_norm.argtypes = [P, P, P, ctypes.POINTER(D)]
    lib.mg_residual_norm_noalloc.argtypes = [P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mg_grad_potential.argtypes = [P, P, P, P]
    lib.mg_prolong.argtypes = [P, I, P, P]
    lib.mg_solve_nested.argtypes = [P, P, P, I, D, D, I, I, ctypes.POINTER(I), ctypes.POINTER(D)]
    lib.mg_time_sweeps.argtypes = [P, I]
    lib.mg_tiles.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I)]
    lib.mg_set_tile.argtypes = [P, I]
    lib.mg_autotune.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mg_sweep_time.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(I)]
    lib.mg_batch_setup.argtypes = [ctypes.POINTER(Params), I, P, ctypes.POINTER(P)]
    lib.mg_batch_destroy.argtypes = [P]
    lib.mg_batch_destroy.restype = None
    lib.mg_batch_problem.argtypes = [P, I, ctypes.POINTER(P)]
    lib.mg_batch_cycle.argtypes = [P, I, ctypes.POINTER(D)]
    lib.mg_batch_autotune.argtypes = [P, I, ctypes.POINTER(I), ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.mg_batch_configs.argtypes = []
    lib.mg_batch_set_config.argtypes = [P, I]
    lib.mg_batch_set_spin_limit.argtypes = [P, ctypes.c_longlong]
    lib.mg_batch_trace.argtypes = [P, I]
    lib.mg_batch_get_trace.argtypes = [P, ctypes.POINTER(ctypes.c_longlong), I, ctypes.POINTER(I)]
    lib.mg_batch_solve.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), D, I, I, ctypes.POINTER(I),
                                   ctypes.POINTER(D)]
    lib.mg_batch_precondition_apply.argtypes = [P, ctypes.POINTER(P), ctypes.POINTER(P), ctypes.POINTER(P)]
    lib.mg_mc_setup.argtypes = [ctypes.POINTER(Params), I, ctypes.POINTER(c128), P, ctypes.POINTER(P)]
    lib.mg_mc_destroy.argtypes = [P]
    lib.mg_mc_destroy.restype = None
    lib.mg_mc_apply.argtypes = [P, P, P]
    lib.mg_mc_set_rhs.argtypes = [P, P]
    lib.mg_mc_set_solution.argtypes = [P, P]
    lib.mg_mc_cycle.argtypes = [P, I, ctypes.POINTER(D)]
    lib.mg_mc_flush.argtypes = [P, P]
    L = ctypes.c_longlong
    lib.mg_amr_setup.argtypes = [I, I, I, I, P, ctypes.POINTER(P)]
    lib.mg_amr_destroy.argtypes = [P]
    lib.mg_amr_destroy.restype = None
    lib.mg_amr_mark.argtypes = [P, I, P, P, c128, P, I, I, I, D, ctypes.POINTER(L), ctypes.POINTER(D)]
    lib.mg_amr_adapt.argtypes = [P, ctypes.POINTER(L)]
    lib.mg_amr_interpolate.argtypes = [P, I, P, P]
    lib.mg_amr_get.argtypes = [P, I, I, P]
    lib.mg_amr_set_cells.argtypes = [P, I, P]
    for name in EXPORTED:
        if name not in ("mg_params_default", "mg_destroy", "mg_last_error", "mg_batch_destroy", "mg_mc_destroy",
                        "mg_amr_destroy"):
            getattr(lib, name).restype = I
    _lib = lib
    return lib


def _check(rc: int, allow=()) -> int:
    if rc != MG_OK and rc not in allow:
        raise MGError(rc, load_library().mg_last_error().decode())
    return rc


def _ptr(t) -> int:
    return t.data_ptr()


def make_params(dim: int, level_max: int, level_min: int = 1, theta: float = 0.0, phi: complex = 0.0,
                phi_field=None, variant: str = "bpx", omega_scheme: str = "const", omega: complex = 0.6,
                omega_L: int = 1, precision: str = "fp64", conjugate: bool = False, restrict_form: str = "auto",
                sweep: str = "auto", inner_rtol: float = 0.0, layer=None):
    """mg_params from keyword values; returns (params, device phi field kept alive or None).
    layer: None or (angle, width, face bits) of an absorbing layer."""
    import torch
    lib = load_library()
    p = Params()
    lib.mg_params_default(ctypes.byref(p))
    p.dim, p.level_min, p.level_max = dim, level_min, level_max
    p.theta = theta
    p.phi = c128(complex(phi).real, complex(phi).imag)
    keep = None
    if phi_field is not None:
        keep = phi_field.to(device="cuda", dtype=torch.complex128).contiguous()
        p.phi_field = _ptr(keep)
    p.variant = VARIANTS[variant]
    p.omega_scheme = OMEGA_SCHEMES[omega_scheme]
    p.omega = c128(complex(omega).real, complex(omega).imag)
    p.omega_L = omega_L
    p.precision = PRECISIONS[precision]
    p.conjugate = 1 if conjugate else 0
    p.restrict_form = RESTRICT_FORMS[restrict_form]
    p.sweep = SWEEPS[sweep]
    p.inner_rtol = inner_rtol
    if layer is not None:
        p.layer_theta, p.layer_width, p.layer_faces = float(layer[0]), float(layer[1]), int(layer[2])
    return p, keep


class Solver:
    """One complex additive multilevel hierarchy on the unit hypercube."""

    def __init__(self, dim: int, level_max: int, level_min: int = 1, theta: float = 0.0,
                 phi: complex = 0.0, phi_field=None, variant: str = "bpx", omega_scheme: str = "const",
                 omega: complex = 0.6, omega_L: int = 1, precision: str = "fp64", conjugate: bool = False,
                 restrict_form: str = "auto", sweep: str = "auto", stream=None, inner_rtol: float = 0.0,
                 layer=None):
        import torch
        lib = load_library()
        p, keep = make_params(dim, level_max, level_min, theta, phi, phi_field, variant, omega_scheme, omega,
                              omega_L, precision, conjugate, restrict_form, sweep, inner_rtol, layer)
        self._phi_keep = keep
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        ctx = ctypes.c_void_p()
        _check(lib.mg_setup(ctypes.byref(p), self.stream.cuda_stream, ctypes.byref(ctx)))
        self._init_view(ctx, dim, level_min, level_max, self.stream, owned=True)

    @classmethod
    def _view(cls, ctx, dim, level_min, level_max, stream):
        """A Solver on a context owned by someone else (a Batch)."""
        obj = cls.__new__(cls)
        obj._phi_keep = None
        obj._init_view(ctx, dim, level_min, level_max, stream, owned=False)
        return obj

    def _init_view(self, ctx, dim, level_min, level_max, stream, owned):
        import torch
        self._torch = torch
        self._ctx = ctx
        self._owned = owned
        self._lib = load_library()
        self.stream = stream
        self.dim, self.level_min, self.level_max = dim, level_min, level_max
        self.n = 3 ** level_max + 1
        self.shape = (self.n,) * dim

    def close(self):
        if not getattr(self, "_owned", False):
            return
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            self._lib.mg_destroy(self._ctx)
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, shape=None, dtype=None):
        t = self._torch
        return t.zeros(shape or self.shape, dtype=dtype or t.complex128, device="cuda")

    def _as_dev(self, x):
        t = self._torch
        if not isinstance(x, t.Tensor):
            x = t.from_numpy(np.ascontiguousarray(x))
        x = x.to(device="cuda", dtype=t.complex128).contiguous()
        if tuple(x.shape) != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {tuple(x.shape)}")
        return x

    def level_size(self, level: int) -> int:
        return _check(self._lib.mg_level_size(self._ctx, level), allow=range(1, 1 << 30))

    def apply(self, x, out=None):
        x = self._as_dev(x)
        y = self._new() if out is None else out
        _check(self._lib.mg_apply(self._ctx, _ptr(x), _ptr(y)))
        return y

    def rhs_from_nodal(self, chi):
        chi = self._as_dev(chi)
        b = self._new()
        _check(self._lib.mg_rhs_from_nodal(self._ctx, _ptr(chi), _ptr(b)))
        return b

    def set_rhs(self, b):
        b = self._as_dev(b)
        _check(self._lib.mg_set_rhs(self._ctx, _ptr(b)))

    def set_solution(self, u):
        u = self._as_dev(u)
        _check(self._lib.mg_set_solution(self._ctx, _ptr(u)))

    def cycle(self, ncycles: int = 1, norms: bool = True):
        if not norms:
            _check(self._lib.mg_cycle(self._ctx, ncycles, None, None))
            return None
        rh = (ctypes.c_double * ncycles)()
        rm = (ctypes.c_double * ncycles)()
        _check(self._lib.mg_cycle(self._ctx, ncycles, rh, rm))
        return np.array(rh[:]), np.array(rm[:])

    def flush(self):
        u = self._new()
        _check(self._lib.mg_flush(self._ctx, _ptr(u)))
        return u

    def get_level(self, level: int, field: str):
        n = 3 ** level + 1
        out = self._new((n,) * self.dim)
        _check(self._lib.mg_get_level(self._ctx, level, FIELDS[field], _ptr(out)))
        return out

    def precondition(self, v):
        v = self._as_dev(v)
        z = self._new()
        _check(self._lib.mg_precondition(self._ctx, _ptr(v), _ptr(z)))
        return z

    def precondition_apply(self, v):
        """(z, y) with z = B v and y = H z (the Krylov driver's fused step)."""
        v = self._as_dev(v)
        z = self._new()
        y = self._new()
        _check(self._lib.mg_precondition_apply(self._ctx, _ptr(v), _ptr(z), _ptr(y)))
        return z, y

    def solve(self, b, u0=None, rtol: float = 1e-10, maxit: int = 500, driver: str = "bicgstab"):
        """Returns (u, iterations, relative residual, status code)."""
        b = self._as_dev(b)
        u = self._new() if u0 is None else self._as_dev(u0).clone()
        its = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        rc = self._lib.mg_solve(self._ctx, _ptr(b), _ptr(u), rtol, maxit, DRIVERS[driver],
                                ctypes.byref(its), ctypes.byref(rel))
        _check(rc, allow=(MG_ENOTCONV, MG_EDIVERGED))
        return u, its.value, rel.value, rc

    def prolong(self, uc, level: int):
        """P uc from level - 1 to `level` (a new complex128 tensor of that level's size)."""
        t = self._torch
        if not isinstance(uc, t.Tensor):
            uc = t.from_numpy(np.ascontiguousarray(uc))
        uc = uc.to(device="cuda", dtype=t.complex128).contiguous()
        if tuple(uc.shape) != (3 ** (level - 1) + 1,) * self.dim:
            raise ValueError(f"expected level {level - 1} shape, got {tuple(uc.shape)}")
        uf = self._new((3 ** level + 1,) * self.dim)
        _check(self._lib.mg_prolong(self._ctx, level, _ptr(uc), _ptr(uf)))
        return uf

    def solve_nested(self, chi, level_start: int, coarse_rtol: float = 1e-2, rtol: float = 1e-10,
                     maxit: int = 500, driver: str = "bicgstab"):
        """Nested solve from the nodal load chi (finest size): levels level_start ..
        level_max - 1 to coarse_rtol, each from the prolonged solution below, then
        the finest level to rtol.  Returns (u, finest iterations, relative residual, status)."""
        chi = self._as_dev(chi)
        u = self._new()
        its = ctypes.c_int(0)
        rel = ctypes.c_double(0.0)
        rc = self._lib.mg_solve_nested(self._ctx, _ptr(chi), _ptr(u), level_start, coarse_rtol, rtol, maxit,
                                       DRIVERS[driver], ctypes.byref(its), ctypes.byref(rel))
        _check(rc, allow=(MG_ENOTCONV, MG_EDIVERGED))
        return u, its.value, rel.value, rc

    def residual_norm(self, u, b) -> float:
        u, b = self._as_dev(u), self._as_dev(b)
        out = ctypes.c_double(0.0)
        _check(self._lib.mg_residual_norm(self._ctx, _ptr(u), _ptr(b), ctypes.byref(out)))
        return out.value

    def residual_norm_noalloc(self, u, b):
        """(|b - H u|_h, max |r|) without any device allocation: u and b must
        already be contiguous complex128 device tensors of the finest shape
        (nothing is converted or copied here)."""
        t = self._torch
        for x in (u, b):
            if (not isinstance(x, t.Tensor) or not x.is_cuda or x.dtype != t.complex128
                    or not x.is_contiguous() or tuple(x.shape) != self.shape):
                raise ValueError("residual_norm_noalloc needs contiguous complex128 device tensors of the finest shape")
        rh, rm = ctypes.c_double(0.0), ctypes.c_double(0.0)
        _check(self._lib.mg_residual_norm_noalloc(self._ctx, _ptr(u), _ptr(b), ctypes.byref(rh), ctypes.byref(rm)))
        return rh.value, rm.value

    def tiles(self):
        """(current tile, number of tile variants) of the fused sweep; (-1, 0) without one."""
        cur, cnt = ctypes.c_int(0), ctypes.c_int(0)
        _check(self._lib.mg_tiles(self._ctx, ctypes.byref(cur), ctypes.byref(cnt)))
        return cur.value, cnt.value

    def set_tile(self, tile: int):
        _check(self._lib.mg_set_tile(self._ctx, tile))

    def autotune(self, reps: int = 5):
        """Times every fused tile variant (state untouched); returns (best tile, best us, all us)."""
        _, cnt = self.tiles()
        best, us = ctypes.c_int(0), ctypes.c_double(0.0)
        times = (ctypes.c_double * max(cnt, 1))()
        _check(self._lib.mg_autotune(self._ctx, reps, ctypes.byref(best), ctypes.byref(us), times))
        return best.value, us.value, list(times[:cnt])

    def time_sweeps(self, enable: bool = True):
        _check(self._lib.mg_time_sweeps(self._ctx, 1 if enable else 0))

    def sweep_time(self):
        """(summed milliseconds, count) of the finest sweeps timed so far."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int(0)
        _check(self._lib.mg_sweep_time(self._ctx, ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def grad_potential(self, u, lam):
        u, lam = self._as_dev(u), self._as_dev(lam)
        g = self._new(dtype=self._torch.float64)
        _check(self._lib.mg_grad_potential(self._ctx, _ptr(u), _ptr(lam), _ptr(g)))
        return g


class Batch:
    """Independent problems advanced together by one persistent launch per cycle.

    `problems` is a list of dicts of Solver keyword arguments (dim, level_max,
    theta, phi, variant, omega, precision, ...; constant phi only).  The
    per-problem contexts are reachable as `batch.solvers[i]` (set_rhs,
    set_solution, get_level, flush, solve work on them as on a Solver)."""

    def __init__(self, problems, stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        self._lib = lib
        arr = (Params * len(problems))()
        for i, kw in enumerate(problems):
            kw = dict(kw)
            if kw.get("phi_field") is not None:
                raise ValueError("batched problems need a constant phi")
            p, _ = make_params(**kw)
            arr[i] = p
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        b = ctypes.c_void_p()
        _check(lib.mg_batch_setup(arr, len(problems), self.stream.cuda_stream, ctypes.byref(b)))
        self._b = b
        self.count = len(problems)
        self.solvers = []
        for i, kw in enumerate(problems):
            ctx = ctypes.c_void_p()
            _check(lib.mg_batch_problem(b, i, ctypes.byref(ctx)))
            self.solvers.append(Solver._view(ctx, kw["dim"], kw.get("level_min", 1), kw["level_max"], self.stream))

    def close(self):
        if getattr(self, "_b", None) is not None and self._b.value:
            self._lib.mg_batch_destroy(self._b)
            self._b = ctypes.c_void_p()
            self.solvers = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cycle(self, ncycles: int = 1, norms: bool = True):
        """ncycles batched cycles; returns an (ncycles, count) array of |r|_h (or None)."""
        if not norms:
            _check(self._lib.mg_batch_cycle(self._b, ncycles, None))
            return None
        res = (ctypes.c_double * (ncycles * self.count))()
        _check(self._lib.mg_batch_cycle(self._b, ncycles, res))
        return np.array(res[:]).reshape(ncycles, self.count)

    def autotune(self, reps: int = 3):
        """Times every configuration; returns (best, us per cycle, all times).
        Advances the problems' state."""
        cfg, us = ctypes.c_int(), ctypes.c_double()
        n = self._lib.mg_batch_configs()
        times = (ctypes.c_double * n)()
        _check(self._lib.mg_batch_autotune(self._b, reps, ctypes.byref(cfg), ctypes.byref(us), times))
        return cfg.value, us.value, list(times)

    def set_config(self, config: int):
        """Selects one of the autotuner's configurations (state kept)."""
        _check(self._lib.mg_batch_set_config(self._b, config))

    def trace(self, enable: bool = True):
        _check(self._lib.mg_batch_trace(self._b, 1 if enable else 0))

    def set_spin_limit(self, polls: int):
        """Bound of the kernel's dependency waits (tests of the error path)."""
        _check(self._lib.mg_batch_set_spin_limit(self._b, polls))

    def cycle_status(self, ncycles: int = 1) -> int:
        """ncycles batched cycles without norms; returns the status code
        (MG_OK or MG_EDEVICE when a dependency wait gave up)."""
        return _check(self._lib.mg_batch_cycle(self._b, ncycles, None), allow=(MG_EDEVICE,))

    def get_trace(self):
        """Last cycle's per-item record as an (items, 8) int64 array: problem,
        phase, tile, kind, wait start, ready, done (10 ns ticks), XCD << 16 | block."""
        cnt = ctypes.c_int()
        _check(self._lib.mg_batch_get_trace(self._b, None, 0, ctypes.byref(cnt)))
        buf = (ctypes.c_longlong * (8 * cnt.value))()
        _check(self._lib.mg_batch_get_trace(self._b, buf, cnt.value, ctypes.byref(cnt)))
        return np.array(buf[:], dtype=np.int64).reshape(cnt.value, 8)

    def precondition_apply(self, vs):
        """(zs, ys) with z_i = B_i v_i (one zero-start cycle) and y_i = H_i z_i,
        every problem in one persistent launch."""
        t = self._torch
        vs = [s._as_dev(v) for s, v in zip(self.solvers, vs)]
        zs = [t.zeros_like(v) for v in vs]
        ys = [t.zeros_like(v) for v in vs]
        n = self.count
        pv = (ctypes.c_void_p * n)(*[_ptr(v) for v in vs])
        pz = (ctypes.c_void_p * n)(*[_ptr(z) for z in zs])
        py = (ctypes.c_void_p * n)(*[_ptr(y) for y in ys])
        _check(self._lib.mg_batch_precondition_apply(self._b, pv, pz, py))
        return zs, ys

    def solve(self, bs, us, rtol: float = 1e-10, maxit: int = 500, driver: str = "bicgstab"):
        """Solves every problem (device complex128 tensors; us[i] initial guess,
        overwritten).  Returns (iterations, relative residuals, status)."""
        n = self.count
        pb = (ctypes.c_void_p * n)(*[_ptr(b) for b in bs])
        pu = (ctypes.c_void_p * n)(*[_ptr(u) for u in us])
        its = (ctypes.c_int * n)()
        rel = (ctypes.c_double * n)()
        rc = self._lib.mg_batch_solve(self._b, pb, pu, rtol, maxit, DRIVERS[driver], its, rel)
        _check(rc, allow=(MG_ENOTCONV, MG_EDIVERGED))
        return np.array(its[:]), np.array(rel[:]), rc


class MultiChannel:
    """Same-grid multichannel problem: nchan channels (one constant phi each)
    on one grid, every vector shaped (n,)*dim + (nchan,) complex128 (the
    channels of a vertex contiguous)."""

    def __init__(self, dim: int, level_max: int, phis, stream=None, **kw):
        import torch
        self._torch = torch
        lib = load_library()
        self._lib = lib
        p, _ = make_params(dim, level_max, **kw)
        self.nchan = len(phis)
        arr = (c128 * self.nchan)(*[c128(complex(f).real, complex(f).imag) for f in phis])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        m = ctypes.c_void_p()
        _check(lib.mg_mc_setup(ctypes.byref(p), self.nchan, arr, self.stream.cuda_stream, ctypes.byref(m)))
        self._m = m
        self.dim, self.level_max = dim, level_max
        self.n = 3 ** level_max + 1
        self.shape = (self.n,) * dim + (self.nchan,)

    def close(self):
        if getattr(self, "_m", None) is not None and self._m.value:
            self._lib.mg_mc_destroy(self._m)
            self._m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _as_dev(self, x):
        t = self._torch
        if not isinstance(x, t.Tensor):
            x = t.from_numpy(np.ascontiguousarray(x))
        x = x.to(device="cuda", dtype=t.complex128).contiguous()
        if tuple(x.shape) != self.shape:
            raise ValueError(f"expected shape {self.shape}, got {tuple(x.shape)}")
        return x

    def apply(self, x):
        x = self._as_dev(x)
        y = self._torch.zeros_like(x)
        _check(self._lib.mg_mc_apply(self._m, _ptr(x), _ptr(y)))
        return y

    def set_rhs(self, b):
        b = self._as_dev(b)
        _check(self._lib.mg_mc_set_rhs(self._m, _ptr(b)))

    def set_solution(self, u):
        u = self._as_dev(u)
        _check(self._lib.mg_mc_set_solution(self._m, _ptr(u)))

    def cycle(self, ncycles: int = 1, norms: bool = True):
        """ncycles cycles; an (ncycles, nchan) array of |r|_h per channel (or None)."""
        if not norms:
            _check(self._lib.mg_mc_cycle(self._m, ncycles, None))
            return None
        res = (ctypes.c_double * (ncycles * self.nchan))()
        _check(self._lib.mg_mc_cycle(self._m, ncycles, res))
        return np.array(res[:]).reshape(ncycles, self.nchan)

    def flush(self):
        u = self._torch.zeros(self.shape, dtype=self._torch.complex128, device="cuda")
        _check(self._lib.mg_mc_flush(self._m, _ptr(u)))
        return u


AMR_CLASSES = {"absent": 0, "persistent": 1, "hanging": 2, "boundary": 3}
AMR_MARKS = {"keep": 0, "refine": 1, "erase": 2}


class Adapt:
    """Feature-based adaptivity state of a dense envelope of levels
    level_min..level_max (one refined flag per cell, one class per vertex)."""

    def __init__(self, dim: int, level_min: int, level_keep: int, level_max: int, stream=None):
        import torch
        self._torch = torch
        lib = load_library()
        self._lib = lib
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        a = ctypes.c_void_p()
        _check(lib.mg_amr_setup(dim, level_min, level_keep, level_max, self.stream.cuda_stream, ctypes.byref(a)))
        self._a = a
        self.dim, self.level_min, self.level_keep, self.level_max = dim, level_min, level_keep, level_max

    def close(self):
        if getattr(self, "_a", None) is not None and self._a.value:
            self._lib.mg_amr_destroy(self._a)
            self._a = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def n(self, level: int) -> int:
        return 3 ** level + 1

    def _field(self, x, level):
        t = self._torch
        if not isinstance(x, t.Tensor):
            x = t.from_numpy(np.ascontiguousarray(x))
        x = x.to(device="cuda", dtype=t.complex128).contiguous()
        if tuple(x.shape) != (self.n(level),) * self.dim:
            raise ValueError(f"expected shape {(self.n(level),) * self.dim}, got {tuple(x.shape)}")
        return x

    def mark(self, level: int, u, r=None, diag=1.0, nbins: int = 20, refine_pct: int = 10,
             erase_pct: int = 2, veto: float = 1e-2, stats: bool = True):
        """Marks a level; diag is a constant or a per-vertex field of the
        level's diagonal; returns a dict of the statistics (or None)."""
        u = self._field(u, level)
        rp = None
        if r is not None:
            r = self._field(r, level)
            rp = _ptr(r)
        dp, d = None, 1.0 + 0j
        if isinstance(diag, self._torch.Tensor):
            scalar = diag.dim() == 0
        else:
            scalar = np.ndim(diag) == 0
        if scalar:
            d = complex(diag)
        else:
            diag = self._field(diag, level)
            dp = _ptr(diag)
        if not stats:
            _check(self._lib.mg_amr_mark(self._a, level, _ptr(u), rp, c128(d.real, d.imag), dp, nbins, refine_pct,
                                         erase_pct, veto, None, None))
            return None
        cnt = (ctypes.c_longlong * (nbins + 5))()
        rng = (ctypes.c_double * 2)()
        _check(self._lib.mg_amr_mark(self._a, level, _ptr(u), rp, c128(d.real, d.imag), dp, nbins, refine_pct,
                                     erase_pct, veto, cnt, rng))
        c = list(cnt)
        return dict(counts=np.array(c[:nbins], dtype=np.int64), k=c[nbins], e=c[nbins + 1], n=c[nbins + 2],
                    refined=c[nbins + 3], erased=c[nbins + 4], s_min=rng[0], s_max=rng[1])

    def adapt(self, counts: bool = True):
        """One adaptation step; per level (absent, persistent, hanging, boundary) counts or None."""
        if not counts:
            _check(self._lib.mg_amr_adapt(self._a, None))
            return None
        nl = self.level_max - self.level_min + 1
        out = (ctypes.c_longlong * (4 * nl))()
        _check(self._lib.mg_amr_adapt(self._a, out))
        return {l: tuple(out[4 * (l - self.level_min):4 * (l - self.level_min) + 4])
                for l in range(self.level_min, self.level_max + 1)}

    def interpolate(self, level: int, u_coarse, u):
        """In place on the device tensor u (level `level`); returns u."""
        uc = self._field(u_coarse, level - 1)
        if not (isinstance(u, self._torch.Tensor) and u.is_cuda and u.dtype == self._torch.complex128
                and u.is_contiguous() and tuple(u.shape) == (self.n(level),) * self.dim):
            raise ValueError("u must be a contiguous complex128 device tensor of the level's shape")
        _check(self._lib.mg_amr_interpolate(self._a, level, _ptr(uc), _ptr(u)))
        return u

    def get(self, level: int, what: str):
        """'classes', 'classes_old', 'cells' or 'marks' of a level (uint8 device tensor)."""
        t = self._torch
        code = {"classes": 0, "classes_old": 1, "cells": 2, "marks": 3}[what]
        shape = (3 ** level,) * self.dim if code == 2 else (self.n(level),) * self.dim
        out = t.empty(shape, dtype=t.uint8, device="cuda")
        _check(self._lib.mg_amr_get(self._a, level, code, _ptr(out)))
        self.stream.synchronize()
        return out

    def set_cells(self, level: int, cells):
        t = self._torch
        if not isinstance(cells, t.Tensor):
            cells = t.from_numpy(np.ascontiguousarray(cells, dtype=np.uint8))
        cells = cells.to(device="cuda", dtype=t.uint8).contiguous()
        if tuple(cells.shape) != (3 ** level,) * self.dim:
            raise ValueError("cells must have (3^level,)*dim entries")
        _check(self._lib.mg_amr_set_cells(self._a, level, _ptr(cells)))
        self.stream.synchronize()
