"""Thin ctypes binding of libhermite_wave.so (include/hermite_wave.h).

Argument marshalling only: every half step runs in the library's HIP kernels.
PyTorch supplies device memory (float64 CUDA tensors) and the stream handle.
There is no fallback: if the library is missing the import of this module works
but every call raises :class:`LibraryMissing`.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhermite_wave.so")

HW_OK, HW_EINVAL, HW_ECFL, HW_ENOMEM, HW_EUNSUPPORTED, HW_EHIP, HW_ESTATE = 0, -1, -2, -3, -4, -5, -6
HW_DISS_FULL, HW_DISS_SIMPLE, HW_CONSERVATIVE = 0, 1, 2
HW_PERIODIC, HW_DIRICHLET, HW_NEUMANN = 0, 1, 2
HW_FP64, HW_FP32, HW_BF16 = 0, 1, 2
HW_KERNEL_AUTO, HW_KERNEL_GENERIC, HW_KERNEL_TILED, HW_KERNEL_SPLIT, HW_KERNEL_DENSE, HW_KERNEL_COMPOSED = 0, 1, 2, 3, 4, 5
HW_KERNEL_BATCH = 6
HW_PRIMAL, HW_DUAL = 0, 1

STATUS_NAMES = {0: "HW_OK", -1: "HW_EINVAL", -2: "HW_ECFL", -3: "HW_ENOMEM",
                -4: "HW_EUNSUPPORTED", -5: "HW_EHIP", -6: "HW_ESTATE"}

# every entry point declared in include/hermite_wave.h
ENTRY_POINTS = ["hw_create", "hw_destroy", "hw_layout", "hw_set_state", "hw_cons_startup",
                "hw_advance", "hw_prepare_advance", "hw_half_steps", "hw_half_step_forced", "hw_half_step_ext", "hw_get_state", "hw_state_grid", "hw_energy",
                "hw_energy_noalloc",
                "hw_time", "hw_last_error", "hw_tuning_report", "hw_probe_stream_triad", "hw_probe_mfma", "hw_probe_coexec", "hw_batch_create", "hw_batch_layout",
                "hw_batch_set_state", "hw_batch_cons_startup", "hw_batch_advance",
                "hw_batch_get_state"]


class LibraryMissing(RuntimeError):
    pass


class HwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class hw_problem(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("m", ctypes.c_int), ("n", ctypes.c_int * 3),
                ("xl", ctypes.c_double * 3), ("xr", ctypes.c_double * 3),
                ("c", ctypes.c_double), ("dt", ctypes.c_double), ("bc", ctypes.c_int * 3),
                ("method", ctypes.c_int), ("precision", ctypes.c_int),
                ("taylor_stages", ctypes.c_int), ("kernel", ctypes.c_int)]


_lib = None


def lib():
    """Load the library (raises LibraryMissing if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} not built: run paper_1802_05246_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, pp = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(hw_problem)
        i64p = ctypes.POINTER(ctypes.c_int64)
        ip = ctypes.POINTER(ctypes.c_int)
        sig = {
            "hw_create": ([pp, ctypes.POINTER(vp)], ctypes.c_int),
            "hw_destroy": ([vp], None),
            "hw_layout": ([vp, ctypes.c_int, i64p, ip, ip], ctypes.c_int),
            "hw_set_state": ([vp, dp, dp, vp], ctypes.c_int),
            "hw_cons_startup": ([vp, dp, dp, vp], ctypes.c_int),
            "hw_advance": ([vp, ctypes.c_int, vp], ctypes.c_int),
            "hw_half_steps": ([vp, ctypes.c_int, vp], ctypes.c_int),
            "hw_prepare_advance": ([vp, ctypes.c_int], ctypes.c_int),
            "hw_half_step_forced": ([vp, dp, ctypes.c_int, vp], ctypes.c_int),
            "hw_half_step_ext": ([vp, dp, ctypes.c_int, dp, dp, vp], ctypes.c_int),
            "hw_get_state": ([vp, dp, dp, vp], ctypes.c_int),
            "hw_state_grid": ([vp], ctypes.c_int),
            "hw_energy": ([vp, ctypes.POINTER(ctypes.c_double), vp], ctypes.c_int),
            "hw_energy_noalloc": ([vp, dp, vp], ctypes.c_int),
            "hw_time": ([vp], ctypes.c_double),
            "hw_last_error": ([], ctypes.c_char_p),
            "hw_tuning_report": ([], ctypes.c_char_p),
            "hw_probe_stream_triad": ([ctypes.c_int64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "hw_probe_mfma": ([ctypes.c_int, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "hw_probe_coexec": ([ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "hw_batch_create": ([pp, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
            "hw_batch_layout": ([vp, ctypes.c_int, ctypes.c_int, i64p, ip, ip], ctypes.c_int),
            "hw_batch_set_state": ([vp, ctypes.c_int, dp, dp, vp], ctypes.c_int),
            "hw_batch_cons_startup": ([vp, ctypes.c_int, dp, dp, vp], ctypes.c_int),
            "hw_batch_advance": ([vp, ctypes.c_int, vp], ctypes.c_int),
            "hw_batch_get_state": ([vp, ctypes.c_int, dp, dp, vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def hw_probe_stream_triad(n: int) -> float:
    g = ctypes.c_double()
    _check(lib().hw_probe_stream_triad(int(n), ctypes.byref(g)))
    return g.value


def hw_probe_mfma(precision: int) -> float:
    t = ctypes.c_double()
    _check(lib().hw_probe_mfma(int(precision), ctypes.byref(t)))
    return t.value


def hw_probe_coexec():
    """(products only, FMAs only, both) in ms per launch: see include/hermite_wave.h."""
    out = (ctypes.c_double * 3)()
    _check(lib().hw_probe_coexec(out))
    return tuple(out)


def hw_tuning_report() -> str:
    return lib().hw_tuning_report().decode()


def last_error() -> str:
    return lib().hw_last_error().decode()


def _check(status):
    if status != HW_OK:
        raise HwError(status, last_error())


def make_problem(spec, precision=HW_FP64, kernel=HW_KERNEL_AUTO) -> hw_problem:
    """hw_problem from a workloads.Spec-like object."""
    p = hw_problem()
    d = spec.d
    p.d, p.m = d, spec.m
    p.n[:] = list(spec.n) + [1] * (3 - d)
    p.xl[:] = list(spec.xl) + [0.0] * (3 - d)
    p.xr[:] = list(spec.xr) + [1.0] * (3 - d)
    p.c, p.dt = spec.c, spec.dt
    p.bc[:] = list(spec.bc) + [0] * (3 - d)
    p.method = spec.method
    p.precision = precision
    p.taylor_stages = getattr(spec, "taylor_stages", 0)
    p.kernel = kernel
    return p


def _stream(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return ctypes.c_void_p(int(stream))


def _ptr(t):
    if t is None:
        return None
    import torch
    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "float64 contiguous CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


# ---- same names as the C ABI -------------------------------------------------
def hw_create(problem: hw_problem):
    h = ctypes.c_void_p()
    _check(lib().hw_create(ctypes.byref(problem), ctypes.byref(h)))
    return h


def hw_batch_create(problems):
    arr = (hw_problem * len(problems))(*problems)
    h = ctypes.c_void_p()
    _check(lib().hw_batch_create(arr, len(problems), ctypes.byref(h)))
    return h


def hw_destroy(h):
    lib().hw_destroy(h)


def hw_layout(h, grid, i=None):
    n = ctypes.c_int64()
    nu, nv = ctypes.c_int(), ctypes.c_int()
    if i is None:
        _check(lib().hw_layout(h, grid, ctypes.byref(n), ctypes.byref(nu), ctypes.byref(nv)))
    else:
        _check(lib().hw_batch_layout(h, i, grid, ctypes.byref(n), ctypes.byref(nu), ctypes.byref(nv)))
    return n.value, nu.value, nv.value


def hw_set_state(h, u, w, stream=None):
    _check(lib().hw_set_state(h, _ptr(u), _ptr(w), _stream(stream)))


def hw_batch_set_state(h, i, u, w, stream=None):
    _check(lib().hw_batch_set_state(h, i, _ptr(u), _ptr(w), _stream(stream)))


def hw_cons_startup(h, u0, v0=None, stream=None):
    _check(lib().hw_cons_startup(h, _ptr(u0), _ptr(v0), _stream(stream)))


def hw_batch_cons_startup(h, i, u0, v0=None, stream=None):
    _check(lib().hw_batch_cons_startup(h, i, _ptr(u0), _ptr(v0), _stream(stream)))


def hw_advance(h, n, stream=None):
    _check(lib().hw_advance(h, n, _stream(stream)))


def hw_batch_advance(h, n, stream=None):
    _check(lib().hw_batch_advance(h, n, _stream(stream)))


def hw_prepare_advance(h, n):
    _check(lib().hw_prepare_advance(h, n))


def hw_half_steps(h, n, stream=None):
    _check(lib().hw_half_steps(h, n, _stream(stream)))


def hw_half_step_forced(h, f_coef, n_orders, stream=None):
    _check(lib().hw_half_step_forced(h, _ptr(f_coef), n_orders, _stream(stream)))


def hw_half_step_ext(h, f_coef, n_orders, wall_u, wall_v, stream=None):
    _check(lib().hw_half_step_ext(h, _ptr(f_coef), n_orders, _ptr(wall_u), _ptr(wall_v), _stream(stream)))


def hw_get_state(h, u, w, stream=None):
    _check(lib().hw_get_state(h, _ptr(u), _ptr(w), _stream(stream)))


def hw_batch_get_state(h, i, u, w, stream=None):
    _check(lib().hw_batch_get_state(h, i, _ptr(u), _ptr(w), _stream(stream)))


def hw_state_grid(h) -> int:
    return int(lib().hw_state_grid(h))


def hw_energy(h, stream=None) -> float:
    e = ctypes.c_double()
    _check(lib().hw_energy(h, ctypes.byref(e), _stream(stream)))
    return e.value


def hw_energy_noalloc(h, e_out_device, stream=None):
    """e_out_device: a float64 CUDA tensor with at least one element; the energy is
    written to its first element asynchronously on the stream."""
    _check(lib().hw_energy_noalloc(h, _ptr(e_out_device), _stream(stream)))


def hw_time(h) -> float:
    return float(lib().hw_time(h))


# ---- convenience wrapper ---------------------------------------------------------
class Solver:
    """One problem (or, with `problems`, a batch) on the current HIP device."""

    def __init__(self, spec=None, precision=HW_FP64, kernel=HW_KERNEL_AUTO, problems=None):
        import torch
        self.torch = torch
        if problems is not None:
            self.specs = list(problems)
            self.h = hw_batch_create([make_problem(s, precision, kernel) for s in self.specs])
        else:
            self.specs = [spec]
            self.h = hw_create(make_problem(spec, precision, kernel))
        self.batch = problems is not None

    def close(self):
        if self.h:
            hw_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def layout(self, grid, i=0):
        return hw_layout(self.h, grid, i if self.batch else None)

    def _dev(self, a):
        t = self.torch
        if isinstance(a, t.Tensor):
            return a.to(device="cuda", dtype=t.float64).contiguous()
        return t.as_tensor(a, dtype=t.float64, device="cuda").contiguous()

    def set_state(self, u, w, i=0):
        u, w = self._dev(u), self._dev(w)
        if self.batch:
            hw_batch_set_state(self.h, i, u, w)
        else:
            hw_set_state(self.h, u, w)
        self.torch.cuda.current_stream().synchronize()

    def cons_startup(self, u0, v0=None, i=0):
        u0 = self._dev(u0)
        v0 = None if v0 is None else self._dev(v0)
        if self.batch:
            hw_batch_cons_startup(self.h, i, u0, v0)
        else:
            hw_cons_startup(self.h, u0, v0)

    def advance(self, n):
        (hw_batch_advance if self.batch else hw_advance)(self.h, n)

    def half_steps(self, n):
        hw_half_steps(self.h, n)

    def half_step_forced(self, f_coef):
        """One half step with forcing coefficients of shape (n_out, R, (2m)^d) (see
        hw_half_step_forced); None or R = 0: no forcing."""
        if f_coef is None:
            hw_half_step_forced(self.h, None, 0)
            return
        f = self._dev(f_coef)
        hw_half_step_forced(self.h, f, int(f.shape[1]))
        self.torch.cuda.current_stream().synchronize()

    def half_step_ext(self, f_coef=None, wall_u=None, wall_v=None):
        """One half step with forcing coefficients of shape (n_out, R, K^d) and / or wall
        records (see hw_half_step_ext); None: no forcing / homogeneous walls."""
        f = None if f_coef is None else self._dev(f_coef)
        wu = None if wall_u is None else self._dev(wall_u)
        wv = None if wall_v is None else self._dev(wall_v)
        hw_half_step_ext(self.h, f, 0 if f is None else int(f.shape[1]), wu, wv)
        self.torch.cuda.current_stream().synchronize()

    def state_grid(self):
        return hw_state_grid(self.h)

    def get_state(self, i=0):
        """(u, v) of the state grid (dissipative) or (u_primal, u_dual)
        (conservative), as float64 CUDA tensors."""
        t = self.torch
        spec = self.specs[i]
        cons = spec.method == HW_CONSERVATIVE
        if cons:
            g0, g1 = HW_PRIMAL, HW_DUAL
        else:
            g0 = g1 = hw_state_grid(self.h)
        n0, nu, nv = self.layout(g0, i)
        n1, _, _ = self.layout(g1, i)
        u = t.empty((n0, nu), dtype=t.float64, device="cuda")
        w = t.empty((n1, nu if cons else nv), dtype=t.float64, device="cuda")
        if self.batch:
            hw_batch_get_state(self.h, i, u, w)
        else:
            hw_get_state(self.h, u, w)
        t.cuda.current_stream().synchronize()
        return u, w

    def energy(self):
        return hw_energy(self.h)

    def time(self):
        return hw_time(self.h)
