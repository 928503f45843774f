"""ctypes binding of libtc.so (include/tc.h).  Argument marshalling only:
every step of the substep runs in the HIP kernels of the library.  The
binding refuses to load when the library has not been built."""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtc.so")

TC_OK, TC_EINVAL, TC_ENOMEM, TC_EDEVICE, TC_ENONFINITE, TC_ESHAPE = 0, -1, -2, -3, -4, -5
TC_PREC_FP64, TC_PREC_MIXED = 0, 1
TC_FLAG_LINEAR = 1
TC_FLAG_DRYRUN = 2
TC_FLAG_GENERIC_FFT = 4


class TcGeometry(ctypes.Structure):
    _fields_ = [
        ("radius_ratio", ctypes.c_double),
        ("gap", ctypes.c_double),
        ("re", ctypes.c_double),
        ("re_outer", ctypes.c_double),
        ("nr", ctypes.c_int),
        ("ntheta", ctypes.c_int),
        ("nz", ctypes.c_int),
        ("theta_period", ctypes.c_double),
        ("lz", ctypes.c_double),
        ("stretch", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("precision", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class TcStats(ctypes.Structure):
    _fields_ = [
        ("time", ctypes.c_double),
        ("torque_in", ctypes.c_double),
        ("torque_out", ctypes.c_double),
        ("tau_in", ctypes.c_double),
        ("tau_out", ctypes.c_double),
        ("retau_in", ctypes.c_double),
        ("retau_out", ctypes.c_double),
        ("energy", ctypes.c_double),
        ("energy_pert", ctypes.c_double),
        ("steps", ctypes.c_longlong),
        ("nonfinite", ctypes.c_int),
    ]


class TcError(RuntimeError):
    def __init__(self, code, message):
        super().__init__(f"libtc error {code}: {message}")
        self.code = code


_lib = None

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGNATURES = {
    "tc_abi_version": (ctypes.c_int, []),
    "tc_create": (ctypes.c_int, [ctypes.POINTER(TcGeometry), ctypes.c_int, ctypes.POINTER(_P)]),
    "tc_destroy": (ctypes.c_int, [_P]),
    "tc_set_stream": (ctypes.c_int, [_P, _P]),
    "tc_mode_shape": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "tc_grid": (ctypes.c_int, [_P, ctypes.c_int, _D]),
    "tc_load_fields": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, _D, _D]),
    "tc_get_fields": (ctypes.c_int, [_P, ctypes.c_int, _D, _D, _D, _D]),
    "tc_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_substep": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_velocity": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
    "tc_products": (ctypes.c_int, [_P, ctypes.c_int, _D]),
    "tc_profiles": (ctypes.c_int, [_P, ctypes.c_int, _D]),
    "tc_set_rhs_rows": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "tc_stats": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(TcStats)]),
    "tc_stats_noalloc": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(TcStats)]),
    "tc_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_use_graphs": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_set_rhs_elimination": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_autotune": (ctypes.c_int, [_P, ctypes.c_int]),
    "tc_tuning": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "tc_set_solve_shape": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "tc_set_tiles": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "tc_tiles": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int)]),
    "tc_kernel_times": (ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_longlong), ctypes.c_int]),
    "tc_kernel_count": (ctypes.c_int, []),
    "tc_kernel_name": (ctypes.c_char_p, [ctypes.c_int]),
    "tc_kernel_bytes": (ctypes.c_double, [_P, ctypes.c_int, ctypes.c_int]),
    "tc_coefficients": (ctypes.c_int, [_P, ctypes.c_int, _D, ctypes.POINTER(ctypes.c_int)]),
    "tc_last_error": (ctypes.c_char_p, [_P]),
}


def load_library(path=LIB_PATH):
    """Load libtc.so; raises ImportError when it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built: run `python -m paper_0711_1429_amd.build` "
                          "(or __graft_entry__.build()) first")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _dptr(a):
    return a.ctypes.data_as(_D)


def make_geometry(zeta, re, nr, ntheta, nz, dt, gap=1.0, re_outer=0.0, theta_period=0.0,
                  lz=0.0, stretch=0.0, precision=TC_PREC_FP64, flags=0):
    return TcGeometry(float(zeta), float(gap), float(re), float(re_outer), int(nr), int(ntheta),
                      int(nz), float(theta_period), float(lz), float(stretch), float(dt),
                      int(precision), int(flags))


class Solver:
    """One libtc context holding one or more Taylor--Couette instances."""

    def __init__(self, geometries):
        self.lib = load_library()
        if isinstance(geometries, TcGeometry):
            geometries = [geometries]
        arr = (TcGeometry * len(geometries))(*geometries)
        ctx = _P()
        rc = self.lib.tc_create(arr, len(geometries), ctypes.byref(ctx))
        if rc != TC_OK:
            raise TcError(rc, self.lib.tc_last_error(None).decode())
        self.ctx = ctx
        self.n_instances = len(geometries)

    # ------------------------------------------------------------- plumbing
    def _check(self, rc):
        if rc != TC_OK:
            raise TcError(rc, self.lib.tc_last_error(self.ctx).decode())

    def close(self):
        if getattr(self, "ctx", None):
            self.lib.tc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------------ ABI
    def set_stream(self, stream_handle):
        self._check(self.lib.tc_set_stream(self.ctx, _P(stream_handle)))

    def mode_shape(self, inst=0):
        nr, nj, nl = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tc_mode_shape(self.ctx, inst, ctypes.byref(nr), ctypes.byref(nj), ctypes.byref(nl)))
        return nr.value, nj.value, nl.value

    def grid(self, inst=0):
        nr = self.mode_shape(inst)[0]
        r = np.empty(nr)
        self._check(self.lib.tc_grid(self.ctx, inst, _dptr(r)))
        return r

    def coefficients(self, inst=0):
        nr = self.mode_shape(inst)[0]
        c = np.empty((5, nr, 5))
        s = np.empty(nr, dtype=np.int32)
        self._check(self.lib.tc_coefficients(self.ctx, inst, _dptr(c), s.ctypes.data_as(ctypes.POINTER(ctypes.c_int))))
        return c, s

    def load_fields(self, v_hat, eta_hat, u_mean, w_mean, inst=0):
        shape = self.mode_shape(inst)
        v = np.ascontiguousarray(v_hat, dtype=np.complex128)
        e = np.ascontiguousarray(eta_hat, dtype=np.complex128)
        um = np.ascontiguousarray(u_mean, dtype=np.float64)
        wm = np.ascontiguousarray(w_mean, dtype=np.float64)
        if v.shape != shape or e.shape != shape or um.shape != (shape[0],) or wm.shape != (shape[0],):
            raise ValueError(f"fields must have shape {shape} and ({shape[0]},)")
        self._check(self.lib.tc_load_fields(self.ctx, inst, v.ctypes.data_as(_D), e.ctypes.data_as(_D),
                                            _dptr(um), _dptr(wm)))

    def get_fields(self, inst=0):
        shape = self.mode_shape(inst)
        v = np.empty(shape, dtype=np.complex128)
        e = np.empty(shape, dtype=np.complex128)
        um = np.empty(shape[0])
        wm = np.empty(shape[0])
        self._check(self.lib.tc_get_fields(self.ctx, inst, v.ctypes.data_as(_D), e.ctypes.data_as(_D),
                                           _dptr(um), _dptr(wm)))
        return v, e, um, wm

    def step(self, nsteps=1):
        self._check(self.lib.tc_step(self.ctx, int(nsteps)))

    def substep(self, k):
        self._check(self.lib.tc_substep(self.ctx, int(k)))

    def velocity(self, inst=0):
        shape = self.mode_shape(inst)
        u = np.empty(shape, dtype=np.complex128)
        w = np.empty(shape, dtype=np.complex128)
        self._check(self.lib.tc_velocity(self.ctx, inst, u.ctypes.data_as(_D), w.ctypes.data_as(_D)))
        return u, w

    def products(self, inst=0):
        shape = self.mode_shape(inst)
        p = np.empty((6,) + shape, dtype=np.complex128)
        self._check(self.lib.tc_products(self.ctx, inst, p.ctypes.data_as(_D)))
        return dict(zip(("uu", "uv", "uw", "vv", "vw", "ww"), p))

    def profiles(self, inst=0):
        nr = self.mode_shape(inst)[0]
        out = np.empty((6, nr), dtype=np.float64)
        self._check(self.lib.tc_profiles(self.ctx, inst, out.ctypes.data_as(_D)))
        return dict(zip(("u_mean", "w_mean", "uu", "vv", "ww", "vw"), out))

    def stats(self, inst=0):
        s = TcStats()
        self._check(self.lib.tc_stats(self.ctx, inst, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in TcStats._fields_}

    def stats_noalloc(self, inst=0):
        s = TcStats()
        self._check(self.lib.tc_stats_noalloc(self.ctx, inst, ctypes.byref(s)))
        return {name: getattr(s, name) for name, _ in TcStats._fields_}

    def use_graphs(self, enable):
        self._check(self.lib.tc_use_graphs(self.ctx, int(bool(enable))))

    def set_rhs_elimination(self, enable):
        self._check(self.lib.tc_set_rhs_elimination(self.ctx, int(bool(enable))))

    def autotune(self, repeats=5):
        self._check(self.lib.tc_autotune(self.ctx, int(repeats)))

    def set_rhs_rows(self, rows, inst=0):
        self._check(self.lib.tc_set_rhs_rows(self.ctx, inst, int(rows)))

    def tuning(self, inst=0):
        rr, sh = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tc_tuning(self.ctx, inst, ctypes.byref(rr), ctypes.byref(sh)))
        return {"rhs_rows": rr.value, "solve_shape": sh.value}

    def set_solve_shape(self, code, inst=0):
        self._check(self.lib.tc_set_solve_shape(self.ctx, inst, int(code)))

    def set_tiles(self, zinv=0, theta=0, zfwd=0, inst=0):
        self._check(self.lib.tc_set_tiles(self.ctx, inst, int(zinv), int(theta), int(zfwd)))

    def tiles(self, inst=0):
        zi, th, zf = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tc_tiles(self.ctx, inst, ctypes.byref(zi), ctypes.byref(th), ctypes.byref(zf)))
        return {"zinv": zi.value, "theta": th.value, "zfwd": zf.value}

    def timing(self, enable):
        self._check(self.lib.tc_timing(self.ctx, int(bool(enable))))

    def kernel_times(self):
        n = self.lib.tc_kernel_count()
        ms = np.zeros(n)
        calls = np.zeros(n, dtype=np.int64)
        self._check(self.lib.tc_kernel_times(self.ctx, _dptr(ms),
                                             calls.ctypes.data_as(ctypes.POINTER(ctypes.c_longlong)), n))
        return {self.lib.tc_kernel_name(i).decode(): (float(ms[i]), int(calls[i])) for i in range(n)}

    def kernel_bytes(self, inst=0):
        n = self.lib.tc_kernel_count()
        return {self.lib.tc_kernel_name(i).decode(): self.lib.tc_kernel_bytes(self.ctx, inst, i) for i in range(n)}
