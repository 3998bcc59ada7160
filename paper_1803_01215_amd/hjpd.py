"""ctypes binding of libhjpd (the C ABI declared in include/hjpd.h).

The functions below carry the C names and only marshal arguments: torch
tensors (device memory) become raw pointers, the stream becomes a
hipStream_t.  Every step of the solve runs in the library's HIP kernels; if
the library is missing, loading raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libhjpd.so")

HJPD_OK, HJPD_EINVAL, HJPD_ENOMEM, HJPD_EDEVICE, HJPD_EUNSUPPORTED = 0, 1, 2, 3, 4
HJPD_PT_CONVERGED, HJPD_PT_MAXITER, HJPD_PT_NONFINITE, HJPD_PT_BADINPUT, HJPD_PT_VALUE_STALLED = 0, 1, 2, 3, 4
HJPD_H_CNORM, HJPD_H_QUADROTOR, HJPD_H_PURSUIT_EVASION, HJPD_H_LINEAR_TANH, HJPD_H_ISAACS = 0, 1, 2, 3, 4
HJPD_G_NORM, HJPD_G_QUAD_SHIFT, HJPD_G_PAIR_DIST, HJPD_G_QUAD_FORM, HJPD_G_SADDLE_QUAD = 0, 1, 2, 3, 4
HJPD_F32, HJPD_F64 = 0, 1
HJPD_PERSISTENT, HJPD_PLAIN, HJPD_FIXED_ITERS, HJPD_GRAPH, HJPD_TIMING, HJPD_NO_ORDER_HINT, HJPD_HOPF = (
    0, 1, 2, 4, 8, 16, 32)
HJPD_FORWARD_EULER, HJPD_TRAPEZOID, HJPD_NO_REFILL = 64, 128, 256

EXPORTED = ["hjpd_create", "hjpd_solve_batch", "hjpd_solve_batch_noalloc", "hjpd_value_grad", "hjpd_autotune",
            "hjpd_get_timing", "hjpd_get_launch_timing", "hjpd_set_plan", "hjpd_get_plan", "hjpd_set_pop_counter",
            "hjpd_calibrate_fma", "hjpd_destroy", "hjpd_last_error"]


class HjpdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hjpd error %d: %s" % (code, msg))
        self.code = code


class hjpd_desc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("d_y", ctypes.c_int), ("H", ctypes.c_int), ("g", ctypes.c_int),
                ("dtype", ctypes.c_int), ("N_max", ctypes.c_int), ("sigma", ctypes.c_double),
                ("tau", ctypes.c_double), ("theta", ctypes.c_double), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("seed", ctypes.c_uint64), ("flags", ctypes.c_uint),
                ("lanes_per_point", ctypes.c_int), ("nodes_per_lane", ctypes.c_int), ("starts", ctypes.c_int),
                ("restarts", ctypes.c_int), ("sigma_inc", ctypes.c_double), ("value_tol", ctypes.c_double)]


_lib = None


def load():
    """Load libhjpd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libhjpd.so not built: run __graft_entry__.build() or "
                              "python paper_1803_01215_amd/build.py")
        # The library and torch must run on one HIP runtime.  Both depend on
        # libamdhip64.so.7 and a process keeps the first copy it loads; torch
        # ships its own, so it is loaded first.  Were the system copy loaded
        # first (by this library), torch would find no GPU, and tensors it
        # allocated could not be handed to the library's kernels.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32p = ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p
        lib.hjpd_create.argtypes = [ctypes.POINTER(hjpd_desc), ctypes.POINTER(ctypes.c_void_p)]
        lib.hjpd_create.restype = ctypes.c_int
        lib.hjpd_solve_batch.argtypes = [vp, i64, vp, vp, i32p, vp, vp, vp, vp, vp, i32p, i32p, vp]
        lib.hjpd_solve_batch.restype = ctypes.c_int
        lib.hjpd_solve_batch_noalloc.argtypes = lib.hjpd_solve_batch.argtypes
        lib.hjpd_solve_batch_noalloc.restype = ctypes.c_int
        lib.hjpd_value_grad.argtypes = [vp, i64, vp, vp, i32p, vp, vp, vp, ctypes.c_int, ctypes.c_int, vp, vp, vp,
                                        vp, vp]
        lib.hjpd_value_grad.restype = ctypes.c_int
        lib.hjpd_autotune.argtypes = [vp, i64, vp, vp, i32p, vp, vp, vp, i32p, i32p, ctypes.c_int, vp]
        lib.hjpd_autotune.restype = ctypes.c_int
        lib.hjpd_get_timing.argtypes = [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        lib.hjpd_get_timing.restype = ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        lib.hjpd_get_launch_timing.argtypes = [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ip, ip, ip, ip]
        lib.hjpd_get_launch_timing.restype = ctypes.c_int
        lib.hjpd_set_pop_counter.argtypes = [vp, vp]
        lib.hjpd_set_pop_counter.restype = ctypes.c_int
        lib.hjpd_set_plan.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        lib.hjpd_set_plan.restype = ctypes.c_int
        lib.hjpd_get_plan.argtypes = [vp, ctypes.c_int, vp, vp, vp, ip, ip]
        lib.hjpd_get_plan.restype = ctypes.c_int
        dp = ctypes.POINTER(ctypes.c_double)
        lib.hjpd_calibrate_fma.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, i64, dp, dp, dp]
        lib.hjpd_calibrate_fma.restype = ctypes.c_int
        lib.hjpd_destroy.argtypes = [vp]
        lib.hjpd_destroy.restype = ctypes.c_int
        lib.hjpd_last_error.argtypes = []
        lib.hjpd_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _ptr(a):
    """Device pointer of a tensor (or None / int passthrough)."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    return a.data_ptr()


def _stream(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(rc):
    if rc != HJPD_OK:
        raise HjpdError(rc, load().hjpd_last_error().decode())


def hjpd_last_error() -> str:
    return load().hjpd_last_error().decode()


def hjpd_create(desc: hjpd_desc) -> int:
    ctx = ctypes.c_void_p()
    _check(load().hjpd_create(ctypes.byref(desc), ctypes.byref(ctx)))
    return ctx.value


def hjpd_calibrate_fma(dtype: int, chains: int, waves_per_simd: int, rounds: int) -> dict:
    """One timed launch of the FMA calibration kernel: device ms, exact flops
    and wave64 FMA instructions."""
    ms, fl, wi = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    _check(load().hjpd_calibrate_fma(int(dtype), int(chains), int(waves_per_simd), int(rounds), ctypes.byref(ms),
                                     ctypes.byref(fl), ctypes.byref(wi)))
    return {"ms": ms.value, "flops": fl.value, "wave_instructions": wi.value}


def hjpd_destroy(ctx: int) -> None:
    _check(load().hjpd_destroy(ctx))


def hjpd_solve_batch(ctx, n, x, t, N, h_params, g_params, phi, x_traj, p_traj, iters, status, stream=None):
    _check(load().hjpd_solve_batch(ctx, int(n), _ptr(x), _ptr(t), _ptr(N), _ptr(h_params), _ptr(g_params),
                                   _ptr(phi), _ptr(x_traj), _ptr(p_traj), _ptr(iters), _ptr(status),
                                   _stream(stream)))


def hjpd_solve_batch_noalloc(ctx, n, x, t, N, h_params, g_params, phi, x_traj, p_traj, iters, status,
                             stream=None):
    _check(load().hjpd_solve_batch_noalloc(ctx, int(n), _ptr(x), _ptr(t), _ptr(N), _ptr(h_params),
                                           _ptr(g_params), _ptr(phi), _ptr(x_traj), _ptr(p_traj), _ptr(iters),
                                           _ptr(status), _stream(stream)))


def hjpd_value_grad(ctx, n, x, t, N, h_params, g_params, grad_phi, K_iters, ckpt_every, phi, dphi_dx,
                    dh_params, dg_params, stream=None):
    _check(load().hjpd_value_grad(ctx, int(n), _ptr(x), _ptr(t), _ptr(N), _ptr(h_params), _ptr(g_params),
                                  _ptr(grad_phi), int(K_iters), int(ckpt_every), _ptr(phi), _ptr(dphi_dx),
                                  _ptr(dh_params), _ptr(dg_params), _stream(stream)))


def hjpd_autotune(ctx, n, x, t, N, h_params, g_params, phi, iters, status, probe_iters=200, stream=None):
    _check(load().hjpd_autotune(ctx, int(n), _ptr(x), _ptr(t), _ptr(N), _ptr(h_params), _ptr(g_params),
                                _ptr(phi), _ptr(iters), _ptr(status), int(probe_iters), _stream(stream)))


def hjpd_get_timing(ctx):
    ms = ctypes.c_double()
    nl = ctypes.c_int()
    _check(load().hjpd_get_timing(ctx, ctypes.byref(ms), ctypes.byref(nl)))
    return ms.value, nl.value


def hjpd_get_launch_timing(ctx, i):
    """(ms, N_lo, N_hi, lanes_per_point, nodes_per_lane) of launch i of the last timed solve."""
    ms = ctypes.c_double()
    v = [ctypes.c_int() for _ in range(4)]
    _check(load().hjpd_get_launch_timing(ctx, int(i), ctypes.byref(ms), *[ctypes.byref(x) for x in v]))
    return (ms.value, *[x.value for x in v])


def hjpd_set_plan(ctx, classes):
    """classes: [(hi, L, K), ...] (host values)."""
    n = len(classes)
    arr = [(ctypes.c_int32 * n)(*[int(c[k]) for c in classes]) for k in range(3)]
    _check(load().hjpd_set_plan(ctx, n, *[ctypes.cast(a, ctypes.c_void_p) for a in arr]))


def hjpd_get_plan(ctx):
    """([(hi, L, K), ...], from_cache) of the context's persistent plan."""
    m = 16
    arr = [(ctypes.c_int32 * m)() for _ in range(3)]
    n, fc = ctypes.c_int(), ctypes.c_int()
    _check(load().hjpd_get_plan(ctx, m, *[ctypes.cast(a, ctypes.c_void_p) for a in arr], ctypes.byref(n),
                                ctypes.byref(fc)))
    return [(arr[0][i], arr[1][i], arr[2][i]) for i in range(n.value)], bool(fc.value)


def hjpd_set_pop_counter(ctx, counts):
    _check(load().hjpd_set_pop_counter(ctx, _ptr(counts)))
