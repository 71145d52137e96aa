"""ctypes binding of libmdjk.so (include/mdjk.h) -- argument marshalling only.

Every numerical step runs in the library's HIP kernels; this module converts
Python/torch objects to the C structs and pointers of the ABI and raises on
error codes.  If the shared library is missing it raises: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmdjk.so")

ERI_OK, ERI_EINVAL, ERI_ENOMEM, ERI_EHIP, ERI_ESTATE = 0, -1, -2, -3, -4
ERI_FP64, ERI_MIXED, ERI_MIXED_ALL = 0, 1, 2
_NAMES = {ERI_EINVAL: "ERI_EINVAL", ERI_ENOMEM: "ERI_ENOMEM", ERI_EHIP: "ERI_EHIP", ERI_ESTATE: "ERI_ESTATE"}


class EriError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_NAMES.get(code, "?"), code, msg))
        self.code = code


class eri_atom(ctypes.Structure):
    _fields_ = [("xyz", ctypes.c_double * 3)]


class eri_shell(ctypes.Structure):
    _fields_ = [("atom", ctypes.c_int32), ("l", ctypes.c_int32), ("nprim", ctypes.c_int32),
                ("exps", ctypes.POINTER(ctypes.c_double)), ("coefs", ctypes.POINTER(ctypes.c_double))]


class eri_opts(ctypes.Structure):
    _fields_ = [("schwarz_thresh", ctypes.c_double), ("prim_thresh", ctypes.c_double),
                ("mixed_thresh", ctypes.c_double), ("precision", ctypes.c_int32),
                ("spherical", ctypes.c_int32), ("stream", ctypes.c_void_p), ("omega", ctypes.c_double)]


class eri_stats_t(ctypes.Structure):
    _fields_ = [("nshell", ctypes.c_int32), ("natom", ctypes.c_int32), ("nbf", ctypes.c_int32),
                ("nbf_cart", ctypes.c_int32), ("n_pairs", ctypes.c_int64), ("n_prim_pairs", ctypes.c_int64),
                ("n_quartets", ctypes.c_int64), ("n_quartets_fp32", ctypes.c_int64),
                ("eris_sph", ctypes.c_double), ("eris_cart", ctypes.c_double),
                ("model_flops_k", ctypes.c_double), ("model_flops_j", ctypes.c_double),
                ("last_ms", ctypes.c_double), ("n_prim_quartets_k", ctypes.c_int64),
                ("n_prim_quartets_j", ctypes.c_int64)]


class eri_tuning_t(ctypes.Structure):
    _fields_ = [("kchunk", ctypes.c_int32 * 100), ("jsplit", ctypes.c_int32 * 100), ("n_kwork", ctypes.c_int32),
                ("kwork_class", ctypes.c_int32 * 64), ("kcap", ctypes.c_int32 * 64), ("ksplit", ctypes.c_int32 * 64),
                ("kinv", ctypes.c_int32 * 64)]


class eri_kernel_time(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 40), ("launches", ctypes.c_int32), ("ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("prim_quartets", ctypes.c_int64)]


EXPORTS = ["eri_default_opts", "eri_setup", "eri_nbf", "eri_set_geometry", "eri_set_precision",
           "build_jk", "jk_grad", "eri_energy", "eri_set_profiling", "eri_profile_read", "eri_stats", "eri_destroy",
           "eri_last_error", "eri_batch_create", "eri_batch_build_jk", "eri_batch_destroy",
           "eri_autotune", "eri_tuning", "build_jk_static", "eri_set_omega", "eri_get_tuning",
           "eri_set_tuning", "eri_potential", "eri_potential_grad", "eri_set_density_screen",
           "eri_one_electron", "eri_grid_density", "eri_grid_matrix", "eri_batch_latency",
           "eri_batch_set_mode", "eri_batch_queue_info"]

ERI_BATCH_QUEUE = 0
ERI_BATCH_STREAMS = 1

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libmdjk.so not found at %s: build it with "
                           "`python -m paper_2406_14920_amd.build` (no CPU fallback exists)" % path)
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.eri_default_opts.argtypes = [ctypes.POINTER(eri_opts)]
    L.eri_default_opts.restype = None
    L.eri_setup.argtypes = [ctypes.POINTER(eri_shell), ctypes.c_int32, ctypes.POINTER(eri_atom),
                            ctypes.c_int32, ctypes.POINTER(eri_opts), ctypes.POINTER(vp)]
    L.eri_nbf.argtypes = [vp, ctypes.POINTER(ctypes.c_int32)]
    L.eri_set_geometry.argtypes = [vp, ctypes.POINTER(eri_atom)]
    L.eri_set_precision.argtypes = [vp, ctypes.c_int32, ctypes.c_double]
    L.eri_set_omega.argtypes = [vp, ctypes.c_double]
    L.eri_get_tuning.argtypes = [vp, ctypes.POINTER(eri_tuning_t)]
    L.eri_set_tuning.argtypes = [vp, ctypes.POINTER(eri_tuning_t)]
    L.build_jk.argtypes = [vp, vp, vp, vp]
    L.build_jk_static.argtypes = [vp, vp, vp, vp]
    L.jk_grad.argtypes = [vp, vp, vp, vp]
    L.eri_energy.argtypes = [vp, vp, vp, vp, vp]
    L.eri_potential.argtypes = [vp, vp, ctypes.c_int32, vp]
    L.eri_set_density_screen.argtypes = [vp, ctypes.c_double]
    L.eri_one_electron.argtypes = [vp, vp, vp]
    L.eri_grid_density.argtypes = [vp, vp, vp, ctypes.c_int64, vp, vp]
    L.eri_grid_matrix.argtypes = [vp, vp, ctypes.c_int64, vp, vp, vp]
    L.eri_potential_grad.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp]
    L.eri_stats.argtypes = [vp, ctypes.POINTER(eri_stats_t)]
    L.eri_set_profiling.argtypes = [vp, ctypes.c_int32]
    L.eri_profile_read.argtypes = [vp, ctypes.POINTER(eri_kernel_time), ctypes.c_int32,
                                   ctypes.POINTER(ctypes.c_int32)]
    L.eri_destroy.argtypes = [vp]
    L.eri_batch_create.argtypes = [ctypes.POINTER(vp), ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.eri_batch_build_jk.argtypes = [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp)]
    L.eri_batch_destroy.argtypes = [vp]
    L.eri_batch_latency.argtypes = [vp, ctypes.POINTER(ctypes.c_float), ctypes.c_int32]
    L.eri_batch_set_mode.argtypes = [vp, ctypes.c_int32]
    L.eri_batch_queue_info.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]
    L.eri_autotune.argtypes = [vp, vp, ctypes.c_int32]
    ip = ctypes.POINTER(ctypes.c_int32)
    L.eri_tuning.argtypes = [vp, ip, ip, ctypes.c_int32, ip]
    L.eri_last_error.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name not in ("eri_default_opts", "eri_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != ERI_OK:
        raise EriError(rc, load().eri_last_error().decode())


def _ptr(x) -> Optional[int]:
    """Device pointer of a torch tensor (or an int address), None for None."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return int(x.data_ptr())


# ---------------------------------------------------------------------------
# ABI calls under their C names
# ---------------------------------------------------------------------------
def eri_default_opts() -> eri_opts:
    o = eri_opts()
    load().eri_default_opts(ctypes.byref(o))
    return o


class _ShellArrays:
    """Keeps the ctypes shell array and the numpy buffers it points into alive."""

    def __init__(self, shells):
        self.bufs = []
        self.arr = (eri_shell * len(shells))()
        for k, s in enumerate(shells):
            e = np.ascontiguousarray(s[2], dtype=np.float64)
            c = np.ascontiguousarray(s[3], dtype=np.float64)
            self.bufs += [e, c]
            self.arr[k].atom = int(s[0])
            self.arr[k].l = int(s[1])
            self.arr[k].nprim = int(e.size)
            self.arr[k].exps = e.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            self.arr[k].coefs = c.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _atoms(xyz) -> ctypes.Array:
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    arr = (eri_atom * len(xyz))()
    for i, r in enumerate(xyz):
        arr[i].xyz[:] = [float(v) for v in r]
    return arr


def eri_setup(shells: Sequence, xyz, opts: Optional[eri_opts] = None) -> int:
    """shells: sequence of (atom, l, exps, coefs); xyz: (natom, 3) bohr.
    Returns the context handle (an int)."""
    L = load()
    sa = _ShellArrays(shells)
    at = _atoms(xyz)
    h = ctypes.c_void_p()
    o = opts if opts is not None else eri_default_opts()
    _check(L.eri_setup(sa.arr, len(shells), at, len(at), ctypes.byref(o), ctypes.byref(h)))
    return int(h.value)


def eri_nbf(ctx: int) -> int:
    n = ctypes.c_int32()
    _check(load().eri_nbf(ctypes.c_void_p(ctx), ctypes.byref(n)))
    return int(n.value)


def eri_set_geometry(ctx: int, xyz) -> None:
    _check(load().eri_set_geometry(ctypes.c_void_p(ctx), _atoms(xyz)))


def eri_set_precision(ctx: int, precision: int, mixed_thresh: float) -> None:
    _check(load().eri_set_precision(ctypes.c_void_p(ctx), int(precision), float(mixed_thresh)))


def build_jk(ctx: int, P, J, K) -> None:
    _check(load().build_jk(ctypes.c_void_p(ctx), _ptr(P), _ptr(J), _ptr(K)))


_CLASSES = ["ss", "ps", "pp", "ds", "dp", "dd", "fs", "fp", "fd", "ff"]


def eri_get_tuning(ctx: int) -> dict:
    """Launch shapes and splits keyed by class names (JSON-serialisable)."""
    t = eri_tuning_t()
    _check(load().eri_get_tuning(ctypes.c_void_p(ctx), ctypes.byref(t)))
    j = {"%s|%s" % (_CLASSES[k // 10], _CLASSES[k % 10]): [int(t.kchunk[k]), int(t.jsplit[k])] for k in range(100)}
    kx = {"%s|%s" % (_CLASSES[t.kwork_class[i] // 10], _CLASSES[t.kwork_class[i] % 10]):
          [int(t.kcap[i]), int(t.ksplit[i]), int(t.kinv[i])] for i in range(t.n_kwork)}
    return {"jengine": j, "exchange": kx}


def eri_set_tuning(ctx: int, tuning: dict) -> None:
    cur = eri_tuning_t()
    _check(load().eri_get_tuning(ctypes.c_void_p(ctx), ctypes.byref(cur)))
    for name, (kc, sp) in tuning.get("jengine", {}).items():
        x, y = name.split("|")
        k = 10 * _CLASSES.index(x) + _CLASSES.index(y)
        cur.kchunk[k], cur.jsplit[k] = int(kc), int(sp)
    for i in range(cur.n_kwork):
        name = "%s|%s" % (_CLASSES[cur.kwork_class[i] // 10], _CLASSES[cur.kwork_class[i] % 10])
        if name in tuning.get("exchange", {}):
            vals = [int(v) for v in tuning["exchange"][name]]
            cur.kcap[i], cur.ksplit[i] = vals[0], vals[1]
            if len(vals) > 2:
                cur.kinv[i] = vals[2]
    _check(load().eri_set_tuning(ctypes.c_void_p(ctx), ctypes.byref(cur)))


def eri_set_omega(ctx: int, omega: float) -> None:
    _check(load().eri_set_omega(ctypes.c_void_p(ctx), float(omega)))


def build_jk_static(ctx: int, P, J, K) -> None:
    """build_jk with the work buffers in the library's static device array
    (allocates nothing; double precision only)."""
    _check(load().build_jk_static(ctypes.c_void_p(ctx), _ptr(P), _ptr(J), _ptr(K)))


def jk_grad(ctx: int, P, grad, E=None) -> None:
    _check(load().jk_grad(ctypes.c_void_p(ctx), _ptr(P), _ptr(grad), _ptr(E)))


def eri_set_density_screen(ctx: int, tau: float) -> None:
    _check(load().eri_set_density_screen(ctypes.c_void_p(ctx), float(tau)))


def eri_one_electron(ctx: int, S, T) -> None:
    """Overlap S and kinetic energy T (device nbf x nbf; either may be None)."""
    _check(load().eri_one_electron(ctypes.c_void_p(ctx), _ptr(S), _ptr(T)))


def eri_grid_density(ctx: int, P, pts, npts: int, rho, grad=None) -> None:
    _check(load().eri_grid_density(ctypes.c_void_p(ctx), _ptr(P), _ptr(pts), int(npts), _ptr(rho), _ptr(grad)))


def eri_grid_matrix(ctx: int, pts, npts: int, v0, v1, V) -> None:
    _check(load().eri_grid_matrix(ctypes.c_void_p(ctx), _ptr(pts), int(npts), _ptr(v0), _ptr(v1), _ptr(V)))


def eri_potential(ctx: int, charges, ncharge: int, V) -> None:
    """V = sum_C q_C (m|1/|r-C||n); charges: device [ncharge][4] x, y, z, q."""
    _check(load().eri_potential(ctypes.c_void_p(ctx), _ptr(charges), int(ncharge), _ptr(V)))


def eri_potential_grad(ctx: int, charges, ncharge: int, P, gatom, gchg) -> None:
    _check(load().eri_potential_grad(ctypes.c_void_p(ctx), _ptr(charges), int(ncharge), _ptr(P), _ptr(gatom),
                                     _ptr(gchg)))


def eri_energy(ctx: int, P, J, K, E) -> None:
    _check(load().eri_energy(ctypes.c_void_p(ctx), _ptr(P), _ptr(J), _ptr(K), _ptr(E)))


def eri_stats(ctx: int) -> dict:
    s = eri_stats_t()
    _check(load().eri_stats(ctypes.c_void_p(ctx), ctypes.byref(s)))
    return {name: getattr(s, name) for name, _ in eri_stats_t._fields_}


def eri_set_profiling(ctx: int, on: bool) -> None:
    _check(load().eri_set_profiling(ctypes.c_void_p(ctx), 1 if on else 0))


def eri_profile_read(ctx: int) -> list:
    cap = 512
    arr = (eri_kernel_time * cap)()
    n = ctypes.c_int32()
    _check(load().eri_profile_read(ctypes.c_void_p(ctx), arr, cap, ctypes.byref(n)))
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
             "flops": arr[i].flops, "prim_quartets": arr[i].prim_quartets} for i in range(min(n.value, cap))]


def eri_destroy(ctx: int) -> None:
    _check(load().eri_destroy(ctypes.c_void_p(ctx)))


def eri_batch_create(ctxs: Sequence[int], stream=None) -> int:
    arr = (ctypes.c_void_p * len(ctxs))(*[ctypes.c_void_p(c) for c in ctxs])
    h = ctypes.c_void_p()
    _check(load().eri_batch_create(arr, len(ctxs), ctypes.c_void_p(_ptr(stream) if stream is not None else None),
                                   ctypes.byref(h)))
    return int(h.value)


def eri_batch_build_jk(batch: int, P: Sequence, J: Sequence, K: Sequence) -> None:
    n = len(P)
    mk = lambda xs: (ctypes.c_void_p * n)(*[ctypes.c_void_p(_ptr(x)) for x in xs])
    _check(load().eri_batch_build_jk(ctypes.c_void_p(batch), mk(P), mk(J), mk(K)))


def eri_batch_destroy(batch: int) -> None:
    _check(load().eri_batch_destroy(ctypes.c_void_p(batch)))


def eri_autotune(ctx: int, P, reps: int = 2) -> None:
    _check(load().eri_autotune(ctypes.c_void_p(ctx), _ptr(P), int(reps)))


def eri_tuning(ctx: int) -> dict:
    kc = (ctypes.c_int32 * 100)()
    n = ctypes.c_int32()
    _check(load().eri_tuning(ctypes.c_void_p(ctx), kc, None, 0, ctypes.byref(n)))
    caps = (ctypes.c_int32 * max(n.value, 1))()
    _check(load().eri_tuning(ctypes.c_void_p(ctx), None, caps, n.value, None))
    return {"kchunk": [kc[i] for i in range(100)], "kcap": [caps[i] for i in range(n.value)]}


def eri_last_error() -> str:
    return load().eri_last_error().decode()


def eri_batch_latency(batch: int, n: int) -> list:
    """Per-molecule completion times (ms) of the last batch build."""
    arr = (ctypes.c_float * max(n, 1))()
    _check(load().eri_batch_latency(ctypes.c_void_p(batch), arr, int(n)))
    return [float(arr[i]) for i in range(n)]


def eri_batch_set_mode(batch: int, mode: int) -> None:
    _check(load().eri_batch_set_mode(ctypes.c_void_p(batch), int(mode)))


def eri_batch_queue_info(batch: int) -> dict:
    """Launches and work items of the batch's current queue plan."""
    n = ctypes.c_int32()
    m = ctypes.c_int64()
    _check(load().eri_batch_queue_info(ctypes.c_void_p(batch), ctypes.byref(n), ctypes.byref(m)))
    return {"launches": int(n.value), "items": int(m.value)}
