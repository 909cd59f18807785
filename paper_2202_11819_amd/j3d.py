"""Thin ctypes binding of libj3d: the C-ABI functions under their own names.

Argument marshalling only: every step of the Jacobi3D path runs in the HIP
library.  Device memory (arenas, dense device arrays) and streams are passed
as raw addresses; PyTorch is one convenient owner of them (see ``Solver``).
If libj3d.so has not been built, importing this module fails loudly.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_char_p, c_double, c_int, c_int32, c_int64, c_uint64, c_void_p

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libj3d.so")
HEADER_PATH = os.path.join(os.path.dirname(_HERE), "include", "j3d.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2202_11819_amd.build` "
                      "(or __graft_entry__.build()); there is no fallback path")

# libj3d must share the process's HIP runtime with whatever owns the device
# memory.  torch ships its own libamdhip64 (same soname); loading torch first
# makes libj3d bind to that copy instead of pulling in a second runtime, which
# would not see the device.
try:
    import torch  # noqa: F401
except ImportError:  # pragma: no cover - torch is only the memory owner
    torch = None

_lib = ctypes.CDLL(LIB_PATH)


def _hip_runtimes_mapped():
    try:
        with open("/proc/self/maps") as f:
            maps = f.read()
    except OSError:
        return set()
    return {line.split()[-1] for line in maps.splitlines() if "libamdhip64" in line}


if len(_hip_runtimes_mapped()) > 1:
    raise ImportError("two HIP runtimes are loaded in this process (" + ", ".join(sorted(_hip_runtimes_mapped()))
                      + "): load torch before any other HIP library")

J3D_OK, J3D_EINVAL, J3D_ENOMEM, J3D_EBUDGET, J3D_EBUSY, J3D_EDEVICE, J3D_ESTATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EBUDGET", -4: "EBUSY", -5: "EDEVICE", -6: "ESTATE"}

J3D_UNFUSED_BLOCK, J3D_UNFUSED_PHASE, J3D_FUSED, J3D_GRAPH = 0, 1, 2, 3
MODES = {"unfused_block": 0, "unfused_phase": 1, "fused": 2, "graph": 3, "block_a": 4, "block_b": 5,
         "block_c": 6, "host_staged": 7, "host_overlap": 8, "two_sweep": 9}
J3D_CAPTURED = 16


def mode_value(mode) -> int:
    """j3d_mode value of a mode name; "<name>+graph" captures it in HIP graphs."""
    if not isinstance(mode, str):
        return int(mode)
    if mode.endswith("+graph"):
        return MODES[mode[: -len("+graph")]] | J3D_CAPTURED
    return MODES[mode]


class J3DError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {message}")


class j3d_problem(ctypes.Structure):
    _fields_ = [("n", c_int64 * 3), ("nblk", c_int32 * 3), ("auto_parts", c_int32),
                ("split", POINTER(c_int64) * 3), ("bc", c_double * 6), ("seed", c_uint64),
                ("pid", c_uint64)]


class j3d_tune(ctypes.Structure):
    _fields_ = [("variant", c_int32), ("zchunk", c_int32), ("blocks_per_cu", c_int32)]


_P = POINTER(j3d_problem)
_DP = POINTER(c_double)
_H = c_void_p  # opaque handles

_SIGS = {
    "j3d_last_error": ([], c_char_p),
    "j3d_version": ([], c_char_p),
    "j3d_auto_split": ([POINTER(c_int64), c_int32, POINTER(c_int32)], c_int),
    "j3d_block_extents": ([_P, POINTER(c_int32), POINTER(c_int64), c_int64], c_int),
    "j3d_arena_bytes": ([_P, POINTER(c_uint64)], c_int),
    "j3d_field_bytes": ([_P, POINTER(c_uint64)], c_int),
    "j3d_variant_info": ([c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int32)], c_int),
    "j3d_create": ([_P, c_void_p, c_uint64, c_void_p, POINTER(_H)], c_int),
    "j3d_set_interior": ([_H, c_void_p, c_int], c_int),
    "j3d_set_face": ([_H, c_int32, c_void_p, c_int], c_int),
    "j3d_set_tune": ([_H, POINTER(j3d_tune)], c_int),
    "j3d_get_tune": ([_H, POINTER(j3d_tune)], c_int),
    "j3d_run": ([_H, c_int64, c_int, _DP], c_int),
    "j3d_iters_done": ([_H, POINTER(c_int64)], c_int),
    "j3d_get_interior": ([_H, c_void_p, c_int], c_int),
    "j3d_destroy": ([_H], c_int),
    "j3d_batch_arena_bytes": ([c_int32, _P, POINTER(c_uint64)], c_int),
    "j3d_batch_create": ([c_int32, _P, POINTER(c_int64), c_void_p, c_uint64, c_void_p,
                          POINTER(j3d_tune), POINTER(_H)], c_int),
    "j3d_batch_run": ([_H, _DP], c_int),
    "j3d_batch_run_two_sweep": ([_H, _DP], c_int),
    "j3d_batch_get_interior": ([_H, c_int32, c_void_p, c_int], c_int),
    "j3d_batch_destroy": ([_H], c_int),
    "j3d_pool_request_bytes": ([_P, POINTER(c_uint64)], c_int),
    "j3d_pool_overhead_bytes": ([c_int32, POINTER(c_uint64)], c_int),
    "j3d_pool_create": ([c_void_p, c_uint64, c_uint64, c_int32, c_void_p, POINTER(_H)], c_int),
    "j3d_pool_admit": ([_H, _P, c_int64, c_double, c_int32, c_void_p, POINTER(c_int32)], c_int),
    "j3d_pool_step": ([_H, c_int32], c_int),
    "j3d_pool_set_policy": ([_H, c_int64, c_int32, c_int32], c_int),
    "j3d_pool_set_tune": ([_H, POINTER(j3d_tune)], c_int),
    "j3d_pool_set_two_sweep": ([_H, c_int32], c_int),
    "j3d_pool_poll": ([_H, POINTER(c_int32), c_int32, POINTER(c_int32), POINTER(c_int32)], c_int),
    "j3d_pool_result": ([_H, c_int32, _DP, POINTER(c_int64)], c_int),
    "j3d_pool_fetch": ([_H, c_int32, c_void_p, _DP, POINTER(c_int64)], c_int),
    "j3d_solve_noalloc": ([_P, c_void_p, c_uint64, c_void_p, c_void_p, c_int64, _DP, c_void_p], c_int),
    "j3d_pool_release": ([_H, c_int32], c_int),
    "j3d_pool_usage": ([_H, POINTER(c_int32), POINTER(c_uint64)], c_int),
    "j3d_pool_destroy": ([_H], c_int),
    "j3d_device_copy": ([c_void_p, c_void_p, c_uint64, c_void_p], c_int),
    "j3d_device_cus": ([POINTER(c_int32)], c_int),
}

for _name, (_args, _res) in _SIGS.items():
    _fn = getattr(_lib, _name)
    _fn.argtypes = _args
    _fn.restype = _res

EXPORTED = tuple(_SIGS)


def _check(status: int, where: str):
    if status != J3D_OK:
        raise J3DError(status, where, j3d_last_error())


def j3d_last_error() -> str:
    return _lib.j3d_last_error().decode()


def j3d_version() -> str:
    return _lib.j3d_version().decode()


# ---- problems -------------------------------------------------------------------

class Problem:
    """A j3d_problem plus the arrays its split pointers refer to."""

    def __init__(self, n, nblk=(1, 1, 1), split=None, bc=0.0, seed=1, pid=0, auto_parts=0):
        self.c = j3d_problem()
        for a in range(3):
            self.c.n[a] = int(n[a])
            self.c.nblk[a] = int(nblk[a]) if nblk is not None else 0
        self.c.auto_parts = int(auto_parts)
        if np.isscalar(bc):
            bc = [float(bc)] * 6
        for f in range(6):
            self.c.bc[f] = float(bc[f])
        self.c.seed = int(seed)
        self.c.pid = int(pid)
        self._keep = []
        if split is not None:
            for a in range(3):
                if split[a] is None:
                    continue
                arr = (c_int64 * len(split[a]))(*[int(v) for v in split[a]])
                self._keep.append(arr)
                self.c.split[a] = ctypes.cast(arr, POINTER(c_int64))

    @property
    def n(self):
        return tuple(self.c.n)

    @property
    def cells(self):
        return int(self.c.n[0]) * int(self.c.n[1]) * int(self.c.n[2])


def j3d_auto_split(n, parts):
    nn = (c_int64 * 3)(*[int(v) for v in n])
    out = (c_int32 * 3)()
    _check(_lib.j3d_auto_split(nn, int(parts), out), "j3d_auto_split")
    return tuple(out)


def j3d_block_extents(p: Problem):
    nb = (c_int32 * 3)()
    _check(_lib.j3d_block_extents(byref(p.c), nb, None, 0), "j3d_block_extents")
    total = nb[0] + nb[1] + nb[2]
    ext = (c_int64 * total)()
    _check(_lib.j3d_block_extents(byref(p.c), nb, ext, total), "j3d_block_extents")
    e = list(ext)
    return tuple(nb), (e[:nb[0]], e[nb[0]:nb[0] + nb[1]], e[nb[0] + nb[1]:])


def j3d_arena_bytes(p: Problem) -> int:
    v = c_uint64()
    _check(_lib.j3d_arena_bytes(byref(p.c), byref(v)), "j3d_arena_bytes")
    return v.value


def j3d_field_bytes(p: Problem) -> int:
    v = c_uint64()
    _check(_lib.j3d_field_bytes(byref(p.c), byref(v)), "j3d_field_bytes")
    return v.value


def j3d_variant_info(v: int):
    tx, ty, th = c_int32(), c_int32(), c_int32()
    _check(_lib.j3d_variant_info(int(v), byref(tx), byref(ty), byref(th)), "j3d_variant_info")
    return tx.value, ty.value, th.value


def variants():
    out = []
    v = 0
    while _lib.j3d_variant_info(v, None, None, None) == J3D_OK:
        out.append(j3d_variant_info(v))
        v += 1
    return out


# ---- plain solver --------------------------------------------------------------

def j3d_create(p: Problem, arena_ptr: int, arena_bytes: int, stream_ptr: int):
    h = _H()
    _check(_lib.j3d_create(byref(p.c), c_void_p(arena_ptr), arena_bytes, c_void_p(stream_ptr), byref(h)),
           "j3d_create")
    return h


def j3d_set_interior(h, src_ptr: int, on_device: bool):
    _check(_lib.j3d_set_interior(h, c_void_p(src_ptr), int(on_device)), "j3d_set_interior")


def j3d_set_face(h, face: int, src_ptr: int, on_device: bool):
    _check(_lib.j3d_set_face(h, int(face), c_void_p(src_ptr), int(on_device)), "j3d_set_face")


def j3d_set_tune(h, variant=-1, zchunk=0, blocks_per_cu=0, default=False):
    if default:
        _check(_lib.j3d_set_tune(h, None), "j3d_set_tune")
        return
    t = j3d_tune(int(variant), int(zchunk), int(blocks_per_cu))
    _check(_lib.j3d_set_tune(h, byref(t)), "j3d_set_tune")


def j3d_get_tune(h):
    t = j3d_tune()
    _check(_lib.j3d_get_tune(h, byref(t)), "j3d_get_tune")
    return t.variant, t.zchunk, t.blocks_per_cu


def j3d_run(h, iters: int, mode, want_residual: bool = False):
    m = mode_value(mode)
    if want_residual:
        r = c_double()
        _check(_lib.j3d_run(h, int(iters), m, byref(r)), "j3d_run")
        return r.value
    _check(_lib.j3d_run(h, int(iters), m, None), "j3d_run")
    return None


def j3d_iters_done(h) -> int:
    v = c_int64()
    _check(_lib.j3d_iters_done(h, byref(v)), "j3d_iters_done")
    return v.value


def j3d_get_interior(h, dst_ptr: int, on_device: bool):
    _check(_lib.j3d_get_interior(h, c_void_p(dst_ptr), int(on_device)), "j3d_get_interior")


def j3d_destroy(h):
    _check(_lib.j3d_destroy(h), "j3d_destroy")


# ---- batched form ---------------------------------------------------------------

def _problem_array(probs):
    arr = (j3d_problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = p.c
    return arr


def j3d_batch_arena_bytes(probs) -> int:
    v = c_uint64()
    _check(_lib.j3d_batch_arena_bytes(len(probs), _problem_array(probs), byref(v)), "j3d_batch_arena_bytes")
    return v.value


def j3d_batch_create(probs, iters, arena_ptr, arena_bytes, stream_ptr, tune=None):
    arr = _problem_array(probs)
    it = (c_int64 * len(probs))(*[int(v) for v in iters])
    t = None
    if tune is not None:
        t = byref(j3d_tune(int(tune[0]), int(tune[1]), int(tune[2])))
    h = _H()
    _check(_lib.j3d_batch_create(len(probs), arr, it, c_void_p(arena_ptr), arena_bytes, c_void_p(stream_ptr),
                                 t, byref(h)), "j3d_batch_create")
    return h


def j3d_batch_run(h, count: int, want_residuals: bool = True):
    if want_residuals:
        r = (c_double * count)()
        _check(_lib.j3d_batch_run(h, r), "j3d_batch_run")
        return np.array(list(r))
    _check(_lib.j3d_batch_run(h, None), "j3d_batch_run")
    return None


def j3d_batch_run_two_sweep(h, count: int, want_residuals: bool = True):
    if want_residuals:
        r = (c_double * count)()
        _check(_lib.j3d_batch_run_two_sweep(h, r), "j3d_batch_run_two_sweep")
        return np.array(list(r))
    _check(_lib.j3d_batch_run_two_sweep(h, None), "j3d_batch_run_two_sweep")
    return None


def j3d_batch_get_interior(h, i: int, dst_ptr: int, on_device: bool):
    _check(_lib.j3d_batch_get_interior(h, int(i), c_void_p(dst_ptr), int(on_device)), "j3d_batch_get_interior")


def j3d_batch_destroy(h):
    _check(_lib.j3d_batch_destroy(h), "j3d_batch_destroy")


# ---- served form ----------------------------------------------------------------

def j3d_pool_request_bytes(p: Problem) -> int:
    v = c_uint64()
    _check(_lib.j3d_pool_request_bytes(byref(p.c), byref(v)), "j3d_pool_request_bytes")
    return v.value


def j3d_pool_overhead_bytes(max_slots: int) -> int:
    v = c_uint64()
    _check(_lib.j3d_pool_overhead_bytes(int(max_slots), byref(v)), "j3d_pool_overhead_bytes")
    return v.value


def j3d_pool_create(arena_ptr, arena_bytes, budget_bytes, max_slots, stream_ptr):
    h = _H()
    _check(_lib.j3d_pool_create(c_void_p(arena_ptr), arena_bytes, budget_bytes, int(max_slots),
                                c_void_p(stream_ptr), byref(h)), "j3d_pool_create")
    return h


def j3d_pool_admit(h, p: Problem, max_iters, tol, check_every, host_result_ptr):
    """Returns the slot, or raises J3DError (status EBUSY / EBUDGET when full)."""
    s = c_int32()
    _check(_lib.j3d_pool_admit(h, byref(p.c), int(max_iters), float(tol), int(check_every),
                               c_void_p(host_result_ptr), byref(s)), "j3d_pool_admit")
    return s.value


def j3d_pool_try_admit(h, p: Problem, max_iters, tol, check_every, host_result_ptr):
    """Like j3d_pool_admit but returns (status, slot) instead of raising on EBUSY/EBUDGET."""
    s = c_int32(-1)
    st = _lib.j3d_pool_admit(h, byref(p.c), int(max_iters), float(tol), int(check_every),
                             c_void_p(host_result_ptr), byref(s))
    if st not in (J3D_OK, J3D_EBUSY, J3D_EBUDGET):
        _check(st, "j3d_pool_admit")
    return st, s.value


def j3d_pool_step(h, sweeps: int):
    _check(_lib.j3d_pool_step(h, int(sweeps)), "j3d_pool_step")


def j3d_pool_set_tune(h, variant=-1, zchunk=32, default=False):
    if default:
        _check(_lib.j3d_pool_set_tune(h, None), "j3d_pool_set_tune")
        return
    t = j3d_tune(int(variant), int(zchunk), 0)
    _check(_lib.j3d_pool_set_tune(h, byref(t)), "j3d_pool_set_tune")


def j3d_pool_set_policy(h, fill_cells: int, max_wait_rounds: int = 32, backlog_share: int = 0):
    _check(_lib.j3d_pool_set_policy(h, int(fill_cells), int(max_wait_rounds), int(backlog_share)),
           "j3d_pool_set_policy")


def j3d_pool_set_two_sweep(h, enable: bool):
    _check(_lib.j3d_pool_set_two_sweep(h, 1 if enable else 0), "j3d_pool_set_two_sweep")


def j3d_pool_poll(h, cap: int = 1024):
    done = (c_int32 * cap)()
    n = c_int32()
    busy = c_int32()
    _check(_lib.j3d_pool_poll(h, done, cap, byref(n), byref(busy)), "j3d_pool_poll")
    return list(done[:n.value]), bool(busy.value)


def j3d_pool_result(h, slot: int):
    r = c_double()
    it = c_int64()
    _check(_lib.j3d_pool_result(h, int(slot), byref(r), byref(it)), "j3d_pool_result")
    return r.value, it.value


def j3d_pool_fetch(h, slot: int, host_dst_ptr=None):
    """(residual, sweeps done) of a finished slot; its interior is copied to
    host_dst_ptr (nx*ny*nz doubles) when given.  Synchronises."""
    r, it = c_double(0.0), c_int64(0)
    _check(_lib.j3d_pool_fetch(h, int(slot), c_void_p(host_dst_ptr) if host_dst_ptr else None, byref(r),
                               byref(it)), "j3d_pool_fetch")
    return r.value, it.value


def j3d_solve_noalloc(p: Problem, fields_ptr, fields_bytes, interior_in_ptr, interior_out_ptr, iters,
                      residual=False, stream_ptr=None):
    """One-shot fused solve with no device allocation (pointers are device
    addresses; interior_in_ptr None: seeded).  Returns the residual or None."""
    r = c_double(0.0)
    _check(_lib.j3d_solve_noalloc(byref(p.c), c_void_p(fields_ptr), int(fields_bytes),
                                  c_void_p(interior_in_ptr) if interior_in_ptr else None,
                                  c_void_p(interior_out_ptr), int(iters), byref(r) if residual else None,
                                  c_void_p(stream_ptr) if stream_ptr else None), "j3d_solve_noalloc")
    return r.value if residual else None


def j3d_pool_release(h, slot: int):
    _check(_lib.j3d_pool_release(h, int(slot)), "j3d_pool_release")


def j3d_pool_usage(h):
    n = c_int32()
    b = c_uint64()
    _check(_lib.j3d_pool_usage(h, byref(n), byref(b)), "j3d_pool_usage")
    return n.value, b.value


def j3d_pool_destroy(h):
    _check(_lib.j3d_pool_destroy(h), "j3d_pool_destroy")


# ---- measurement helpers ------------------------------------------------------

def j3d_device_copy(dst_ptr, src_ptr, nbytes, stream_ptr):
    _check(_lib.j3d_device_copy(c_void_p(dst_ptr), c_void_p(src_ptr), int(nbytes), c_void_p(stream_ptr)),
           "j3d_device_copy")


def j3d_device_cus() -> int:
    v = c_int32()
    _check(_lib.j3d_device_cus(byref(v)), "j3d_device_cus")
    return v.value
