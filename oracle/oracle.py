"""ctypes wrapper around the plain CPU oracle (``j3d_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg; never by the product path.  It shares no code
with the HIP library.  What each function computes, and the passages of the
paper it follows, are documented in ``j3d_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "j3d_oracle.c")
LIB = os.path.join(HERE, "liboracle_j3d.so")

# IEEE binary64, no contraction, no fast-math (denormals stay on).  One flag
# list serves both builds below; neither option changes a result bit
# (tests/test_oracle_pins.py compares the two builds).
CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-Wall", "-Wextra"]
# The timing copy is also tuned for the host it runs on.  It is compiled on
# that host, into a private directory, and never shipped: code built for one
# machine's vector extensions may not run on another's.
NATIVE_CFLAGS = CFLAGS + ["-march=native"]


def compile_oracle(force: bool = False) -> str:
    """Compile the parity build (portable code) with gcc; returns the library path."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"])
        os.replace(tmp, LIB)
    return LIB


_native_path = None


def compile_native() -> str:
    """Compile the timing copy (-march=native) for this host, once per process."""
    global _native_path
    if _native_path is None:
        import tempfile
        d = tempfile.mkdtemp(prefix="j3d_oracle_native_")
        path = os.path.join(d, "liboracle_j3d_native.so")
        subprocess.check_call(["gcc", *NATIVE_CFLAGS, SRC, "-o", path, "-lm"])
        _native_path = path
    return _native_path


_libs = {}


def lib(native: bool = False) -> ctypes.CDLL:
    """The parity build, or (native=True) the host-tuned timing copy."""
    if native not in _libs:
        L = ctypes.CDLL(compile_native() if native else compile_oracle())
        i64, u64, dp = ctypes.c_int64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double)
        L.oracle_splitmix64_seq.argtypes = [u64, i64, ctypes.POINTER(u64)]
        L.oracle_splitmix64_seq.restype = None
        L.oracle_init_interior.argtypes = [i64, i64, i64, u64, u64, dp]
        L.oracle_init_interior.restype = None
        L.oracle_init_cell.argtypes = [i64, i64, u64, u64, i64, i64, i64]
        L.oracle_init_cell.restype = ctypes.c_double
        L.oracle_jacobi.argtypes = [i64, i64, i64, dp, u64, u64, dp,
                                    ctypes.POINTER(dp), i64, ctypes.c_double, i64,
                                    dp, dp, ctypes.POINTER(i64), ctypes.c_int]
        L.oracle_jacobi.restype = ctypes.c_int
        L.oracle_cell_after.argtypes = [i64, i64, i64, u64, u64, dp, i64, i64, i64,
                                        i64, dp]
        L.oracle_cell_after.restype = ctypes.c_int
        L.oracle_max_threads.argtypes = []
        L.oracle_max_threads.restype = ctypes.c_int
        _libs[native] = L
    return _libs[native]


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def splitmix64_seq(seed: int, n: int) -> np.ndarray:
    out = np.zeros(n, dtype=np.uint64)
    lib().oracle_splitmix64_seq(seed, n, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def init_interior(n, seed: int, pid: int = 0) -> np.ndarray:
    """Seeded u0, shape (nz, ny, nx) (x fastest in memory)."""
    nx, ny, nz = (int(v) for v in n)
    u = np.empty((nz, ny, nx), dtype=np.float64)
    lib().oracle_init_interior(nx, ny, nz, seed, pid, _dp(u))
    return u


def init_cell(n, seed: int, pid: int, i: int, j: int, k: int) -> float:
    return lib().oracle_init_cell(int(n[0]), int(n[1]), seed, pid, i, j, k)


def jacobi(n, t_max: int, bc=(0.0,) * 6, u0=None, seed: int = 1, pid: int = 0,
           faces=None, tol: float = 0.0, check_every: int = 0, nthreads: int = 1, native: bool = False):
    """Run the oracle; returns (u (nz,ny,nx), residual, iters_done).
    native=True runs the host-tuned timing copy (same bits)."""
    nx, ny, nz = (int(v) for v in n)
    out = np.empty((nz, ny, nx), dtype=np.float64)
    bca = np.ascontiguousarray(np.asarray(bc, dtype=np.float64))
    assert bca.shape == (6,)
    u0p = None
    if u0 is not None:
        u0 = np.ascontiguousarray(np.asarray(u0, dtype=np.float64)).reshape(nz, ny, nx)
        u0p = _dp(u0)
    face_ptrs = None
    keep = []
    if faces is not None:
        arr = (ctypes.POINTER(ctypes.c_double) * 6)()
        shapes = [(nz, ny), (nz, ny), (nz, nx), (nz, nx), (ny, nx), (ny, nx)]
        for f in range(6):
            if faces[f] is None:
                arr[f] = ctypes.POINTER(ctypes.c_double)()
            else:
                a = np.ascontiguousarray(np.asarray(faces[f], dtype=np.float64)).reshape(shapes[f])
                keep.append(a)
                arr[f] = _dp(a)
        face_ptrs = arr
    res = ctypes.c_double(0.0)
    done = ctypes.c_int64(0)
    rc = lib(native).oracle_jacobi(nx, ny, nz, u0p, seed, pid, _dp(bca), face_ptrs, int(t_max),
                             float(tol), int(check_every), _dp(out), ctypes.byref(res),
                             ctypes.byref(done), int(nthreads))
    if rc != 0:
        raise ValueError("oracle_jacobi rejected its arguments")
    return out, res.value, done.value


def cell_after(n, seed: int, pid: int, bc, t: int, i: int, j: int, k: int) -> float:
    """One cell's value after t sweeps, from its domain of dependence."""
    bca = np.ascontiguousarray(np.asarray(bc, dtype=np.float64))
    v = ctypes.c_double(0.0)
    rc = lib().oracle_cell_after(int(n[0]), int(n[1]), int(n[2]), seed, pid, _dp(bca), int(t),
                                 int(i), int(j), int(k), ctypes.byref(v))
    if rc != 0:
        raise ValueError("oracle_cell_after rejected its arguments")
    return v.value


def max_threads() -> int:
    return int(lib().oracle_max_threads())
