"""Torch-owned device memory around the C ABI: Solver, Batch and Pool.

These classes only allocate the arena (a uint8 CUDA/HIP tensor), pick the
stream and marshal arrays; every computation runs in libj3d.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import j3d as C


def _stream(stream):
    return stream if stream is not None else torch.cuda.current_stream()


class Solver:
    """One Jacobi3D problem, over-decomposed into blocks on one GPU."""

    def __init__(self, n, nblk=(1, 1, 1), split=None, bc=0.0, seed=1, pid=0, auto_parts=0,
                 stream=None, device="cuda"):
        self.problem = C.Problem(n, nblk, split, bc, seed, pid, auto_parts)
        self.n = tuple(int(v) for v in n)
        self.arena_bytes = C.j3d_arena_bytes(self.problem)
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        self.stream = _stream(stream)
        self.h = C.j3d_create(self.problem, self.arena.data_ptr(), self.arena_bytes, self.stream.cuda_stream)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    def run(self, iters, mode="graph", residual=False):
        return C.j3d_run(self.h, iters, mode, residual)

    def set_tune(self, variant=-1, zchunk=0, blocks_per_cu=0):
        C.j3d_set_tune(self.h, variant, zchunk, blocks_per_cu)

    def get_tune(self):
        """(variant, zchunk, blocks_per_cu) in use."""
        return C.j3d_get_tune(self.h)

    def set_interior(self, u):
        if isinstance(u, torch.Tensor) and u.is_cuda:
            u = u.contiguous().to(torch.float64)
            C.j3d_set_interior(self.h, u.data_ptr(), True)
            self.stream.synchronize()
        else:
            a = np.ascontiguousarray(np.asarray(u, dtype=np.float64))
            assert a.size == self.n[0] * self.n[1] * self.n[2]
            C.j3d_set_interior(self.h, a.ctypes.data, False)

    def set_face(self, face, values):
        a = np.ascontiguousarray(np.asarray(values, dtype=np.float64))
        C.j3d_set_face(self.h, face, a.ctypes.data, False)

    def get_interior(self) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.float64)
        C.j3d_get_interior(self.h, out.ctypes.data, False)
        return out

    def get_interior_device(self) -> torch.Tensor:
        out = torch.empty(self.shape, dtype=torch.float64, device=self.arena.device)
        C.j3d_get_interior(self.h, out.data_ptr(), True)
        self.stream.synchronize()
        return out

    def iters_done(self):
        return C.j3d_iters_done(self.h)

    def close(self):
        if self.h is not None:
            C.j3d_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Many independent problems advanced by one launch per sweep."""

    def __init__(self, problems, iters, tune=None, stream=None, device="cuda"):
        self.problems = list(problems)
        self.iters = [int(v) for v in iters]
        self.arena_bytes = C.j3d_batch_arena_bytes(self.problems)
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        self.stream = _stream(stream)
        self.h = C.j3d_batch_create(self.problems, self.iters, self.arena.data_ptr(), self.arena_bytes,
                                    self.stream.cuda_stream, tune)

    def run(self, residuals=True, two_sweep=False):
        if two_sweep:
            return C.j3d_batch_run_two_sweep(self.h, len(self.problems), residuals)
        return C.j3d_batch_run(self.h, len(self.problems), residuals)

    def get_interior(self, i) -> np.ndarray:
        n = self.problems[i].n
        out = np.empty((n[2], n[1], n[0]), dtype=np.float64)
        C.j3d_batch_get_interior(self.h, i, out.ctypes.data, False)
        return out

    def close(self):
        if self.h is not None:
            C.j3d_batch_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Pool:
    """Continuous batching of solve requests under an HBM budget.

    Finished results are copied asynchronously into page-locked host buffers
    (one per admitted request).  Those buffers are recycled: a released
    request's buffer goes back to a free list of size classes (1/8 octave
    apart), and a buffer is allocated only when no free one fits, and only
    after a cheap check that the pool has a free slot and budget, so a request
    that cannot be admitted yet costs no allocation."""

    def __init__(self, budget_bytes, max_slots=256, stream=None, device="cuda"):
        self.overhead = C.j3d_pool_overhead_bytes(max_slots)
        self.budget = int(budget_bytes)
        self.arena_bytes = self.overhead + self.budget
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        self.stream = _stream(stream)
        self.max_slots = max_slots
        self.h = C.j3d_pool_create(self.arena.data_ptr(), self.arena_bytes, self.budget, max_slots,
                                   self.stream.cuda_stream)
        self.results = {}       # slot -> (pinned host buffer or None, (nz, ny, nx))
        self._free_host = []    # released pinned buffers, reused by later requests

    @staticmethod
    def _size_class(cells):
        return max(1, int(2.0 ** (math.ceil(8 * math.log2(max(cells, 1))) / 8)))

    def _host_buffer(self, cells):
        best = None
        for i, buf in enumerate(self._free_host):
            if buf.numel() >= cells and (best is None or buf.numel() < self._free_host[best].numel()):
                best = i
        if best is not None and self._free_host[best].numel() <= 2 * cells:
            return self._free_host.pop(best)
        return torch.empty(max(cells, self._size_class(cells)), dtype=torch.float64, pin_memory=True)

    def try_admit(self, problem, max_iters, tol=0.0, check_every=50, host=True):
        """Returns the slot or None when no slot / budget is free.  host=False:
        the result stays on the device until fetch()."""
        n = problem.n
        cells = n[0] * n[1] * n[2]
        buf = None
        if host:
            used, nbytes = C.j3d_pool_usage(self.h)
            if used >= self.max_slots or nbytes + C.j3d_pool_request_bytes(problem) > self.budget:
                return None
            buf = self._host_buffer(cells)
        st, slot = C.j3d_pool_try_admit(self.h, problem, max_iters, tol, check_every,
                                        buf.data_ptr() if buf is not None else None)
        if st != C.J3D_OK:
            if buf is not None:
                self._free_host.append(buf)  # fragmented budget: keep the buffer for the retry
            return None
        self.results[slot] = (buf, (n[2], n[1], n[0]))
        return slot

    def step(self, sweeps=50):
        """Enqueue one round.  Returns whether a round is in flight afterwards:
        False when no admitted request was still running (all finished ones
        wait for their result copy or their release), so nothing was enqueued."""
        C.j3d_pool_step(self.h, sweeps)
        return C.j3d_pool_poll(self.h, 0)[1]

    def set_policy(self, fill_cells, max_wait_rounds=32, backlog_share=0):
        C.j3d_pool_set_policy(self.h, fill_cells, max_wait_rounds, backlog_share)

    def set_tune(self, variant=-1, zchunk=32):
        """Tile shape of the rounds; only while no request is admitted."""
        C.j3d_pool_set_tune(self.h, variant, zchunk)

    def set_two_sweep(self, enable=True):
        """Two sweeps per launch in the rounds; only while no request is admitted."""
        C.j3d_pool_set_two_sweep(self.h, enable)

    def poll(self):
        return C.j3d_pool_poll(self.h, self.max_slots)

    def result(self, slot):
        """(interior as numpy (nz,ny,nx), residual, sweeps done) of a finished slot.
        The array views the slot's host buffer: copy it to keep it past release."""
        buf, shape = self.results[slot]
        if buf is None:
            return self.fetch(slot)
        r, it = C.j3d_pool_result(self.h, slot)
        return buf.numpy()[: shape[0] * shape[1] * shape[2]].reshape(shape), r, it

    def fetch(self, slot):
        """(interior, residual, sweeps done) copied from the device by j3d_pool_fetch (synchronous)."""
        _, shape = self.results[slot]
        out = np.empty(shape, dtype=np.float64)
        r, it = C.j3d_pool_fetch(self.h, slot, out.ctypes.data)
        return out, r, it

    def release(self, slot):
        C.j3d_pool_release(self.h, slot)
        buf, _ = self.results.pop(slot, (None, None))
        if buf is not None:
            self._free_host.append(buf)
            if len(self._free_host) > 64:  # bound the idle page-locked memory
                self._free_host.pop(0)

    def usage(self):
        return C.j3d_pool_usage(self.h)

    def close(self):
        if self.h is not None:
            C.j3d_pool_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
