"""Batched form: many snapshots through one persistent launch per stage.

Thin binding of the gpz_batch_* C ABI.  torch owns every device buffer (the
snapshots, their stream buffers, decompression outputs and the shared
workspace); the library owns only its small job tables.  Launch geometry
(persistent grid, blocks per work-queue grab) comes from the autotuner.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np

from . import (BatchConfig, Job, Params, _check, _lib, _ptr_array, _stream_handle,
               max_compressed_bytes, params)


def default_config() -> BatchConfig:
    c = BatchConfig()
    _lib().gpz_default_batch_config(ctypes.byref(c))
    return c


class _JobArrays:
    """Keeps the host pointer arrays of a job list alive for the C call."""

    def __init__(self, fields, ebs, outs, decs, wss=None):
        outs = outs or []
        self.njobs = len(outs)
        self.jobs = (Job * max(1, self.njobs))()
        self.keep = []
        for j in range(self.njobs):
            J = self.jobs[j]
            fl = fields[j] if fields is not None else None
            dl = decs[j] if decs is not None else None
            F = len(fl) if fl is not None else len(dl)
            n = (fl[0] if fl is not None else dl[0]).numel()
            e = np.ascontiguousarray(np.broadcast_to(np.asarray(ebs[j], np.float32), (F,)))
            fa = _ptr_array(fl) if fl is not None else None
            da = _ptr_array(dl) if dl is not None else None
            self.keep += [e, fa, da]
            J.fields = ctypes.cast(fa, ctypes.c_void_p) if fa is not None else None
            J.n = n
            J.nfields = F
            J.eb = e.ctypes.data_as(ctypes.c_void_p)
            J.out = outs[j].data_ptr()
            J.out_capacity = outs[j].numel()
            J.dec_fields = ctypes.cast(da, ctypes.c_void_p) if da is not None else None
            J.ws = wss[j].data_ptr() if wss is not None and wss[j] is not None else None


class PreparedJob:
    """One job's C struct and the host arrays it points at, built once (a
    serving loop builds it when a request is admitted and its bound known)
    and copied into a job list at launch."""

    __slots__ = ("job", "keep", "blocks")

    def __init__(self, fields, eb, out, dec=None, ws=None, block_size: int = 1024):
        fl, dl = fields, dec
        F = len(fl) if fl is not None else len(dl)
        n = (fl[0] if fl is not None else dl[0]).numel()
        e = np.ascontiguousarray(np.broadcast_to(np.asarray(eb, np.float32), (F,)))
        fa = _ptr_array(fl) if fl is not None else None
        da = _ptr_array(dl) if dl is not None else None
        J = Job()
        J.fields = ctypes.cast(fa, ctypes.c_void_p) if fa is not None else None
        J.n = n
        J.nfields = F
        J.eb = e.ctypes.data_as(ctypes.c_void_p)
        J.out = out.data_ptr()
        J.out_capacity = out.numel()
        J.dec_fields = ctypes.cast(da, ctypes.c_void_p) if da is not None else None
        J.ws = ws.data_ptr() if ws is not None else None
        self.job = J
        self.keep = (e, fa, da)
        self.blocks = (n + block_size - 1) // block_size


class Batch:
    """A bound batch of jobs.  `fields[j]` / `dec[j]` are lists of float32 CUDA
    tensors (either may be None), `outs[j]` uint8 CUDA stream buffers of at
    least max_compressed_bytes, `ebs[j]` absolute bounds (scalar or per field)."""

    def __init__(self, fields: Optional[Sequence[Sequence]], ebs: Sequence, outs: Sequence,
                 dec: Optional[Sequence[Sequence]] = None, p: Optional[Params] = None,
                 config: Optional[BatchConfig] = None, workspace=None, max_jobs: int = 0,
                 max_blocks: int = 0):
        import torch
        self.p = p if p is not None else params(3)
        self.config = config if config is not None else default_config()
        if max_jobs:
            self.config.max_jobs = max_jobs
        if max_blocks:
            self.config.max_blocks = max_blocks
        arrays = _JobArrays(fields, ebs, outs, dec)
        need = int(_lib().gpz_batch_workspace_bytes(arrays.jobs, arrays.njobs,
                                                    ctypes.byref(self.p)))
        if need == 0:
            raise ValueError("invalid job list")
        if workspace is None:
            workspace = torch.empty(need, dtype=torch.uint8, device="cuda")
        self.ws = workspace
        self.handle = ctypes.c_void_p()
        rc = _lib().gpz_batch_create(ctypes.byref(self.handle), arrays.jobs, arrays.njobs,
                                     ctypes.byref(self.p), ctypes.byref(self.config),
                                     self.ws.data_ptr(), self.ws.numel())
        _check(rc, "gpz_batch_create")
        self.njobs = arrays.njobs
        self._arrays = arrays

    @classmethod
    def empty(cls, max_jobs: int, max_blocks: int, p: Optional[Params] = None,
              config: Optional[BatchConfig] = None):
        """A batch with no jobs yet (bind them with rebind)."""
        import torch
        ws = torch.empty(256, dtype=torch.uint8, device="cuda")
        return cls(None, [], [], dec=None, p=p, config=config, workspace=ws, max_jobs=max_jobs,
                   max_blocks=max_blocks)

    @staticmethod
    def workspace_bytes(fields, ebs, outs, dec=None, p=None) -> int:
        arrays = _JobArrays(fields, ebs, outs, dec)
        pp = p if p is not None else params(3)
        return int(_lib().gpz_batch_workspace_bytes(arrays.jobs, arrays.njobs, ctypes.byref(pp)))

    def rebind(self, fields, ebs, outs, dec=None, workspace=None, stream=None, job_ws=None):
        """Bind new jobs; `job_ws[j]` optionally gives job j its own record-slot
        workspace (then `workspace` only has to hold the others)."""
        arrays = _JobArrays(fields, ebs, outs, dec, job_ws)
        ws = workspace if workspace is not None else self.ws
        rc = _lib().gpz_batch_rebind(self.handle, arrays.jobs, arrays.njobs, ws.data_ptr(),
                                     ws.numel(), _stream_handle(stream))
        _check(rc, "gpz_batch_rebind")
        self.njobs = arrays.njobs
        self._arrays = arrays
        self.ws = ws

    def rebind_prepared(self, jobs: Sequence[PreparedJob], workspace, stream=None):
        """Bind prepared jobs: only their structs are copied into one array
        (the host arrays they point at were built once, with the job)."""
        arr = (Job * max(1, len(jobs)))()
        for j, pj in enumerate(jobs):
            arr[j] = pj.job
        rc = _lib().gpz_batch_rebind(self.handle, arr, len(jobs), workspace.data_ptr(),
                                     workspace.numel(), _stream_handle(stream))
        _check(rc, "gpz_batch_rebind")
        self.njobs = len(jobs)
        self._arrays = (arr, list(jobs))
        self.ws = workspace

    def compress(self, stream=None):
        _check(_lib().gpz_batch_compress(self.handle, _stream_handle(stream)), "gpz_batch_compress")

    def decompress(self, stream=None):
        _check(_lib().gpz_batch_decompress(self.handle, _stream_handle(stream)),
               "gpz_batch_decompress")

    def sizes_device(self):
        """Stream sizes as a device tensor view (uint64, one per job)."""
        return device_view(_lib().gpz_batch_sizes(self.handle), self.njobs, "<i8")

    def capacity_views(self):
        """(sizes, errors): device tensor views of the batch's whole size and
        error tables (int64 / int32, max_jobs entries each).  The tables stay
        at the same address for the life of the batch, so the views are made
        once and sliced by the caller."""
        if getattr(self, "_views", None) is None:
            cap = max(1, self.config.max_jobs or self.njobs)
            self._views = (device_view(_lib().gpz_batch_sizes(self.handle), cap, "<i8"),
                           device_view(_lib().gpz_batch_errors(self.handle), cap, "<i4"))
        return self._views

    def sizes(self) -> np.ndarray:
        """Stream size per job (synchronizes the device)."""
        import torch
        torch.cuda.synchronize()
        ptr = _lib().gpz_batch_sizes(self.handle)
        out = np.zeros(self.njobs, np.uint64)
        _device_to_host(ptr, out)
        return out

    def errors(self) -> np.ndarray:
        import torch
        torch.cuda.synchronize()
        ptr = _lib().gpz_batch_errors(self.handle)
        out = np.zeros(self.njobs, np.uint32)
        _device_to_host(ptr, out)
        return out

    def close(self):
        if self.handle:
            _lib().gpz_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Zero-copy view of a library-owned device array for torch.as_tensor."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr,
                                         "data": (ptr, False), "version": 3, "strides": None}


def device_view(ptr: int, n: int, typestr: str):
    import torch
    return torch.as_tensor(_DeviceArray(ptr, n, typestr), device="cuda")


def _device_to_host(ptr: int, out: np.ndarray):
    typestr = {np.dtype(np.uint64): "<i8", np.dtype(np.uint32): "<i4"}[out.dtype]
    t = device_view(ptr, out.size, typestr)
    out[:] = t.cpu().numpy().view(out.dtype)
