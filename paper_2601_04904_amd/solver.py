"""Thin Python binding over the C ABI: same names, argument marshalling only.

PyTorch provides device memory and the HIP stream; every step of SI and SQ
runs in the library's HIP kernels.  There is no CPU path.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BT_DIAG_ONLY, BT_FP64, BT_FUSED, BT_GRAPH, BT_MIXED, BT_PLAIN, BT_SIGMA_ANTIHERMITIAN, BTError,
                   BTToleranceError, check, check_tol, make_desc)

FIELDS = ("diag", "upper", "lower", "arrow_right", "arrow_bottom", "tip")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("a ROCm GPU is required (torch.cuda.is_available() is False)")
    return torch


class DeviceBlocks:
    """Six complex128 device tensors in the layout of include/bt_si_sq.h."""

    def __init__(self, diag, upper, lower, arrow_right, arrow_bottom, tip):
        self.diag, self.upper, self.lower = diag, upper, lower
        self.arrow_right, self.arrow_bottom, self.tip = arrow_right, arrow_bottom, tip

    @property
    def n(self):
        return self.diag.shape[0]

    @property
    def b(self):
        return self.diag.shape[1]

    @property
    def a(self):
        return self.tip.shape[0]

    @staticmethod
    def empty(n: int, b: int, a: int, device="cuda", zero=False):
        torch = _torch()
        f = torch.zeros if zero else torch.empty
        z = torch.complex128
        m = max(n - 1, 0)
        return DeviceBlocks(f((n, b, b), dtype=z, device=device), f((m, b, b), dtype=z, device=device),
                            f((m, b, b), dtype=z, device=device), f((n, b, a), dtype=z, device=device),
                            f((n, a, b), dtype=z, device=device), f((a, a), dtype=z, device=device))

    @staticmethod
    def from_host(M, device="cuda"):
        torch = _torch()
        t = [torch.from_numpy(np.ascontiguousarray(getattr(M, f), dtype=np.complex128)).to(device)
             for f in FIELDS]
        return DeviceBlocks(*t)

    def to_host(self):
        from types import SimpleNamespace
        return SimpleNamespace(**{f: getattr(self, f).cpu().numpy() for f in FIELDS})

    def c_blocks(self) -> _lib.bt_blocks:
        bl = _lib.bt_blocks()
        for f in FIELDS:
            t = getattr(self, f)
            assert t.is_contiguous() and t.dtype.is_complex
            setattr(bl, f, t.data_ptr() if t.numel() > 0 else None)
        return bl


class VarDeviceBlocks:
    """Device storage for diagonal blocks of different sizes, in the layout of
    include/bt_si_sq.h: one flat complex128 tensor per field, block i of a
    field after blocks 0..i-1 of that field."""

    def __init__(self, sizes, a, diag, upper, lower, arrow_right, arrow_bottom, tip):
        self.sizes, self.a = [int(v) for v in sizes], int(a)
        self.diag, self.upper, self.lower = diag, upper, lower
        self.arrow_right, self.arrow_bottom, self.tip = arrow_right, arrow_bottom, tip

    @property
    def n(self):
        return len(self.sizes)

    @staticmethod
    def _counts(sizes, a):
        n = len(sizes)
        return dict(diag=[s * s for s in sizes],
                    upper=[sizes[i] * sizes[i + 1] for i in range(n - 1)],
                    lower=[sizes[i] * sizes[i + 1] for i in range(n - 1)],
                    arrow_right=[s * a for s in sizes], arrow_bottom=[s * a for s in sizes],
                    tip=[a * a])

    @staticmethod
    def empty(sizes, a, device="cuda", zero=False):
        torch = _torch()
        f = torch.zeros if zero else torch.empty
        cnt = VarDeviceBlocks._counts(sizes, a)
        return VarDeviceBlocks(sizes, a, *[f(sum(cnt[k]), dtype=torch.complex128, device=device)
                                           for k in FIELDS])

    @staticmethod
    def from_host(M, device="cuda"):
        """From any object with list-of-blocks fields (synth.VBTA)."""
        torch = _torch()
        sizes = [int(np.shape(d)[0]) for d in M.diag]
        a = int(np.shape(M.tip)[0])
        flat = []
        for k in FIELDS:
            v = getattr(M, k)
            parts = [np.asarray(v, dtype=np.complex128).ravel()] if k == "tip" else \
                [np.asarray(x, dtype=np.complex128).ravel() for x in v]
            arr = np.concatenate(parts) if parts else np.zeros(0, np.complex128)
            flat.append(torch.from_numpy(np.ascontiguousarray(arr)).to(device))
        return VarDeviceBlocks(sizes, a, *flat)

    def to_host(self):
        """Lists of blocks (tip as one array)."""
        from types import SimpleNamespace
        n, sz, a = self.n, self.sizes, self.a
        shapes = dict(diag=[(s, s) for s in sz],
                      upper=[(sz[i], sz[i + 1]) for i in range(n - 1)],
                      lower=[(sz[i + 1], sz[i]) for i in range(n - 1)],
                      arrow_right=[(s, a) for s in sz], arrow_bottom=[(a, s) for s in sz])
        out = {}
        for k in FIELDS:
            flat = getattr(self, k).cpu().numpy()
            if k == "tip":
                out[k] = flat.reshape(a, a)
                continue
            blocks, off = [], 0
            for r, c in shapes[k]:
                blocks.append(flat[off:off + r * c].reshape(r, c))
                off += r * c
            out[k] = blocks
        return SimpleNamespace(**out)

    def c_blocks(self) -> _lib.bt_blocks:
        bl = _lib.bt_blocks()
        for f in FIELDS:
            t = getattr(self, f)
            assert t.is_contiguous() and t.dtype.is_complex
            setattr(bl, f, t.data_ptr() if t.numel() > 0 else None)
        return bl


def workspace_bytes(n, b, a=0, partitions=1, bounds=None, precision=BT_FP64, sizes=None,
                    reduced_parts=0) -> int:
    d = make_desc(n, b, a, partitions, bounds, precision, sizes=sizes, reduced_parts=reduced_parts)
    return int(_lib.lib().bt_si_sq_workspace_bytes(C.byref(d)))


def partition_bounds(n, b, a=0, partitions=1, bounds=None, sizes=None):
    d = make_desc(n, b, a, partitions, bounds, sizes=sizes)
    out = (C.c_int32 * (partitions + 1))()
    check(_lib.lib().bt_si_sq_partition_bounds(C.byref(d), out))
    return list(out)


def flops(n, b, a=0, partitions=1, bounds=None, flags=0, sizes=None, reduced_parts=0):
    """(executed, useful) real flops of one fused SI+SQ solve."""
    d = make_desc(n, b, a, partitions, bounds, flags=flags, sizes=sizes, reduced_parts=reduced_parts)
    ex, us = C.c_double(), C.c_double()
    check(_lib.lib().bt_si_sq_flops(C.byref(d), C.byref(ex), C.byref(us)))
    return ex.value, us.value


class Solver:
    """bt_si_sq_create / _factor / _selected_solve / _solve / _sync / _destroy.

    flags: BT_PLAIN (reference schedule), BT_GRAPH (launch lists replayed as
    HIP graphs), BT_SIGMA_ANTIHERMITIAN (Sigma^< anti-Hermitian, asserted by
    the caller and not checked; fewer X^< products), BT_DIAG_ONLY (diagonal
    blocks only), BT_FUSED (blocks and tip <= 64: the whole solve in one
    workgroup, one launch).
    """

    def __init__(self, n, b, a=0, partitions=1, bounds=None, precision=BT_FP64, tol=1e-4,
                 stream=None, flags=0, sizes=None, reduced_parts=0):
        torch = _torch()
        self.n, self.b, self.a = n, b, a
        self._desc = make_desc(n, b, a, partitions, bounds, precision, tol, flags, sizes, reduced_parts)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        check(_lib.lib().bt_si_sq_create(C.byref(self._desc), C.c_void_p(self.stream.cuda_stream),
                                         C.byref(h)))
        self._h = h
        self._keep = []

    def _blocks(self, M):
        if M is None:
            return None
        bl = M.c_blocks()
        self._keep.append(M)
        return C.byref(bl)

    def factor(self, A: DeviceBlocks, XR: DeviceBlocks = None):
        self._keep = [A, XR]
        check(_lib.lib().bt_si_sq_factor(self._h, self._blocks(A), self._blocks(XR)), self._h)

    def selected_solve(self, B: DeviceBlocks, XL: DeviceBlocks):
        err, fb = C.c_double(), C.c_int()
        self._keep.extend([B, XL])
        st = _lib.lib().bt_si_sq_selected_solve(self._h, self._blocks(B), self._blocks(XL),
                                                C.byref(err), C.byref(fb))
        check_tol(st, self._h, err.value, bool(fb.value))
        return err.value, bool(fb.value)

    def solve(self, A: DeviceBlocks, B: DeviceBlocks, XR: DeviceBlocks, XL: DeviceBlocks):
        err, fb = C.c_double(), C.c_int()
        self._keep = [A, B, XR, XL]
        st = _lib.lib().bt_si_sq_solve(self._h, self._blocks(A), self._blocks(B), self._blocks(XR),
                                       self._blocks(XL), C.byref(err), C.byref(fb))
        check_tol(st, self._h, err.value, bool(fb.value))
        return err.value, bool(fb.value)

    def sync(self):
        check(_lib.lib().bt_si_sq_sync(self._h), self._h)

    def last_launch_count(self) -> int:
        return int(_lib.lib().bt_si_sq_last_launch_count(self._h))

    def profile(self, enable: bool = True):
        check(_lib.lib().bt_si_sq_profile(self._h, int(bool(enable))), self._h)

    def profile_stats(self):
        """{kernel name: dict(launches, total_ms, flops, bytes)} since profile(True)."""
        arr = (_lib.bt_kernel_stat * 8)()
        cnt = C.c_int32()
        check(_lib.lib().bt_si_sq_profile_stats(self._h, arr, 8, C.byref(cnt)), self._h)
        return {_lib.KERNEL_NAMES[arr[i].kind]: dict(launches=arr[i].launches, total_ms=arr[i].total_ms,
                                                      flops=arr[i].flops, bytes=arr[i].bytes)
                for i in range(cnt.value)}

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.lib().bt_si_sq_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class BatchSolver:
    """bt_si_sq_batch_create / _batch_solve: many uneven instances in one schedule.

    specs: list of dicts with n, b, a and optionally partitions, bounds,
    precision, tol, flags, sizes.  workspace: None (the library allocates
    the handle's device memory), or a contiguous device tensor of at least
    batch_workspace_bytes(specs) bytes that the handle uses instead
    (bt_si_sq_batch_create_in; kept alive by the solver until destroy).
    """

    def __init__(self, specs, stream=None, workspace=None):
        torch = _torch()
        self.count = len(specs)
        self._descs = [make_desc(sp["n"], sp.get("b", 0), sp.get("a", 0), sp.get("partitions", 1),
                                 sp.get("bounds"), sp.get("precision", BT_FP64), sp.get("tol", 1e-4),
                                 sp.get("flags", 0), sp.get("sizes"), sp.get("reduced_parts", 0))
                       for sp in specs]
        arr = (_lib.bt_desc * self.count)(*self._descs)
        self._arr = arr
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = C.c_void_p()
        self._workspace = workspace
        if workspace is None:
            check(_lib.lib().bt_si_sq_batch_create(self.count, arr, C.c_void_p(self.stream.cuda_stream),
                                                   C.byref(h)))
        else:
            assert workspace.is_cuda and workspace.is_contiguous()
            nbytes = workspace.numel() * workspace.element_size()
            check(_lib.lib().bt_si_sq_batch_create_in(self.count, arr, C.c_void_p(self.stream.cuda_stream),
                                                      C.c_void_p(workspace.data_ptr()), nbytes, C.byref(h)))
        self._h = h

    def solve(self, A, B, XR, XL):
        """Lists of DeviceBlocks (XR may be None).  Returns (err_estimates, used_fp64_fallback)."""
        n = self.count

        def arr(ms):
            if ms is None:
                return None
            return (_lib.bt_blocks * n)(*[m.c_blocks() for m in ms])

        self._keep = (A, B, XR, XL)
        err = (C.c_double * n)()
        fb = (C.c_int * n)()
        st = _lib.lib().bt_si_sq_batch_solve(self._h, arr(A), arr(B), arr(XR), arr(XL), err, fb)
        check_tol(st, self._h, list(err), [bool(x) for x in fb])
        return list(err), [bool(x) for x in fb]

    def selected_solve(self, B, XL):
        """New right-hand sides on the resident factors; entries of XL may be None (skipped)."""
        n = self.count
        empty = _lib.bt_blocks()
        barr = (_lib.bt_blocks * n)(*[(b.c_blocks() if b is not None else empty) for b in B])
        larr = (_lib.bt_blocks * n)(*[(x.c_blocks() if x is not None else empty) for x in XL])
        self._keep2 = (B, XL)
        err = (C.c_double * n)()
        fb = (C.c_int * n)()
        st = _lib.lib().bt_si_sq_batch_selected_solve(self._h, barr, larr, err, fb)
        check_tol(st, self._h, list(err), [bool(x) for x in fb])
        return list(err), [bool(x) for x in fb]

    def sync(self):
        check(_lib.lib().bt_si_sq_sync(self._h), self._h)

    def last_launch_count(self) -> int:
        return int(_lib.lib().bt_si_sq_last_launch_count(self._h))

    def destroy(self):
        if getattr(self, "_h", None):
            _lib.lib().bt_si_sq_destroy(self._h)
            self._h = None
        self._workspace = None      # the caller's memory may be reused only now

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def batch_workspace_bytes(specs) -> int:
    descs = [make_desc(sp["n"], sp.get("b", 0), sp.get("a", 0), sp.get("partitions", 1), sp.get("bounds"),
                       sp.get("precision", BT_FP64), sp.get("tol", 1e-4), sp.get("flags", 0),
                       sp.get("sizes"), sp.get("reduced_parts", 0)) for sp in specs]
    arr = (_lib.bt_desc * len(descs))(*descs)
    return int(_lib.lib().bt_si_sq_batch_workspace_bytes(len(descs), arr))


__all__ = ["DeviceBlocks", "VarDeviceBlocks", "Solver", "BatchSolver", "workspace_bytes", "batch_workspace_bytes",
           "partition_bounds", "flops", "BT_FP64", "BT_MIXED", "BT_PLAIN", "BT_GRAPH", "BT_SIGMA_ANTIHERMITIAN",
           "BT_DIAG_ONLY", "BT_FUSED", "BTError", "BTToleranceError",
           "autotune", "tune_table", "set_tune_table"]


def tune_table():
    """The product tile-shape tuning table as a list of BT_TUNE_ENTRIES ints
    ([precision][size class][work class], -1 = default rule)."""
    t = (C.c_int32 * _lib.BT_TUNE_ENTRIES)()
    check(_lib.lib().bt_si_sq_tune_table(t, 1))
    return list(t)


def set_tune_table(table):
    vals = [int(v) for v in table]
    if len(vals) != _lib.BT_TUNE_ENTRIES:
        raise ValueError(f"tuning table needs {_lib.BT_TUNE_ENTRIES} entries, got {len(vals)}")
    t = (C.c_int32 * _lib.BT_TUNE_ENTRIES)(*vals)
    check(_lib.lib().bt_si_sq_tune_table(t, 0))


def autotune(stream=None, cache=None):
    """Time the product tile shapes on this device and fill the tuning table.

    Returns the report lines ("prec size_class work_class shape us0 us1 us2").
    With cache (a file path) the table is loaded from it if present, else
    tuned and written there (JSON)."""
    import json
    import os
    if cache and os.path.exists(cache):
        with open(cache) as f:
            rec = json.load(f)
        set_tune_table(rec["table"])
        return rec.get("report", [])
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    buf = C.create_string_buffer(1 << 16)
    check(_lib.lib().bt_si_sq_autotune(C.c_void_p(st.cuda_stream), buf, len(buf)))
    report = [ln for ln in buf.value.decode().splitlines() if ln]
    if cache:
        os.makedirs(os.path.dirname(os.path.abspath(cache)), exist_ok=True)
        with open(cache, "w") as f:
            json.dump({"table": tune_table(), "report": report}, f)
    return report


def diag_gemm(alpha, A, opA, B, opB, beta=0.0, Cin=None, D=None, mixed=False, stream=None, shape=-1):
    """D = beta Cin + alpha op(A) op(B) on the device (2-D complex128 tensors); returns D.
    shape: product tile shape, -1 for the tuning table's choice."""
    torch = _torch()
    m = A.shape[1] if opA else A.shape[0]
    k = A.shape[0] if opA else A.shape[1]
    n = B.shape[0] if opB else B.shape[1]
    if D is None:
        D = torch.empty((m, n), dtype=torch.complex128, device=A.device)
    st = stream if stream is not None else torch.cuda.current_stream()
    al = (C.c_double * 2)(complex(alpha).real, complex(alpha).imag)
    be = (C.c_double * 2)(complex(beta).real, complex(beta).imag)
    check(_lib.lib().bt_si_sq_diag_gemm(
        m, n, k, al, A.data_ptr(), A.stride(0), int(bool(opA)), B.data_ptr(), B.stride(0),
        int(bool(opB)), be, Cin.data_ptr() if Cin is not None else None,
        Cin.stride(0) if Cin is not None else 0, D.data_ptr(), D.stride(0), int(bool(mixed)),
        int(shape), C.c_void_p(st.cuda_stream)))
    return D


def diag_inverse(src, stream=None):
    """Batched inverse of a (count, d, d) complex128 device tensor; returns (dst, bad_index)."""
    torch = _torch()
    src = src.contiguous()
    dst = torch.empty_like(src)
    st = stream if stream is not None else torch.cuda.current_stream()
    bad = C.c_int32(-1)
    status = _lib.lib().bt_si_sq_diag_inverse(src.data_ptr(), dst.data_ptr(), src.shape[-1],
                                              src.shape[0], C.byref(bad), C.c_void_p(st.cuda_stream))
    if status not in (_lib.BT_OK, _lib.BT_ERR_SINGULAR):
        check(status)
    return dst, (bad.value if status == _lib.BT_ERR_SINGULAR else -1)


def diag_inverse_noalloc(src, dst=None, stream=None):
    """bt_si_sq_diag_inverse_noalloc: the batched inverse with the library's fixed
    scratch array (no device allocation by the library).  dst may be given
    (preallocated) so that the call allocates nothing at all."""
    torch = _torch()
    assert src.is_contiguous()
    if dst is None:
        dst = torch.empty_like(src)
    st = stream if stream is not None else torch.cuda.current_stream()
    bad = C.c_int32(-1)
    status = _lib.lib().bt_si_sq_diag_inverse_noalloc(src.data_ptr(), dst.data_ptr(), src.shape[-1],
                                                      src.shape[0], C.byref(bad), C.c_void_p(st.cuda_stream))
    if status not in (_lib.BT_OK, _lib.BT_ERR_SINGULAR):
        check(status)
    return dst, (bad.value if status == _lib.BT_ERR_SINGULAR else -1)
