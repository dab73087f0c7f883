"""Python binding of libprony with torch tensors (device memory and streams only).

The functions carry the C ABI's names without the `prony_` prefix. Each call
checks dtypes, devices and shapes, passes raw device pointers and strides to the
library on torch's current stream, and returns torch tensors. No arithmetic of
the method happens here.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib

_handles: dict = {}
_call_locks: dict = {}
_lock = threading.Lock()


def _handle(device: torch.device):
    """One library handle per device (created on first use)."""
    idx = device.index if device.index is not None else torch.cuda.current_device()
    with _lock:
        h = _handles.get(idx)
        if h is None:
            lib = _lib.load()
            hp = ctypes.c_void_p()
            st = lib.prony_create(ctypes.byref(hp), idx)
            if st != _lib.PRONY_OK:
                raise _lib.PronyError(st, f"prony_create(device={idx}) failed")
            h = hp
            _handles[idx] = h
            _call_locks[idx] = threading.Lock()
    return h


def _call(name: str, device: torch.device, *args):
    """Run one library call on torch's current stream. The handle is shared by the
    threads of the process; its lock keeps one call (stream switch and call) at a
    time. The library orders a new stream after the previous one's queued work."""
    lib = _lib.load()
    h = _handle(device)
    idx = device.index if device.index is not None else torch.cuda.current_device()
    stream = torch.cuda.current_stream(device)
    with _call_locks[idx]:
        st = lib.prony_set_stream(h, ctypes.c_void_p(stream.cuda_stream))
        if st != _lib.PRONY_OK:
            msg = lib.prony_last_error(h)
            raise _lib.PronyError(st, f"prony_set_stream: {msg.decode() if msg else ''}")
        st = getattr(lib, name)(h, *args)
        if st != _lib.PRONY_OK:
            msg = lib.prony_last_error(h)
            raise _lib.PronyError(st, f"{name}: {msg.decode() if msg else ''}")


def _ptr(x):
    return ctypes.c_void_p(x.data_ptr()) if x is not None else ctypes.c_void_p(0)


def _require(x: torch.Tensor, name: str, dtype, device=None, contiguous=True):
    if not isinstance(x, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")
    if not x.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if device is not None and x.device != device:
        raise ValueError(f"{name} is on {x.device}, expected {device}")
    if contiguous and not x.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def grid_size(d: int, n: int) -> int:
    return (2 * n + 2) ** d


def samples(t: torch.Tensor, c: torch.Tensor, n: int, noise: torch.Tensor | None = None,
            out: torch.Tensor | None = None) -> torch.Tensor:
    """Sample grid f(p), p in {-n..n+1}^d (prony_samples). t: (m, d) float64, c: (m,) complex128."""
    _require(t, "t", torch.float64)
    dev = t.device
    _require(c, "c", torch.complex128, dev)
    m, d = t.shape
    if c.shape != (m,):
        raise ValueError("c must have shape (m,)")
    G = grid_size(d, n)
    if noise is not None:
        _require(noise, "noise", torch.complex128, dev)
        if noise.numel() != G:
            raise ValueError("noise must have (2n+2)^d entries")
    if out is None:
        out = torch.empty(G, dtype=torch.complex128, device=dev)
    else:
        _require(out, "out", torch.complex128, dev)
        if out.numel() != G:
            raise ValueError("out must have (2n+2)^d entries")
    _call("prony_samples", dev, d, n, m, _ptr(t), _ptr(c), _ptr(noise), _ptr(out))
    return out


def build_T(f: torch.Tensor, d: int, n: int, which: int = 0, out: torch.Tensor | None = None) -> torch.Tensor:
    """T (which=0) or T_which as an N x N complex128 matrix (prony_build_T)."""
    _require(f, "f", torch.complex128)
    N = (n + 1) ** d
    if f.numel() != grid_size(d, n):
        raise ValueError("f must hold the (2n+2)^d sample grid")
    if out is None:
        out = torch.empty((N, N), dtype=torch.complex128, device=f.device)
    if out.dtype != torch.complex128 or out.dim() != 2 or out.shape[0] != N or out.shape[1] != N \
            or out.stride(1) != 1:
        raise ValueError("out must be an N x N complex128 matrix with unit column stride")
    _call("prony_build_T", f.device, d, n, which, _ptr(f), _ptr(out), out.stride(0))
    return out


_S_PRECS = {"fp64": _lib.PRONY_FP64, "fp32": _lib.PRONY_FP32, "bf16x3": _lib.PRONY_BF16X3}


def _build_S(entry: str, f, d, n, U, sigma, V, prec, with_s0, out):
    _require(f, "f", torch.complex128)
    dev = f.device
    if f.numel() != grid_size(d, n):
        raise ValueError("f must hold the (2n+2)^d sample grid")
    _require(U, "U", torch.complex128, dev, contiguous=False)
    _require(V, "V", torch.complex128, dev, contiguous=False)
    _require(sigma, "sigma", torch.float64, dev)
    N = (n + 1) ** d
    if U.dim() != 2 or U.shape[0] != N or V.shape != U.shape:
        raise ValueError("U and V must be N x m")
    m = U.shape[1]
    if sigma.shape != (m,):
        raise ValueError("sigma must have shape (m,)")
    if prec not in _S_PRECS:
        raise ValueError("prec must be 'fp64', 'fp32' or 'bf16x3'")
    ells = d + (1 if with_s0 else 0)
    if out is None:
        out = torch.empty((ells, m, m), dtype=torch.complex128, device=dev)
    else:
        _require(out, "out", torch.complex128, dev)
        if out.shape != (ells, m, m):
            raise ValueError("out has the wrong shape")
    _call(entry, dev, d, n, m, _ptr(f), _ptr(U), U.stride(0), U.stride(1), _ptr(sigma),
          _ptr(V), V.stride(0), V.stride(1), _S_PRECS[prec], _lib.PRONY_WITH_S0 if with_s0 else 0, _ptr(out))
    return out


def build_S(f: torch.Tensor, d: int, n: int, U: torch.Tensor, sigma: torch.Tensor, V: torch.Tensor,
            prec: str = "fp64", with_s0: bool = False, out: torch.Tensor | None = None) -> torch.Tensor:
    """S_l = U^* T_l V Sigma^{-1}, l = 1..d (prony_build_S); shape (d[+1], m, m).

    V is the right factor itself (torch.linalg.svd returns V^* as Vh: pass Vh.mH).
    prec: 'fp64', 'fp32' or 'bf16x3' (three-term bfloat16 splits on the bf16 MFMA,
    same error scale as 'fp32').
    """
    return _build_S("prony_build_S", f, d, n, U, sigma, V, prec, with_s0, out)


def build_S_noalloc(f: torch.Tensor, d: int, n: int, U: torch.Tensor, sigma: torch.Tensor, V: torch.Tensor,
                    out: torch.Tensor, prec: str = "fp64", with_s0: bool = False) -> torch.Tensor:
    """build_S through prony_build_S_noalloc: the library allocates no device memory
    (the caller passes `out`; the scratch is the library's fixed per-device array)."""
    if out is None:
        raise ValueError("build_S_noalloc needs a preallocated out")
    return _build_S("prony_build_S_noalloc", f, d, n, U, sigma, V, prec, with_s0, out)


class Factors:
    """Prepared factors (prony_factors_create): U, sigma and V packed once for
    S-builds with many sample grids; `build_S(f)` runs only the tile and finishing
    launches (prony_build_S_factors) and returns what build_S would under the plan
    current at creation. The packed copy is the factors' own: U, sigma and V may
    be released afterwards."""

    def __init__(self, d: int, n: int, U: torch.Tensor, sigma: torch.Tensor, V: torch.Tensor,
                 prec: str = "fp64", with_s0: bool = False):
        dev = U.device
        _require(U, "U", torch.complex128, dev, contiguous=False)
        _require(V, "V", torch.complex128, dev, contiguous=False)
        _require(sigma, "sigma", torch.float64, dev)
        N = (n + 1) ** d
        if U.dim() != 2 or U.shape[0] != N or V.shape != U.shape:
            raise ValueError("U and V must be N x m")
        m = U.shape[1]
        if sigma.shape != (m,):
            raise ValueError("sigma must have shape (m,)")
        if prec not in _S_PRECS:
            raise ValueError("prec must be 'fp64', 'fp32' or 'bf16x3'")
        self.d, self.n, self.m, self.prec, self.with_s0 = d, n, m, prec, with_s0
        self.device = dev
        self.handle = None
        out = ctypes.c_void_p()
        _call("prony_factors_create", dev, d, n, m, _ptr(U), U.stride(0), U.stride(1), _ptr(sigma), _ptr(V),
              V.stride(0), V.stride(1), _S_PRECS[prec], _lib.PRONY_WITH_S0 if with_s0 else 0, ctypes.byref(out))
        self.handle = out

    def build_S(self, f: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if self.handle is None:
            raise ValueError("factors are closed")
        _require(f, "f", torch.complex128, self.device)
        if f.numel() != grid_size(self.d, self.n):
            raise ValueError("f must hold the (2n+2)^d sample grid")
        ells = self.d + (1 if self.with_s0 else 0)
        if out is None:
            out = torch.empty((ells, self.m, self.m), dtype=torch.complex128, device=self.device)
        else:
            _require(out, "out", torch.complex128, self.device)
            if out.shape != (ells, self.m, self.m):
                raise ValueError("out has the wrong shape")
        _call("prony_build_S_factors", self.device, self.handle, _ptr(f), _ptr(out))
        return out

    def close(self) -> None:
        if self.handle is not None:
            st = _lib.load().prony_factors_destroy(self.handle)
            self.handle = None
            if st != _lib.PRONY_OK:
                raise _lib.PronyError(st, "prony_factors_destroy")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build_S_adjoint(gS: torch.Tensor, d: int, n: int, U: torch.Tensor, sigma: torch.Tensor, V: torch.Tensor,
                    prec: str = "fp32", out: torch.Tensor | None = None) -> torch.Tensor:
    """Gradient on the sample grid of a loss with dL/dS_l = gS[l-1] (prony_build_S_adjoint)."""
    _require(gS, "gS", torch.complex128)
    dev = gS.device
    _require(U, "U", torch.complex128, dev, contiguous=False)
    _require(V, "V", torch.complex128, dev, contiguous=False)
    _require(sigma, "sigma", torch.float64, dev)
    N = (n + 1) ** d
    if U.dim() != 2 or U.shape[0] != N or V.shape != U.shape:
        raise ValueError("U and V must be N x m")
    m = U.shape[1]
    if gS.shape != (d, m, m) or sigma.shape != (m,):
        raise ValueError("gS must be (d, m, m) and sigma (m,)")
    if prec not in ("fp64", "fp32"):
        raise ValueError("prec must be 'fp64' or 'fp32'")
    if out is None:
        out = torch.empty(grid_size(d, n), dtype=torch.complex128, device=dev)
    else:
        _require(out, "out", torch.complex128, dev)
        if out.numel() != grid_size(d, n):
            raise ValueError("out must hold (2n+2)^d values")
    _call("prony_build_S_adjoint", dev, d, n, m, _ptr(U), U.stride(0), U.stride(1), _ptr(sigma),
          _ptr(V), V.stride(0), V.stride(1), _ptr(gS), _lib.PRONY_FP32 if prec == "fp32" else _lib.PRONY_FP64,
          _ptr(out))
    return out


def toeplitz_mm(f: torch.Tensor, d: int, n: int, X: torch.Tensor, adjoint: bool = False, prec: str = "fp64",
                out: torch.Tensor | None = None) -> torch.Tensor:
    """Y = T X or T^* X for the multilevel Toeplitz matrix T of the grid f, without
    forming T (prony_toeplitz_mm). X: N x r complex128 with unit column stride."""
    _require(f, "f", torch.complex128)
    dev = f.device
    _require(X, "X", torch.complex128, dev, contiguous=False)
    N = (n + 1) ** d
    if f.numel() != grid_size(d, n):
        raise ValueError("f must hold the (2n+2)^d sample grid")
    if X.dim() != 2 or X.shape[0] != N or (X.shape[1] > 1 and X.stride(1) != 1):
        raise ValueError("X must be N x r with unit column stride")
    if prec not in ("fp64", "fp32"):
        raise ValueError("prec must be 'fp64' or 'fp32'")
    r = X.shape[1]
    if out is None:
        out = torch.empty((N, r), dtype=torch.complex128, device=dev)
    else:
        _require(out, "out", torch.complex128, dev, contiguous=False)
        if out.shape != (N, r) or (r > 1 and out.stride(1) != 1):
            raise ValueError("out must be N x r with unit column stride")
    _call("prony_toeplitz_mm", dev, d, n, 1 if adjoint else 0, _ptr(f), r, _ptr(X), X.stride(0),
          _lib.PRONY_FP32 if prec == "fp32" else _lib.PRONY_FP64, _ptr(out), out.stride(0))
    return out


def coeffs(z: torch.Tensor, f: torch.Tensor, d: int, n: int, want_AT: bool = False):
    """Gram (A^T)^* A^T and rhs (A^T)^* f_I (prony_coeffs); optionally A^T (N x m)."""
    _require(z, "z", torch.complex128)
    dev = z.device
    _require(f, "f", torch.complex128, dev)
    if f.numel() != grid_size(d, n):
        raise ValueError("f must hold the (2n+2)^d sample grid")
    if z.dim() != 2 or z.shape[1] != d:
        raise ValueError("z must be m x d")
    m = z.shape[0]
    gram = torch.empty((m, m), dtype=torch.complex128, device=dev)
    rhs = torch.empty(m, dtype=torch.complex128, device=dev)
    AT = torch.empty(((n + 1) ** d, m), dtype=torch.complex128, device=dev) if want_AT else None
    _call("prony_coeffs", dev, d, n, m, _ptr(z), _ptr(f), _ptr(gram), _ptr(rhs), _ptr(AT))
    return (gram, rhs, AT) if want_AT else (gram, rhs)


def reserve(device: torch.device, d_max: int, n_max: int, m_max: int) -> None:
    """Pre-size the library workspace (prony_reserve)."""
    _call("prony_reserve", device, d_max, n_max, m_max)


def synchronize(device: torch.device) -> None:
    _call("prony_synchronize", device)


def profile_enable(device: torch.device, kernel: str | None) -> None:
    """Bracket every later launch of `kernel` with HIP events (None stops; resets records)."""
    _call("prony_profile_enable", device, kernel.encode() if kernel else None)


def profile_read(device: torch.device):
    """(launches, total milliseconds) of the profiled kernel since profile_enable."""
    launches = ctypes.c_int()
    total = ctypes.c_double()
    _call("prony_profile_read", device, ctypes.byref(launches), ctypes.byref(total))
    return launches.value, total.value


class Batch:
    """A planned S-build of many instances (prony_batch_create).

    instances: sequence of (d, n, f, U, sigma, V) with U, V contiguous N x m
    complex128 device tensors; the outputs S (d, m, m) are allocated here (or
    taken from `outputs`, contiguous (d, m, m) complex128 tensors) and exposed as
    `batch.S`. The tensors are referenced for the batch's lifetime.
    """

    def __init__(self, instances, prec: str = "fp32", outputs=None):
        if prec not in ("fp64", "fp32"):
            raise ValueError("prec must be 'fp64' or 'fp32'")
        if not instances:
            raise ValueError("empty batch")
        dev = instances[0][2].device
        descs = (_lib.InstanceDesc * len(instances))()
        self._keep = []
        self.S = []
        for i, (d, n, f, U, sigma, V) in enumerate(instances):
            N = (n + 1) ** d
            _require(f, "f", torch.complex128, dev)
            _require(U, "U", torch.complex128, dev)
            _require(V, "V", torch.complex128, dev)
            _require(sigma, "sigma", torch.float64, dev)
            if f.numel() != grid_size(d, n) or U.dim() != 2 or U.shape[0] != N or V.shape != U.shape:
                raise ValueError(f"instance {i}: shapes do not match d={d}, n={n}")
            m = U.shape[1]
            if outputs is None:
                S = torch.empty((d, m, m), dtype=torch.complex128, device=dev)
            else:
                S = outputs[i]
                _require(S, "S", torch.complex128, dev)
                if S.shape != (d, m, m):
                    raise ValueError(f"instance {i}: output must be ({d}, {m}, {m})")
            descs[i] = _lib.InstanceDesc(d, n, m, f.data_ptr(), U.data_ptr(), sigma.data_ptr(),
                                         V.data_ptr(), S.data_ptr())
            self._keep += [f, U, sigma, V, S]
            self.S.append(S)
        self.shapes = [(d, n, U.shape[1]) for d, n, f, U, sigma, V in instances]
        self.gs_sizes = [d * m * m for d, n, m in self.shapes]
        self.gf_sizes = [grid_size(d, n) for d, n, m in self.shapes]
        self.device = dev
        self.prec = prec
        self.graph = None
        out = ctypes.c_void_p()
        _call("prony_batch_create", dev, len(instances), descs,
              _lib.PRONY_FP32 if prec == "fp32" else _lib.PRONY_FP64, ctypes.byref(out))
        self.handle = out

    def set_schedule(self, schedule: str) -> None:
        """'classes' (one launch per tile class over four streams; the default)
        or 'queue' (one persistent launch over all tiles, FP32 only) —
        prony_batch_set_schedule. Results are bitwise equal."""
        codes = {"queue": _lib.PRONY_SCHEDULE_QUEUE, "classes": _lib.PRONY_SCHEDULE_CLASSES}
        if schedule not in codes:
            raise ValueError("schedule must be 'queue' or 'classes'")
        lib = _lib.load()
        if self.graph is not None:     # a captured graph holds the old schedule's launches
            lib.prony_graph_destroy(self.graph)
            self.graph = None
        st = lib.prony_batch_set_schedule(self.handle, codes[schedule])
        if st != _lib.PRONY_OK:
            msg = lib.prony_last_error(_handle(self.device))
            raise _lib.PronyError(st, f"prony_batch_set_schedule: {msg.decode() if msg else ''}")

    def run(self) -> None:
        """Enqueue the S-build of every instance (prony_build_S_batched)."""
        _call("prony_build_S_batched", self.device, self.handle)

    def adjoint(self, gS_all: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Grid gradients of all instances from their dL/dS (prony_build_S_adjoint_batched).

        gS_all: the (d, m, m) gradients of all instances flattened and concatenated
        in instance order (sum of gs_sizes complex128 values). Returns the grid
        gradients concatenated the same way (sum of gf_sizes values)."""
        _require(gS_all, "gS_all", torch.complex128, self.device)
        if gS_all.numel() != sum(self.gs_sizes):
            raise ValueError("gS_all must hold sum(gs_sizes) values")
        if out is None:
            out = torch.empty(sum(self.gf_sizes), dtype=torch.complex128, device=self.device)
        else:
            _require(out, "out", torch.complex128, self.device)
            if out.numel() != sum(self.gf_sizes):
                raise ValueError("out must hold sum(gf_sizes) values")
        _call("prony_build_S_adjoint_batched", self.device, self.handle, _ptr(gS_all), _ptr(out))
        return out

    def capture(self) -> None:
        """Capture run() into a HIP graph (prony_graph_capture)."""
        if self.graph is None:
            g = ctypes.c_void_p()
            _call("prony_graph_capture", self.device, self.handle, ctypes.byref(g))
            self.graph = g

    def replay(self) -> None:
        """Launch the captured graph on torch's current stream (prony_graph_launch)."""
        if self.graph is None:
            self.capture()
        _call("prony_graph_launch", self.device, self.graph)

    def close(self) -> None:
        lib = _lib.load()
        if self.graph is not None:
            lib.prony_graph_destroy(self.graph)
            self.graph = None
        if self.handle is not None and self.handle.value:
            lib.prony_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
