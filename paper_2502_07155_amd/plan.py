"""Thin torch-facing wrapper of the blnfft C ABI.

Only argument checking and marshalling happen here: every step of the transform runs
in the library's HIP kernels on the plan's stream.  Torch provides device memory and
the stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from ._lib import METHODS, PRECISIONS, WINDOWS, Stats, check, load


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def window_transform(v, M: int, L: int, m: int, beta: float = 0.0, window: str = "sinh",
                     method: str = "shannon") -> np.ndarray:
    """Host-side univariate psihat (shannon) or phihat (nfft) at frequencies v, as used
    for the deconvolution factors."""
    lib = load()
    v = np.ascontiguousarray(np.atleast_1d(np.asarray(v, dtype=np.float64)))
    out = np.empty_like(v)
    P = ctypes.POINTER(ctypes.c_double)
    check(lib.bl_window_transform(WINDOWS[window], METHODS[method], M, L, m, float(beta), v.size,
                                  v.ctypes.data_as(P), out.ctypes.data_as(P)),
          "bl_window_transform")
    return out


class Plan:
    """One transform configuration (Algorithm 4.2 or Algorithm 2.1) on one device/stream.

    precision: "f64", "f32" (plain float), "f32c" (float data and FFT arithmetic with FP64
    twiddles and deconvolution factors, two-sum compensated short sums) or "f32d" (float
    data, FP64 FFT arithmetic and FP64 accumulation of the short sums).
    Inputs/outputs are torch tensors on the plan's device: fhat (M,)*d complex, nodes (N, d)
    real, f (N,) complex, in the plan's precision."""

    def __init__(self, d: int, M: int, L: int, m: int, window: str = "sinh", beta: float = 0.0,
                 method: str = "shannon", precision: str = "f32c", device=None, stream=None):
        self._lib = load()
        self.d, self.M, self.L, self.m = int(d), int(M), int(L), int(m)
        self.method, self.precision, self.window = method, precision, window
        self.real_dtype = torch.float64 if precision == "f64" else torch.float32
        self.complex_dtype = torch.complex128 if precision == "f64" else torch.complex64
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(self._lib.bl_plan_create(ctypes.byref(h), self.d, self.M, self.L, self.m,
                                           WINDOWS[window], float(beta), METHODS[method],
                                           PRECISIONS[precision],
                                           ctypes.c_void_p(self.stream.cuda_stream)),
                  "bl_plan_create")
        self._h = h
        self.N = 0
        self._nodes_version = 0
        self._forward_version = 0

    # -- helpers
    def _check(self, t: torch.Tensor, shape, dtype, name: str):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} must be on {self.device}, got {t.device}")
        if t.dtype != dtype:
            raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _dev(self):
        return torch.cuda.device(self.device)

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    # -- calls
    def set_nodes(self, x: torch.Tensor) -> None:
        N = int(x.shape[0]) if x.dim() >= 1 else 0
        self._check(x, (N, self.d), self.real_dtype, "x")
        with self._dev():
            check(self._lib.bl_set_nodes(self.handle, N, _ptr(x)), "bl_set_nodes")
        self.N = N
        self._nodes_version += 1

    def bind_nodes(self, x: torch.Tensor) -> None:
        """set_nodes, skipped when x is the tensor (same storage, shape and version) that
        is bound already."""
        key = (x.data_ptr(), tuple(x.shape), x._version, x.dtype)
        if getattr(self, "_bound_key", None) == key and self._bound_nodes == self._nodes_version:
            return
        self.set_nodes(x)
        self._bound_key = key
        self._bound_nodes = self._nodes_version

    def forward(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(fhat, (self.M,) * self.d, self.complex_dtype, "fhat")
        if out is None:
            out = torch.empty(self.N, dtype=self.complex_dtype, device=self.device)
        self._check(out, (self.N,), self.complex_dtype, "out")
        with self._dev():
            check(self._lib.bl_forward(self.handle, _ptr(fhat), _ptr(out)), "bl_forward")
        self._forward_version += 1
        return out

    def samples(self, fhat: torch.Tensor) -> None:
        """bl_samples: steps 1-2 alone; the samples theta stay in the plan (theta())."""
        self._check(fhat, (self.M,) * self.d, self.complex_dtype, "fhat")
        with self._dev():
            check(self._lib.bl_samples(self.handle, _ptr(fhat)), "bl_samples")
        self._forward_version += 1

    def state(self) -> tuple:
        """(node binding, forward) counters: identifies the samples theta the plan holds."""
        return (self._nodes_version, self._forward_version)

    def precompute_weights(self, enable: bool = True) -> None:
        """Store the bound nodes' window weights once (Algorithm 4.2, step 0b) for later
        transforms with the same nodes; enable=False returns to on-the-fly weights."""
        with self._dev():
            check(self._lib.bl_precompute_weights(self.handle, int(bool(enable))),
                  "bl_precompute_weights")

    def interpolate(self, theta: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(theta, (self.L,) * self.d, self.complex_dtype, "theta")
        if out is None:
            out = torch.empty(self.N, dtype=self.complex_dtype, device=self.device)
        self._check(out, (self.N,), self.complex_dtype, "out")
        with self._dev():
            check(self._lib.bl_interpolate(self.handle, _ptr(theta), _ptr(out)), "bl_interpolate")
        return out

    def theta(self) -> torch.Tensor:
        out = torch.empty((self.L,) * self.d, dtype=self.complex_dtype, device=self.device)
        with self._dev():
            check(self._lib.bl_get_theta(self.handle, _ptr(out)), "bl_get_theta")
        return out

    def adjoint(self, g: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(g, (self.N,), self.complex_dtype, "g")
        if out is None:
            out = torch.empty((self.M,) * self.d, dtype=self.complex_dtype, device=self.device)
        self._check(out, (self.M,) * self.d, self.complex_dtype, "out")
        with self._dev():
            check(self._lib.bl_adjoint(self.handle, _ptr(g), _ptr(out)), "bl_adjoint")
        return out

    def adjoint_noalloc(self, g: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """bl_adjoint_noalloc: the adjoint without any device allocation (the caller passes
        the output; the spreading grid lives in the library's fixed device scratch)."""
        self._check(g, (self.N,), self.complex_dtype, "g")
        self._check(out, (self.M,) * self.d, self.complex_dtype, "out")
        with self._dev():
            check(self._lib.bl_adjoint_noalloc(self.handle, _ptr(g), _ptr(out)), "bl_adjoint_noalloc")
        return out

    def grad_x(self, g: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(g, (self.N,), self.complex_dtype, "g")
        if out is None:
            out = torch.empty((self.N, self.d), dtype=self.real_dtype, device=self.device)
        self._check(out, (self.N, self.d), self.real_dtype, "out")
        with self._dev():
            check(self._lib.bl_grad_x(self.handle, _ptr(g), _ptr(out)), "bl_grad_x")
        return out

    def stats(self) -> dict:
        s = Stats()
        check(self._lib.bl_plan_stats(self.handle, ctypes.byref(s)), "bl_plan_stats")
        return {"n_nodes": s.n_nodes, "n_outside": s.n_outside, "n_chunks": s.n_chunks,
                "tile": tuple(s.tile), "chunk_cap": s.chunk_cap,
                "workspace_bytes": s.workspace_bytes, "beta": s.beta,
                "weight_fit_err": s.weight_fit_err,
                "fft_lines": (tuple(s.fft_lines[0:3]), tuple(s.fft_lines[3:6])),
                "fft_radix": (tuple(s.fft_radix[0:3]), tuple(s.fft_radix[3:6])),
                "tuned": {"fft": int(s.tuned[0]), "tiles": int(s.tuned[1])}}

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            self._lib.bl_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class BatchPlan:
    """Many independent d = 1 transforms (Algorithm 4.2) with their own (M_i, L_i, m_i, N_i),
    run together: one graph launch per forward call.

    Packed buffers: fhat (sum M_i,) complex64, instance after instance, each in the order
    k = -M_i/2 .. M_i/2 - 1; nodes (sum N_i,) float32; f (sum N_i,) complex64."""

    def __init__(self, M, L, m, N, precision: str = "f32", device=None, stream=None):
        self._lib = load()
        self.M = [int(v) for v in M]
        self.L = [int(v) for v in L]
        self.m = [int(v) for v in m]
        self.N = [int(v) for v in N]
        if not (len(self.M) == len(self.L) == len(self.m) == len(self.N)):
            raise ValueError("M, L, m and N must have the same length")
        self.count = len(self.M)
        self.precision = precision
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.fhat_offsets = np.concatenate([[0], np.cumsum(self.M)]).astype(np.int64)
        self.node_offsets = np.concatenate([[0], np.cumsum(self.N)]).astype(np.int64)
        self.total_M = int(self.fhat_offsets[-1])
        self.total_N = int(self.node_offsets[-1])
        i64 = ctypes.c_int64 * max(self.count, 1)
        i32 = ctypes.c_int * max(self.count, 1)
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(self._lib.bl_batch_create(ctypes.byref(h), self.count, i64(*self.M), i64(*self.L),
                                            i32(*self.m), i64(*self.N), PRECISIONS[precision],
                                            ctypes.c_void_p(self.stream.cuda_stream)),
                  "bl_batch_create")
        self._h = h

    def _check(self, t: torch.Tensor, n: int, dtype, name: str):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device or t.dtype != dtype or tuple(t.shape) != (n,) \
                or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous ({n},) {dtype} tensor on {self.device}")

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("batch destroyed")
        return self._h

    def set_nodes(self, x: torch.Tensor) -> None:
        self._check(x, self.total_N, torch.float32, "x")
        with torch.cuda.device(self.device):
            check(self._lib.bl_batch_set_nodes(self.handle, _ptr(x)), "bl_batch_set_nodes")

    def forward(self, fhat: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check(fhat, self.total_M, torch.complex64, "fhat")
        if out is None:
            out = torch.empty(self.total_N, dtype=torch.complex64, device=self.device)
        self._check(out, self.total_N, torch.complex64, "out")
        with torch.cuda.device(self.device):
            check(self._lib.bl_batch_forward(self.handle, _ptr(fhat), _ptr(out)), "bl_batch_forward")
        return out

    def split(self, f: torch.Tensor) -> list:
        """Per-instance views of a packed output."""
        return [f[self.node_offsets[i]:self.node_offsets[i + 1]] for i in range(self.count)]

    def close(self) -> None:
        if getattr(self, "_h", None) is not None:
            self._lib.bl_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
