"""Python binding of libbzq (include/bzq.h): argument marshalling only.

Every step of the collision operator runs in the HIP library; this module
passes device pointers of torch tensors (PyTorch provides device memory and
the current stream) and turns status codes into exceptions.  There is no CPU
fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbzq.so")

FP64 = 0
FP32_ACC64 = 1
_PREC = {"fp64": FP64, "f64": FP64, FP64: FP64, "fp32": FP32_ACC64, "fp32_acc64": FP32_ACC64,
         FP32_ACC64: FP32_ACC64}

STATUS = {0: "BZQ_OK", 1: "BZQ_EINVAL", 2: "BZQ_ENOMEM", 3: "BZQ_EDEVICE", 4: "BZQ_EUNSUPPORTED",
          5: "BZQ_ENONFINITE"}


class BzqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2004_11239_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i, sz = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
    sigs = {
        "bzq_plan_create": ([ctypes.POINTER(vp), i, d, d, d, d, i, i, i, vp], i),
        "bzq_plan_create_general": ([ctypes.POINTER(vp), i, d, d, d, d, d, d, i, i, i, i, vp], i),
        "bzq_collision": ([vp, vp, vp, vp], i),
        "bzq_step": ([vp, vp, d, i, vp], i),
        "bzq_moments": ([vp, vp, vp, ctypes.POINTER(d), vp], i),
        "bzq_check_finite": ([vp, vp, vp], i),
        "bzq_collision_batch": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i, vp], i),
        "bzq_plan_device_bytes": ([vp], sz),
        "bzq_request_device_bytes": ([i], sz),
        "bzq_plan_info": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_pairs": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_weights": ([vp, i, ctypes.POINTER(d)], i),
        "bzq_plan_set_timing": ([vp, i], i),
        "bzq_plan_stage_times": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_destroy": ([vp], i),
        "bzq_status_string": ([i], ctypes.c_char_p),
        "bzq_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED = ("bzq_plan_create", "bzq_plan_create_general", "bzq_collision", "bzq_step", "bzq_moments",
            "bzq_check_finite", "bzq_collision_batch", "bzq_plan_device_bytes",
            "bzq_request_device_bytes", "bzq_plan_info", "bzq_plan_pairs", "bzq_plan_weights",
            "bzq_plan_set_timing", "bzq_plan_stage_times", "bzq_plan_destroy", "bzq_status_string", "bzq_last_error")


def lib():
    return _lib


def _check(code: int):
    if code != 0:
        raise BzqError(code, _lib.bzq_last_error().decode())


def _stream(stream=None) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _spectral(t: torch.Tensor, N: int, name: str):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 CUDA tensor")
    if tuple(t.shape) != (N, N, N) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous ({N},{N},{N}) tensor")
    return ctypes.c_void_p(t.data_ptr())


class Plan:
    """Plan of the collision operator for one (N, L, R, gamma, kernel, N_rho, M, precision)."""

    def __init__(self, N: int, L: float, R: float, gamma: float, s: float, N_rho: int, M: int,
                 precision="fp64", kernel: Optional[Sequence[float]] = None, n_jacobi: int = 64,
                 stream=None):
        """kernel=None: b = c_s sin^{-(2+2s)}(th/2), c_s = (1-s)(2-s)/(24 pi).
        kernel=(c, s_b, r): b = c t^{-1-s_b} (1-t)^{-r}, t = sin^2(th/2) (then `s` is ignored)."""
        self.N, self.L, self.R, self.gamma = int(N), float(L), float(R), float(gamma)
        self.N_rho, self.M = int(N_rho), int(M)
        self.precision = _PREC[precision]
        h = ctypes.c_void_p()
        st = _stream(stream)
        if kernel is None:
            self.kernel = ((1 - s) * (2 - s) / (24 * math.pi), float(s), 0.0)
            code = _lib.bzq_plan_create(ctypes.byref(h), self.N, self.L, self.R, self.gamma, float(s),
                                        self.N_rho, self.M, self.precision, st)
        else:
            self.kernel = tuple(float(x) for x in kernel)
            c, sb, r = self.kernel
            code = _lib.bzq_plan_create_general(ctypes.byref(h), self.N, self.L, self.R, self.gamma,
                                                c, sb, r, int(n_jacobi), self.N_rho, self.M,
                                                self.precision, st)
        _check(code)
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def collision(self, f_hat: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """Q(f, f) of eq. realQ; complex128 (N,N,N) in FFT order on the GPU."""
        fp = _spectral(f_hat, self.N, "f_hat")
        if out is None:
            out = torch.empty_like(f_hat)
        qp = _spectral(out, self.N, "out")
        _check(_lib.bzq_collision(self.handle, fp, qp, _stream(stream)))
        return out

    def step(self, f_hat: torch.Tensor, dt: float, n_steps: int = 1, stream=None):
        """n_steps Heun steps of d f/dt = Q(f, f), in place."""
        fp = _spectral(f_hat, self.N, "f_hat")
        _check(_lib.bzq_step(self.handle, fp, float(dt), int(n_steps), _stream(stream)))
        return f_hat

    def moments(self, f_hat: torch.Tensor, Q_hat: Optional[torch.Tensor] = None, stream=None):
        fp = _spectral(f_hat, self.N, "f_hat")
        qp = _spectral(Q_hat, self.N, "Q_hat") if Q_hat is not None else None
        out = (ctypes.c_double * 6)()
        _check(_lib.bzq_moments(self.handle, fp, qp, out, _stream(stream)))
        return {"mass": out[0], "momentum": (out[1], out[2], out[3]), "energy": out[4],
                "entropy_dissipation": out[5]}

    def check_finite(self, f_hat: torch.Tensor, stream=None) -> bool:
        fp = _spectral(f_hat, self.N, "f_hat")
        code = _lib.bzq_check_finite(self.handle, fp, _stream(stream))
        if code == 5:
            return False
        _check(code)
        return True

    def info(self) -> dict:
        out = (ctypes.c_double * 8)()
        _check(_lib.bzq_plan_info(self.handle, out))
        keys = ("N", "P", "npairs", "pairs_per_chunk", "splits", "precision", "n_jacobi", "table_bytes")
        return {k: (int(v) if k != "table_bytes" else float(v)) for k, v in zip(keys, out)}

    def pairs(self):
        import numpy as np
        n = self.info()["npairs"]
        out = (ctypes.c_double * (6 * n))()
        _check(_lib.bzq_plan_pairs(self.handle, out))
        return np.frombuffer(out, dtype=np.float64).reshape(n, 6).copy()

    def weights(self, pair: int):
        import numpy as np
        n1 = self.N - 1
        nh = (n1 * n1 + 1) // 2
        out = (ctypes.c_double * (nh * n1))()
        _check(_lib.bzq_plan_weights(self.handle, int(pair), out))
        return np.frombuffer(out, dtype=np.float64).reshape(nh, n1).copy()

    STAGES = ("prep", "zinv", "plane", "zfwd", "finalize")

    def set_timing(self, enable: bool):
        _check(_lib.bzq_plan_set_timing(self.handle, int(bool(enable))))

    def stage_times(self) -> dict:
        """{stage: (total_ms, launches)} since timing was enabled (synchronous)."""
        out = (ctypes.c_double * 10)()
        _check(_lib.bzq_plan_stage_times(self.handle, out))
        return {k: (out[i], int(out[5 + i])) for i, k in enumerate(self.STAGES)}

    def device_bytes(self) -> int:
        return int(_lib.bzq_plan_device_bytes(self.handle))

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.bzq_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def collision_batch(plans: Sequence[Plan], f_hats: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
                    stream=None):
    n = len(plans)
    if not (len(f_hats) == len(outs) == n):
        raise ValueError("plans, f_hats and outs must have the same length")
    P = (ctypes.c_void_p * n)(*[p.handle for p in plans])
    F = (ctypes.c_void_p * n)(*[_spectral(f, p.N, "f_hat") for p, f in zip(plans, f_hats)])
    Q = (ctypes.c_void_p * n)(*[_spectral(q, p.N, "out") for p, q in zip(plans, outs)])
    _check(_lib.bzq_collision_batch(P, F, Q, n, _stream(stream)))
    return outs


def request_device_bytes(N: int) -> int:
    return int(_lib.bzq_request_device_bytes(int(N)))
