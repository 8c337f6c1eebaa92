"""Python binding of libbzq (include/bzq.h): argument marshalling only.

Every step of the collision operator runs in the HIP library; this module
passes device pointers of torch tensors (PyTorch provides device memory and
the current stream) and turns status codes into exceptions.  There is no CPU
fallback: if the library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbzq.so")

FP64 = 0
FP32_ACC64 = 1
_PREC = {"fp64": FP64, "f64": FP64, FP64: FP64, "fp32": FP32_ACC64, "fp32_acc64": FP32_ACC64,
         FP32_ACC64: FP32_ACC64}

KERNEL_POWER = 0
KERNEL_CUTOFF_CONST = 1
KERNEL_GENERAL = 2

STATUS = {0: "BZQ_OK", 1: "BZQ_EINVAL", 2: "BZQ_ENOMEM", 3: "BZQ_EDEVICE", 4: "BZQ_EUNSUPPORTED",
          5: "BZQ_ENONFINITE", 6: "BZQ_EBUSY"}
REQ_STEP = 0
REQ_COLLISION = 1
SERVER_TUNE = 1


class BzqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class BzqRequest(ctypes.Structure):
    """Mirror of bzq_request (include/bzq.h)."""
    _fields_ = [("N", ctypes.c_int), ("L", ctypes.c_double), ("R", ctypes.c_double),
                ("gamma", ctypes.c_double), ("s", ctypes.c_double), ("N_rho", ctypes.c_int),
                ("M", ctypes.c_int), ("precision", ctypes.c_int), ("dt", ctypes.c_double),
                ("n_steps", ctypes.c_int), ("kind", ctypes.c_int)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python -m paper_2004_11239_amd.build)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, d, i, sz = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_size_t
    sigs = {
        "bzq_plan_create": ([ctypes.POINTER(vp), i, d, d, d, d, i, i, i, i, vp], i),
        "bzq_plan_create_general": ([ctypes.POINTER(vp), i, d, d, d, d, d, d, i, i, i, i, vp], i),
        "bzq_plan_create_otf": ([ctypes.POINTER(vp), i, d, d, d, i, d, d, d, i, i, i, vp], i),
        "bzq_plan_create_debye": ([ctypes.POINTER(vp), i, d, d, d, i, i, i, vp], i),
        "bzq_plan_derive_gamma": ([ctypes.POINTER(vp), vp, d, vp], i),
        "bzq_plan_shared_bytes": ([vp], sz),
        "bzq_collision": ([vp, vp, vp, vp], i),
        "bzq_collision_noalloc": ([vp, vp, vp, vp], i),
        "bzq_step": ([vp, vp, d, i, vp], i),
        "bzq_step_rk4": ([vp, vp, d, i, vp], i),
        "bzq_plan_set_schedule": ([vp, vp], i),
        "bzq_plan_schedule": ([vp, vp], i),
        "bzq_plan_autotune": ([vp, vp, i, vp], i),
        "bzq_moments": ([vp, vp, vp, ctypes.POINTER(d), vp], i),
        "bzq_check_finite": ([vp, vp, vp], i),
        "bzq_collision_batch": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i, vp], i),
        "bzq_plan_device_bytes": ([vp], sz),
        "bzq_request_device_bytes": ([i, i], sz),
        "bzq_plan_info": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_pairs": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_weights": ([vp, i, ctypes.POINTER(d)], i),
        "bzq_workspace_create": ([ctypes.POINTER(vp), vp], i),
        "bzq_collision_ws": ([vp, vp, vp, vp, vp], i),
        "bzq_step_ws": ([vp, vp, vp, d, i, vp], i),
        "bzq_workspace_bytes": ([vp], sz),
        "bzq_workspace_destroy": ([vp], i),
        "bzq_batch_create": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp), i, i, vp], i),
        "bzq_batch_collision": ([vp, ctypes.POINTER(vp), vp], i),
        "bzq_batch_step": ([vp, d, i, i, vp], i),
        "bzq_batch_groups": ([vp], i),
        "bzq_batch_rounds": ([vp], i),
        "bzq_batch_group_info": ([vp, i, ctypes.POINTER(i)], i),
        "bzq_batch_device_bytes": ([vp], sz),
        "bzq_batch_destroy": ([vp], i),
        "bzq_server_create": ([ctypes.POINTER(vp), sz, i, i, i], i),
        "bzq_server_submit": ([vp, ctypes.POINTER(BzqRequest), vp, ctypes.POINTER(ctypes.c_ulonglong)], i),
        "bzq_server_poll": ([vp, ctypes.c_ulonglong, vp, ctypes.POINTER(d)], i),
        "bzq_server_wait": ([vp, ctypes.c_ulonglong, d], i),
        "bzq_server_stats": ([vp, ctypes.POINTER(d)], i),
        "bzq_server_destroy": ([vp], i),
        "bzq_plan_bytes_estimate": ([i, i, i, i], sz),
        "bzq_plan_set_timing": ([vp, i], i),
        "bzq_plan_stage_times": ([vp, ctypes.POINTER(d)], i),
        "bzq_plan_destroy": ([vp], i),
        "bzq_plan2d_create": ([ctypes.POINTER(vp), i, d, d, d, d, d, d, i, i, i, i, vp], i),
        "bzq_collision2d": ([vp, vp, vp, vp], i),
        "bzq_step2d": ([vp, vp, d, i, i, vp], i),
        "bzq_plan2d_destroy": ([vp], i),
        "bzq_status_string": ([i], ctypes.c_char_p),
        "bzq_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()
EXPORTED_EXTRA = ("bzq_workspace_create", "bzq_collision_ws", "bzq_step_ws", "bzq_workspace_bytes",
                  "bzq_workspace_destroy", "bzq_batch_create", "bzq_batch_collision", "bzq_batch_step",
                  "bzq_batch_groups", "bzq_batch_group_info", "bzq_batch_device_bytes",
                  "bzq_batch_destroy", "bzq_server_create", "bzq_server_submit", "bzq_server_poll",
                  "bzq_server_wait", "bzq_server_stats", "bzq_server_destroy", "bzq_plan_bytes_estimate")
EXPORTED = ("bzq_plan_create", "bzq_plan_create_general", "bzq_plan_create_otf", "bzq_plan_create_debye",
            "bzq_plan_derive_gamma",
            "bzq_plan_shared_bytes", "bzq_collision", "bzq_step", "bzq_step_rk4", "bzq_moments",
            "bzq_check_finite", "bzq_collision_batch", "bzq_plan_device_bytes",
            "bzq_request_device_bytes", "bzq_plan_info", "bzq_plan_pairs", "bzq_plan_weights",
            "bzq_plan_set_timing", "bzq_plan_stage_times", "bzq_plan_destroy", "bzq_status_string", "bzq_last_error",
            "bzq_plan_set_schedule", "bzq_plan_schedule", "bzq_plan_autotune", "bzq_plan2d_create",
            "bzq_collision2d", "bzq_step2d", "bzq_plan2d_destroy")


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
                 stream=None, weights: str = "table"):
        """kernel=None: b = c_s sin^{-(2+2s)}(th/2), c_s = (1-s)(2-s)/(24 pi) (BZQ_KERNEL_POWER);
        kernel="cutoff": b = 1/(4 pi) (BZQ_KERNEL_CUTOFF_CONST; `s` is ignored);
        kernel=(c, s_b, r): b = c t^{-1-s_b} (1-t)^{-r}, t = sin^2(th/2) (then `s` is ignored).
        weights="table" stores the weights at creation; "otf" evaluates them per
        chunk of pairs from their series (bzq_plan_create_otf)."""
        self.N, self.L, self.R, self.gamma = int(N), float(L), float(R), float(gamma)
        self.N_rho, self.M = int(N_rho), int(M)
        self.precision = _PREC[precision]
        if weights not in ("table", "otf"):
            raise ValueError("weights must be 'table' or 'otf'")
        self.weights_mode = weights
        h = ctypes.c_void_p()
        st = _stream(stream)
        if kernel is None:
            self.kernel, ksel, kargs = ("power", float(s)), KERNEL_POWER, (0.0, float(s), 0.0)
        elif isinstance(kernel, str):
            if kernel != "cutoff":
                raise ValueError("kernel must be None, 'cutoff' or (c, s, r)")
            self.kernel, ksel, kargs = ("cutoff",), KERNEL_CUTOFF_CONST, (0.0, 0.0, 0.0)
        else:
            self.kernel = tuple(float(x) for x in kernel)
            ksel, kargs = KERNEL_GENERAL, self.kernel
        if weights == "otf":
            c, sb, r = kargs
            code = _lib.bzq_plan_create_otf(ctypes.byref(h), self.N, self.L, self.R, self.gamma, ksel, c, sb, r,
                                            self.N_rho, self.M, self.precision, st)
        elif ksel != KERNEL_GENERAL:
            code = _lib.bzq_plan_create(ctypes.byref(h), self.N, self.L, self.R, self.gamma, kargs[1],
                                        self.N_rho, self.M, self.precision, ksel, st)
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

    @classmethod
    def debye(cls, N: int, L: float, R: float, theta_cut: float, N_rho: int, M: int, precision="fp64",
              stream=None) -> "Plan":
        """The Debye-Yukawa kernel of Section 5.6 (gamma = 1), zero below theta_cut
        (pi/10 for the paper's cutoff version, 0 for the non-cutoff kernel)."""
        h = ctypes.c_void_p()
        prec = _PREC[precision]
        _check(_lib.bzq_plan_create_debye(ctypes.byref(h), int(N), float(L), float(R), float(theta_cut),
                                          int(N_rho), int(M), prec, _stream(stream)))
        p = cls.__new__(cls)
        p.N, p.L, p.R, p.gamma = int(N), float(L), float(R), 1.0
        p.N_rho, p.M, p.precision = int(N_rho), int(M), prec
        p.weights_mode, p.kernel = "table", ("debye", float(theta_cut))
        p._h = h
        return p

    def with_gamma(self, gamma: float, stream=None) -> "Plan":
        """A plan for another gamma sharing this plan's tables (bzq_plan_derive_gamma)."""
        h = ctypes.c_void_p()
        _check(_lib.bzq_plan_derive_gamma(ctypes.byref(h), self.handle, float(gamma), _stream(stream)))
        p = Plan.__new__(Plan)
        p.N, p.L, p.R, p.gamma = self.N, self.L, self.R, float(gamma)
        p.N_rho, p.M, p.precision = self.N_rho, self.M, self.precision
        p.weights_mode, p.kernel = self.weights_mode, self.kernel
        p._h = h
        return p

    def shared_bytes(self) -> int:
        return int(_lib.bzq_plan_shared_bytes(self.handle))

    def collision(self, f_hat: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """Q(f, f) of eq. realQ; complex128 (N,N,N) in FFT order on the GPU."""
        fp = _spectral(f_hat, self.N, "f_hat")
        if out is None:
            out = torch.empty_like(f_hat)
        qp = _spectral(out, self.N, "out")
        _check(_lib.bzq_collision(self.handle, fp, qp, _stream(stream)))
        return out

    def collision_noalloc(self, f_hat: torch.Tensor, out: torch.Tensor, stream=None):
        """Q(f, f) with the library's static device scratch (bzq_collision_noalloc):
        no allocation in the call; `out` must be given."""
        fp = _spectral(f_hat, self.N, "f_hat")
        qp = _spectral(out, self.N, "out")
        _check(_lib.bzq_collision_noalloc(self.handle, fp, qp, _stream(stream)))
        return out

    def step(self, f_hat: torch.Tensor, dt: float, n_steps: int = 1, stream=None, method: str = "heun"):
        """n_steps steps of d f/dt = Q(f, f), in place: Heun's method (default)
        or the classical fourth-order Runge-Kutta method (method="rk4")."""
        fp = _spectral(f_hat, self.N, "f_hat")
        if method == "heun":
            _check(_lib.bzq_step(self.handle, fp, float(dt), int(n_steps), _stream(stream)))
        elif method == "rk4":
            _check(_lib.bzq_step_rk4(self.handle, fp, float(dt), int(n_steps), _stream(stream)))
        else:
            raise ValueError("method must be 'heun' or 'rk4'")
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

    def set_timing(self, enable, stages=None):
        """Per-launch HIP events on the timed stages (all stages, or the listed
        stage names: prep, zinv, plane, zfwd, finalize)."""
        if not enable:
            mask = 0
        elif stages is None:
            mask = 1
        else:
            mask = sum(1 << self.STAGES.index(n) for n in stages)
            if mask == 1:
                raise ValueError("the prep stage cannot be timed alone")
        _check(_lib.bzq_plan_set_timing(self.handle, int(mask)))

    def schedule(self) -> dict:
        """Kernel variant per stage (as used), the last stage's workgroup target and splits."""
        out = (ctypes.c_int * 5)()
        _check(_lib.bzq_plan_schedule(self.handle, out))
        return {"zinv": out[0], "plane": out[1], "zfwd": out[2], "s_target": out[3], "splits": out[4]}

    def set_schedule(self, zinv: int = 0, plane: int = 0, zfwd: int = 0, s_target: int = 1024):
        arr = (ctypes.c_int * 4)(int(zinv), int(plane), int(zfwd), int(s_target))
        _check(_lib.bzq_plan_set_schedule(self.handle, arr))
        return self.schedule()

    def autotune(self, f_hat: torch.Tensor, use_cache: bool = True, stream=None) -> dict:
        """Time the kernel variants on f_hat and keep the fastest schedule (synchronous)."""
        fp = _spectral(f_hat, self.N, "f_hat")
        _check(_lib.bzq_plan_autotune(self.handle, fp, int(bool(use_cache)), _stream(stream)))
        return self.schedule()

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


class Plan2D:
    """Plan of the two-dimensional operator (d = 2, Section 5.2): kernel
    b = c t^{-1-s} (1-t)^{-r} with t = sin^2(th/2), N_rho Gauss-Legendre nodes on
    [0, R], the midpoint rule of N_sigma points on the circle."""

    def __init__(self, N: int, L: float, R: float, gamma: float, kernel: Sequence[float], N_rho: int,
                 N_sigma: int, precision="fp64", n_jacobi: int = 64, stream=None):
        self.N, self.L, self.R, self.gamma = int(N), float(L), float(R), float(gamma)
        self.kernel = tuple(float(x) for x in kernel)
        self.N_rho, self.N_sigma = int(N_rho), int(N_sigma)
        self.precision = _PREC[precision]
        c, sb, r = self.kernel
        h = ctypes.c_void_p()
        _check(_lib.bzq_plan2d_create(ctypes.byref(h), self.N, self.L, self.R, self.gamma, c, sb, r,
                                      int(n_jacobi), self.N_rho, self.N_sigma, self.precision,
                                      _stream(stream)))
        self._h = h

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("plan destroyed")
        return self._h

    def _spectral2d(self, t: torch.Tensor, name: str):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
            raise TypeError(f"{name} must be a complex128 CUDA tensor")
        if tuple(t.shape) != (self.N, self.N) or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous ({self.N},{self.N}) tensor")
        return ctypes.c_void_p(t.data_ptr())

    def collision(self, f_hat: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None):
        """Q(f, f) of eq. realQ in 2-D; complex128 (N,N) in FFT order on the GPU."""
        fp = self._spectral2d(f_hat, "f_hat")
        if out is None:
            out = torch.empty_like(f_hat)
        qp = self._spectral2d(out, "out")
        _check(_lib.bzq_collision2d(self.handle, fp, qp, _stream(stream)))
        return out

    def step(self, f_hat: torch.Tensor, dt: float, n_steps: int = 1, method: str = "rk4", stream=None):
        """n_steps of Heun's method ("heun") or classical RK4 ("rk4"), in place."""
        fp = self._spectral2d(f_hat, "f_hat")
        m = {"heun": 0, "rk4": 1}[method]
        _check(_lib.bzq_step2d(self.handle, fp, float(dt), int(n_steps), m, _stream(stream)))
        return f_hat

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.bzq_plan2d_destroy(self._h)
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


def request_device_bytes(N: int, precision="fp32") -> int:
    return int(_lib.bzq_request_device_bytes(int(N), _PREC[precision]))


class Workspace:
    """Extra scratch so that one plan can be evaluated on several streams at once."""

    def __init__(self, plan: Plan):
        h = ctypes.c_void_p()
        _check(_lib.bzq_workspace_create(ctypes.byref(h), plan.handle))
        self.plan = plan
        self._h = h

    def collision(self, f_hat, out=None, stream=None):
        fp = _spectral(f_hat, self.plan.N, "f_hat")
        if out is None:
            out = torch.empty_like(f_hat)
        _check(_lib.bzq_collision_ws(self.plan.handle, self._h, fp, _spectral(out, self.plan.N, "out"),
                                     _stream(stream)))
        return out

    def step(self, f_hat, dt, n_steps=1, stream=None):
        _check(_lib.bzq_step_ws(self.plan.handle, self._h, _spectral(f_hat, self.plan.N, "f_hat"),
                                float(dt), int(n_steps), _stream(stream)))
        return f_hat

    def device_bytes(self):
        return int(_lib.bzq_workspace_bytes(self._h))

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.bzq_workspace_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Batch:
    """Fused evaluation of many independent cells (see bzq_batch_create)."""

    def __init__(self, plans: Sequence[Plan], f_hats: Sequence[torch.Tensor], cells_per_launch: int = 0,
                 stream=None):
        n = len(plans)
        if n != len(f_hats) or n == 0:
            raise ValueError("plans and f_hats must be non-empty and of equal length")
        self.plans = list(plans)
        self.f_hats = list(f_hats)          # kept alive: the batch holds their pointers
        P = (ctypes.c_void_p * n)(*[p.handle for p in plans])
        F = (ctypes.c_void_p * n)(*[_spectral(f, p.N, "f_hat") for p, f in zip(plans, f_hats)])
        h = ctypes.c_void_p()
        _check(_lib.bzq_batch_create(ctypes.byref(h), P, F, n, int(cells_per_launch), _stream(stream)))
        self._h = h

    def collision(self, outs: Sequence[torch.Tensor], stream=None):
        n = len(self.plans)
        Q = (ctypes.c_void_p * n)(*[_spectral(q, p.N, "out") for p, q in zip(self.plans, outs)])
        _check(_lib.bzq_batch_collision(self._h, Q, _stream(stream)))
        return outs

    def step(self, dt: float, n_steps: int = 1, use_graph: bool = True, stream=None):
        _check(_lib.bzq_batch_step(self._h, float(dt), int(n_steps), int(bool(use_graph)), _stream(stream)))

    def rounds(self) -> int:
        """Rounds of the mixed-size launches (0: one group of launches per plan)."""
        return int(_lib.bzq_batch_rounds(self._h))

    def groups(self):
        out = []
        for g in range(_lib.bzq_batch_groups(self._h)):
            v = (ctypes.c_int * 4)()
            _check(_lib.bzq_batch_group_info(self._h, g, v))
            out.append({"N": v[0], "cells": v[1], "cells_per_launch": v[2], "tuned": bool(v[3])})
        return out

    def device_bytes(self):
        return int(_lib.bzq_batch_device_bytes(self._h))

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.bzq_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


class Server:
    """Request server with continuous batching (see bzq_server_create):
    max_queued bounds the waiting requests (0: unbounded; a full queue makes
    submit raise BzqError with code BZQ_EBUSY), tune times each new plan's
    schedule on its first request."""

    def __init__(self, budget_bytes: int, slots: int = 4, max_queued: int = 0, tune: bool = False):
        h = ctypes.c_void_p()
        _check(_lib.bzq_server_create(ctypes.byref(h), int(budget_bytes), int(slots), int(max_queued),
                                      SERVER_TUNE if tune else 0))
        self._h = h

    def submit(self, f_hat_host, N, L, R, gamma, s, N_rho, M, precision="fp32", dt=0.01, n_steps=10,
               kind="step"):
        """kind="step": n_steps Heun steps of f; kind="collision": Q(f) (dt, n_steps unused)."""
        import numpy as np
        f = np.ascontiguousarray(f_hat_host, dtype=np.complex128)
        if f.shape != (N, N, N):
            raise ValueError("f_hat must be (N, N, N)")
        k = {"step": REQ_STEP, "collision": REQ_COLLISION}[kind]
        req = BzqRequest(N, L, R, gamma, s, N_rho, M, _PREC[precision], dt, n_steps, k)
        rid = ctypes.c_ulonglong()
        _check(_lib.bzq_server_submit(self._h, ctypes.byref(req), f.ctypes.data_as(ctypes.c_void_p),
                                      ctypes.byref(rid)))
        return rid.value

    def poll(self, rid: int, N: int):
        """None if not finished, else (f_hat_result, (arrival, start, done))."""
        import numpy as np
        out = np.empty((N, N, N), dtype=np.complex128)
        t = (ctypes.c_double * 3)()
        r = _lib.bzq_server_poll(self._h, ctypes.c_ulonglong(rid), out.ctypes.data_as(ctypes.c_void_p), t)
        if r == 0:
            return None
        if r == -1:
            raise KeyError(rid)
        if r == -2:
            raise BzqError(2, _lib.bzq_last_error().decode())
        return out, (t[0], t[1], t[2])

    def wait(self, rid: int, timeout: float = 600.0):
        _check(_lib.bzq_server_wait(self._h, ctypes.c_ulonglong(rid), float(timeout)))

    def stats(self):
        v = (ctypes.c_double * 9)()
        _check(_lib.bzq_server_stats(self._h, v))
        keys = ("submitted", "completed", "failed", "queued", "running", "device_bytes", "peak_device_bytes",
                "evictions", "rejected")
        return {k: v[i] for i, k in enumerate(keys)}

    def destroy(self):
        if getattr(self, "_h", None) is not None:
            _lib.bzq_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def plan_bytes_estimate(N: int, N_rho: int, M: int, precision="fp32") -> int:
    return int(_lib.bzq_plan_bytes_estimate(int(N), int(N_rho), int(M), _PREC[precision]))
