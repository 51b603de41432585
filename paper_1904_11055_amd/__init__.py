"""MI355X (gfx950) angle-averaged polyspectrum estimator.

Thin Python binding over ``libpolyspec.so`` (see ``include/polyspec.h``).  The
functions named ``polyspec_*`` marshal arguments to the C calls of the same name;
every step of the computation runs in the library's HIP kernels.  PyTorch is used
only for device memory and the current stream.  ``Plan`` and ``polyspectrum``
are conveniences on top (``polyspectrum`` is differentiable for orders 3 and 4).

The estimator is the FFT form of Tomlinson, Jeong & Kim (2019), Sec. 2 and
Appendix A: B_t = sum_x prod_j d_{t_j}[x] / (N^3 n_t) over sorted shell tuples t,
with d_s the unnormalised inverse transform of the density restricted to shell s
and n_t the number of closed n-gons with sides in those shells.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

__all__ = [
    "PolyspecError", "Plan", "polyspectrum", "load_library",
    "FP32", "SPLIT_BF16", "SPLIT_FP16", "INPUT_HALF_SPECTRUM", "ALLOW_ALIASING", "NAN_GUARD", "STREAM_SLABS", "MULTIPOLE",
    "polyspec_plan", "polyspec_shells", "polyspec_contract", "polyspec_backward", "polyspec_forward_static",
    "polyspec_workspace_size", "polyspec_set_workspace", "polyspec_set_precision", "polyspec_set_multipole",
    "polyspec_set_slab_planes", "polyspec_slab_planes",
    "polyspec_tuples", "polyspec_candidates", "polyspec_fields", "polyspec_destroy",
    "polyspec_profile", "polyspec_profile_read", "PHASES",
    "polyspec_status_string", "polyspec_last_error",
]

FP32, SPLIT_BF16, SPLIT_FP16 = 0, 1, 2
STATIC_SCRATCH_BYTES = 128 << 20   # POLYSPEC_STATIC_SCRATCH_BYTES
INPUT_HALF_SPECTRUM, ALLOW_ALIASING, NAN_GUARD, STREAM_SLABS, MULTIPOLE = 1, 2, 8, 16, 32

STATUS = {0: "POLYSPEC_OK", 1: "POLYSPEC_ERR_INVALID_ARG", 2: "POLYSPEC_ERR_ALIASING",
          3: "POLYSPEC_ERR_OUT_OF_MEMORY", 4: "POLYSPEC_ERR_DEVICE",
          5: "POLYSPEC_ERR_COUNT_NOT_INTEGRAL", 6: "POLYSPEC_ERR_STATE", 7: "POLYSPEC_ERR_UNSUPPORTED"}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpolyspec.so")


class PolyspecError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")


class polyspec_desc(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("order", ctypes.c_int32), ("n_shells", ctypes.c_int32),
                ("shell_width", ctypes.c_double), ("batch", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("box_length", ctypes.c_double),
                ("flags", ctypes.c_uint32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Loads the HIP library; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_1904_11055_amd.build`")
    try:  # bind to the HIP runtime torch already carries, when torch is present
        import torch  # noqa: F401
    except Exception:
        pass
    lib = ctypes.CDLL(path)
    P, V, D = ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER
    sig = {
        "polyspec_plan": (ctypes.c_int, [D(polyspec_desc), V, D(P)]),
        "polyspec_shells": (ctypes.c_int, [P, V]),
        "polyspec_contract": (ctypes.c_int, [P, V, V]),
        "polyspec_forward_static": (ctypes.c_int, [P, V, V, V]),
        "polyspec_backward": (ctypes.c_int, [P, V, V]),
        "polyspec_workspace_size": (ctypes.c_int, [P, D(ctypes.c_size_t)]),
        "polyspec_set_workspace": (ctypes.c_int, [P, V, ctypes.c_size_t]),
        "polyspec_set_precision": (ctypes.c_int, [P, ctypes.c_int32]),
        "polyspec_set_multipole": (ctypes.c_int, [P, ctypes.c_int32]),
        "polyspec_set_slab_planes": (ctypes.c_int, [P, ctypes.c_int32]),
        "polyspec_slab_planes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_int32)]),
        "polyspec_tuples": (ctypes.c_int, [P, D(ctypes.c_int64), V, V]),
        "polyspec_candidates": (ctypes.c_int, [P, D(ctypes.c_int64), V, V]),
        "polyspec_fields": (ctypes.c_int, [P, D(ctypes.c_void_p)]),
        "polyspec_destroy": (ctypes.c_int, [P]),
        "polyspec_profile": (ctypes.c_int, [P, ctypes.c_int32]),
        "polyspec_profile_read": (ctypes.c_int, [P, V, V]),
        "polyspec_issued_flops": (ctypes.c_int, [P, ctypes.c_int32, D(ctypes.c_double)]),
        "polyspec_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "polyspec_last_error": (ctypes.c_char_p, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int, where: str, plan=None):
    if st != 0:
        lib = load_library()
        detail = lib.polyspec_last_error(plan).decode(errors="replace")
        raise PolyspecError(st, where, detail)


# --- same-name marshalling wrappers -------------------------------------------
def polyspec_status_string(status: int) -> str:
    return load_library().polyspec_status_string(status).decode()


def polyspec_last_error(plan) -> str:
    return load_library().polyspec_last_error(plan).decode(errors="replace")


def polyspec_plan(N, order, n_shells, shell_width, batch=1, precision=FP32, box_length=0.0,
                  flags=0, stream=None):
    lib = load_library()
    d = polyspec_desc(N, order, n_shells, float(shell_width), batch, precision, float(box_length), flags)
    h = ctypes.c_void_p()
    _check(lib.polyspec_plan(ctypes.byref(d), stream, ctypes.byref(h)), "polyspec_plan")
    return h


def polyspec_shells(plan, d_delta_ptr: int):
    _check(load_library().polyspec_shells(plan, ctypes.c_void_p(d_delta_ptr)), "polyspec_shells", plan)


def polyspec_contract(plan, d_out_ptr: int, d_raw_ptr: int | None = None):
    _check(load_library().polyspec_contract(plan, ctypes.c_void_p(d_out_ptr),
                                            ctypes.c_void_p(d_raw_ptr) if d_raw_ptr else None),
           "polyspec_contract", plan)


def polyspec_forward_static(plan, d_delta_ptr: int, d_out_ptr: int, d_raw_ptr: int | None = None):
    _check(load_library().polyspec_forward_static(plan, ctypes.c_void_p(d_delta_ptr), ctypes.c_void_p(d_out_ptr),
                                                  ctypes.c_void_p(d_raw_ptr) if d_raw_ptr else None),
           "polyspec_forward_static", plan)


def polyspec_backward(plan, d_grad_out_ptr: int, d_grad_delta_ptr: int):
    _check(load_library().polyspec_backward(plan, ctypes.c_void_p(d_grad_out_ptr),
                                            ctypes.c_void_p(d_grad_delta_ptr)), "polyspec_backward", plan)


def polyspec_workspace_size(plan) -> int:
    n = ctypes.c_size_t()
    _check(load_library().polyspec_workspace_size(plan, ctypes.byref(n)), "polyspec_workspace_size", plan)
    return n.value


def polyspec_set_workspace(plan, d_ptr: int, nbytes: int):
    _check(load_library().polyspec_set_workspace(plan, ctypes.c_void_p(d_ptr), nbytes),
           "polyspec_set_workspace", plan)


def polyspec_set_precision(plan, precision: int):
    _check(load_library().polyspec_set_precision(plan, precision), "polyspec_set_precision", plan)


def polyspec_set_multipole(plan, ell: int):
    _check(load_library().polyspec_set_multipole(plan, ell), "polyspec_set_multipole", plan)


def polyspec_set_slab_planes(plan, planes: int):
    _check(load_library().polyspec_set_slab_planes(plan, planes), "polyspec_set_slab_planes", plan)


def polyspec_slab_planes(plan) -> int:
    v = ctypes.c_int32()
    _check(load_library().polyspec_slab_planes(plan, ctypes.byref(v)), "polyspec_slab_planes", plan)
    return v.value


def polyspec_tuples(plan, order: int):
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.polyspec_tuples(plan, ctypes.byref(n), None, None), "polyspec_tuples", plan)
    bins = np.zeros((n.value, order), dtype=np.int32)
    counts = np.zeros(n.value, dtype=np.int64)
    _check(lib.polyspec_tuples(plan, ctypes.byref(n), bins.ctypes.data_as(ctypes.c_void_p),
                               counts.ctypes.data_as(ctypes.c_void_p)), "polyspec_tuples", plan)
    return bins, counts


def polyspec_candidates(plan, order: int):
    lib = load_library()
    n = ctypes.c_int64()
    _check(lib.polyspec_candidates(plan, ctypes.byref(n), None, None), "polyspec_candidates", plan)
    bins = np.zeros((n.value, order), dtype=np.int32)
    quot = np.zeros(n.value, dtype=np.float64)
    _check(lib.polyspec_candidates(plan, ctypes.byref(n), bins.ctypes.data_as(ctypes.c_void_p),
                                   quot.ctypes.data_as(ctypes.c_void_p)), "polyspec_candidates", plan)
    return bins, quot


def polyspec_fields(plan) -> int:
    ptr = ctypes.c_void_p()
    _check(load_library().polyspec_fields(plan, ctypes.byref(ptr)), "polyspec_fields", plan)
    return ptr.value


PHASES = ["input_q3", "input_q2", "input_q1", "shell_p1", "shell_p2", "shell_p3", "contract",
          "reduce", "gather", "adj_weights", "adj_gemm", "adj_q3", "adj_q2", "adj_q1",
          "grad_p1", "grad_p2", "grad_p3"]


def polyspec_profile(plan, enable: bool):
    _check(load_library().polyspec_profile(plan, 1 if enable else 0), "polyspec_profile", plan)


def polyspec_profile_read(plan):
    """{phase: (milliseconds, launches)} since the last read (synchronises the stream)."""
    ms = np.zeros(len(PHASES), dtype=np.float64)
    calls = np.zeros(len(PHASES), dtype=np.int64)
    _check(load_library().polyspec_profile_read(plan, ms.ctypes.data_as(ctypes.c_void_p),
                                                calls.ctypes.data_as(ctypes.c_void_p)),
           "polyspec_profile_read", plan)
    return {name: (float(ms[i]), int(calls[i])) for i, name in enumerate(PHASES)}


def polyspec_issued_flops(plan, phase: str) -> float:
    """Matrix-core flops one call issues in `phase` ("contract" or "adj_gemm")."""
    out = ctypes.c_double(0.0)
    _check(load_library().polyspec_issued_flops(plan, PHASES.index(phase), ctypes.byref(out)),
           "polyspec_issued_flops", plan)
    return out.value


def polyspec_destroy(plan):
    _check(load_library().polyspec_destroy(plan), "polyspec_destroy")


# --- conveniences ------------------------------------------------------------
class Plan:
    """One geometry (grid, order, shells) and batch, bound to torch's current stream."""

    def __init__(self, N, order, n_shells, shell_width, batch=1, precision=FP32, box_length=0.0,
                 flags=0, device=None, slab_planes=None, multipole=None):
        """multipole=ell (even, 0..16) selects the bispectrum multipole B_ell about the third grid
        axis: the plan's tuples are then (u, v, w) with the Legendre weight on shell w."""
        import torch
        if multipole is not None:
            flags |= MULTIPOLE
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.N, self.order, self.n_shells, self.width = N, order, n_shells, float(shell_width)
        self.batch, self.flags = batch, flags
        self._precision = precision
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self.handle = polyspec_plan(N, order, n_shells, shell_width, batch, precision, box_length,
                                        flags, ctypes.c_void_p(self.stream.cuda_stream))
        self._multipole = None
        if multipole is not None:
            self.multipole = multipole
        if slab_planes is not None:
            polyspec_set_slab_planes(self.handle, slab_planes)
        self.slab_planes = polyspec_slab_planes(self.handle)
        self.tuples, self.counts = polyspec_tuples(self.handle, order)
        self.n_closing = len(self.counts)
        self._workspace = None   # torch-allocated on the first shells() (after any slab setting)
        self.generation = 0      # bumped by every shells(); the autograd backward checks it

    def _ensure_workspace(self):
        """Hands the library device memory from torch's allocator (256-byte aligned), once."""
        if self._workspace is not None:
            return
        import torch
        nbytes = polyspec_workspace_size(self.handle)
        ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = ws.data_ptr()
        polyspec_set_workspace(self.handle, base + (-base) % 256, nbytes)
        self._workspace = ws     # the plan keeps the tensor alive
        self.workspace_bytes = nbytes

    @property
    def precision(self):
        return self._precision

    @precision.setter
    def precision(self, value):
        polyspec_set_precision(self.handle, value)
        self._precision = value

    @property
    def multipole(self):
        return self._multipole

    @multipole.setter
    def multipole(self, ell):
        """Switches a MULTIPOLE plan to another even ell; the next shells() recomputes the fields."""
        polyspec_set_multipole(self.handle, ell)
        self._multipole = ell

    def candidates(self):
        return polyspec_candidates(self.handle, self.order)

    def shells(self, delta):
        """delta: float32 [batch, N, N, N] (or complex64 half spectrum) on the plan's device."""
        import torch
        N = self.N
        if self.flags & INPUT_HALF_SPECTRUM:
            want, dt = (self.batch, N, N, N // 2 + 1), torch.complex64
        else:
            want, dt = (self.batch, N, N, N), torch.float32
        if tuple(delta.shape) != want or delta.dtype != dt or delta.device != self.device:
            raise ValueError(f"expected {dt} {want} on {self.device}, got {delta.dtype} {tuple(delta.shape)} "
                             f"on {delta.device}")
        delta = delta.contiguous()
        self._ensure_workspace()
        polyspec_shells(self.handle, delta.data_ptr())
        self._last_input = delta  # keep alive until the stream has consumed it
        self.generation += 1

    def contract(self, raw=False):
        import torch
        out = torch.empty((self.batch, self.n_closing), dtype=torch.float64, device=self.device)
        rs = torch.empty_like(out) if raw else None
        polyspec_contract(self.handle, out.data_ptr(), rs.data_ptr() if raw else None)
        return (out, rs) if raw else out

    def backward(self, grad_out):
        """dL/d(input) of the last shells() input, in its space (real field or half spectrum)."""
        import torch
        if tuple(grad_out.shape) != (self.batch, self.n_closing):
            raise ValueError(f"grad_out must have shape {(self.batch, self.n_closing)}, got {tuple(grad_out.shape)}")
        grad_out = grad_out.to(device=self.device, dtype=torch.float64).contiguous()
        N = self.N
        if self.flags & INPUT_HALF_SPECTRUM:
            g = torch.empty((self.batch, N, N, N // 2 + 1), dtype=torch.complex64, device=self.device)
        else:
            g = torch.empty((self.batch, N, N, N), dtype=torch.float32, device=self.device)
        polyspec_backward(self.handle, grad_out.data_ptr(), g.data_ptr())
        return g

    def fields(self):
        """A copy of the kept float32 shell fields [batch, n_fields, N, N, N] (n_fields is
        n_shells, or 2 n_shells for a multipole plan: the shells, then their weighted copies)."""
        import torch
        ptr = polyspec_fields(self.handle)
        n_fields = self.n_shells * (2 if self.flags & MULTIPOLE else 1)
        shape = (self.batch, n_fields, self.N, self.N, self.N)
        view = torch.as_tensor(_DeviceArray(ptr, shape, "<f4"), device=self.device)
        return view.clone()

    def close(self):
        if getattr(self, "handle", None):
            polyspec_destroy(self.handle)   # waits for the stream, then the workspace may go
            self.handle = None
        self._workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _DeviceArray:
    """Describes library-owned device memory to torch without copying."""

    def __init__(self, ptr, shape, typestr):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": typestr,
                                         "data": (int(ptr), False), "version": 2}


def polyspectrum(delta, plan: Plan):
    """B [batch, n_closing] (float64) of delta; differentiable for orders 3 and 4.

    delta is the real field [batch, N, N, N], or the half spectrum [batch, N, N, N/2+1]
    (complex64) for plans made with INPUT_HALF_SPECTRUM; the gradient is in the same
    space.  The plan keeps only the shell fields of its last input, so the backward of
    a result raises if the plan has run another forward since (its fields are stale).
    """
    import torch

    class _Fn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x):
            plan.shells(x.detach())
            ctx.generation = plan.generation
            return plan.contract()

        @staticmethod
        def backward(ctx, g):
            if plan.generation != ctx.generation:
                raise RuntimeError("polyspectrum backward: the plan has run another forward since this result "
                                   "was computed, so its shell fields belong to another input; use one plan per "
                                   "pending backward or run the backward first")
            return plan.backward(g)

    return _Fn.apply(delta)
