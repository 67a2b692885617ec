"""Python binding of libcme.so: the C ABI of include/cme.h, argument marshalling only.

The functions keep the C names (cme_init, cme_step, cme_run, cme_adjoint,
cme_status, cme_destroy, cme_strerror, ...) and take torch tensors that live
on the GPU; every step of the computation runs in the library's HIP kernels.
PyTorch only provides device memory and the stream.  There is no CPU
fallback: if the library is not built or cannot load, these calls raise.

`Plan` is a small convenience wrapper that owns the handle.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcme.so")

CME_OK, CME_EINVAL, CME_ENOMEM, CME_EHIP = 0, -1, -2, -3
CME_EUNSTABLE, CME_ENONFINITE, CME_EUNSUPPORTED, CME_ENODEVICE = -4, -5, -6, -7
CME_ESCRATCH = -8
CME_NOALLOC_SCRATCH_BYTES = 64 * 1024 * 1024
CME_F64, CME_F32 = 0, 1
CME_RK4, CME_RK4IP, CME_SPLIT_STEP = 0, 1, 2
CME_FWM_CYCLIC, CME_FWM_PADDED = 0, 1
CME_INIT_DEFAULT, CME_INIT_SKIP_STABILITY, CME_INIT_AUTOTUNE = 0, 1, 2

EXPORTED = (
    "cme_init", "cme_step", "cme_run", "cme_fwm", "cme_adjoint", "cme_adjoint_noalloc",
    "cme_status", "cme_set_stream",
    "cme_plan_kernel", "cme_plan_select", "cme_list_kernels", "cme_kernel_info", "cme_destroy",
    "cme_strerror", "cme_version",
)

KERNEL_INFO_FIELDS = ("precision", "n_modes", "elems_per_thread", "sub_transforms", "pad_shift",
                      "kind", "instances_per_group", "threads", "lds_bytes", "exchange")


class CmeError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {cme_strerror(code)} ({code})")


class CmeInstance(ctypes.Structure):
    """Mirror of cme_instance in include/cme.h."""
    _fields_ = [
        ("n_modes", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("mode_offset", ctypes.c_int64), ("kappa_ext", ctypes.c_double),
        ("g0", ctypes.c_double), ("a_in_re", ctypes.c_double), ("a_in_im", ctypes.c_double),
        ("sigma0", ctypes.c_double), ("sigma1", ctypes.c_double), ("tau_ramp", ctypes.c_double),
    ]


_lib: Optional[ctypes.CDLL] = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libcme.so and declare its signatures.  Raises if it is missing.

    torch is imported first so that the HIP runtime torch ships with is the
    one already mapped when libcme.so resolves its libamdhip64 dependency:
    device pointers and streams then belong to a single runtime."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run python -m paper_1307_3428_amd._build first")
    import torch  # noqa: F401  (must precede the dlopen below)
    lib = ctypes.CDLL(path)
    P, i32, i64, u32, dbl = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                             ctypes.c_double)
    sig = {
        "cme_init": (ctypes.c_int, [ctypes.POINTER(P), i32, P, P, P, i32, i32, i32, dbl, P, u32]),
        "cme_step": (ctypes.c_int, [P, P, i64]),
        "cme_run": (ctypes.c_int, [P, P, i64, i64, i32, P]),
        "cme_fwm": (ctypes.c_int, [P, P, P]),
        "cme_adjoint": (ctypes.c_int, [P, P, P, i64, i64, i32, P, P, P, P, P]),
        "cme_adjoint_noalloc": (ctypes.c_int, [P, P, P, i64, i64, i32, P, P, P, P, P]),
        "cme_status": (ctypes.c_int, [P, P]),
        "cme_set_stream": (ctypes.c_int, [P, P]),
        "cme_plan_kernel": (ctypes.c_int, [P, i32, P]),
        "cme_plan_select": (ctypes.c_int, [P, i32, i32]),
        "cme_list_kernels": (ctypes.c_int, [i32, i32, P, i32]),
        "cme_kernel_info": (ctypes.c_int, [i32, P, i32]),
        "cme_destroy": (ctypes.c_int, [P]),
        "cme_strerror": (ctypes.c_char_p, [ctypes.c_int]),
        "cme_version": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def cme_strerror(code: int) -> str:
    return load_library().cme_strerror(int(code)).decode()


def cme_version() -> int:
    return int(load_library().cme_version())


def _check(rc: int, what: str) -> int:
    if rc != CME_OK:
        raise CmeError(rc, what)
    return rc


def _dptr(t) -> Optional[int]:
    """Device address of a CUDA (HIP) tensor, None for None."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a GPU tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return t.data_ptr()


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def make_instances(n_modes: Sequence[int], offsets: Sequence[int], kappa_ext, g0, a_in,
                   sigma0, sigma1, tau_ramp) -> ctypes.Array:
    arr = (CmeInstance * len(n_modes))()
    for b in range(len(n_modes)):
        ai = complex(a_in[b])
        arr[b] = CmeInstance(int(n_modes[b]), 0, int(offsets[b]), float(kappa_ext[b]),
                             float(g0[b]), ai.real, ai.imag, float(sigma0[b]),
                             float(sigma1[b]), float(tau_ramp[b]))
    return arr


# ---------------------------------------------------------------------------
# C-named entry points
# ---------------------------------------------------------------------------

def cme_init(instances: ctypes.Array, kappa, omega, h: float, precision: int = CME_F64,
             integrator: int = CME_RK4, fwm: int = CME_FWM_CYCLIC, stream=None,
             flags: int = CME_INIT_DEFAULT) -> int:
    """Returns the plan handle.  kappa, omega: float64 tensors (GPU or CPU)."""
    lib = load_library()
    handle = ctypes.c_void_p()
    kp = kappa.data_ptr() if kappa is not None else None
    op = omega.data_ptr() if omega is not None else None
    rc = lib.cme_init(ctypes.byref(handle), len(instances), instances, kp, op, int(precision),
                      int(integrator), int(fwm), float(h), _stream_handle(stream), int(flags))
    _check(rc, "cme_init")
    return handle.value


def cme_step(plan: int, A, step0: int) -> None:
    _check(load_library().cme_step(plan, _dptr(A), int(step0)), "cme_step")


def cme_run(plan: int, A, step0: int, n_steps: int, ckpt_every: int = 0, ckpt=None) -> None:
    _check(load_library().cme_run(plan, _dptr(A), int(step0), int(n_steps), int(ckpt_every),
                                  _dptr(ckpt)), "cme_run")


def cme_fwm(plan: int, A, K) -> None:
    _check(load_library().cme_fwm(plan, _dptr(A), _dptr(K)), "cme_fwm")


def cme_adjoint(plan: int, A0, ckpt, step0: int, n_steps: int, ckpt_every: int, gA_T,
                gA_0=None, g_omega=None, g_kappa=None, g_ain=None) -> None:
    _check(load_library().cme_adjoint(plan, _dptr(A0), _dptr(ckpt), int(step0), int(n_steps),
                                      int(ckpt_every), _dptr(gA_T), _dptr(gA_0), _dptr(g_omega),
                                      _dptr(g_kappa), _dptr(g_ain)), "cme_adjoint")


def cme_adjoint_noalloc(plan: int, A0, ckpt, step0: int, n_steps: int, ckpt_every: int, gA_T,
                        gA_0=None, g_omega=None, g_kappa=None, g_ain=None) -> None:
    _check(load_library().cme_adjoint_noalloc(
        plan, _dptr(A0), _dptr(ckpt), int(step0), int(n_steps), int(ckpt_every), _dptr(gA_T),
        _dptr(gA_0), _dptr(g_omega), _dptr(g_kappa), _dptr(g_ain)), "cme_adjoint_noalloc")


def cme_status(plan: int, batch: int) -> np.ndarray:
    """Per-instance non-finite flags (synchronises the plan's stream)."""
    flags = np.zeros(batch, dtype=np.int32)
    rc = load_library().cme_status(plan, flags.ctypes.data_as(ctypes.c_void_p))
    if rc not in (CME_OK, CME_ENONFINITE):
        raise CmeError(rc, "cme_status")
    return flags


def cme_set_stream(plan: int, stream=None) -> None:
    _check(load_library().cme_set_stream(plan, _stream_handle(stream)), "cme_set_stream")


def cme_plan_kernel(plan: int, n_modes: int) -> int:
    kid = ctypes.c_int32()
    _check(load_library().cme_plan_kernel(plan, int(n_modes), ctypes.byref(kid)),
           "cme_plan_kernel")
    return kid.value


def cme_plan_select(plan: int, n_modes: int, kernel_id: int) -> None:
    _check(load_library().cme_plan_select(plan, int(n_modes), int(kernel_id)), "cme_plan_select")


def cme_list_kernels(precision: int, n_modes: int) -> list:
    out = np.zeros(64, dtype=np.int32)
    k = load_library().cme_list_kernels(int(precision), int(n_modes),
                                        out.ctypes.data_as(ctypes.c_void_p), 64)
    return [int(x) for x in out[:min(k, 64)]]


def cme_kernel_info(kernel_id: int) -> dict:
    out = np.zeros(len(KERNEL_INFO_FIELDS), dtype=np.int32)
    rc = load_library().cme_kernel_info(int(kernel_id), out.ctypes.data_as(ctypes.c_void_p),
                                        len(KERNEL_INFO_FIELDS))
    if rc < 0:
        raise CmeError(rc, "cme_kernel_info")
    info = dict(zip(KERNEL_INFO_FIELDS, (int(x) for x in out)))
    info["id"] = int(kernel_id)
    info["threads_per_instance"] = info["n_modes"] // info["elems_per_thread"]
    info["name"] = ({0: "rk4_persistent", 1: "rk4_wave", 2: "rk4_duo", 3: "rk4_lean", 4: "split_lean", 5: "rk4_wave_pad", 6: "rk4_staged", 7: "rk4ip_wave", 8: "rk4ip_staged", 9: "split_staged", 10: "rk4_staged_pad", 11: "rk4_lean_pad", 12: "rk4ip_lean",
                     13: "rk4_stream", 14: "rk4ip_stream"}[info["kind"]]
                    + "<{},{},{},{},{}{}>".format(
                        "double" if info["precision"] == 0 else "float", info["n_modes"],
                        info["elems_per_thread"], info["sub_transforms"], info["pad_shift"],
                        "," + str(info["exchange"]) if info["kind"] >= 1 else ""))
    return info


def cme_destroy(plan: Optional[int]) -> None:
    if plan:
        _check(load_library().cme_destroy(plan), "cme_destroy")


# ---------------------------------------------------------------------------
# Convenience owner of a plan over a packed batch (workloads.Packed layout)
# ---------------------------------------------------------------------------

class Plan:
    """Owns a cme_plan for one packed batch.  `packed` provides n_modes,
    offsets, kappa, omega, kappa_ext, g0, a_in, sigma0, sigma1, tau_ramp
    (numpy arrays, as workloads.pack returns)."""

    def __init__(self, packed, h: float, precision: int = CME_F64, flags: int = CME_INIT_DEFAULT,
                 device: str = "cuda", stream=None, integrator: int = CME_RK4,
                 fwm: int = CME_FWM_CYCLIC):
        import torch
        self.torch = torch
        self.batch = int(packed.batch)
        self.total = int(packed.total)
        self.h = float(h)
        self.precision = precision
        self.device = torch.device(device)
        self.cdtype = torch.complex128 if precision == CME_F64 else torch.complex64
        self._inst = make_instances(packed.n_modes, packed.offsets, packed.kappa_ext, packed.g0,
                                    packed.a_in, packed.sigma0, packed.sigma1, packed.tau_ramp)
        kappa = torch.as_tensor(np.ascontiguousarray(packed.kappa, np.float64), device=self.device)
        omega = torch.as_tensor(np.ascontiguousarray(packed.omega, np.float64), device=self.device)
        self.handle = cme_init(self._inst, kappa, omega, self.h, precision=precision,
                               integrator=integrator, fwm=fwm, stream=stream, flags=flags)

    def state(self, a0) -> "object":
        """A device tensor of the plan's complex dtype holding a0 (packed)."""
        return self.torch.as_tensor(np.ascontiguousarray(a0), device=self.device).to(self.cdtype)

    def run(self, A, n_steps: int, step0: int = 0, ckpt_every: int = 0, ckpt=None):
        cme_run(self.handle, A, step0, n_steps, ckpt_every, ckpt)
        return A

    def step(self, A, step0: int):
        cme_step(self.handle, A, step0)
        return A

    def fwm(self, A, K=None):
        """The four-wave-mixing sum K of every instance (a new tensor unless K is given)."""
        if K is None:
            K = self.torch.empty_like(A)
        cme_fwm(self.handle, A, K)
        return K

    def adjoint(self, A0, gA_T, n_steps: int, step0: int = 0, ckpt_every: int = 0, ckpt=None,
                want=("gA_0", "g_omega", "g_kappa", "g_ain")):
        torch = self.torch
        out = {}
        gA_0 = torch.empty_like(A0) if "gA_0" in want else None
        g_om = torch.zeros(self.total, dtype=torch.float64, device=self.device) if "g_omega" in want else None
        g_ka = torch.zeros(self.total, dtype=torch.float64, device=self.device) if "g_kappa" in want else None
        g_ai = torch.zeros(2 * self.batch, dtype=torch.float64, device=self.device) if "g_ain" in want else None
        cme_adjoint(self.handle, A0, ckpt, step0, n_steps, ckpt_every, gA_T, gA_0, g_om, g_ka, g_ai)
        out.update({"gA_0": gA_0, "g_omega": g_om, "g_kappa": g_ka, "g_ain": g_ai})
        return out

    def status(self) -> np.ndarray:
        return cme_status(self.handle, self.batch)

    def set_stream(self, stream=None):
        """Enqueue later calls on `stream` (a torch.cuda.Stream, a raw handle,
        or None for the null stream)."""
        cme_set_stream(self.handle, stream)

    def kernel(self, n_modes: int) -> dict:
        """Shape of the kernel variant the plan uses for this size."""
        return cme_kernel_info(cme_plan_kernel(self.handle, n_modes))

    def select(self, n_modes: int, kernel_id: int):
        cme_plan_select(self.handle, n_modes, kernel_id)

    def close(self):
        if getattr(self, "handle", None):
            cme_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


# ---------------------------------------------------------------------------
# torch.autograd binding of cme_run / cme_adjoint
# ---------------------------------------------------------------------------

class _Handle:
    """Owns a plan handle (destroyed with the object)."""

    def __init__(self, handle: int, batch: int, total: int):
        self.handle, self.batch, self.total = handle, batch, total

    def __del__(self):
        try:
            cme_destroy(self.handle)
        except Exception:
            pass


def _evolve_function():
    import torch

    class Evolve(torch.autograd.Function):
        """A(T) = RK4 map applied n_steps times to A0 (cme_run); backward is the
        library's discrete adjoint (cme_adjoint) from the checkpoints written by
        the forward call.  Differentiable inputs: A0 (complex128), omega and
        kappa (float64, per mode, packed) and a_in (complex128, per instance).
        Complex gradients follow torch's convention dL/dRe + i dL/dIm, which is
        the library's."""

        @staticmethod
        def forward(ctx, A0, omega, kappa, a_in, meta):
            n_modes, offsets, kappa_ext, g0, sigma0, sigma1, tau_ramp, h, n_steps, step0, K = meta
            ain = a_in.detach().cpu().numpy()
            inst = make_instances(n_modes, offsets, kappa_ext, g0, ain, sigma0, sigma1, tau_ramp)
            plan = _Handle(cme_init(inst, kappa.detach().contiguous(),
                                    omega.detach().contiguous(), h, precision=CME_F64),
                           len(n_modes), int(A0.numel()))
            A = A0.detach().clone().contiguous()
            K = max(1, min(K, n_steps)) if n_steps > 0 else 1
            nck = n_steps // K
            ckpt = torch.empty((max(nck, 1), plan.total), dtype=torch.complex128, device=A.device)
            if n_steps > 0:
                cme_run(plan.handle, A, step0, n_steps, K if nck > 0 else 0, ckpt if nck > 0 else None)
            ctx.plan, ctx.ckpt, ctx.K = plan, ckpt, K
            ctx.meta = (n_steps, step0)
            ctx.save_for_backward(A0.detach().contiguous())
            return A

        @staticmethod
        def backward(ctx, gA):
            (A0,) = ctx.saved_tensors
            n_steps, step0 = ctx.meta
            plan = ctx.plan
            gA = gA.detach().to(torch.complex128).contiguous()
            g0_ = torch.empty_like(A0)
            g_om = torch.zeros(plan.total, dtype=torch.float64, device=A0.device)
            g_ka = torch.zeros(plan.total, dtype=torch.float64, device=A0.device)
            g_ai = torch.zeros(2 * plan.batch, dtype=torch.float64, device=A0.device)
            cme_adjoint(plan.handle, A0, ctx.ckpt if n_steps >= ctx.K else None, step0, n_steps,
                        ctx.K, gA, g0_, g_om, g_ka, g_ai)
            g_ain = torch.complex(g_ai[0::2], g_ai[1::2])
            return g0_, g_om, g_ka, g_ain, None

    return Evolve


_EVOLVE = None


def evolve(A0, omega, kappa, a_in, *, n_modes, offsets, kappa_ext, g0, sigma0, sigma1, tau_ramp,
           h: float, n_steps: int, step0: int = 0, ckpt_every: int = 100):
    """Differentiable FP64 time stepping of a packed batch (see Evolve).  The
    per-instance scalars are plain sequences; A0 / omega / kappa / a_in are
    CUDA tensors that may require grad."""
    global _EVOLVE
    if _EVOLVE is None:
        _EVOLVE = _evolve_function()
    meta = (list(n_modes), list(offsets), list(kappa_ext), list(g0), list(sigma0), list(sigma1),
            list(tau_ramp), float(h), int(n_steps), int(step0), int(ckpt_every))
    return _EVOLVE.apply(A0, omega, kappa, a_in, meta)
