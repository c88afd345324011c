"""ctypes binding of ``libdtrg.so`` (the C ABI in include/dtrg.h), with the same entry-point names.

Argument marshalling only: every step of the HOTRG forward and backward runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  If the library has not
been built, importing this module raises (there is no fallback implementation).
"""

from __future__ import annotations

import atexit
import ctypes
import os
import weakref
from ctypes import POINTER, byref, c_double, c_int, c_longlong, c_size_t, c_void_p

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdtrg.so")

DTRG_OK, DTRG_EINVAL, DTRG_ENOMEM, DTRG_EHIP, DTRG_ENOCONV, DTRG_ENONPOS, DTRG_ESTATE = range(7)
STATUS_NAMES = {0: "DTRG_OK", 1: "DTRG_EINVAL", 2: "DTRG_ENOMEM", 3: "DTRG_EHIP", 4: "DTRG_ENOCONV",
                5: "DTRG_ENONPOS", 6: "DTRG_ESTATE"}
DTRG_FP64, DTRG_FP32, DTRG_BF16X3, DTRG_BF16X6 = 0, 1, 2, 3
PRECISIONS = {"fp64": DTRG_FP64, "fp32": DTRG_FP32, "bf16x3": DTRG_BF16X3, "bf16x6": DTRG_BF16X6}

EXPORTED = ["dtrg_default_options", "dtrg_hotrg_forward", "dtrg_plan_create", "dtrg_plan_forward",
            "dtrg_hotrg_backward", "dtrg_plan_step_info", "dtrg_plan_profile", "dtrg_batch_create", "dtrg_batch_run",
            "dtrg_hotrg_batched",
            "dtrg_batch_step_info", "dtrg_batch_profile", "dtrg_batch_device_bytes", "dtrg_batch_destroy", "dtrg_tuned_shapes",
            "dtrg_plan_device_bytes", "dtrg_plan_destroy", "dtrg_last_error", "dtrg_contract", "dtrg_contract_config", "dtrg_version",
            "dtrg_contract_noalloc", "dtrg_plan_isometry", "dtrg_plan_fix_isometry", "dtrg_plan_isometry_grad",
            "dtrg_isometry_optimize"]


ALLOC_FN = ctypes.CFUNCTYPE(c_void_p, c_size_t, c_void_p, c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, c_void_p, c_size_t, c_void_p, c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("contract", c_int), ("gram_fp64", c_int), ("eig_broadening", c_double),
                ("max_subspace_iters", c_int), ("subspace_tol", c_double), ("block_size", c_int),
                ("autotune", c_int), ("profile", c_int), ("checkpoint_gib", c_double), ("oversample", c_int),
                ("max_fp32_chain", c_int), ("max_fp32_chain_wide", c_int),
                ("tile_table", ctypes.c_char_p), ("alloc_fn", ALLOC_FN), ("free_fn", FREE_FN),
                ("alloc_user", c_void_p), ("chain_phys", c_int), ("side_rule", c_int), ("polar_newton", c_int),
                ("subspace_shift", c_int), ("rr_skip", c_int)]


class StepInfo(ctypes.Structure):
    _fields_ = [("X", c_int), ("Y", c_int), ("chi_kept", c_int), ("full_eig", c_int), ("iters", c_int),
                ("c", c_double), ("trace_G", c_double), ("lam_last_kept", c_double),
                ("lam_first_dropped", c_double), ("resid", c_double), ("cheb_degree", c_int),
                ("trunc_weight", c_double), ("cut_gap", c_double), ("min_kept_gap", c_double), ("mixed", c_int),
                ("lnZ_at_step", c_double), ("side", c_int), ("trunc_weight_left", c_double),
                ("trunc_weight_right", c_double), ("rr_stride", c_int)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class DtrgError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1912_02780_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.dtrg_default_options.argtypes = [POINTER(Options)]
    lib.dtrg_default_options.restype = None
    lib.dtrg_hotrg_forward.argtypes = [c_void_p, c_int, c_int, c_int, POINTER(Options), c_void_p,
                                       POINTER(c_void_p), POINTER(c_double)]
    lib.dtrg_hotrg_forward.restype = c_int
    lib.dtrg_plan_create.argtypes = [c_int, c_int, c_int, POINTER(Options), POINTER(c_void_p)]
    lib.dtrg_plan_create.restype = c_int
    lib.dtrg_plan_forward.argtypes = [c_void_p, c_void_p, c_void_p, POINTER(c_double)]
    lib.dtrg_plan_forward.restype = c_int
    lib.dtrg_plan_profile.argtypes = [c_void_p, POINTER(c_longlong), POINTER(c_double), POINTER(c_double), c_int]
    lib.dtrg_plan_profile.restype = c_int
    lib.dtrg_hotrg_backward.argtypes = [c_void_p, c_double, c_void_p, c_void_p, POINTER(c_double), c_void_p]
    lib.dtrg_hotrg_backward.restype = c_int
    lib.dtrg_plan_step_info.argtypes = [c_void_p, c_int, POINTER(StepInfo)]
    lib.dtrg_plan_step_info.restype = c_int
    lib.dtrg_batch_create.argtypes = [c_int, c_int, POINTER(c_int), c_int, POINTER(Options), POINTER(c_void_p)]
    lib.dtrg_batch_create.restype = c_int
    lib.dtrg_batch_run.argtypes = [c_void_p, c_void_p, c_void_p, c_double, POINTER(c_double), c_void_p,
                                   POINTER(c_double), c_int, c_void_p]
    lib.dtrg_batch_run.restype = c_int
    lib.dtrg_hotrg_batched.argtypes = [c_void_p, c_int, POINTER(c_int), c_int, c_int, POINTER(c_double),
                                       POINTER(Options), c_void_p, POINTER(c_double), c_void_p, c_void_p,
                                       POINTER(c_double)]
    lib.dtrg_hotrg_batched.restype = c_int
    lib.dtrg_batch_step_info.argtypes = [c_void_p, c_int, c_int, POINTER(StepInfo)]
    lib.dtrg_batch_step_info.restype = c_int
    lib.dtrg_batch_profile.argtypes = [c_void_p, POINTER(c_longlong), POINTER(c_double), POINTER(c_double), c_int]
    lib.dtrg_batch_profile.restype = c_int
    lib.dtrg_batch_device_bytes.argtypes = [c_void_p]
    lib.dtrg_batch_device_bytes.restype = c_size_t
    lib.dtrg_batch_destroy.argtypes = [c_void_p]
    lib.dtrg_batch_destroy.restype = None
    lib.dtrg_tuned_shapes.argtypes = []
    lib.dtrg_tuned_shapes.restype = c_int
    lib.dtrg_plan_device_bytes.argtypes = [c_void_p]
    lib.dtrg_plan_device_bytes.restype = c_size_t
    lib.dtrg_plan_destroy.argtypes = [c_void_p]
    lib.dtrg_plan_destroy.restype = None
    lib.dtrg_last_error.argtypes = []
    lib.dtrg_last_error.restype = ctypes.c_char_p
    lib.dtrg_version.argtypes = []
    lib.dtrg_version.restype = ctypes.c_char_p
    lib.dtrg_contract.argtypes = [c_int, c_int, c_int, c_int, c_void_p, c_longlong, c_int, c_void_p, c_longlong,
                                  c_int, c_void_p, c_longlong, c_int, c_double, c_double, c_void_p]
    lib.dtrg_contract.restype = c_int
    lib.dtrg_contract_config.argtypes = [c_int, c_int, c_int, c_int, c_void_p, c_longlong, c_int, c_void_p,
                                         c_longlong, c_int, c_void_p, c_longlong, c_int, c_double, c_double, c_int,
                                         c_int, c_void_p]
    lib.dtrg_contract_config.restype = c_int
    lib.dtrg_contract_noalloc.argtypes = lib.dtrg_contract.argtypes
    lib.dtrg_contract_noalloc.restype = c_int
    for name in ("dtrg_plan_isometry", "dtrg_plan_fix_isometry", "dtrg_plan_isometry_grad"):
        getattr(lib, name).argtypes = [c_void_p, c_int, c_void_p, c_void_p]
        getattr(lib, name).restype = c_int
    lib.dtrg_isometry_optimize.argtypes = [c_void_p, c_void_p, c_int, c_int, c_int, c_void_p, POINTER(c_double),
                                           POINTER(c_double), POINTER(c_double)]
    lib.dtrg_isometry_optimize.restype = c_int
    return lib


lib = _load()


def _check(status: int):
    if status != DTRG_OK:
        raise DtrgError(status, lib.dtrg_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return c_void_p(stream.cuda_stream)


# PyTorch's caching allocator behind the library's allocator callbacks: plan memory is then part of
# torch's pool (torch.cuda.memory_allocated counts it, and it is reused after the plan is released).
# The callbacks run on the calling thread with the GIL taken by ctypes.
def _torch_alloc(nbytes, stream, user):
    try:
        return torch.cuda.caching_allocator_alloc(int(nbytes), torch.cuda.current_device(), int(stream or 0))
    except Exception:   # out of memory: the library reports DTRG_ENOMEM
        return None


def _torch_free(ptr, nbytes, stream, user):
    torch.cuda.caching_allocator_delete(int(ptr))


TORCH_ALLOC = ALLOC_FN(_torch_alloc)
TORCH_FREE = FREE_FN(_torch_free)

# plans and batches still alive at exit are released while PyTorch's allocator is still there
_LIVE = weakref.WeakSet()


@atexit.register
def _release_live():
    for obj in list(_LIVE):
        try:
            obj.close()
        except Exception:
            pass


def default_options(torch_allocator: bool = True, **overrides) -> Options:
    """The library's defaults with `overrides` applied; plan memory comes from PyTorch's caching
    allocator unless torch_allocator is False (then hipMalloc)."""
    o = Options()
    lib.dtrg_default_options(byref(o))
    if torch_allocator:
        o.alloc_fn = TORCH_ALLOC
        o.free_fn = TORCH_FREE
    for k, v in overrides.items():
        if k == "contract" and isinstance(v, str):
            v = PRECISIONS[v]
        if k == "tile_table" and isinstance(v, str):
            v = v.encode()
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _opts(options: Options | None) -> Options:
    """The options to pass: the caller's, or the defaults (PyTorch's allocator) when None."""
    return default_options() if options is None else options


def _dev_f64(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


class Plan:
    """Owns a dtrg_plan (the forward checkpoints); released with the object."""

    def __init__(self, handle: int, D: int, n_steps: int, device, phys: int = 0):
        self._h = c_void_p(handle)
        self.D = D
        self.phys = phys
        # input layout [l][u][r][d]: D^4, or an MPO cell D x d x D x d (scheme (b))
        self.in_shape = (D, phys, D, phys) if phys else (D, D, D, D)
        self.n_steps = n_steps
        self.device = device
        _LIVE.add(self)

    def step_info(self, k: int) -> dict:
        info = StepInfo()
        _check(lib.dtrg_plan_step_info(self._h, k, byref(info)))
        return info.as_dict()

    def profile(self, reset: bool = True):
        """(launches, total_ms, flops) of the timed chi^7 contractions since the last reset."""
        n, ms, fl = c_longlong(), c_double(), c_double()
        _check(lib.dtrg_plan_profile(self._h, byref(n), byref(ms), byref(fl), int(reset)))
        return n.value, ms.value, fl.value

    def device_bytes(self) -> int:
        return int(lib.dtrg_plan_device_bytes(self._h))

    def close(self):
        if self._h is not None and self._h.value:
            lib.dtrg_plan_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dtrg_hotrg_forward(T0: torch.Tensor, chi: int, n_steps: int, options: Options | None = None, stream=None):
    """Returns (plan, lnZ_per_site).  T0: [l][u][r][d] float64 CUDA tensor."""
    T0 = _dev_f64(T0, "T0")
    if T0.dim() != 4 or len(set(T0.shape)) != 1:
        raise ValueError("T0 must be D x D x D x D")
    D = int(T0.shape[0])
    h = c_void_p()
    out = c_double()
    with torch.cuda.device(T0.device):
        _check(lib.dtrg_hotrg_forward(c_void_p(T0.data_ptr()), D, int(chi), int(n_steps),
                                      byref(_opts(options)), _stream(stream),
                                      byref(h), byref(out)))
    return Plan(h.value, D, n_steps, T0.device), out.value


def dtrg_plan_create(D: int, chi: int, n_steps: int, options: Options | None = None, device=None) -> Plan:
    """Allocate a plan (checkpoints and workspaces) for D^4 inputs on `device` (default: current)."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = c_void_p()
    with torch.cuda.device(device):
        _check(lib.dtrg_plan_create(int(D), int(chi), int(n_steps), byref(_opts(options)),
                                    byref(h)))
    return Plan(h.value, D, n_steps, device)


def _chain_options(options: Options | None, d: int) -> Options:
    """A copy of the options (or the defaults) with chain_phys = d."""
    src = _opts(options)
    o = Options()
    ctypes.pointer(o)[0] = src
    o.chain_phys = int(d)
    return o


def dtrg_chain_forward(M0: torch.Tensor, chi: int, n_steps: int, options: Options | None = None, stream=None):
    """Scheme (b): returns (plan, ln Z per cell per Trotter slice) of the infinite chain of the MPO cell
    M0 [l][u][r][d] (D x d x D x d float64 CUDA tensor) squared n_steps times."""
    M0 = _dev_f64(M0, "M0")
    if M0.dim() != 4 or M0.shape[0] != M0.shape[2] or M0.shape[1] != M0.shape[3]:
        raise ValueError("M0 must be D x d x D x d")
    D, d = int(M0.shape[0]), int(M0.shape[1])
    h = c_void_p()
    out = c_double()
    with torch.cuda.device(M0.device):
        _check(lib.dtrg_hotrg_forward(c_void_p(M0.data_ptr()), D, int(chi), int(n_steps),
                                      byref(_chain_options(options, d)), _stream(stream), byref(h), byref(out)))
    return Plan(h.value, D, n_steps, M0.device, d), out.value


def dtrg_chain_plan_create(D: int, d: int, chi: int, n_steps: int, options: Options | None = None,
                           device=None) -> Plan:
    """Allocate a scheme-(b) plan for MPO cells of bond D and physical dimension d."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    h = c_void_p()
    with torch.cuda.device(device):
        _check(lib.dtrg_plan_create(int(D), int(chi), int(n_steps), byref(_chain_options(options, d)), byref(h)))
    return Plan(h.value, D, n_steps, device, d)


def dtrg_plan_forward(plan: Plan, T0: torch.Tensor, stream=None) -> float:
    T0 = _dev_f64(T0, "T0")
    if tuple(T0.shape) != plan.in_shape:
        raise ValueError("T0 does not match the plan's input shape")
    out = c_double()
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_plan_forward(plan._h, c_void_p(T0.data_ptr()), _stream(stream), byref(out)))
    return out.value


def dtrg_hotrg_backward(plan: Plan, gbar: float = 1.0, dT0: torch.Tensor | None = None, stream=None):
    """Returns (T0bar, <T0bar, dT0> or None)."""
    T0bar = torch.empty(plan.in_shape, dtype=torch.float64, device=plan.device)
    dptr = None
    if dT0 is not None:
        dT0 = _dev_f64(dT0, "dT0")
        if tuple(dT0.shape) != plan.in_shape:
            raise ValueError("dT0 must have the shape of T0")
        dptr = c_void_p(dT0.data_ptr())
    val = c_double()
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_hotrg_backward(plan._h, float(gbar), c_void_p(T0bar.data_ptr()), dptr,
                                       byref(val) if dT0 is not None else None, _stream(stream)))
    return T0bar, (val.value if dT0 is not None else None)


def dtrg_plan_isometry(plan: Plan, k: int, stream=None) -> torch.Tensor:
    """Step k's isometry w[x1][x2][a] (float64, X x X x chi') after a forward pass."""
    info = plan.step_info(k)
    X, K = info["X"], info["chi_kept"]
    w = torch.empty((X, X, K), dtype=torch.float64, device=plan.device)
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_plan_isometry(plan._h, int(k), c_void_p(w.data_ptr()), _stream(stream)))
    return w


def dtrg_plan_fix_isometry(plan: Plan, k: int, w: torch.Tensor | None, stream=None):
    """Project step k with the given isometry w[x1][x2][a] in later passes (None: HOTRG's own again)."""
    ptr = None
    if w is not None:
        w = _dev_f64(w, "w")
        if w.dim() != 3 or w.shape[0] != w.shape[1]:
            raise ValueError("w must be X x X x chi'")
        ptr = c_void_p(w.data_ptr())
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_plan_fix_isometry(plan._h, int(k), ptr, _stream(stream)))
        plan.fixed_shapes = getattr(plan, "fixed_shapes", {})
        if w is None:
            plan.fixed_shapes.pop(int(k), None)
        else:
            plan.fixed_shapes[int(k)] = tuple(w.shape)


def dtrg_plan_isometry_grad(plan: Plan, k: int, stream=None) -> torch.Tensor:
    """d(gbar lnZ/N)/dw of step k's fixed isometry after a backward pass (shape of w)."""
    shape = getattr(plan, "fixed_shapes", {}).get(int(k))
    if shape is None:
        info = plan.step_info(k)
        shape = (info["X"], info["X"], info["chi_kept"])
    g = torch.empty(shape, dtype=torch.float64, device=plan.device)
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_plan_isometry_grad(plan._h, int(k), c_void_p(g.data_ptr()), _stream(stream)))
    return g


def dtrg_isometry_optimize(plan: Plan, T0: torch.Tensor, layers: int = 1, n_inner: int = 5, n_sweeps: int = 4,
                           stream=None):
    """Differentiable-TRG isometry optimisation (see include/dtrg.h).
    Returns (ln Z / N of plain HOTRG, ln Z / N after the optimisation, history list)."""
    T0 = _dev_f64(T0, "T0")
    if tuple(T0.shape) != plan.in_shape:
        raise ValueError("T0 does not match the plan's input shape")
    hist = (c_double * max(1, n_sweeps * layers * n_inner))()
    l0, l1 = c_double(), c_double()
    with torch.cuda.device(plan.device):
        _check(lib.dtrg_isometry_optimize(plan._h, c_void_p(T0.data_ptr()), int(layers), int(n_inner), int(n_sweeps),
                                          _stream(stream), byref(l0), byref(l1), hist))
    return l0.value, l1.value, list(hist)[:n_sweeps * layers * n_inner]


class Batch:
    """Owns a dtrg_batch: n_inst instances of D^4 inputs with per-instance chi; released with the object."""

    def __init__(self, handle: int, n_inst: int, D: int, n_steps: int, device):
        self._h = c_void_p(handle)
        self.n_inst = n_inst
        self.D = D
        self.n_steps = n_steps
        self.device = device
        _LIVE.add(self)

    def step_info(self, inst: int, k: int) -> dict:
        info = StepInfo()
        _check(lib.dtrg_batch_step_info(self._h, int(inst), int(k), byref(info)))
        return info.as_dict()

    def profile(self, reset: bool = True):
        """(launches, total_ms, flops) of the timed chi^7 contractions of adaptive runs since the last reset."""
        n, ms, fl = c_longlong(), c_double(), c_double()
        _check(lib.dtrg_batch_profile(self._h, byref(n), byref(ms), byref(fl), int(reset)))
        return n.value, ms.value, fl.value

    def device_bytes(self) -> int:
        return int(lib.dtrg_batch_device_bytes(self._h))

    def close(self):
        if self._h is not None and self._h.value:
            lib.dtrg_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def dtrg_batch_create(D: int, chis, n_steps: int, options: Options | None = None, device=None) -> Batch:
    """Allocate a batch of len(chis) instances (instance i with bond dimension chis[i])."""
    device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    n = len(chis)
    arr = (c_int * n)(*[int(c) for c in chis])
    h = c_void_p()
    with torch.cuda.device(device):
        _check(lib.dtrg_batch_create(n, int(D), arr, int(n_steps), byref(_opts(options)),
                                     byref(h)))
    return Batch(h.value, n, D, n_steps, device)


def dtrg_batch_run(batch: Batch, T0s: torch.Tensor, dT0s: torch.Tensor | None = None, gbar: float = 1.0,
                   backward: bool = True, replay: bool = False, T0bar: torch.Tensor | None = None, stream=None):
    """Forward (+ backward) of every instance.  T0s: [n_inst][D][D][D][D] float64 CUDA tensor.
    Returns (lnZ per instance (list), T0bar tensor or None, <T0bar_i, dT0_i> list or None)."""
    n, D = batch.n_inst, batch.D
    T0s = _dev_f64(T0s, "T0s")
    if tuple(T0s.shape) != (n, D, D, D, D):
        raise ValueError("T0s must be n_inst x D x D x D x D")
    dptr = None
    if dT0s is not None:
        dT0s = _dev_f64(dT0s, "dT0s")
        if tuple(dT0s.shape) != tuple(T0s.shape):
            raise ValueError("dT0s must have the shape of T0s")
        dptr = c_void_p(dT0s.data_ptr())
    bptr = None
    if backward:
        if T0bar is None:
            T0bar = torch.empty_like(T0s)
        T0bar = _dev_f64(T0bar, "T0bar")
        if tuple(T0bar.shape) != tuple(T0s.shape):
            raise ValueError("T0bar must have the shape of T0s")
        bptr = c_void_p(T0bar.data_ptr())
    lnZ = (c_double * n)()
    dirs = (c_double * n)()
    want_dir = backward and dT0s is not None
    with torch.cuda.device(batch.device):
        _check(lib.dtrg_batch_run(batch._h, c_void_p(T0s.data_ptr()), dptr, float(gbar), lnZ, bptr,
                                  dirs if want_dir else None, int(bool(replay)), _stream(stream)))
    return list(lnZ), (T0bar if backward else None), (list(dirs) if want_dir else None)


def dtrg_hotrg_batched(T0s: torch.Tensor, chis, n_steps: int, gbar: float | None = 1.0,
                       dT0s: torch.Tensor | None = None, options: Options | None = None, stream=None):
    """One call for a whole batch (create, one adaptive run, release).  T0s: [n_inst][D]^4 float64
    CUDA tensor, chis: per-instance bond dimensions.  gbar None: forward only.
    Returns (lnZ per instance (list), T0bar tensor or None, <T0bar_i, dT0_i> list or None)."""
    T0s = _dev_f64(T0s, "T0s")
    n = len(chis)
    if T0s.dim() != 5 or T0s.shape[0] != n or len(set(T0s.shape[1:])) != 1:
        raise ValueError("T0s must be n_inst x D x D x D x D with n_inst = len(chis)")
    D = int(T0s.shape[1])
    arr = (c_int * n)(*[int(c) for c in chis])
    dptr = None
    if dT0s is not None:
        dT0s = _dev_f64(dT0s, "dT0s")
        if tuple(dT0s.shape) != tuple(T0s.shape):
            raise ValueError("dT0s must have the shape of T0s")
        dptr = c_void_p(dT0s.data_ptr())
    T0bar = torch.empty_like(T0s) if gbar is not None else None
    lnZ = (c_double * n)()
    dirs = (c_double * n)()
    want_dir = gbar is not None and dT0s is not None
    g = c_double(float(gbar)) if gbar is not None else None
    with torch.cuda.device(T0s.device):
        _check(lib.dtrg_hotrg_batched(c_void_p(T0s.data_ptr()), D, arr, n, int(n_steps),
                                      byref(g) if g is not None else None, byref(_opts(options)), _stream(stream),
                                      lnZ, c_void_p(T0bar.data_ptr()) if T0bar is not None else None, dptr,
                                      dirs if want_dir else None))
    return list(lnZ), T0bar, (list(dirs) if want_dir else None)


def tuned_shapes() -> int:
    return int(lib.dtrg_tuned_shapes())


def dtrg_contract(precision: str, A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, a_kmajor=False, b_kmajor=False,
                  alpha=1.0, beta=0.0, stream=None, tile=0, splits=0, noalloc=False):
    """C = alpha * A' B'^T + beta * C with A' = A or A.T (a_kmajor), B' = B or B.T (b_kmajor).

    tile / splits: the kernel configuration (0 = the library's choice; dtrg_contract_config).
    noalloc: run through dtrg_contract_noalloc (the library's static scratch; tile and splits 0)."""
    prec = PRECISIONS[precision]
    if a_kmajor:
        K, M = A.shape
    else:
        M, K = A.shape
    N = B.shape[1] if b_kmajor else B.shape[0]
    for t in (A, B, C):
        if not (t.is_cuda and t.is_contiguous()):
            raise TypeError("operands must be contiguous CUDA tensors")
    in_dt = torch.float64 if prec == DTRG_FP64 else torch.float32
    if A.dtype != in_dt or B.dtype != in_dt:
        raise TypeError("operand dtype does not match the precision")
    out_f64 = C.dtype == torch.float64
    if prec == DTRG_FP64 and not out_f64:
        raise TypeError("fp64 contraction writes float64")
    if tuple(C.shape) != (M, N):
        raise ValueError("C has the wrong shape")
    if noalloc:
        if tile or splits:
            raise ValueError("dtrg_contract_noalloc takes no tile or split configuration")
        _check(lib.dtrg_contract_noalloc(prec, M, N, K, c_void_p(A.data_ptr()), A.shape[1], int(a_kmajor),
                                         c_void_p(B.data_ptr()), B.shape[1], int(b_kmajor), c_void_p(C.data_ptr()), N,
                                         int(out_f64), float(alpha), float(beta), _stream(stream)))
    elif tile or splits:
        _check(lib.dtrg_contract_config(prec, M, N, K, c_void_p(A.data_ptr()), A.shape[1], int(a_kmajor),
                                        c_void_p(B.data_ptr()), B.shape[1], int(b_kmajor), c_void_p(C.data_ptr()),
                                        N, int(out_f64), float(alpha), float(beta), int(tile), int(splits),
                                        _stream(stream)))
    else:
        _check(lib.dtrg_contract(prec, M, N, K, c_void_p(A.data_ptr()), A.shape[1], int(a_kmajor),
                                 c_void_p(B.data_ptr()), B.shape[1], int(b_kmajor), c_void_p(C.data_ptr()), N,
                                 int(out_f64), float(alpha), float(beta), _stream(stream)))
    return C


def version() -> str:
    return lib.dtrg_version().decode()
