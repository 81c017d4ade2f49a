"""Python binding of libkpm.so, the MI355X kernel polynomial method library.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libkpm.so``.  PyTorch is used for device memory (matrices
uploaded with :class:`DeviceCSR`) and for the HIP stream handle.  If the
library is not built this module raises on first use; there is no fallback.

The functions carry the C names of ``include/kpm.h`` (``kpm_bounds``,
``kpm_moments``, ``kpm_dos`` ...) and take a :class:`Context`.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkpm.so")
# Damping-network weights shipped with the library (kpm_mlp_save format):
# trained on the library's device path against exact blurred densities of
# the training family (random sparse n = 2,048, 2D Anderson 32 x 64, 3D
# Anderson 12^3); load with kpm_mlp_load for KPM_DAMP_LEARNED.
DAMPING_WEIGHTS = os.path.join(_HERE, "damping_net.bin")

KPM_FP32, KPM_FP64 = 0, 1
KPM_DAMP_NONE, KPM_DAMP_JACKSON, KPM_DAMP_LEARNED = 0, 1, 2
STATUS = {0: "KPM_OK", -1: "KPM_ERR_ARG", -2: "KPM_ERR_ALLOC", -3: "KPM_ERR_HIP",
          -4: "KPM_ERR_SPECTRUM", -5: "KPM_ERR_NOCONV", -6: "KPM_ERR_UNSUPPORTED",
          -7: "KPM_ERR_NOMODEL"}

# Every symbol include/kpm.h declares.
EXPORTS = [
    "kpm_create", "kpm_destroy", "kpm_set_stream", "kpm_last_error", "kpm_bounds", "kpm_moments",
    "kpm_moments_noalloc", "kpm_locality_order",
    "kpm_moments_batched", "kpm_damping_factors", "kpm_dos", "kpm_dos_bins", "kpm_rademacher",
    "kpm_slq", "kpm_slq_dos", "kpm_haydock_dos", "kpm_tridiag_eig", "kpm_legendre_moments", "kpm_dgl_dos",
    "kpm_legendre_dos", "kpm_functional", "kpm_functional_nodes", "kpm_heat_capacity", "kpm_slq_heat_capacity", "kpm_dos_pipeline", "kpm_autotune", "kpm_autotune_batched",
    "kpm_mlp_param_count", "kpm_mlp_set_params", "kpm_mlp_get_params", "kpm_mlp_forward",
    "kpm_mlp_loss_grad", "kpm_mlp_train", "kpm_mlp_init", "kpm_mlp_save", "kpm_mlp_load",
    "kpm_profile_enable", "kpm_profile_query", "kpm_profile_reset", "kpm_hbm_copy_probe",
    "kpm_gershgorin", "kpm_moments_robust", "kpm_bounds_batched", "kpm_dos_batched", "kpm_dos_pipeline_batched",
]


class KpmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.message = message


class kpm_csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col_idx", ctypes.c_void_p), ("val", ctypes.c_void_p), ("val_is_f64", ctypes.c_int32),
                ("on_device", ctypes.c_int32)]


class kpm_moment_opts(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("nvec", ctypes.c_int32), ("block", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("seed", ctypes.c_uint64), ("validate", ctypes.c_int32),
                ("rows_per_block", ctypes.c_int32), ("flags", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libkpm.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_1308_5467_amd.build`")
    # torch first: its HIP runtime (soname libamdhip64.so.7, requested by its
    # own libraries as libamdhip64.so) must be the one libkpm.so binds to.
    # Loaded the other way round, the process would hold two HIP runtimes
    # and the library's calls would fail.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I32, I64, U64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    sig = {
        "kpm_create": ([I32, P, P], I32),
        "kpm_destroy": ([P], I32),
        "kpm_set_stream": ([P, P], I32),
        "kpm_last_error": ([P], ctypes.c_char_p),
        "kpm_bounds": ([P, P, I32, U64, D, P, P], I32),
        "kpm_bounds_batched": ([P, I32, P, I32, U64, D, P, P], I32),
        "kpm_moments": ([P, P, D, D, P, P, P], I32),
        "kpm_moments_noalloc": ([P, P, D, D, P, P, P], I32),
        "kpm_moments_batched": ([P, I32, P, P, P, P, P, P], I32),
        "kpm_gershgorin": ([P, P, P, P], I32),
        "kpm_moments_robust": ([P, P, I32, U64, D, P, P, P, P, P, P], I32),
        "kpm_damping_factors": ([P, I32, I32, P, P], I32),
        "kpm_slq": ([P, P, D, D, P, P, P, P, P, P], I32),
        "kpm_autotune": ([P, P, D, D, P, P, P], I32),
        "kpm_autotune_batched": ([P, I32, P, P, P, P, P, P], I32),
        "kpm_slq_dos": ([P, P, P, I32, I32, D, P, I32, P], I32),
        "kpm_haydock_dos": ([P, P, P, P, I32, I32, D, D, D, P, I32, P], I32),
        "kpm_legendre_moments": ([P, P, D, D, P, P, P], I32),
        "kpm_dgl_dos": ([P, P, I32, D, D, D, D, P, I32, P, P], I32),
        "kpm_legendre_dos": ([P, P, P, I32, D, D, P, I32, P], I32),
        "kpm_functional": ([P, P, P, I32, D, D, P, I32, P], I32),
        "kpm_functional_nodes": ([I32, D, D, P], I32),
        "kpm_locality_order": ([I64, I64, P, P, P, P], I32),
        "kpm_dos_pipeline": ([P, P, I32, U64, D, P, I32, P, I32, P, P, P, P], I32),
        "kpm_heat_capacity": ([P, P, P, I32, D, D, P, I32, I32, P], I32),
        "kpm_slq_heat_capacity": ([P, P, P, I32, I32, P, I32, P], I32),
        "kpm_tridiag_eig": ([I32, P, P, P, P], I32),
        "kpm_dos": ([P, P, P, I32, D, D, P, I32, P], I32),
        "kpm_dos_batched": ([P, I32, P, P, I32, I32, P, P, P, I32, P], I32),
        "kpm_dos_pipeline_batched": ([P, I32, P, I32, U64, D, P, I32, P, I32, P, P, P, P, P], I32),
        "kpm_dos_bins": ([P, P, P, I32, D, D, P, I32, P], I32),
        "kpm_rademacher": ([P, U64, I64, I32, I64, I64, I32, P], I32),
        "kpm_mlp_param_count": ([], I64),
        "kpm_mlp_set_params": ([P, P], I32),
        "kpm_mlp_get_params": ([P, P], I32),
        "kpm_mlp_forward": ([P, I32, P, P], I32),
        "kpm_mlp_loss_grad": ([P, I32, P, P, ctypes.c_float, P, P], I32),
        "kpm_mlp_train": ([P, I32, P, P, ctypes.c_float, I32, I32, ctypes.c_float, U64, P], I32),
        "kpm_mlp_init": ([P, U64], I32),
        "kpm_mlp_save": ([P, ctypes.c_char_p], I32),
        "kpm_mlp_load": ([P, ctypes.c_char_p], I32),
        "kpm_profile_enable": ([P, I32], I32),
        "kpm_profile_query": ([P, ctypes.c_char_p, P, P], I32),
        "kpm_profile_reset": ([P], I32),
        "kpm_hbm_copy_probe": ([P, I64, I32, P], I32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Matrices
# --------------------------------------------------------------------------
@dataclass
class DeviceCSR:
    """CSR matrix in device memory (torch tensors own the storage)."""

    n: int
    row_ptr: "object"
    col_idx: "object"
    val: "object"

    @classmethod
    def from_host(cls, n, row_ptr, col_idx, val, dtype="f32", device="cuda:0") -> "DeviceCSR":
        import torch
        tdt = torch.float32 if dtype in ("f32", "float32", KPM_FP32) else torch.float64
        rp = torch.as_tensor(np.ascontiguousarray(row_ptr, dtype=np.int32)).to(device)
        ci = torch.as_tensor(np.ascontiguousarray(col_idx, dtype=np.int32)).to(device)
        va = torch.as_tensor(np.ascontiguousarray(val)).to(device=device, dtype=tdt)
        return cls(int(n), rp, ci, va)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.numel())

    def as_c(self) -> kpm_csr:
        import torch
        return kpm_csr(self.n, self.nnz, self.row_ptr.data_ptr(), self.col_idx.data_ptr(),
                       self.val.data_ptr(), 1 if self.val.dtype == torch.float64 else 0, 1)


@dataclass
class HostCSR:
    """CSR matrix in host memory (copied into the context on each call)."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray

    def __post_init__(self):
        self.row_ptr = np.ascontiguousarray(self.row_ptr, dtype=np.int32)
        self.col_idx = np.ascontiguousarray(self.col_idx, dtype=np.int32)
        if self.val.dtype not in (np.float32, np.float64):
            self.val = self.val.astype(np.float64)
        self.val = np.ascontiguousarray(self.val)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)

    def as_c(self) -> kpm_csr:
        return kpm_csr(self.n, self.nnz, _p(self.row_ptr), _p(self.col_idx), _p(self.val),
                       1 if self.val.dtype == np.float64 else 0, 0)


# --------------------------------------------------------------------------
# Context and entry points
# --------------------------------------------------------------------------
class Context:
    """A library context on one device, enqueueing on one HIP stream."""

    def __init__(self, device: int = 0, stream: int | None = None):
        self.lib = load_library()
        if stream is None:
            import torch
            torch.cuda.set_device(device)
            stream = torch.cuda.current_stream(device).cuda_stream
        self.handle = ctypes.c_void_p()
        st = self.lib.kpm_create(device, ctypes.c_void_p(stream), ctypes.byref(self.handle))
        if st != 0:
            raise KpmError(st, "kpm_create failed")

    def check(self, st: int):
        if st != 0:
            raise KpmError(st, self.lib.kpm_last_error(self.handle).decode())

    def close(self):
        if self.handle:
            self.lib.kpm_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kpm_create(device: int = 0, stream: int | None = None) -> Context:
    return Context(device, stream)


def kpm_destroy(ctx: Context) -> None:
    ctx.close()


def kpm_set_stream(ctx: Context, stream: int) -> None:
    ctx.check(ctx.lib.kpm_set_stream(ctx.handle, ctypes.c_void_p(stream)))


def kpm_bounds(ctx: Context, A, steps: int = 20, seed: int = 0, margin: float = 0.01):
    lb, ub = ctypes.c_double(), ctypes.c_double()
    c = A.as_c()
    ctx.check(ctx.lib.kpm_bounds(ctx.handle, ctypes.byref(c), steps, seed, margin,
                                 ctypes.byref(lb), ctypes.byref(ub)))
    return lb.value, ub.value


KPM_FLAG_NO_GRAPH, KPM_FLAG_GATHER4, KPM_FLAG_GATHER8, KPM_FLAG_GATHER7 = 1, 2, 4, 8
KPM_FLAG_LEGENDRE_RECURRENCE = 16
KPM_FLAG_BATCH_STREAM, KPM_FLAG_BATCH_RESIDENT = 32, 64
KPM_FLAG_LOCALITY = 128


def _opts(M, nvec, seed, precision, block, validate, rows_per_block, flags=0) -> kpm_moment_opts:
    prec = KPM_FP64 if precision in ("f64", "float64", KPM_FP64) else KPM_FP32
    return kpm_moment_opts(M, nvec, block, prec, seed & (2**64 - 1), 1 if validate else 0, rows_per_block,
                           flags)


def _gather_flags(gather: int) -> int:
    if gather not in (0, 4, 7, 8):
        raise ValueError("gather must be 0 (library default), 4, 7 or 8")
    return {0: 0, 4: KPM_FLAG_GATHER4, 7: KPM_FLAG_GATHER7, 8: KPM_FLAG_GATHER8}[gather]


def kpm_moments(ctx: Context, A, lb: float, ub: float, M: int, nvec: int, seed: int,
                precision="f32", block: int = 0, validate: bool = True, per_vector: bool = False,
                rows_per_block: int = 0, gather: int = 0, locality: bool = False):
    """Normalised moments mu[0..M]; with per_vector=True also [nvec, M+1] per-probe moments.
    locality=True: KPM_FLAG_LOCALITY (grid matrices renumbered along a Morton curve inside the library)."""
    o = _opts(M, nvec, seed, precision, block, validate, rows_per_block,
              _gather_flags(gather) | (KPM_FLAG_LOCALITY if locality else 0))
    mu = np.zeros(M + 1)
    pv = np.zeros((nvec, M + 1)) if per_vector else None
    c = A.as_c()
    st = ctx.lib.kpm_moments(ctx.handle, ctypes.byref(c), lb, ub, ctypes.byref(o), _p(mu),
                             _p(pv) if pv is not None else None)
    ctx.check(st)
    return (mu, pv) if per_vector else mu


def kpm_moments_noalloc(ctx: Context, A, lb: float, ub: float, M: int, nvec: int, seed: int, mu_out,
                        per_vector_out=None, precision="f32", block: int = 0, rows_per_block: int = 0,
                        gather: int = 0) -> None:
    """kpm_moments into caller-owned device tensors (float64 CUDA tensors of
    M+1 and nvec*(M+1) elements), enqueued on the context's stream without a
    wait and without device allocation; A must be a DeviceCSR."""
    import torch
    if mu_out is None:
        raise ValueError("mu_out is required")
    for t, size in ((mu_out, M + 1), (per_vector_out, nvec * (M + 1))):
        if t is not None and not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
                                  and t.numel() >= size):
            raise ValueError(f"outputs must be contiguous float64 CUDA tensors of at least {size} elements")
    o = _opts(M, nvec, seed, precision, block, False, rows_per_block, _gather_flags(gather))
    c = A.as_c()
    ctx.check(ctx.lib.kpm_moments_noalloc(ctx.handle, ctypes.byref(c), lb, ub, ctypes.byref(o),
                                          ctypes.c_void_p(mu_out.data_ptr()),
                                          ctypes.c_void_p(per_vector_out.data_ptr())
                                          if per_vector_out is not None else None))


def kpm_legendre_moments(ctx: Context, A, lb: float, ub: float, M: int, nvec: int, seed: int,
                         precision="f32", block: int = 0, validate: bool = True, per_vector: bool = False,
                         rows_per_block: int = 0, recurrence: bool = False, locality: bool = False):
    """Normalised Legendre moments mu[0..M] (tr L_k(B)/n estimates); with
    recurrence=True by the Legendre three-term recurrence in the fused step."""
    o = _opts(M, nvec, seed, precision, block, validate, rows_per_block,
              (KPM_FLAG_LEGENDRE_RECURRENCE if recurrence else 0) | (KPM_FLAG_LOCALITY if locality else 0))
    mu = np.zeros(M + 1)
    pv = np.zeros((nvec, M + 1)) if per_vector else None
    c = A.as_c()
    ctx.check(ctx.lib.kpm_legendre_moments(ctx.handle, ctypes.byref(c), lb, ub, ctypes.byref(o), _p(mu),
                                           _p(pv) if pv is not None else None))
    return (mu, pv) if per_vector else mu


def kpm_dgl_dos(ctx: Context, mu, lb: float, ub: float, sigma: float, x, tol: float = 1e-6):
    """Delta-Gauss-Legendre density at x (A's units) from Legendre moments;
    returns (phi, degree used per point)."""
    m = _f64(mu)
    x = _f64(x)
    phi = np.zeros(x.size)
    deg = np.zeros(x.size, dtype=np.int32)
    ctx.check(ctx.lib.kpm_dgl_dos(ctx.handle, _p(m), m.size - 1, lb, ub, sigma, tol, _p(x), x.size, _p(phi),
                                  deg.ctypes.data_as(ctypes.c_void_p)))
    return phi, deg


def kpm_legendre_dos(ctx: Context, mu, lb: float, ub: float, x, g=None) -> np.ndarray:
    """KPM-Legendre density at x (A's units); g = damping factors or None."""
    m = _f64(mu)
    gg = None if g is None else _f64(g)
    if gg is not None and gg.size != m.size:
        raise ValueError("g must have the length of mu")
    x = _f64(x)
    phi = np.zeros(x.size)
    ctx.check(ctx.lib.kpm_legendre_dos(ctx.handle, _p(m), _p(gg) if gg is not None else None, m.size - 1, lb, ub,
                                       _p(x), x.size, _p(phi)))
    return phi


def kpm_dos_pipeline(ctx: Context, A, M: int, nvec: int, seed: int, x, precision="f32", block: int = 0,
                     damping: int = KPM_DAMP_JACKSON, lanczos_steps: int = 20, lanczos_seed: int = 3002,
                     margin: float = 0.01, validate: bool = False, rows_per_block: int = 0,
                     locality: bool = False):
    """Bounds, moments, damping and density in one call: (phi, mu, lb, ub).
    locality=True: KPM_FLAG_LOCALITY."""
    o = _opts(M, nvec, seed, precision, block, validate, rows_per_block, KPM_FLAG_LOCALITY if locality else 0)
    x = _f64(x)
    phi = np.zeros(x.size)
    mu = np.zeros(M + 1)
    lb = ctypes.c_double()
    ub = ctypes.c_double()
    c = A.as_c()
    ctx.check(ctx.lib.kpm_dos_pipeline(ctx.handle, ctypes.byref(c), lanczos_steps, lanczos_seed, margin,
                                       ctypes.byref(o), damping, _p(x), x.size, _p(phi), _p(mu), ctypes.byref(lb),
                                       ctypes.byref(ub)))
    return phi, mu, lb.value, ub.value


def kpm_locality_order(row_ptr, col_idx):
    """(perm, dims): the grid found behind a CSR matrix and its rows in Morton
    order (perm[new] = old), or the identity and zeros (host only)."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    n = rp.size - 1
    perm = np.zeros(max(n, 0), dtype=np.int32)
    dims = np.zeros(3, dtype=np.int32)
    st = load_library().kpm_locality_order(n, ci.size, _p(rp), _p(ci), _p(perm), _p(dims))
    if st != 0:
        raise KpmError(st, "kpm_locality_order: bad argument")
    return perm, tuple(int(d) for d in dims)


def kpm_functional_nodes(Q: int, lb: float, ub: float) -> np.ndarray:
    """The Q points of A's axis at which kpm_functional samples f (computed
    by the library)."""
    x = np.zeros(int(Q))
    st = load_library().kpm_functional_nodes(int(Q), float(lb), float(ub), _p(x))
    if st != 0:
        raise KpmError(st, "kpm_functional_nodes: bad argument")
    return x


def kpm_functional(ctx: Context, mu, lb: float, ub: float, f, Q: int = 1024, g=None) -> float:
    """<phi~, f> of the KPM density; f is a callable evaluated (on the host)
    at the Q quadrature nodes, or an array of its values there."""
    m = _f64(mu)
    fv = _f64(f(kpm_functional_nodes(Q, lb, ub)) if callable(f) else f)
    if fv.size != Q:
        raise ValueError("need one value of f per node")
    gg = None if g is None else _f64(g)
    out = np.zeros(1)
    ctx.check(ctx.lib.kpm_functional(ctx.handle, _p(m), _p(gg) if gg is not None else None, m.size - 1, lb, ub,
                                     _p(fv), Q, _p(out)))
    return float(out[0])


def kpm_heat_capacity(ctx: Context, mu, lb: float, ub: float, T, g=None, Q: int = 0) -> np.ndarray:
    """C_v(T) = <phi~, g_T> of the KPM density (section 4.3)."""
    m = _f64(mu)
    t = _f64(T)
    gg = None if g is None else _f64(g)
    cv = np.zeros(t.size)
    ctx.check(ctx.lib.kpm_heat_capacity(ctx.handle, _p(m), _p(gg) if gg is not None else None, m.size - 1, lb, ub,
                                        _p(t), t.size, Q, _p(cv)))
    return cv


def kpm_slq_heat_capacity(ctx: Context, theta, tau2, T) -> np.ndarray:
    """C_v(T) for the Lanczos density from kpm_slq's nodes and weights."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    w = np.ascontiguousarray(tau2, dtype=np.float64)
    if th.ndim != 2 or th.shape != w.shape:
        raise ValueError("theta and tau2 must be [nvec, M] arrays of the same shape")
    t = _f64(T)
    cv = np.zeros(t.size)
    ctx.check(ctx.lib.kpm_slq_heat_capacity(ctx.handle, _p(th), _p(w), th.shape[0], th.shape[1], _p(t), t.size,
                                            _p(cv)))
    return cv


class MatrixBatch:
    """The device matrices of batched calls with their C descriptors built
    once: calls that pass the same MatrixBatch skip rebuilding them (for
    thousands of matrices that costs tens of ms per call).  The descriptors
    hold the tensors' addresses: after replacing a matrix's tensors, build
    a new MatrixBatch (values changed in place need nothing)."""

    def __init__(self, mats):
        self.mats = list(mats)
        self.arr = (kpm_csr * len(self.mats))(*[m.as_c() for m in self.mats])

    def __len__(self):
        return len(self.mats)


def _batch_arr(mats):
    if isinstance(mats, MatrixBatch):
        return mats.arr
    return (kpm_csr * len(mats))(*[m.as_c() for m in mats])


def kpm_bounds_batched(ctx: Context, mats, steps: int = 20, seed: int = 0, margin: float = 0.01):
    """kpm_bounds for every matrix of a list of device matrices (or a
    MatrixBatch) in one launch sequence: arrays lb, ub [nmat], bitwise the
    values of per-matrix kpm_bounds calls with the same arguments."""
    arr = _batch_arr(mats)
    lb = np.zeros(len(mats))
    ub = np.zeros(len(mats))
    ctx.check(ctx.lib.kpm_bounds_batched(ctx.handle, len(mats), arr, steps, seed, margin,
                                         lb.ctypes.data_as(ctypes.c_void_p), ub.ctypes.data_as(ctypes.c_void_p)))
    return lb, ub


def kpm_moments_batched(ctx: Context, mats, lb, ub, M: int, nvec: int, seed: int, precision="f32",
                        block: int = 0, validate: bool = False, graph: bool = True, rows_per_block: int = 0,
                        return_max_abs: bool = False, path: str = "auto"):
    """Moments [nmat, M+1] of several device-resident matrices (a list of
    DeviceCSR or a MatrixBatch).

    path: "auto" (the on-chip path when block is 0 and every matrix fits it,
    else streaming), "stream" or "resident" (KPM_FLAG_BATCH_STREAM /
    KPM_FLAG_BATCH_RESIDENT).  With return_max_abs=True returns (mu,
    max_abs) and does not raise on a spectrum escape (max_abs[m] > 1 marks
    the matrices whose [lb, ub] was too narrow).
    """
    flags = {"auto": 0, "stream": KPM_FLAG_BATCH_STREAM, "resident": KPM_FLAG_BATCH_RESIDENT}[path]
    if not graph:
        flags |= KPM_FLAG_NO_GRAPH
    o = _opts(M, nvec, seed, precision, block, validate, rows_per_block, flags)
    arr = _batch_arr(mats)
    lbv, ubv = _f64(lb), _f64(ub)
    mu = np.zeros((len(mats), M + 1))
    mx = np.zeros(len(mats))
    st = ctx.lib.kpm_moments_batched(ctx.handle, len(mats), arr, _p(lbv), _p(ubv), ctypes.byref(o), _p(mu), _p(mx))
    if return_max_abs:
        if st not in (0, -4):
            ctx.check(st)
        return mu, mx
    ctx.check(st)
    return mu


def kpm_dos_batched(ctx: Context, mu, g, lb, ub, x) -> np.ndarray:
    """Densities phi [nmat, npts] of several matrices in one launch: mu
    [nmat, M+1], g [M+1] (shared) or [nmat, M+1], lb, ub [nmat], x [nmat,
    npts] (each matrix's own points)."""
    mu = _f64(np.atleast_2d(mu))
    nmat, M1 = mu.shape
    g = _f64(g)
    per = 1 if g.ndim == 2 else 0
    x = _f64(np.atleast_2d(x))
    lbv, ubv = _f64(lb), _f64(ub)
    phi = np.zeros(x.shape)
    ctx.check(ctx.lib.kpm_dos_batched(ctx.handle, nmat, _p(mu), _p(g), per, M1 - 1, _p(lbv), _p(ubv), _p(x),
                                      x.shape[1], _p(phi)))
    return phi


def kpm_dos_pipeline_batched(ctx: Context, mats, M: int, nvec: int, seed: int, x, precision="f32", block: int = 0,
                             damping: int = KPM_DAMP_JACKSON, lanczos_steps: int = 20, lanczos_seed: int = 3003,
                             margin: float = 0.01, rows_per_block: int = 0, path: str = "auto"):
    """The whole path for several device matrices (a list of DeviceCSR or a
    MatrixBatch) in one call, escapes recovered per matrix: (phi [nmat,
    npts], mu [nmat, M+1], lb, ub, attempts [nmat]); x [nmat, npts]."""
    flags = {"auto": 0, "stream": KPM_FLAG_BATCH_STREAM, "resident": KPM_FLAG_BATCH_RESIDENT}[path]
    o = _opts(M, nvec, seed, precision, block, False, rows_per_block, flags)
    arr = _batch_arr(mats)
    n = len(mats)
    x = _f64(np.atleast_2d(x))
    if x.shape[0] != n:
        raise ValueError("x needs one row of points per matrix")
    phi = np.zeros(x.shape)
    mu = np.zeros((n, M + 1))
    lb, ub = np.zeros(n), np.zeros(n)
    att = np.zeros(n, dtype=np.int32)
    ctx.check(ctx.lib.kpm_dos_pipeline_batched(ctx.handle, n, arr, lanczos_steps, lanczos_seed, margin,
                                               ctypes.byref(o), damping, _p(x), x.shape[1], _p(phi), _p(mu),
                                               _p(lb), _p(ub), _p(att)))
    return phi, mu, lb, ub, att


def kpm_slq(ctx: Context, A, lb: float, ub: float, M: int, nvec: int, seed: int, block: int = 0,
            validate: bool = False, rows_per_block: int = 0, coefficients: bool = False, nodes: bool = True,
            locality: bool = False):
    """Stochastic Lanczos nodes: theta [nvec, M] (A's units), tau2 [nvec, M],
    steps_used [nvec]; with coefficients=True also alpha, beta [nvec, M] of B.
    nodes=False (with coefficients=True) skips the eigenvalue problems and
    returns (steps_used, alpha, beta).  locality=True: KPM_FLAG_LOCALITY."""
    if not nodes and not coefficients:
        raise ValueError("nodes=False needs coefficients=True")
    o = _opts(M, nvec, seed, "f64", block, validate, rows_per_block, KPM_FLAG_LOCALITY if locality else 0)
    theta = np.zeros((nvec, M)) if nodes else None
    tau2 = np.zeros((nvec, M)) if nodes else None
    used = np.zeros(nvec, dtype=np.int32)
    al = np.zeros((nvec, M)) if coefficients else None
    be = np.zeros((nvec, M)) if coefficients else None
    c = A.as_c()
    ctx.check(ctx.lib.kpm_slq(ctx.handle, ctypes.byref(c), lb, ub, ctypes.byref(o),
                              _p(theta) if nodes else None, _p(tau2) if nodes else None,
                              used.ctypes.data_as(ctypes.c_void_p), _p(al) if coefficients else None,
                              _p(be) if coefficients else None))
    if not nodes:
        return used, al, be
    return (theta, tau2, used, al, be) if coefficients else (theta, tau2, used)


def kpm_slq_dos(ctx: Context, theta, tau2, sigma: float, x) -> np.ndarray:
    """Eq. (landos) at points x (A's units)."""
    th = np.ascontiguousarray(theta, dtype=np.float64)
    w = np.ascontiguousarray(tau2, dtype=np.float64)
    if th.ndim != 2 or th.shape != w.shape:
        raise ValueError("theta and tau2 must be [nvec, M] arrays of the same shape")
    x = _f64(x)
    phi = np.zeros(x.size)
    ctx.check(ctx.lib.kpm_slq_dos(ctx.handle, _p(th), _p(w), th.shape[0], th.shape[1], sigma, _p(x), x.size,
                                  _p(phi)))
    return phi


def kpm_haydock_dos(ctx: Context, alpha, beta, steps_used, lb: float, ub: float, eta: float, x) -> np.ndarray:
    """Haydock's Lorentzian density at points x (A's units) from kpm_slq's
    coefficients alpha, beta [nvec, M] (of B) and steps_used [nvec]."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    u = np.ascontiguousarray(steps_used, dtype=np.int32)
    if a.ndim != 2 or a.shape != b.shape or u.shape != (a.shape[0],):
        raise ValueError("alpha and beta must be [nvec, M] and steps_used [nvec]")
    x = _f64(x)
    phi = np.zeros(x.size)
    ctx.check(ctx.lib.kpm_haydock_dos(ctx.handle, _p(a), _p(b), u.ctypes.data_as(ctypes.c_void_p), a.shape[0],
                                      a.shape[1], lb, ub, eta, _p(x), x.size, _p(phi)))
    return phi


def kpm_tridiag_eig(alpha, beta):
    """Host-only: eigenvalues and squared first eigenvector components of tridiag(beta, alpha, beta)."""
    lib = load_library()
    a = _f64(alpha)
    b = _f64(beta) if a.size > 1 else np.zeros(1)
    th = np.zeros(a.size)
    w = np.zeros(a.size)
    st = lib.kpm_tridiag_eig(a.size, _p(a), _p(b), _p(th), _p(w))
    if st != 0:
        raise KpmError(st, "kpm_tridiag_eig failed")
    return th, w


def kpm_autotune(ctx: Context, A, lb: float, ub: float, nvec: int, seed: int = 0, precision="f32",
                 block: int = 0, rows_per_block: int = 0, locality: bool = False) -> dict:
    """Measured choice of block, rows_per_block and gather for kpm_moments on A
    (on the renumbered matrix with locality=True: KPM_FLAG_LOCALITY)."""
    o = _opts(16, nvec, seed, precision, block, False, rows_per_block, KPM_FLAG_LOCALITY if locality else 0)
    best = kpm_moment_opts()
    us = ctypes.c_double()
    c = A.as_c()
    ctx.check(ctx.lib.kpm_autotune(ctx.handle, ctypes.byref(c), lb, ub, ctypes.byref(o), ctypes.byref(best),
                                   ctypes.byref(us)))
    return {"block": best.block, "rows_per_block": best.rows_per_block,
            "gather": 4 if best.flags & KPM_FLAG_GATHER4 else (7 if best.flags & KPM_FLAG_GATHER7 else 8),
            "us_per_step": us.value}


def kpm_autotune_batched(ctx: Context, mats, lb, ub, nvec: int, seed: int = 0, precision="f32",
                         block: int = 0, rows_per_block: int = 0) -> dict:
    """Measured choice of block and rows_per_block for kpm_moments_batched."""
    o = _opts(16, nvec, seed, precision, block, False, rows_per_block)
    arr = _batch_arr(mats)
    lbv, ubv = _f64(lb), _f64(ub)
    best = kpm_moment_opts()
    us = ctypes.c_double()
    ctx.check(ctx.lib.kpm_autotune_batched(ctx.handle, len(mats), arr, _p(lbv), _p(ubv), ctypes.byref(o),
                                           ctypes.byref(best), ctypes.byref(us)))
    return {"block": best.block, "rows_per_block": best.rows_per_block, "us_per_step": us.value}


def kpm_gershgorin(ctx: Context, A):
    lo, hi = ctypes.c_double(), ctypes.c_double()
    c = A.as_c()
    ctx.check(ctx.lib.kpm_gershgorin(ctx.handle, ctypes.byref(c), ctypes.byref(lo), ctypes.byref(hi)))
    return lo.value, hi.value


def kpm_moments_robust(ctx: Context, A, M: int, nvec: int, seed: int, steps: int = 20, lanczos_seed: int = 0,
                       margin: float = 0.01, precision="f32", block: int = 0, validate: bool = True,
                       per_vector: bool = False):
    """Bounds + moments with escape recovery; returns (mu, lb, ub, attempts) (+ per-probe moments)."""
    o = _opts(M, nvec, seed, precision, block, validate, 0)
    mu = np.zeros(M + 1)
    pv = np.zeros((nvec, M + 1)) if per_vector else None
    lb, ub, att = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
    c = A.as_c()
    ctx.check(ctx.lib.kpm_moments_robust(ctx.handle, ctypes.byref(c), steps, lanczos_seed, margin, ctypes.byref(o),
                                         _p(mu), _p(pv) if pv is not None else None, ctypes.byref(lb),
                                         ctypes.byref(ub), ctypes.byref(att)))
    out = (mu, lb.value, ub.value, att.value)
    return out + (pv,) if per_vector else out


def kpm_damping_factors(ctx: Context, kind: int, M: int, mu=None) -> np.ndarray:
    g = np.zeros(M + 1)
    mu_a = _f64(mu) if mu is not None else None
    ctx.check(ctx.lib.kpm_damping_factors(ctx.handle, kind, M, _p(mu_a) if mu_a is not None else None, _p(g)))
    return g


def kpm_dos(ctx: Context, mu, g, lb: float, ub: float, x) -> np.ndarray:
    mu, g, x = _f64(mu), _f64(g), _f64(x)
    phi = np.zeros(x.size)
    ctx.check(ctx.lib.kpm_dos(ctx.handle, _p(mu), _p(g), mu.size - 1, lb, ub, _p(x), x.size, _p(phi)))
    return phi


def kpm_dos_bins(ctx: Context, mu, g, lb: float, ub: float, edges) -> np.ndarray:
    mu, g, e = _f64(mu), _f64(g), _f64(edges)
    mass = np.zeros(max(e.size - 1, 0))
    ctx.check(ctx.lib.kpm_dos_bins(ctx.handle, _p(mu), _p(g), mu.size - 1, lb, ub, _p(e), mass.size, _p(mass)))
    return mass


def kpm_rademacher(ctx: Context, seed: int, vec0: int, nvec: int, n: int, ld: int, precision, out) -> None:
    """Fill device tensor ``out`` ([n, ld] row-major) with probe vectors."""
    prec = KPM_FP64 if precision in ("f64", "float64", KPM_FP64) else KPM_FP32
    ctx.check(ctx.lib.kpm_rademacher(ctx.handle, seed, vec0, nvec, n, ld, prec, ctypes.c_void_p(out.data_ptr())))


# ---- damping network -------------------------------------------------------
def kpm_mlp_param_count() -> int:
    return int(load_library().kpm_mlp_param_count())


def kpm_mlp_set_params(ctx: Context, params) -> None:
    p = np.ascontiguousarray(params, dtype=np.float32)
    assert p.size == kpm_mlp_param_count()
    ctx.check(ctx.lib.kpm_mlp_set_params(ctx.handle, _p(p)))


def kpm_mlp_get_params(ctx: Context) -> np.ndarray:
    p = np.zeros(kpm_mlp_param_count(), dtype=np.float32)
    ctx.check(ctx.lib.kpm_mlp_get_params(ctx.handle, _p(p)))
    return p


def kpm_mlp_init(ctx: Context, seed: int) -> None:
    ctx.check(ctx.lib.kpm_mlp_init(ctx.handle, seed))


def kpm_mlp_forward(ctx: Context, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float32)
    g = np.zeros_like(x)
    ctx.check(ctx.lib.kpm_mlp_forward(ctx.handle, x.shape[0], _p(x), _p(g)))
    return g


def kpm_mlp_loss_grad(ctx: Context, x, target, sigma: float):
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(target, dtype=np.float32)
    loss = ctypes.c_float()
    grads = np.zeros(kpm_mlp_param_count(), dtype=np.float32)
    ctx.check(ctx.lib.kpm_mlp_loss_grad(ctx.handle, x.shape[0], _p(x), _p(t), sigma, ctypes.byref(loss), _p(grads)))
    return loss.value, grads


def kpm_mlp_train(ctx: Context, x, target, sigma: float, epochs: int, batch: int, lr: float, seed: int):
    x = np.ascontiguousarray(x, dtype=np.float32)
    t = np.ascontiguousarray(target, dtype=np.float32)
    losses = np.zeros(epochs, dtype=np.float32)
    ctx.check(ctx.lib.kpm_mlp_train(ctx.handle, x.shape[0], _p(x), _p(t), sigma, epochs, batch, lr, seed, _p(losses)))
    return losses


def kpm_mlp_save(ctx: Context, path: str) -> None:
    ctx.check(ctx.lib.kpm_mlp_save(ctx.handle, path.encode()))


def kpm_mlp_load(ctx: Context, path: str) -> None:
    ctx.check(ctx.lib.kpm_mlp_load(ctx.handle, path.encode()))


# ---- device timing -------------------------------------------------------
def kpm_profile_enable(ctx: Context, enable: bool = True) -> None:
    ctx.check(ctx.lib.kpm_profile_enable(ctx.handle, 1 if enable else 0))


def kpm_profile_query(ctx: Context, kernel: str):
    n, ms = ctypes.c_int64(), ctypes.c_double()
    ctx.check(ctx.lib.kpm_profile_query(ctx.handle, kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def kpm_profile_reset(ctx: Context) -> None:
    ctx.check(ctx.lib.kpm_profile_reset(ctx.handle))


def kpm_hbm_copy_probe(ctx: Context, nbytes: int = 1 << 30, iters: int = 20) -> float:
    """Achievable copy bandwidth in GB/s (read + write bytes)."""
    g = ctypes.c_double()
    ctx.check(ctx.lib.kpm_hbm_copy_probe(ctx.handle, nbytes, iters, ctypes.byref(g)))
    return g.value


# MLP parameter layout (matches include/kpm.h)
MLP_SHAPES = [("W1", (128, 256)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("W3", (256, 128)), ("b3", (128,))]


def mlp_pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[k], dtype=np.float32).reshape(-1) for k, _ in MLP_SHAPES])


def mlp_unpack(flat) -> dict:
    out, off = {}, 0
    for k, shp in MLP_SHAPES:
        sz = int(np.prod(shp))
        out[k] = np.asarray(flat[off:off + sz]).reshape(shp)
        off += sz
    return out
