"""Python binding of the C ABI in include/sfk.h (argument marshalling only).

Every step of the method runs in the HIP library libsfk.so; PyTorch only
provides device memory and the stream.  If the library is not built, or no GPU
is present, the calls raise: there is no CPU fallback.

Names follow the C entry points without the ``sfk_`` prefix:
    init, iterate, solution, solution_at, residual_norms, true_residual,
    destroy, validate, workspace_bytes, sketch_sparse_sign, sketch_srht,
    coefficients.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsfk.so")

OK, EINVAL, ENOMEM, EDEVICE, BREAKDOWN, ESTATE = range(6)
SFLSQR, SFLSMR, FLSQR, FLSMR = 0, 1, 2, 3
SK_SPARSE_SIGN, SK_SRHT, SK_IDENTITY = 0, 1, 2
TAU_IDENTITY, TAU_REWEIGHT_L1, TAU_LOWRANK, TAU_LOWRANK_RND = 0, 1, 2, 3
DRIVER_AUTO, DRIVER_MULTI, DRIVER_GRAPH = 0, 1, 2
RES_SKETCHED, RES_TRUE_RECURRENCE, RES_TRUE_EXPLICIT = 0, 1, 2

_METHODS = {"sflsqr": SFLSQR, "sflsmr": SFLSMR, "flsqr": FLSQR, "flsmr": FLSMR}
_SKETCHES = {"sparse_sign": SK_SPARSE_SIGN, "countsketch": SK_SPARSE_SIGN, "srht": SK_SRHT,
             "identity": SK_IDENTITY}
_TAUS = {"identity": TAU_IDENTITY, "reweight_l1": TAU_REWEIGHT_L1, "lowrank": TAU_LOWRANK,
         "lowrank_rnd": TAU_LOWRANK_RND}
_DRIVERS = {"auto": DRIVER_AUTO, "multi": DRIVER_MULTI, "graph": DRIVER_GRAPH}
_RES = {"sketched": RES_SKETCHED, "true_recurrence": RES_TRUE_RECURRENCE,
        "true_explicit": RES_TRUE_EXPLICIT}


class SfkError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"sfk status {status}: {msg}")
        self.status = status


class CSR(ctypes.Structure):
    _fields_ = [("rows", ctypes.c_int64), ("cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p), ("val", ctypes.c_void_p)]


class Params(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("ell", ctypes.c_int32), ("maxit", ctypes.c_int32),
                ("sketch", ctypes.c_int32), ("s", ctypes.c_int32), ("zeta", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("instance", ctypes.c_int32), ("tau", ctypes.c_int32),
                ("eps", ctypes.c_double), ("eta", ctypes.c_double), ("noise_norm", ctypes.c_double),
                ("tol", ctypes.c_double), ("driver", ctypes.c_int32), ("vw", ctypes.c_int32),
                ("vw_b", ctypes.c_int32), ("vw_split", ctypes.c_int32),
                ("wg_per_cu", ctypes.c_int32), ("resid", ctypes.c_int32),
                ("copies", ctypes.c_int32), ("tape", ctypes.c_int32),
                ("perm", ctypes.c_void_p),
                ("lr_rows", ctypes.c_int32), ("lr_rank", ctypes.c_int32),
                ("lr_over", ctypes.c_int32), ("lr_q", ctypes.c_int32),
                ("lr_maxit", ctypes.c_int32), ("lr_reserved", ctypes.c_int32),
                ("lr_tol", ctypes.c_double)]


class Beam(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("nz", ctypes.c_int32), ("n_angles", ctypes.c_int32),
                ("n_det", ctypes.c_int32), ("cos_a", ctypes.c_void_p), ("sin_a", ctypes.c_void_p),
                ("back", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libsfk.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2605_22281_amd/build.py")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64, PI32, PI8, PD = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64,
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int8),
                                  ctypes.POINTER(ctypes.c_double))
    PCSR, PPAR = ctypes.POINTER(CSR), ctypes.POINTER(Params)
    sig = {
        "sfk_params_default": (None, [PPAR]),
        "sfk_validate": (I32, [PCSR, PCSR, PPAR]),
        "sfk_workspace_bytes": (ctypes.c_size_t, [PCSR, PCSR, PPAR]),
        "sfk_init": (I32, [ctypes.POINTER(P), PCSR, PCSR, P, PPAR, P, ctypes.c_size_t, P]),
        "sfk_iterate": (I32, [P, I32, PI32, PI32]),
        "sfk_solution": (I32, [P, P]),
        "sfk_solution_at": (I32, [P, I32, P]),
        "sfk_residual_norms": (I32, [P, I32, PD, I32, PI32, PD]),
        "sfk_basis_vector": (I32, [P, I32, I32, I32, P]),
        "sfk_adjoint": (I32, [P, P, P, PD]),
        "sfk_init_beam": (I32, [ctypes.POINTER(P), ctypes.POINTER(Beam), P, PPAR, P, ctypes.c_size_t, P]),
        "sfk_apply": (I32, [P, I32, P, P]),
        "sfk_tau_apply": (I32, [P, P, P, I32]),
        "sfk_tau_stats": (I32, [P, PI32, PD]),
        "sfk_solve_noalloc": (I32, [PCSR, PCSR, P, PPAR, I32, P, PD, PI32, PI32, P]),
        "sfk_memory": (I32, [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]),
        "sfk_true_residual": (I32, [P, PD]),
        "sfk_destroy": (I32, [P]),
        "sfk_last_error": (ctypes.c_char_p, [P]),
        "sfk_sketch_sparse_sign": (I32, [P, PI32, PI8]),
        "sfk_sketch_srht": (I32, [P, PI32, PI8, ctypes.POINTER(I64)]),
        "sfk_coefficients": (I32, [P, PD, PD, I32]),
        "sfk_version": (ctypes.c_char_p, []),
        "sfk_set_timing": (I32, [P, I32]),
        "sfk_init_batch": (I32, [ctypes.POINTER(P), I32, PCSR, PCSR, ctypes.POINTER(P), PPAR, P]),
        "sfk_batch_size": (I32, [P]),
        "sfk_instance_status": (I32, [P, I32, PI32, PI32, PI32]),
        "sfk_instance_solution": (I32, [P, I32, P]),
        "sfk_instance_solution_at": (I32, [P, I32, I32, P]),
        "sfk_instance_residual_norms": (I32, [P, I32, I32, PD, I32, PI32, PD]),
        "sfk_instance_true_residual": (I32, [P, I32, PD]),
        "sfk_init_multi": (I32, [ctypes.POINTER(P), PCSR, PCSR, P, I32, PPAR, P]),
        "sfk_stage_times": (I32, [P, PD, PI32]),
        "sfk_spmv_variant": (I32, [P, PI32, PI32]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def exported_symbols() -> list[str]:
    return ["sfk_params_default", "sfk_validate", "sfk_workspace_bytes", "sfk_init", "sfk_iterate",
            "sfk_solution", "sfk_solution_at", "sfk_residual_norms", "sfk_true_residual",
            "sfk_destroy", "sfk_last_error", "sfk_sketch_sparse_sign", "sfk_sketch_srht",
            "sfk_coefficients", "sfk_version", "sfk_set_timing", "sfk_stage_times",
            "sfk_init_batch", "sfk_batch_size", "sfk_instance_status", "sfk_instance_solution",
            "sfk_instance_residual_norms", "sfk_instance_true_residual", "sfk_init_multi",
            "sfk_instance_solution_at", "sfk_spmv_variant", "sfk_memory", "sfk_basis_vector",
            "sfk_solve_noalloc", "sfk_adjoint", "sfk_init_beam", "sfk_apply", "sfk_tau_apply",
            "sfk_tau_stats"]


def _check(status: int, ctx=None):
    if status != OK:
        msg = lib().sfk_last_error(ctx)
        raise SfkError(status, msg.decode() if msg else "")


def params(method="sflsqr", *, ell=2, maxit=50, sketch="sparse_sign", s=101, zeta=8, seed=0,
           instance=0, tau="identity", eps=1e-3, eta=1.01, noise_norm=0.0, tol=0.0,
           driver="auto", vw=-2, vw_b=None, wg_per_cu=0, resid=0, copies=0, tape=0,
           perm=None, lr_rows=0, lr_rank=0, lr_over=0, lr_q=1, lr_maxit=0,
           lr_tol=0.0) -> Params:
    """perm: optional order of the unknowns, a torch.int32 device tensor of n
    distinct values in [0, n) (unknown j stored at position perm[j] inside the
    library; results come back in the caller's order).
    vw: SpMV kernel, as sfk_params.vw: -2 automatic (timed at init), 0
    CSR-stream, 1 SELL-64, 8/16/32/64 lanes per row, -1 lanes from the mean row
    length; for right-hand sides sharing A and B (init_multi) -2 automatic, 0
    column-sliced L2 gathers, 2 LDS-staged units, any other value the row
    kernel.
    vw_b: SpMV kernel of B (coded as vw) when it differs from A's (sets
    vw_split); resid: 0, 1 (record ||b - A x_k|| every iteration) or 2 (record
    it and stop on it); copies: 1 forbids device copies of the operators
    beyond the workspace.
    tau "lowrank" / "lowrank_rnd": rank-lr_rank truncation of each basis vector
    viewed as an lr_rows x (n / lr_rows) image (truncated SVD to a Ritz-residual
    tolerance lr_tol, or the randomized SVD with lr_q power iterations), with
    l = lr_rank + lr_over test vectors (0: automatic)."""
    p = Params()
    lib().sfk_params_default(ctypes.byref(p))
    p.method = _METHODS[method] if isinstance(method, str) else int(method)
    p.ell, p.maxit = ell, maxit
    p.sketch = _SKETCHES[sketch] if isinstance(sketch, str) else int(sketch)
    if sketch == "countsketch":
        zeta = 1
    p.s, p.zeta, p.seed, p.instance = s, zeta, seed, instance
    p.tau = _TAUS[tau] if isinstance(tau, str) else int(tau)
    p.eps, p.eta, p.noise_norm, p.tol = eps, eta, noise_norm, tol
    p.driver = _DRIVERS[driver] if isinstance(driver, str) else int(driver)
    p.vw, p.wg_per_cu = vw, wg_per_cu
    if vw_b is not None:
        p.vw_b, p.vw_split = int(vw_b), 1
    p.resid, p.copies, p.tape = int(resid), int(copies), int(tape)
    p.lr_rows, p.lr_rank, p.lr_over = int(lr_rows), int(lr_rank), int(lr_over)
    p.lr_q, p.lr_maxit, p.lr_tol = int(lr_q), int(lr_maxit), float(lr_tol)
    if perm is not None:
        import torch
        if perm.dtype != torch.int32 or not perm.is_cuda or not perm.is_contiguous():
            raise ValueError("perm must be a contiguous torch.int32 device tensor")
        p.perm = perm.data_ptr()
        p._perm = perm           # kept alive with the parameters (copied at init)
    return p


# ----------------------------------------------------------------------------
# device matrices
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class DeviceCSR:
    """CSR arrays resident on the GPU (torch tensors keep the memory alive)."""
    rows: int
    cols: int
    rowptr: object
    colind: object
    val: object

    @property
    def nnz(self) -> int:
        return int(self.colind.numel())

    def c(self) -> CSR:
        return CSR(self.rows, self.cols, self.nnz, self.rowptr.data_ptr(),
                   self.colind.data_ptr() if self.nnz else self.rowptr.data_ptr(),
                   self.val.data_ptr() if self.nnz else self.rowptr.data_ptr())


def to_device_csr(M, device="cuda") -> DeviceCSR:
    """scipy CSR -> DeviceCSR (int32 indices, float64 values)."""
    import torch
    M = M.tocsr()
    return DeviceCSR(M.shape[0], M.shape[1],
                     torch.from_numpy(np.ascontiguousarray(M.indptr, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(M.indices, dtype=np.int32)).to(device),
                     torch.from_numpy(np.ascontiguousarray(M.data, dtype=np.float64)).to(device))


def host_csr_descriptor(rows: int, cols: int, nnz: int) -> CSR:
    """A descriptor with NULL arrays, for host-only validation."""
    return CSR(rows, cols, nnz, None, None, None)


def validate(A: CSR, B: CSR | None, p: Params) -> tuple[int, str]:
    st = lib().sfk_validate(ctypes.byref(A), ctypes.byref(B) if B is not None else None,
                            ctypes.byref(p))
    msg = lib().sfk_last_error(None).decode() if st != OK else ""
    return st, msg


def workspace_bytes(A: CSR, B: CSR | None, p: Params) -> int:
    return int(lib().sfk_workspace_bytes(ctypes.byref(A),
                                         ctypes.byref(B) if B is not None else None, ctypes.byref(p)))


# ----------------------------------------------------------------------------
# context
# ----------------------------------------------------------------------------

class Context:
    """Owns an sfk_ctx; keeps the borrowed device buffers alive."""

    def __init__(self, handle, A: DeviceCSR, B: DeviceCSR | None, b, p: Params, ws, stream):
        self.handle = handle
        self.A, self.B, self.b, self.p, self.ws, self.stream = A, B, b, p, ws, stream
        self.m, self.n = A.rows, A.cols
        self.k = 0
        self.stopped = False

    def __del__(self):
        try:
            destroy(self)
        except Exception:
            pass


def init(A: DeviceCSR, B: DeviceCSR | None, b, p: Params, *, stream=None,
         library_workspace: bool = False) -> Context:
    """sfk_init: A (m x n), B (n x m) or None for A^T, b (m) float64 on the GPU."""
    import torch
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()):
        raise ValueError("b must be a contiguous float64 CUDA tensor")
    Ac = A.c()
    Bc = B.c() if B is not None else None
    ws = None
    ws_ptr, ws_len = None, 0
    if not library_workspace:
        nbytes = workspace_bytes(Ac, Bc, p)
        if nbytes == 0:
            _check(validate(Ac, Bc, p)[0])
        ws = torch.empty(nbytes, dtype=torch.uint8, device=b.device)
        ws_ptr, ws_len = ws.data_ptr(), nbytes
    st_obj = stream if stream is not None else torch.cuda.current_stream(b.device)
    h = ctypes.c_void_p()
    st = lib().sfk_init(ctypes.byref(h), ctypes.byref(Ac), ctypes.byref(Bc) if Bc is not None else None,
                        b.data_ptr(), ctypes.byref(p), ws_ptr, ws_len, st_obj.cuda_stream)
    _check(st)
    return Context(h, A, B, b, p, ws, st_obj)


NOALLOC_BYTES = 64 << 20


def solve_noalloc(A: DeviceCSR, B: DeviceCSR | None, b, p: Params, k: int, *, x=None,
                  stream=None):
    """sfk_solve_noalloc: k iterations of one instance with the library's fixed
    device scratch (no device allocation inside the call).  x: optional CUDA
    float64 n-vector for the result (allocated here by torch when None, i.e. by
    the caller's side).  Returns (x, rho, iterations done, stopped, status)."""
    import torch
    if x is None:
        x = torch.empty(A.cols, dtype=torch.float64, device=b.device)
    st_obj = stream if stream is not None else torch.cuda.current_stream(b.device)
    rho = (ctypes.c_double * max(1, k))()
    done, stopped = ctypes.c_int32(), ctypes.c_int32()
    Bc = ctypes.byref(B.c()) if B is not None else None
    st = lib().sfk_solve_noalloc(ctypes.byref(A.c()), Bc, b.data_ptr(), ctypes.byref(p), int(k),
                                 x.data_ptr(), rho, ctypes.byref(done), ctypes.byref(stopped),
                                 st_obj.cuda_stream)
    if st not in (OK, BREAKDOWN):
        _check(st)
    return x, np.array(rho[: done.value]), done.value, bool(stopped.value), st


class BeamGeometry:
    """Parallel-beam geometry for the matrix-free operators (sfk_beam): the
    direction tables live on the device as long as this object."""

    def __init__(self, N, n_angles, n_det, *, nz=1, back=0, cos_a=None, sin_a=None, device="cuda"):
        import math
        import torch
        theta = np.arange(n_angles, dtype=np.float64) * (math.pi / n_angles)
        ca = np.cos(theta) if cos_a is None else np.asarray(cos_a, dtype=np.float64)
        sa = np.sin(theta) if sin_a is None else np.asarray(sin_a, dtype=np.float64)
        self.cos = torch.from_numpy(np.ascontiguousarray(ca)).to(device)
        self.sin = torch.from_numpy(np.ascontiguousarray(sa)).to(device)
        self.N, self.nz, self.n_angles, self.n_det, self.back = N, nz, n_angles, n_det, back
        self.m = nz * n_angles * n_det
        self.n = nz * N * N

    def c(self) -> Beam:
        return Beam(self.N, self.nz, self.n_angles, self.n_det, self.cos.data_ptr(),
                    self.sin.data_ptr(), self.back, 0)


def init_beam(geo: BeamGeometry, b, p: Params, *, stream=None) -> Context:
    """sfk_init_beam: matrix-free operators of the parallel-beam geometry."""
    import torch
    if not (b.is_cuda and b.dtype == torch.float64 and b.is_contiguous() and b.numel() == geo.m):
        raise ValueError("b must be a contiguous float64 CUDA tensor of length m")
    st_obj = stream if stream is not None else torch.cuda.current_stream(b.device)
    h = ctypes.c_void_p()
    g = geo.c()
    st = lib().sfk_init_beam(ctypes.byref(h), ctypes.byref(g), b.data_ptr(), ctypes.byref(p), None, 0,
                             st_obj.cuda_stream)
    _check(st)
    A = DeviceCSR(geo.m, geo.n, None, None, None)
    ctx = Context(h, A, None, b, p, None, st_obj)
    ctx.geo = geo
    return ctx


def apply(ctx: Context, op: str, x):
    """sfk_apply: y = A x (op "A") or y = B x (op "B")."""
    import torch
    y = torch.empty(ctx.m if op == "A" else ctx.n, dtype=torch.float64, device=x.device)
    _check(lib().sfk_apply(ctx.handle, 0 if op == "A" else 1, x.contiguous().data_ptr(), y.data_ptr()),
           ctx.handle)
    return y


def tau_apply(ctx: Context, x, call: int = 1):
    """sfk_tau_apply: the context's low-rank operator applied to x (as to basis
    vector `call`)."""
    import torch
    xc = x.contiguous()
    y = torch.empty_like(xc)
    _check(lib().sfk_tau_apply(ctx.handle, xc.data_ptr(), y.data_ptr(), int(call)), ctx.handle)
    return y


def tau_stats(ctx: Context) -> dict:
    """sfk_tau_stats: power iterations and residual test of the last application,
    unconverged applications so far, last relative Ritz residual."""
    out = (ctypes.c_int32 * 3)()
    rm = ctypes.c_double()
    _check(lib().sfk_tau_stats(ctx.handle, out, ctypes.byref(rm)), ctx.handle)
    return {"iterations": out[0], "converged": bool(out[1]), "unconverged_calls": out[2],
            "resmax": rm.value}


def iterate(ctx: Context, k: int) -> tuple[int, bool, int]:
    """sfk_iterate: returns (iterations done, stopped, status); BREAKDOWN is not raised."""
    done, stopped = ctypes.c_int32(), ctypes.c_int32()
    st = lib().sfk_iterate(ctx.handle, int(k), ctypes.byref(done), ctypes.byref(stopped))
    if st not in (OK, BREAKDOWN):
        _check(st, ctx.handle)
    ctx.k, ctx.stopped = done.value, bool(stopped.value)
    return done.value, bool(stopped.value), st


def solution(ctx: Context, out=None):
    import torch
    x = out if out is not None else torch.empty(ctx.n, dtype=torch.float64, device=ctx.b.device)
    _check(lib().sfk_solution(ctx.handle, x.data_ptr()), ctx.handle)
    return x


def solution_at(ctx: Context, j: int, out=None):
    import torch
    x = out if out is not None else torch.empty(ctx.n, dtype=torch.float64, device=ctx.b.device)
    _check(lib().sfk_solution_at(ctx.handle, int(j), x.data_ptr()), ctx.handle)
    return x


def _res_kind(kind) -> int:
    return _RES[kind] if isinstance(kind, str) else int(kind)


def residual_norms(ctx: Context, kind="sketched") -> tuple[np.ndarray, float]:
    """Residual history j = 1..k of the given kind ("sketched": rho_j,
    "true_recurrence": ||beta e_1 - H y_j||, "true_explicit": ||b - A x_j||) and
    the scale of its stop test (||S b|| or ||S B b|| for "sketched", ||b||
    otherwise)."""
    cap = max(1, ctx.p.maxit)
    buf = (ctypes.c_double * cap)()
    cnt = ctypes.c_int32()
    rn = ctypes.c_double()
    _check(lib().sfk_residual_norms(ctx.handle, _res_kind(kind), buf, cap, ctypes.byref(cnt),
                                    ctypes.byref(rn)), ctx.handle)
    return np.array(buf[: cnt.value]), rn.value


def memory(ctx) -> tuple[int, int]:
    """(workspace bytes, bytes the library allocated besides it) of a context."""
    ws, lb = ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().sfk_memory(ctx.handle, ctypes.byref(ws), ctypes.byref(lb)), ctx.handle)
    return ws.value, lb.value


def true_residual(ctx: Context) -> float:
    out = ctypes.c_double()
    _check(lib().sfk_true_residual(ctx.handle, ctypes.byref(out)), ctx.handle)
    return out.value


def destroy(ctx: Context):
    if ctx.handle is not None and _lib is not None:
        lib().sfk_destroy(ctx.handle)
        ctx.handle = None


def sketch_sparse_sign(ctx: Context) -> tuple[np.ndarray, np.ndarray]:
    d = ctx.m if ctx.p.method == SFLSQR else ctx.n
    z = ctx.p.zeta
    rows = np.zeros(d * z, dtype=np.int32)
    neg = np.zeros(d * z, dtype=np.int8)
    _check(lib().sfk_sketch_sparse_sign(ctx.handle, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        neg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))), ctx.handle)
    return rows.reshape(d, z), neg.reshape(d, z)


def sketch_srht(ctx: Context) -> tuple[np.ndarray, np.ndarray]:
    d = ctx.m if ctx.p.method == SFLSQR else ctx.n
    N = 1
    while N < d:
        N *= 2
    rows = np.zeros(ctx.p.s, dtype=np.int32)
    neg = np.zeros(N, dtype=np.int8)
    Nout = ctypes.c_int64()
    _check(lib().sfk_sketch_srht(ctx.handle, rows.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                 neg.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)),
                                 ctypes.byref(Nout)), ctx.handle)
    return rows, neg


def coefficients(ctx: Context, k: int) -> tuple[np.ndarray, np.ndarray]:
    H = np.zeros((k, k + 1))
    T = np.zeros((k, k))
    _check(lib().sfk_coefficients(ctx.handle, H.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  T.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(k)),
           ctx.handle)
    return H.T.copy(), T.T.copy()


STAGES = ("spmv_A", "w_update", "sketch", "ls", "spmv_B", "p_update", "tau")


def set_timing(ctx: Context, on: bool = True):
    _check(lib().sfk_set_timing(ctx.handle, 1 if on else 0), ctx.handle)


def stage_times(ctx: Context) -> dict:
    """{stage: (total ms, launches)} accumulated since set_timing."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (ctypes.c_int32 * len(STAGES))()
    _check(lib().sfk_stage_times(ctx.handle, ms, cnt), ctx.handle)
    return {name: (ms[i], cnt[i]) for i, name in enumerate(STAGES)}


class BatchContext:
    """A context of independent instances advancing in lockstep."""

    def __init__(self, handle, As, Bs, bs, ps, stream):
        self.handle = handle
        self.As, self.Bs, self.bs, self.ps, self.stream = As, Bs, bs, ps, stream
        self.nb = len(ps)

    def __del__(self):
        try:
            if self.handle is not None and _lib is not None:
                lib().sfk_destroy(self.handle)
                self.handle = None
        except Exception:
            pass


def init_batch(As: list, Bs: list | None, bs: list, ps: list, *, stream=None) -> BatchContext:
    """sfk_init_batch: lists of DeviceCSR A_i, DeviceCSR-or-None B_i, CUDA b_i, Params p_i."""
    import torch
    nb = len(As)
    Aarr = (CSR * nb)(*[A.c() for A in As])
    Barr = None
    if Bs is not None and any(B is not None for B in Bs):
        Barr = (CSR * nb)(*[(B.c() if B is not None else CSR(0, 0, 0, None, None, None)) for B in Bs])
    barr = (ctypes.c_void_p * nb)(*[b.data_ptr() for b in bs])
    parr = (Params * nb)(*ps)
    st_obj = stream if stream is not None else torch.cuda.current_stream(bs[0].device)
    h = ctypes.c_void_p()
    st = lib().sfk_init_batch(ctypes.byref(h), nb, Aarr, Barr, barr, parr, st_obj.cuda_stream)
    _check(st)
    return BatchContext(h, As, Bs, bs, ps, st_obj)


def init_multi(A: DeviceCSR, B: DeviceCSR | None, b_block, ps: list, *, stream=None) -> BatchContext:
    """sfk_init_multi: R right-hand sides sharing A and B.  b_block is a CUDA
    float64 tensor of shape (R, m) (right-hand side r in row r, contiguous);
    ps holds R Params that agree except in seed, instance, eta, noise_norm, tol."""
    import torch
    R = len(ps)
    if tuple(b_block.shape) != (R, A.rows) or not b_block.is_contiguous() \
            or b_block.dtype != torch.float64:
        raise ValueError(f"b_block must be a contiguous float64 tensor of shape ({R}, {A.rows})")
    parr = (Params * R)(*ps)
    st_obj = stream if stream is not None else torch.cuda.current_stream(b_block.device)
    h = ctypes.c_void_p()
    Bc = ctypes.byref(B.c()) if B is not None else None
    st = lib().sfk_init_multi(ctypes.byref(h), ctypes.byref(A.c()), Bc, b_block.data_ptr(), R, parr,
                              st_obj.cuda_stream)
    _check(st)
    return BatchContext(h, [A], [B], [b_block], ps, st_obj)


def instance_true_residual(ctx, i: int) -> float:
    out = ctypes.c_double()
    _check(lib().sfk_instance_true_residual(ctx.handle, i, ctypes.byref(out)), ctx.handle)
    return out.value


def instance_status(ctx, i: int) -> tuple[int, bool, int]:
    d, s, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sfk_instance_status(ctx.handle, i, ctypes.byref(d), ctypes.byref(s), ctypes.byref(b)),
           ctx.handle)
    return d.value, bool(s.value), b.value


def instance_solution(ctx, i: int, n: int, out=None):
    import torch
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device="cuda")
    _check(lib().sfk_instance_solution(ctx.handle, i, x.data_ptr()), ctx.handle)
    return x


def instance_solution_at(ctx, i: int, j: int, n: int, out=None):
    import torch
    x = out if out is not None else torch.empty(n, dtype=torch.float64, device="cuda")
    _check(lib().sfk_instance_solution_at(ctx.handle, i, j, x.data_ptr()), ctx.handle)
    return x


def instance_residual_norms(ctx, i: int, cap: int, kind="sketched") -> tuple[np.ndarray, float]:
    buf = (ctypes.c_double * max(1, cap))()
    cnt = ctypes.c_int32()
    rn = ctypes.c_double()
    _check(lib().sfk_instance_residual_norms(ctx.handle, i, _res_kind(kind), buf, max(1, cap),
                                             ctypes.byref(cnt), ctypes.byref(rn)), ctx.handle)
    return np.array(buf[: min(cnt.value, cap)]), rn.value


BASIS = {"w": 0, "p": 1, "z": 2}


def basis_vector(ctx, kind: str, j: int, i: int = 0):
    """Basis vector w_j, p_j or z_j of instance i (see sfk_basis_vector), as a
    CUDA float64 tensor (n-vectors in the caller's order)."""
    import torch
    inst_ctx = ctx
    length = None
    if isinstance(ctx, Context):
        length = ctx.m if kind == "w" else ctx.n
    else:
        A = ctx.As[0] if len(ctx.As) == 1 else ctx.As[i]
        length = A.rows if kind == "w" else A.cols
    x = torch.empty(length, dtype=torch.float64, device="cuda")
    _check(lib().sfk_basis_vector(inst_ctx.handle, int(i), BASIS[kind], int(j), x.data_ptr()),
           inst_ctx.handle)
    return x


def adjoint(ctx: Context, xbar):
    """sfk_adjoint: (dL/db as a CUDA float64 m-vector, dL/deps) for xbar = dL/dx_K."""
    import torch
    xb = xbar.contiguous()
    if not (xb.is_cuda and xb.dtype == torch.float64 and xb.numel() == ctx.n):
        raise ValueError("xbar must be a CUDA float64 n-vector")
    bb = torch.empty(ctx.m, dtype=torch.float64, device=xb.device)
    eb = ctypes.c_double()
    _check(lib().sfk_adjoint(ctx.handle, xb.data_ptr(), bb.data_ptr(), ctypes.byref(eb)), ctx.handle)
    return bb, eb.value


def spmv_variant(ctx) -> tuple[int, int]:
    """(variant for A, variant for B) actually launched (see sfk_spmv_variant)."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().sfk_spmv_variant(ctx.handle, ctypes.byref(a), ctypes.byref(b)), ctx.handle)
    return a.value, b.value


def version() -> str:
    return lib().sfk_version().decode()


# ----------------------------------------------------------------------------
# convenience
# ----------------------------------------------------------------------------

class Solver:
    """Owns device copies of a problem and one context."""

    def __init__(self, A, b, *, B=None, device="cuda", **kw):
        import torch
        self.dA = A if isinstance(A, DeviceCSR) else to_device_csr(A, device)
        self.dB = None if B is None else (B if isinstance(B, DeviceCSR) else to_device_csr(B, device))
        self.b = b if hasattr(b, "is_cuda") else torch.from_numpy(np.ascontiguousarray(b, np.float64)).to(device)
        self.p = params(**kw)
        self.ctx = init(self.dA, self.dB, self.b, self.p)

    def iterate(self, k: int):
        return iterate(self.ctx, k)

    def solution(self):
        return solution(self.ctx)

    def solution_at(self, j: int):
        return solution_at(self.ctx, j)

    def residual_norms(self, kind="sketched"):
        return residual_norms(self.ctx, kind)

    def true_residual(self):
        return true_residual(self.ctx)
