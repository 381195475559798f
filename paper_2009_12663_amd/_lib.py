"""ctypes binding of libbfgsuq.so (include/bfgsuq.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the computation runs in the library's HIP kernels.  The
library must be built (``paper_2009_12663_amd.build``); there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbfgsuq.so")

F64, F32, BF16 = 0, 1, 2
STORAGE_CODES = {"f64": F64, "f32": F32, "bf16": BF16}
STORAGE_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}
RESULT_TORCH = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.float32}

BFGS_OK = 0
BFGS_ERR_ARG = -1
BFGS_ERR_FULL = -2
BFGS_ERR_STATE = -3
BFGS_ERR_CURVATURE = -4
BFGS_ERR_NONFINITE = -5
BFGS_ERR_NUMERIC = -6
BFGS_ERR_ALLOC = -7
BFGS_ERR_HIP = -8
MAX_COLS = 256
MAX_PAIRS = 1024

EXPORTS = [
    "bfgs_create", "bfgs_create_streamed", "bfgs_destroy", "bfgs_push_pair", "bfgs_pop_oldest", "bfgs_num_pairs",
    "bfgs_apply_Hinv",
    "bfgs_apply_Hinv_noalloc",
    "bfgs_apply_Hdiff", "bfgs_generate_probes", "bfgs_rsvd", "bfgs_rsvd_ex", "bfgs_posterior_diag",
    "bfgs_get_pair", "bfgs_get_h0", "bfgs_get_status", "bfgs_status_string",
    "bfgs_profile", "bfgs_profile_report", "bfgs_autotune", "bfgs_tuning", "bfgs_set_tuning", "bfgs_sync", "bfgs_tsqr_shape",
    "bfgs_batch_create", "bfgs_batch_handle", "bfgs_batch_push_pairs", "bfgs_batch_apply_Hinv", "bfgs_batch_rsvd",
    "bfgs_batch_autotune", "bfgs_batch_graph_build", "bfgs_batch_graph_launch", "bfgs_batch_destroy",
    "bfgs_precond_diag", "bfgs_gridop_create", "bfgs_gridop_apply", "bfgs_gridop_destroy", "bfgs_minimize_quadratic",
    "bfgs_minimize_quadratic_ex",
    "bfgs_mlp_create", "bfgs_mlp_destroy", "bfgs_mlp_set_params", "bfgs_mlp_get_params", "bfgs_mlp_features",
    "bfgs_mlp_forward", "bfgs_mlp_grad", "bfgs_mlp_train_step",
]
MLP_NPARAM = 4801

_lib = None


class BfgsError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__(f"{where}: {status_string(code)} ({code})")


def load(path: str = LIB_PATH):
    """Load the library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libbfgsuq.so not built at {path}; run paper_2009_12663_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    sig = {
        "bfgs_create": [i64, i32, vp, ctypes.c_int, vp, ctypes.POINTER(vp)],
        "bfgs_create_streamed": [i64, i32, vp, ctypes.c_int, i64, vp, ctypes.POINTER(vp)],
        "bfgs_destroy": [vp],
        "bfgs_push_pair": [vp, vp, vp, ctypes.c_int],
        "bfgs_num_pairs": [vp, ctypes.POINTER(i32)],
        "bfgs_apply_Hinv": [vp, vp, i32, vp],
        "bfgs_apply_Hinv_noalloc": [vp, vp, i32, vp],
        "bfgs_apply_Hdiff": [vp, vp, i32, vp],
        "bfgs_generate_probes": [vp, u64, i32, vp],
        "bfgs_rsvd": [vp, i32, i32, u64, vp, vp],
        "bfgs_rsvd_ex": [vp, i32, i32, u64, ctypes.c_uint32, vp, vp],
        "bfgs_posterior_diag": [vp, vp],
        "bfgs_get_pair": [vp, i32, vp, vp],
        "bfgs_get_h0": [vp, vp],
        "bfgs_get_status": [vp],
        "bfgs_status_string": [ctypes.c_int],
        "bfgs_profile": [vp, i32],
        "bfgs_profile_report": [vp, ctypes.c_char_p, i32],
        "bfgs_autotune": [vp, i32, i32, i32, vp, vp, vp, vp],
        "bfgs_tuning": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "bfgs_set_tuning": [vp, i32, i32],
        "bfgs_sync": [vp],
        "bfgs_tsqr_shape": [i32, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "bfgs_batch_create": [i32, vp, vp, vp, ctypes.c_int, vp, ctypes.POINTER(vp)],
        "bfgs_batch_handle": [vp, i32, ctypes.POINTER(vp)],
        "bfgs_batch_push_pairs": [vp, vp, vp, vp, ctypes.c_int],
        "bfgs_batch_apply_Hinv": [vp, vp, vp, vp],
        "bfgs_batch_rsvd": [vp, vp, i32, u64, vp, vp],
        "bfgs_batch_autotune": [vp, vp, vp, vp, vp, i32, vp, vp],
        "bfgs_batch_graph_build": [vp, vp, vp, vp, vp, i32, u64, vp, vp],
        "bfgs_batch_graph_launch": [vp],
        "bfgs_batch_destroy": [vp],
        "bfgs_precond_diag": [i64, i64, i32, vp, ctypes.c_double, i32, ctypes.c_double, vp, vp,
                              ctypes.POINTER(ctypes.c_double), vp],
        "bfgs_gridop_create": [i64, i64, i32, vp, ctypes.c_double, i32, ctypes.c_double, vp, ctypes.POINTER(vp)],
        "bfgs_gridop_apply": [vp, vp, i32, vp],
        "bfgs_gridop_destroy": [vp],
        "bfgs_minimize_quadratic": [vp, vp, vp, i32, ctypes.c_double, vp, ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(i32)],
        "bfgs_minimize_quadratic_ex": [vp, vp, vp, i32, ctypes.c_double, i32, ctypes.c_double, vp,
                                       ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i32)],
        "bfgs_pop_oldest": [vp],
        "bfgs_mlp_create": [vp, ctypes.POINTER(vp)],
        "bfgs_mlp_destroy": [vp],
        "bfgs_mlp_set_params": [vp, vp],
        "bfgs_mlp_get_params": [vp, vp],
        "bfgs_mlp_features": [i64, i64, vp, vp, ctypes.c_float, vp, vp],
        "bfgs_mlp_forward": [vp, vp, i64, vp, i32],
        "bfgs_mlp_grad": [vp, vp, vp, i64, vp, vp],
        "bfgs_mlp_train_step": [vp, vp, vp, i64, ctypes.c_float, vp],
    }
    for name, args in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = ctypes.c_char_p if name == "bfgs_status_string" else ctypes.c_int
    _lib = L
    return L


def status_string(code: int) -> str:
    try:
        return load().bfgs_status_string(code).decode()
    except Exception:  # pragma: no cover
        return "status"


def _check(code: int, where: str) -> int:
    if code < 0:
        raise BfgsError(code, where)
    return code


def tsqr_shape(c: int):
    """(slot_f64, ring) of the tall-skinny QR for a c-column block."""
    a, b = ctypes.c_int32(), ctypes.c_int32()
    _check(load().bfgs_tsqr_shape(int(c), ctypes.byref(a), ctypes.byref(b)), "bfgs_tsqr_shape")
    return bool(a.value), int(b.value)


def precond_diag(hdiag: torch.Tensor, nx: int, nz: int, nparam: int, sigma: float, half: int,
                 damping: float = 1.0, stream: torch.cuda.Stream | None = None):
    """B_0 of eq. (4) from a diagonal Hessian estimate (bfgs_precond_diag):
    returns (h0, hs, lambda) with h0 and the smoothed estimate hs as float32 tensors."""
    L = load()
    h = hdiag.to(torch.float32).contiguous()
    assert h.is_cuda and h.numel() == nx * nz * nparam
    h0 = torch.empty_like(h)
    hs = torch.empty_like(h)
    lam = ctypes.c_double()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(L.bfgs_precond_diag(int(nx), int(nz), int(nparam), _ptr(h), float(sigma), int(half), float(damping),
                               _ptr(h0), _ptr(hs), ctypes.byref(lam), ctypes.c_void_p(st.cuda_stream)),
           "bfgs_precond_diag")
    return h0, hs, lam.value


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Bfgs:
    """One BFGS history on the current CUDA/HIP device and stream.

    Vectors and blocks are torch tensors on the device; a block of ncols
    vectors of length n has shape (ncols, n) (column-major n x ncols)."""

    def __init__(self, n: int, k_max: int, h0: torch.Tensor | None = None, storage: str = "f32",
                 stream: torch.cuda.Stream | None = None, _handle=None, slice_rows: int | None = None):
        """slice_rows: keep the pairs in host memory and stream them to the device in
        row slices of this many rows (bfgs_create_streamed)."""
        self.L = load()
        self.n, self.k_max, self.storage = int(n), int(k_max), storage
        self.sdt = STORAGE_TORCH[storage]
        self.rdt = RESULT_TORCH[storage]
        self.hdt = torch.float64 if storage == "f64" else torch.float32
        self._owns = _handle is None
        if _handle is not None:          # a problem handle owned by a BfgsBatch
            self.h = _handle
            self.stream = None
            return
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h0 = None
        if h0 is not None:
            assert h0.is_cuda and h0.numel() == self.n
            self._h0 = h0.to(self.hdt).contiguous()
        handle = ctypes.c_void_p()
        if slice_rows is None:
            _check(self.L.bfgs_create(self.n, self.k_max, _ptr(self._h0), STORAGE_CODES[storage],
                                      ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
                   "bfgs_create")
        else:
            _check(self.L.bfgs_create_streamed(self.n, self.k_max, _ptr(self._h0), STORAGE_CODES[storage],
                                               int(slice_rows), ctypes.c_void_p(self.stream.cuda_stream),
                                               ctypes.byref(handle)),
                   "bfgs_create_streamed")
        self.h = handle

    # -- life cycle -------------------------------------------------------------------
    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owns", True):
                self.L.bfgs_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- calls ------------------------------------------------------------------------
    def _enter(self):
        # A batch-owned handle runs on its own side stream: order it after torch's stream.
        if not self._owns:
            torch.cuda.current_stream().synchronize()

    def _leave(self):
        if not self._owns:
            _check(self.L.bfgs_sync(self.h), "bfgs_sync")

    def push_pair(self, s: torch.Tensor, y: torch.Tensor) -> None:
        dt = torch.float64 if s.dtype == torch.float64 else torch.float32
        s = s.to(dt).contiguous()
        y = y.to(dt).contiguous()
        assert s.numel() == self.n and y.numel() == self.n and s.is_cuda and y.is_cuda
        self._enter()
        _check(self.L.bfgs_push_pair(self.h, _ptr(s), _ptr(y), F64 if dt == torch.float64 else F32),
               "bfgs_push_pair")
        self._leave()

    def pop_oldest(self) -> None:
        """bfgs_pop_oldest: forget the oldest stored pair (the limited-memory form)."""
        self._enter()
        _check(self.L.bfgs_pop_oldest(self.h), "bfgs_pop_oldest")
        self._leave()

    @property
    def k(self) -> int:
        out = ctypes.c_int32()
        _check(self.L.bfgs_num_pairs(self.h, ctypes.byref(out)), "bfgs_num_pairs")
        return out.value

    def _block(self, V):
        assert V.is_cuda and V.dim() == 2 and V.shape[1] == self.n
        return V.to(self.sdt).contiguous()

    def apply_Hinv(self, V: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        V = self._block(V)
        if out is None:
            out = torch.empty(V.shape, dtype=self.rdt, device=V.device)
        self._enter()
        _check(self.L.bfgs_apply_Hinv(self.h, _ptr(V), V.shape[0], _ptr(out)), "bfgs_apply_Hinv")
        self._leave()
        return out

    def apply_Hdiff(self, V: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        V = self._block(V)
        if out is None:
            out = torch.empty(V.shape, dtype=self.rdt, device=V.device)
        self._enter()
        _check(self.L.bfgs_apply_Hdiff(self.h, _ptr(V), V.shape[0], _ptr(out)), "bfgs_apply_Hdiff")
        self._leave()
        return out

    def generate_probes(self, seed: int, ncols: int) -> torch.Tensor:
        X = torch.empty((ncols, self.n), dtype=self.sdt, device="cuda")
        self._enter()
        _check(self.L.bfgs_generate_probes(self.h, ctypes.c_uint64(seed), ncols, _ptr(X)),
               "bfgs_generate_probes")
        self._leave()
        return X

    def rsvd(self, rank: int, oversample: int, seed: int, U: torch.Tensor | None = None,
             Sigma: torch.Tensor | None = None):
        if U is None:
            U = torch.empty((rank, self.n), dtype=self.rdt, device="cuda")
        if Sigma is None:
            Sigma = torch.empty(rank, dtype=torch.float64, device="cuda")
        self._enter()
        _check(self.L.bfgs_rsvd(self.h, rank, oversample, ctypes.c_uint64(seed), _ptr(U), _ptr(Sigma)),
               "bfgs_rsvd")
        self._leave()
        return U, Sigma

    def rsvd_ex(self, rank: int, oversample: int, seed: int, precond: bool = False, two_pass: bool = False,
                U: torch.Tensor | None = None, Sigma: torch.Tensor | None = None):
        """bfgs_rsvd_ex: the preconditioned (whitened) and/or two-pass variants."""
        if U is None:
            U = torch.empty((rank, self.n), dtype=self.rdt, device="cuda")
        if Sigma is None:
            Sigma = torch.empty(rank, dtype=torch.float64, device="cuda")
        flags = (1 if precond else 0) | (2 if two_pass else 0)
        self._enter()
        _check(self.L.bfgs_rsvd_ex(self.h, rank, oversample, ctypes.c_uint64(seed), flags, _ptr(U), _ptr(Sigma)),
               "bfgs_rsvd_ex")
        self._leave()
        return U, Sigma

    def posterior_diag(self, out: torch.Tensor | None = None) -> torch.Tensor:
        if out is None:
            out = torch.empty(self.n, dtype=self.rdt, device="cuda")
        self._enter()
        _check(self.L.bfgs_posterior_diag(self.h, _ptr(out)), "bfgs_posterior_diag")
        self._leave()
        return out

    def get_pair(self, j: int):
        s = torch.empty(self.n, dtype=self.rdt, device="cuda")
        y = torch.empty(self.n, dtype=self.rdt, device="cuda")
        self._enter()
        _check(self.L.bfgs_get_pair(self.h, j, _ptr(s), _ptr(y)), "bfgs_get_pair")
        self._leave()
        return s, y

    def get_pairs(self):
        """All stored pairs, upcast exactly: (S, Y) of shape (k, n) on the device."""
        k = self.k
        S = torch.empty((k, self.n), dtype=self.rdt, device="cuda")
        Y = torch.empty((k, self.n), dtype=self.rdt, device="cuda")
        self._enter()
        for j in range(k):
            _check(self.L.bfgs_get_pair(self.h, j, _ptr(S[j]), _ptr(Y[j])), "bfgs_get_pair")
        self._leave()
        return S, Y

    def get_h0(self) -> torch.Tensor:
        out = torch.empty(self.n, dtype=self.hdt, device="cuda")
        self._enter()
        _check(self.L.bfgs_get_h0(self.h, _ptr(out)), "bfgs_get_h0")
        self._leave()
        return out

    def get_status(self) -> int:
        return self.L.bfgs_get_status(self.h)

    def autotune(self, V: torch.Tensor, out: torch.Tensor | None = None, rank: int = 0, oversample: int = 0):
        """Times the tunable launch shapes on these buffers and keeps the fastest."""
        V = self._block(V)
        if out is None:
            out = torch.empty(V.shape, dtype=self.rdt, device=V.device)
        U = Sig = None
        if rank:
            U = torch.empty((rank, self.n), dtype=self.rdt, device="cuda")
            Sig = torch.empty(rank, dtype=torch.float64, device="cuda")
        _check(self.L.bfgs_autotune(self.h, V.shape[0], rank, oversample, _ptr(V), _ptr(out), _ptr(U), _ptr(Sig)),
               "bfgs_autotune")
        return self.tuning()

    def tuning(self):
        a, b = ctypes.c_int32(), ctypes.c_int32()
        _check(self.L.bfgs_tuning(self.h, ctypes.byref(a), ctypes.byref(b)), "bfgs_tuning")
        return {"g1_rows": a.value, "qr_chains": b.value}

    def set_tuning(self, g1_rows: int = 0, qr_chains: int = 0):
        """bfgs_set_tuning: pin the launch shapes (0 keeps a choice)."""
        _check(self.L.bfgs_set_tuning(self.h, int(g1_rows), int(qr_chains)), "bfgs_set_tuning")

    def profile(self, enable: bool):
        _check(self.L.bfgs_profile(self.h, 1 if enable else 0), "bfgs_profile")

    def profile_report(self) -> dict:
        import json
        buf = ctypes.create_string_buffer(1 << 16)
        _check(self.L.bfgs_profile_report(self.h, buf, len(buf)), "bfgs_profile_report")
        return json.loads(buf.value.decode())


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))()
    for i, t in enumerate(tensors):
        arr[i] = None if t is None else t.data_ptr()
    return arr


def _i32_array(vals):
    return (ctypes.c_int32 * len(vals))(*[int(v) for v in vals])


class GridOp:
    """The synthetic grid Hessian A = diag(D) + P (x) (G_z (x) G_x) (bfgs_gridop_*)."""

    def __init__(self, nx: int, nz: int, nparam: int, D: torch.Tensor, sigma: float, half: int, coupling: float,
                 stream: torch.cuda.Stream | None = None):
        self.L = load()
        self.nx, self.nz, self.nparam = int(nx), int(nz), int(nparam)
        self.n = self.nx * self.nz * self.nparam
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        D = D.to(torch.float64).contiguous()
        assert D.is_cuda and D.numel() == self.n
        h = ctypes.c_void_p()
        _check(self.L.bfgs_gridop_create(self.nx, self.nz, self.nparam, _ptr(D), float(sigma), int(half),
                                         float(coupling), ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)),
               "bfgs_gridop_create")
        self.op = h

    def apply(self, x: torch.Tensor) -> torch.Tensor:
        x = x.to(torch.float64).contiguous()
        single = x.dim() == 1
        xb = x.view(1, -1) if single else x
        assert xb.is_cuda and xb.shape[1] == self.n
        y = torch.empty_like(xb)
        _check(self.L.bfgs_gridop_apply(self.op, _ptr(xb), xb.shape[0], _ptr(y)), "bfgs_gridop_apply")
        return y[0] if single else y

    def close(self):
        if getattr(self, "op", None):
            self.L.bfgs_gridop_destroy(self.op)
            self.op = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def minimize_quadratic(H: "Bfgs", op: GridOp, b: torch.Tensor, max_iter: int, rel_tol: float, memory: int = 0,
                       damping: float = 1.0):
    """bfgs_minimize_quadratic (memory 0, damping 1) or bfgs_minimize_quadratic_ex:
    returns (m, gnorms) with gnorms |g_0| .. |g_iters|."""
    L = load()
    b = b.to(torch.float64).contiguous()
    m = torch.empty_like(b)
    gn = (ctypes.c_double * (max_iter + 1))()
    it = ctypes.c_int32()
    if memory == 0 and damping == 1.0:
        _check(L.bfgs_minimize_quadratic(H.h, op.op, _ptr(b), int(max_iter), float(rel_tol), _ptr(m), gn,
                                         ctypes.byref(it)), "bfgs_minimize_quadratic")
    else:
        _check(L.bfgs_minimize_quadratic_ex(H.h, op.op, _ptr(b), int(max_iter), float(rel_tol), int(memory),
                                            float(damping), _ptr(m), gn, ctypes.byref(it)),
               "bfgs_minimize_quadratic_ex")
    return m, [gn[i] for i in range(it.value + 1)]


class BfgsBatch:
    """nprob independent histories driven together (bfgs_batch_* of the C ABI).

    `problems[i]` is a non-owning Bfgs view of problem i (push pairs through it).
    Blocks are lists of per-problem tensors."""

    def __init__(self, n: list, k_max: list, h0: list | None = None, storage: str = "f32",
                 stream: torch.cuda.Stream | None = None):
        self.L = load()
        self.nprob = len(n)
        self.storage = storage
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        hdt = torch.float64 if storage == "f64" else torch.float32
        self._h0 = None if h0 is None else [None if x is None else x.to(hdt).contiguous() for x in h0]
        n_arr = (ctypes.c_int64 * self.nprob)(*[int(x) for x in n])
        k_arr = _i32_array(k_max)
        h0_arr = None if self._h0 is None else _ptr_array(self._h0)
        handle = ctypes.c_void_p()
        _check(self.L.bfgs_batch_create(self.nprob, n_arr, k_arr, h0_arr, STORAGE_CODES[storage],
                                        ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(handle)),
               "bfgs_batch_create")
        self.b = handle
        self.problems = []
        for i in range(self.nprob):
            hp = ctypes.c_void_p()
            _check(self.L.bfgs_batch_handle(self.b, i, ctypes.byref(hp)), "bfgs_batch_handle")
            self.problems.append(Bfgs(n[i], k_max[i], storage=storage, _handle=hp))
        self._keep = []

    def close(self):
        if getattr(self, "b", None):
            for p in self.problems:
                p.h = None
            self.L.bfgs_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def push_pairs(self, S: list, Y: list):
        """S[i], Y[i]: (k_i, n_i) float32 or float64 tensors on the device (row j = pair j).
        Returns the status of bfgs_batch_push_pairs (0, or the first pair error met;
        rejected pairs are dropped); argument and capacity errors raise."""
        dt = S[0].dtype
        code = F64 if dt == torch.float64 else F32
        S = [s.to(dt).contiguous() for s in S]
        Y = [y.to(dt).contiguous() for y in Y]
        for p, s, y in zip(self.problems, S, Y):
            assert s.shape == y.shape and (s.numel() == 0 or s.shape[1] == p.n)
        rc = self.L.bfgs_batch_push_pairs(self.b, _ptr_array(S), _ptr_array(Y), _i32_array([s.shape[0] for s in S]),
                                          code)
        if rc in (BFGS_ERR_ARG, BFGS_ERR_FULL, BFGS_ERR_HIP, BFGS_ERR_ALLOC):
            raise BfgsError(rc, "bfgs_batch_push_pairs")
        return rc

    def apply_Hinv(self, V: list, out: list | None = None) -> list:
        V = [p._block(v) for p, v in zip(self.problems, V)]
        if out is None:
            out = [torch.empty(v.shape, dtype=p.rdt, device=v.device) for p, v in zip(self.problems, V)]
        self._keep = [V, out]
        _check(self.L.bfgs_batch_apply_Hinv(self.b, _ptr_array(V), _i32_array([v.shape[0] for v in V]),
                                            _ptr_array(out)), "bfgs_batch_apply_Hinv")
        return out

    def _rsvd_bufs(self, rank):
        U = [torch.empty((r, p.n), dtype=p.rdt, device="cuda") for p, r in zip(self.problems, rank)]
        Sig = [torch.empty(r, dtype=torch.float64, device="cuda") for r in rank]
        return U, Sig

    def rsvd(self, rank: list, oversample: int, seed: int, U=None, Sigma=None):
        if U is None:
            U, Sigma = self._rsvd_bufs(rank)
        self._keep = [U, Sigma]
        _check(self.L.bfgs_batch_rsvd(self.b, _i32_array(rank), oversample, ctypes.c_uint64(seed), _ptr_array(U),
                                      _ptr_array(Sigma)), "bfgs_batch_rsvd")
        return U, Sigma

    def autotune(self, V: list, rank: list | None = None, oversample: int = 0):
        V = [p._block(v) for p, v in zip(self.problems, V)]
        out = [torch.empty(v.shape, dtype=p.rdt, device=v.device) for p, v in zip(self.problems, V)]
        U = Sig = None
        if rank is not None:
            U, Sig = self._rsvd_bufs(rank)
        _check(self.L.bfgs_batch_autotune(self.b, _ptr_array(V), _i32_array([v.shape[0] for v in V]), _ptr_array(out),
                                          None if rank is None else _i32_array(rank), oversample,
                                          None if U is None else _ptr_array(U),
                                          None if Sig is None else _ptr_array(Sig)), "bfgs_batch_autotune")
        return [p.tuning() for p in self.problems]

    def graph_build(self, V: list, out: list, rank: list, oversample: int, seed: int, U: list, Sigma: list):
        V = [p._block(v) for p, v in zip(self.problems, V)]
        self._graph_keep = [V, out, U, Sigma]
        _check(self.L.bfgs_batch_graph_build(self.b, _ptr_array(V), _i32_array([v.shape[0] for v in V]),
                                             _ptr_array(out), _i32_array(rank), oversample, ctypes.c_uint64(seed),
                                             _ptr_array(U), _ptr_array(Sigma)), "bfgs_batch_graph_build")

    def graph_launch(self):
        _check(self.L.bfgs_batch_graph_launch(self.b), "bfgs_batch_graph_launch")


# Same names as the C ABI.
def bfgs_create(n, k, H0=None, storage="f32", stream=None) -> Bfgs:
    return Bfgs(n, k, H0, storage, stream)


def bfgs_push_pair(h: Bfgs, s, y):
    return h.push_pair(s, y)


def bfgs_apply_Hinv(h: Bfgs, V, out=None):
    return h.apply_Hinv(V, out)


def bfgs_apply_Hdiff(h: Bfgs, V, out=None):
    return h.apply_Hdiff(V, out)


def bfgs_rsvd(h: Bfgs, rank, oversample, seed, U=None, Sigma=None):
    return h.rsvd(rank, oversample, seed, U, Sigma)


def bfgs_posterior_diag(h: Bfgs, out=None):
    return h.posterior_diag(out)


def bfgs_generate_probes(h: Bfgs, seed, ncols):
    return h.generate_probes(seed, ncols)


def bfgs_destroy(h: Bfgs):
    h.close()


class Mlp:
    """The learned-B_0 network (bfgs_mlp_* of the C ABI)."""

    def __init__(self, params: torch.Tensor | None = None, stream: torch.cuda.Stream | None = None):
        self.L = load()
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        _check(self.L.bfgs_mlp_create(ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "bfgs_mlp_create")
        self.m = h
        if params is not None:
            self.set_params(params)

    def close(self):
        if getattr(self, "m", None):
            self.L.bfgs_mlp_destroy(self.m)
            self.m = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params: torch.Tensor):
        p = params.to("cuda", torch.float32).contiguous()
        assert p.numel() == MLP_NPARAM
        _check(self.L.bfgs_mlp_set_params(self.m, _ptr(p)), "bfgs_mlp_set_params")
        torch.cuda.current_stream().synchronize()

    def get_params(self) -> torch.Tensor:
        p = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        _check(self.L.bfgs_mlp_get_params(self.m, _ptr(p)), "bfgs_mlp_get_params")
        return p

    @staticmethod
    def features(logD: torch.Tensor, gabs: torch.Tensor, nx: int, nz: int, sigma_scale: float = 1.0) -> torch.Tensor:
        L = load()
        logD = logD.to("cuda", torch.float32).contiguous()
        gabs = gabs.to("cuda", torch.float32).contiguous()
        X = torch.empty((logD.numel(), 8), dtype=torch.float32, device="cuda")
        _check(L.bfgs_mlp_features(nx, nz, _ptr(logD), _ptr(gabs), ctypes.c_float(sigma_scale), _ptr(X),
                                   ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)), "bfgs_mlp_features")
        return X

    def forward(self, X: torch.Tensor, exp_out: bool = False) -> torch.Tensor:
        X = X.to("cuda", torch.float32).contiguous()
        out = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(self.L.bfgs_mlp_forward(self.m, _ptr(X), X.shape[0], _ptr(out), 1 if exp_out else 0),
               "bfgs_mlp_forward")
        return out

    def grad(self, X: torch.Tensor, target: torch.Tensor):
        X = X.to("cuda", torch.float32).contiguous()
        t = target.to("cuda", torch.float32).contiguous()
        g = torch.empty(MLP_NPARAM, dtype=torch.float32, device="cuda")
        loss = torch.empty(1, dtype=torch.float32, device="cuda")
        _check(self.L.bfgs_mlp_grad(self.m, _ptr(X), _ptr(t), X.shape[0], _ptr(g), _ptr(loss)), "bfgs_mlp_grad")
        return g, loss

    def train_step(self, X: torch.Tensor, target: torch.Tensor, lr: float, loss: torch.Tensor | None = None):
        """One Adam step; X, target (and loss, if given) should already be float32 device tensors."""
        X = X.to("cuda", torch.float32).contiguous()
        target = target.to("cuda", torch.float32).contiguous()
        _check(self.L.bfgs_mlp_train_step(self.m, _ptr(X), _ptr(target), X.shape[0], ctypes.c_float(lr), _ptr(loss)),
               "bfgs_mlp_train_step")
        return loss
