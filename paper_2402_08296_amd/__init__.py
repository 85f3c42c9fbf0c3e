"""Python binding of libddmgnn (DDM-GNN preconditioned flexible CG on MI355X).

Argument marshalling only: every step of the solve runs in the HIP library.
Device buffers are torch CUDA (HIP) tensors, passed by pointer; torch supplies
device memory and the stream, nothing else. There is no CPU fallback: when the
library is missing every call raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

from ._build import LIB as _LIB_PATH

FCG, PCG, CG, FGMRES = 0, 1, 2, 3
FP64, FP32, BF16 = 0, 1, 2
PROLONG_POU, PROLONG_UNWEIGHTED = 0, 1
LOCAL_GNN, LOCAL_LU = 0, 1
MEM_HOST, MEM_DEVICE = 0, 1
STATUS = {0: "OK", -1: "E_INVALID", -2: "E_NOMEM", -3: "E_HIP", -4: "E_NOT_SPD", -5: "E_BREAKDOWN",
          -6: "E_MAXIT", -7: "E_NONFINITE", -8: "E_BUDGET", -9: "E_PENDING"}
PRECISION = {"fp64": FP64, "fp32": FP32, "bf16": BF16}

_p = ctypes.c_void_p
_i32, _i64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double


class DDMGNNError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class ModelDesc(ctypes.Structure):
    _fields_ = [("kbar", _i32), ("d", _i32), ("alpha", _f64)]


class ProblemDesc(ctypes.Structure):
    _fields_ = [("n_nodes", _i64), ("xy", _p), ("n_tri", _i64), ("tri", _p), ("dirichlet", _p),
                ("a_rowptr", _p), ("a_col", _p), ("a_val", _p), ("b", _p), ("u0", _p),
                ("n_sub", _i32), ("sub_ptr", _p), ("sub_nodes", _p), ("weights", _p), ("mem_kind", _i32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("krylov", _i32), ("m_max", _i32), ("rtol", _f64), ("max_it", _i32), ("precision", _i32),
                ("prolong", _i32), ("coarse", _i32), ("check_every", _i32), ("profile", _i32),
                ("graph", _i32), ("local_solver", _i32), ("restart", _i32)]


class Tuning(ctypes.Structure):
    _fields_ = [("small_lds", _i32), ("vec_blocks", _i32)]

    def as_dict(self):
        return {"small_lds": self.small_lds, "vec_blocks": self.vec_blocks}


class SimRequest(ctypes.Structure):
    _fields_ = [("arrival", _f64), ("setup_s", _f64), ("bytes", _i64), ("group", ctypes.c_uint64),
                ("chunks", _i32), ("setup_ok", _i32)]


class SimResult(ctypes.Structure):
    _fields_ = [("admitted", _f64), ("finished", _f64), ("status", _i32)]


class Stats(ctypes.Structure):
    _fields_ = [("iterations", _i32), ("converged", _i32), ("rel_residual", _f64),
                ("true_rel_residual", _f64), ("solve_ms", _f64), ("dss_launches", _i32), ("dss_ms", _f64),
                ("coarse_ms", _f64), ("prolong_ms", _f64), ("krylov_ms", _f64), ("dss_kernel", _i32),
                ("status", _i32), ("latency_ms", _f64), ("setup_ms", _f64), ("queue_ms", _f64),
                ("upload_ms", _f64)]


_lib = None


def lib():
    """Load the in-tree libddmgnn.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build()")
    # torch bundles its own HIP runtime, loaded by file name; loading ours first
    # would put two HIP runtimes in the process (the second then finds no
    # device). With torch loaded first, the library binds to torch's runtime.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    L = ctypes.CDLL(_LIB_PATH)
    sig = {
        "ddmgnn_last_error": (ctypes.c_char_p, []),
        "ddmgnn_version": (ctypes.c_char_p, []),
        "ddmgnn_ctx_create": (ctypes.c_int, [_p, ctypes.POINTER(_p)]),
        "ddmgnn_ctx_destroy": (ctypes.c_int, [_p]),
        "ddmgnn_model_create": (ctypes.c_int, [_p, ctypes.POINTER(ModelDesc), _p, _i64, ctypes.POINTER(_p)]),
        "ddmgnn_model_destroy": (ctypes.c_int, [_p]),
        "ddmgnn_validate_problem": (ctypes.c_int, [ctypes.POINTER(ProblemDesc)]),
        "ddmgnn_max_subdomain_nodes": (_i32, []),
        "ddmgnn_problem_create": (ctypes.c_int, [_p, ctypes.POINTER(ProblemDesc), _p, ctypes.POINTER(_p)]),
        "ddmgnn_problem_destroy": (ctypes.c_int, [_p]),
        "ddmgnn_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
        "ddmgnn_solve": (ctypes.c_int, [_p, _p, ctypes.POINTER(SolveOpts), _p, ctypes.POINTER(Stats)]),
        "ddmgnn_solve_batch": (ctypes.c_int, [_p, ctypes.POINTER(_p), _i32, ctypes.POINTER(SolveOpts),
                                              ctypes.POINTER(_p), ctypes.POINTER(Stats)]),
        "ddmgnn_server_create": (ctypes.c_int, [_p, _p, _i64, _i32, _i32, ctypes.POINTER(_p)]),
        "ddmgnn_server_submit": (ctypes.c_int, [_p, ctypes.POINTER(ProblemDesc), ctypes.POINTER(SolveOpts),
                                                ctypes.POINTER(ctypes.c_uint64)]),
        "ddmgnn_server_poll": (ctypes.c_int, [_p, ctypes.c_uint64, _p, ctypes.POINTER(Stats)]),
        "ddmgnn_server_drain": (ctypes.c_int, [_p]),
        "ddmgnn_server_destroy": (ctypes.c_int, [_p]),
        "ddmgnn_problem_device_bytes": (ctypes.c_int, [_p, ctypes.POINTER(_i64)]),
        "ddmgnn_problem_set_tuning": (ctypes.c_int, [_p, ctypes.POINTER(Tuning)]),
        "ddmgnn_server_simulate": (ctypes.c_int, [ctypes.POINTER(SimRequest), _i32, _i64, _i32, _i32, _f64,
                                                  ctypes.POINTER(SimResult)]),
        "ddmgnn_time_apply_stages": (ctypes.c_int, [_p, _p, ctypes.POINTER(SolveOpts), _p, _p, _i32,
                                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                                    ctypes.POINTER(ctypes.c_double)]),
        "ddmgnn_problem_get_tuning": (ctypes.c_int, [_p, ctypes.POINTER(Tuning)]),
        "ddmgnn_autotune": (ctypes.c_int, [_p, _p, ctypes.POINTER(SolveOpts), _i32, ctypes.POINTER(Tuning),
                                           ctypes.POINTER(ctypes.c_double)]),
        "ddmgnn_precond_apply": (ctypes.c_int, [_p, _p, ctypes.POINTER(SolveOpts), _p, _p]),
        "ddmgnn_apply_intermediates": (ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
        "ddmgnn_dss_forward": (ctypes.c_int, [_p, _p, _i32, _p, _p]),
        "ddmgnn_spmv": (ctypes.c_int, [_p, _p, _p, _p]),
        "ddmgnn_dot": (ctypes.c_int, [_p, _i64, _p, _p, ctypes.POINTER(_f64)]),
        "ddmgnn_dot_noalloc": (ctypes.c_int, [_p, _i64, _p, _p, _p]),
        "ddmgnn_expand_overlap": (ctypes.c_int, [_i64, _i64, _p, _p, _i32, _i32, ctypes.POINTER(_p),
                                                 ctypes.POINTER(_p)]),
        "ddmgnn_pou_weights": (ctypes.c_int, [_i64, _p, _i32, _p, _p, _p]),
        "ddmgnn_free": (None, [_p]),
        "ddmgnn_expand_overlap_device": (ctypes.c_int, [_p, _i64, _i64, _p, _p, _p, _i32, _i32, _p, _p, _p, _i64]),
        "ddmgnn_problem_sizes": (ctypes.c_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                                ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
        "ddmgnn_setup_local_graph": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), _i32, _p, _p,
                                                    ctypes.POINTER(_i64)]),
        "ddmgnn_setup_coarse": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), _p, _p]),
        "ddmgnn_setup_local_inverse": (ctypes.c_int, [ctypes.POINTER(ProblemDesc), _i32, _p]),
        "ddmgnn_dss_forward_sub": (ctypes.c_int, [_p, _p, _i32, _i32, _p, _p]),
        "ddmgnn_train_rhs": (ctypes.c_int, [_p, _p, _p, _p]),
        "ddmgnn_train_grad": (ctypes.c_int, [_p, _p, ctypes.POINTER(ModelDesc), _p, ctypes.POINTER(_i32), _i32, _p,
                                             ctypes.POINTER(_i64), _f64, _p, ctypes.POINTER(_f64),
                                             ctypes.POINTER(_f64)]),
        "ddmgnn_adam_step": (ctypes.c_int, [_p, _p, _p, _p, _p, _i64, _f64, _i32, _f64, _f64, _f64, _f64, _f64]),
        "ddmgnn_model_init_xavier": (ctypes.c_int, [ctypes.POINTER(ModelDesc), ctypes.c_uint64, _p, _i64]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _check(rc: int):
    if rc != 0:
        raise DDMGNNError(rc, lib().ddmgnn_last_error().decode())


def _np(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data_as(_p)


def _shape_check(t, dtype_name="float64", n=None, what="tensor"):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_contiguous() or str(t.dtype) != f"torch.{dtype_name}":
        raise TypeError(f"{what}: expected a contiguous {dtype_name} tensor")
    if n is not None and t.numel() != n:
        raise ValueError(f"{what}: expected {n} values, got {t.numel()}")


def _dev(t, dtype_name="float64", n=None, what="tensor"):
    """Pointer of a contiguous torch device tensor of the given dtype holding exactly
    n values (n = None: any length). The C ABI takes bare pointers, so every length the
    library will read or write is checked here, before the device is touched."""
    _shape_check(t, dtype_name, n, what)
    if not t.is_cuda:
        raise TypeError(f"{what}: expected a torch device tensor")
    return _p(t.data_ptr())


def _devs(*specs):
    """_dev over several (tensor, dtype, n, what) at once: every length is checked
    before any device check."""
    for sp in specs:
        _shape_check(*sp)
    return [_dev(*sp) for sp in specs]


def _disjoint(a, b, what: str):
    """Raises when two tensors share memory (the ABI requires distinct buffers)."""
    a0, b0 = a.data_ptr(), b.data_ptr()
    if a0 < b0 + b.numel() * b.element_size() and b0 < a0 + a.numel() * a.element_size():
        raise ValueError(f"{what} must not alias")


def n_theta(kbar: int, d: int) -> int:
    """Weights of DSS_theta with kbar blocks of latent width d (Table II: kbar (11 d^2 + 15 d + 1))."""
    return kbar * (11 * d * d + 15 * d + 1)


# ------------------------------------------------------------------ host-only helpers
def expand_overlap(n: int, tri, part, n_part: int, delta: int):
    """Overlapping sub-meshes (library implementation); returns (sub_ptr int64, sub_nodes int32)."""
    tri, tp = _np(tri, np.int32)
    part, pp = _np(part, np.int32)
    sp, sn = _p(), _p()
    _check(lib().ddmgnn_expand_overlap(n, tri.size // 3, tp, pp, n_part, delta, ctypes.byref(sp), ctypes.byref(sn)))
    try:
        ptr = np.ctypeslib.as_array(ctypes.cast(sp, ctypes.POINTER(_i64)), (n_part + 1,)).copy()
        nodes = np.ctypeslib.as_array(ctypes.cast(sn, ctypes.POINTER(_i32)), (int(ptr[-1]),)).copy()
    finally:
        lib().ddmgnn_free(sp)
        lib().ddmgnn_free(sn)
    return ptr, nodes


def pou_weights(n: int, dirichlet, sub_ptr, sub_nodes):
    dirichlet, dp = _np(dirichlet, np.uint8)
    sub_ptr, spp = _np(sub_ptr, np.int64)
    sub_nodes, snp = _np(sub_nodes, np.int32)
    w = np.empty(sub_nodes.size, np.float64)
    _check(lib().ddmgnn_pou_weights(n, dp, sub_ptr.size - 1, spp, snp, w.ctypes.data_as(_p)))
    return w


@dataclass
class HostProblem:
    """Host arrays of one problem in the layout of ddmgnn_problem_desc."""
    xy: np.ndarray
    tri: np.ndarray
    dirichlet: np.ndarray
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    b: np.ndarray
    u0: np.ndarray
    sub_ptr: np.ndarray
    sub_nodes: np.ndarray
    weights: np.ndarray

    def __post_init__(self):
        self.xy = np.ascontiguousarray(self.xy, np.float64)
        self.tri = np.ascontiguousarray(self.tri, np.int32)
        self.dirichlet = np.ascontiguousarray(self.dirichlet, np.uint8)
        self.rowptr = np.ascontiguousarray(self.rowptr, np.int32)
        self.col = np.ascontiguousarray(self.col, np.int32)
        self.val = np.ascontiguousarray(self.val, np.float64)
        self.b = np.ascontiguousarray(self.b, np.float64)
        self.u0 = np.ascontiguousarray(self.u0, np.float64)
        self.sub_ptr = np.ascontiguousarray(self.sub_ptr, np.int64)
        self.sub_nodes = np.ascontiguousarray(self.sub_nodes, np.int32)
        self.weights = np.ascontiguousarray(self.weights, np.float64)
        n = self.xy.shape[0] if self.xy.ndim == 2 else -1
        K = self.sub_ptr.size - 1
        checks = [
            (self.xy.ndim == 2 and self.xy.shape[1] == 2, "xy must be (N, 2)"),
            (self.tri.size % 3 == 0 and self.tri.size > 0, "tri must hold 3 node ids per triangle"),
            (self.dirichlet.size == n and self.b.size == n and self.u0.size == n,
             "dirichlet, b and u0 must hold N values"),
            (self.rowptr.size == n + 1, "a_rowptr must hold N + 1 values"),
            (self.rowptr.size == n + 1 and self.col.size == self.val.size == int(self.rowptr[-1]),
             "a_col and a_val must hold a_rowptr[N] values"),
            (K >= 1 and self.sub_nodes.size == self.weights.size == int(self.sub_ptr[-1]),
             "sub_nodes and weights must hold sub_ptr[K] values"),
        ]
        for ok, msg in checks:
            if not ok:
                raise ValueError(msg)

    @property
    def n(self) -> int:
        return self.xy.shape[0]

    @property
    def K(self) -> int:
        return self.sub_ptr.size - 1

    def desc(self) -> ProblemDesc:
        P = lambda a: a.ctypes.data_as(_p)
        return ProblemDesc(self.n, P(self.xy), self.tri.size // 3, P(self.tri), P(self.dirichlet),
                           P(self.rowptr), P(self.col), P(self.val), P(self.b), P(self.u0), self.K,
                           P(self.sub_ptr), P(self.sub_nodes), P(self.weights))


def host_problem(xy, tri, dirichlet, rowptr, col, val, b, u0, part, n_part, delta=2) -> HostProblem:
    """Problem arrays with the library's overlap expansion and partition-of-unity weights."""
    n = np.asarray(xy).shape[0]
    sub_ptr, sub_nodes = expand_overlap(n, tri, part, n_part, delta)
    w = pou_weights(n, dirichlet, sub_ptr, sub_nodes)
    return HostProblem(xy, tri, dirichlet, rowptr, col, val, b, u0, sub_ptr, sub_nodes, w)


def validate(hp: HostProblem):
    d = hp.desc()
    _check(lib().ddmgnn_validate_problem(ctypes.byref(d)))


def setup_local_graph(hp: HostProblem, sub: int):
    d = hp.desc()
    ne = _i64()
    _check(lib().ddmgnn_setup_local_graph(ctypes.byref(d), sub, None, None, ctypes.byref(ne)))
    k = int(hp.sub_ptr[sub + 1] - hp.sub_ptr[sub])
    rowptr = np.empty(k + 1, np.int32)
    col = np.empty(max(1, ne.value), np.int32)
    _check(lib().ddmgnn_setup_local_graph(ctypes.byref(d), sub, rowptr.ctypes.data_as(_p),
                                          col.ctypes.data_as(_p), ctypes.byref(ne)))
    return rowptr, col[:ne.value]


def setup_coarse(hp: HostProblem):
    d = hp.desc()
    a0 = np.empty((hp.K, hp.K))
    a0inv = np.empty((hp.K, hp.K))
    _check(lib().ddmgnn_setup_coarse(ctypes.byref(d), a0.ctypes.data_as(_p), a0inv.ctypes.data_as(_p)))
    return a0, a0inv


def setup_local_inverse(hp: HostProblem, sub: int):
    """(R_i A R_i^T)^{-1} of sub-mesh `sub` as the library's exact local solver forms it."""
    d = hp.desc()
    k = int(hp.sub_ptr[sub + 1] - hp.sub_ptr[sub]) if 0 <= sub < hp.K else 0
    inv = np.empty((k, k))
    _check(lib().ddmgnn_setup_local_inverse(ctypes.byref(d), sub, inv.ctypes.data_as(_p)))
    return inv


def init_xavier(seed: int, kbar: int = 30, d: int = 10, alpha: float = 1e-3) -> np.ndarray:
    """Seeded Xavier-uniform weights from the library (host only)."""
    desc = ModelDesc(kbar, d, alpha)
    n = kbar * (11 * d * d + 15 * d + 1)
    th = np.empty(n, dtype=np.float32)
    _check(lib().ddmgnn_model_init_xavier(ctypes.byref(desc), seed, th.ctypes.data_as(_p), n))
    return th


def simulate_server(requests, hbm_budget: int, max_active: int, setup_threads: int = 4, chunk_s: float = 0.01):
    """Host-only model of the serving loop: requests are dicts with arrival, setup_s, bytes,
    group, chunks and setup_ok (default 1); returns a list of (admitted, finished, status)."""
    n = len(requests)
    reqs = (SimRequest * max(n, 1))()
    for i, r in enumerate(requests):
        reqs[i] = SimRequest(r["arrival"], r["setup_s"], r["bytes"], r.get("group", 0), r["chunks"],
                             r.get("setup_ok", 1))
    out = (SimResult * max(n, 1))()
    _check(lib().ddmgnn_server_simulate(reqs, n, hbm_budget, max_active, setup_threads, chunk_s, out))
    return [(out[i].admitted, out[i].finished, out[i].status) for i in range(n)]


def default_opts(**kw) -> SolveOpts:
    o = SolveOpts()
    lib().ddmgnn_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision" and isinstance(v, str):
            v = PRECISION[v]
        setattr(o, k, v)
    return o


# ------------------------------------------------------------------ device objects
class Context:
    """A library context bound to the current device and a torch stream."""

    def __init__(self, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device available")
        s = stream if stream is not None else torch.cuda.current_stream()
        self.stream = s
        h = _p()
        _check(lib().ddmgnn_ctx_create(_p(s.cuda_stream), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ddmgnn_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def dot(self, x, y) -> float:
        out = _f64()
        xp, yp = _devs((x, "float64", None, "x"), (y, "float64", x.numel(), "y"))
        _check(lib().ddmgnn_dot(self.h, x.numel(), xp, yp, ctypes.byref(out)))
        return out.value

    def expand_overlap_device(self, n: int, tri, part, dirichlet, n_part: int, delta: int):
        """Overlapping sub-meshes and partition-of-unity weights computed on the device:
        (sub_ptr int64 numpy, sub_nodes int32 device tensor, weights float64 device tensor)."""
        import torch
        tri_d, part_d, dir_d = _devs((tri, "int32", None, "tri"), (part, "int32", n, "part"),
                                     (dirichlet, "uint8", n, "dirichlet"))
        if tri.numel() % 3:
            raise ValueError("tri: expected 3 node ids per triangle")
        sp = np.empty(n_part + 1, np.int64)
        L = lib()
        args = (self.h, n, tri.numel() // 3, tri_d, part_d, dir_d, n_part, delta,
                sp.ctypes.data_as(ctypes.POINTER(_i64)))
        rc = L.ddmgnn_expand_overlap_device(*args, None, None, 0)
        if rc != 0 and not (sp[n_part] > 0 and b"capacity" in L.ddmgnn_last_error()):
            _check(rc)
        dev = tri.device
        nodes = torch.empty(int(sp[n_part]), dtype=torch.int32, device=dev)
        weights = torch.empty(int(sp[n_part]), dtype=torch.float64, device=dev)
        _check(L.ddmgnn_expand_overlap_device(*args, _p(nodes.data_ptr()), _p(weights.data_ptr()), nodes.numel()))
        return sp, nodes, weights

    def dot_noalloc(self, x, y, out):
        """x . y into the one-double device tensor out, asynchronously on the
        context's stream, with no device allocation (ddmgnn_dot_noalloc)."""
        xp, yp, op = _devs((x, "float64", None, "x"), (y, "float64", x.numel(), "y"), (out, "float64", 1, "out"))
        _check(lib().ddmgnn_dot_noalloc(self.h, x.numel(), xp, yp, op))


class Model:
    def __init__(self, ctx: Context, theta, kbar: int = 30, d: int = 10, alpha: float = 1e-3):
        th, tp = _np(theta, np.float32)
        self._theta = th
        desc = ModelDesc(kbar, d, alpha)
        h = _p()
        _check(lib().ddmgnn_model_create(ctx.h, ctypes.byref(desc), tp, th.size, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            lib().ddmgnn_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Problem:
    def __init__(self, ctx: Context, hp: HostProblem, model: Model, desc: ProblemDesc | None = None):
        """desc: a descriptor to use instead of hp's host arrays (e.g. device pointers
        with mem_kind = MEM_DEVICE); hp still describes the problem's sizes."""
        self.ctx = ctx
        self.hp = hp
        d = desc if desc is not None else hp.desc()
        h = _p()
        _check(lib().ddmgnn_problem_create(ctx.h, ctypes.byref(d), model.h, ctypes.byref(h)))
        self.h = h
        n, nnz, e = _i64(), _i64(), _i64()
        k, sk = _i32(), _i64()
        _check(lib().ddmgnn_problem_sizes(h, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(k), ctypes.byref(sk),
                                          ctypes.byref(e)))
        self.n, self.nnz, self.K, self.sum_k, self.n_edges = n.value, nnz.value, k.value, sk.value, e.value

    def close(self):
        if getattr(self, "h", None):
            lib().ddmgnn_problem_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def solve(self, u_out, opts: SolveOpts | None = None, check=True) -> Stats:
        o = opts or default_opts()
        st = Stats()
        rc = lib().ddmgnn_solve(self.ctx.h, self.h, ctypes.byref(o), _dev(u_out, n=self.n, what="u_out"),
                                ctypes.byref(st))
        if check:
            _check(rc)
        return st

    def time_apply_stages(self, r, z, opts: SolveOpts | None = None, reps: int = 10):
        """(local, coarse, glue) milliseconds of one apply, each stage replayed as a HIP graph."""
        o = opts or default_opts()
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rp, zp = _devs((r, "float64", self.n, "r"), (z, "float64", self.n, "z"))
        _disjoint(r, z, "r and z")
        _check(lib().ddmgnn_time_apply_stages(self.ctx.h, self.h, ctypes.byref(o), rp, zp, reps,
                                              ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def set_tuning(self, small_lds: int = 0, vec_blocks: int = 0):
        t = Tuning(small_lds, vec_blocks)
        _check(lib().ddmgnn_problem_set_tuning(self.h, ctypes.byref(t)))

    def tuning(self) -> Tuning:
        t = Tuning()
        _check(lib().ddmgnn_problem_get_tuning(self.h, ctypes.byref(t)))
        return t

    def autotune(self, opts: SolveOpts | None = None, iterations: int = 16):
        """Runs the library's autotuner; returns (Tuning, ms per iteration)."""
        o = opts or default_opts()
        t = Tuning()
        ms = ctypes.c_double()
        _check(lib().ddmgnn_autotune(self.ctx.h, self.h, ctypes.byref(o), iterations, ctypes.byref(t),
                                     ctypes.byref(ms)))
        return t, ms.value

    def device_bytes(self) -> int:
        b = _i64()
        _check(lib().ddmgnn_problem_device_bytes(self.h, ctypes.byref(b)))
        return b.value

    def apply(self, r, z, opts: SolveOpts | None = None):
        o = opts or default_opts()
        rp, zp = _devs((r, "float64", self.n, "r"), (z, "float64", self.n, "z"))
        _disjoint(r, z, "r and z")
        _check(lib().ddmgnn_precond_apply(self.ctx.h, self.h, ctypes.byref(o), rp, zp))

    def intermediates(self):
        import torch
        dev = self.ctx.stream.device
        s = torch.empty(self.K, dtype=torch.float64, device=dev)
        y0 = torch.empty_like(s)
        y = torch.empty_like(s)
        loc = torch.empty(self.sum_k, dtype=torch.float64, device=dev)
        _check(lib().ddmgnn_apply_intermediates(self.ctx.h, self.h, _dev(s), _dev(y0), _dev(y), _dev(loc)))
        return s, y0, y, loc

    def dss_forward(self, c, out, precision=FP32):
        if isinstance(precision, str):
            precision = PRECISION[precision]
        cp, op = _devs((c, "float64", self.sum_k, "c"), (out, "float64", self.sum_k, "out"))
        _check(lib().ddmgnn_dss_forward(self.ctx.h, self.h, precision, cp, op))

    def dss_forward_sub(self, sub: int, c, out, precision=FP32):
        """DSS forward of sub-mesh `sub` alone (c, out: its k_sub values)."""
        if isinstance(precision, str):
            precision = PRECISION[precision]
        if not 0 <= sub < self.K:
            raise ValueError(f"sub-mesh {sub} out of range [0, {self.K})")
        k = int(self.hp.sub_ptr[sub + 1] - self.hp.sub_ptr[sub])
        cp, op = _devs((c, "float64", k, "c"), (out, "float64", k, "out"))
        _check(lib().ddmgnn_dss_forward_sub(self.ctx.h, self.h, precision, sub, cp, op))

    def spmv(self, x, y):
        xp, yp = _devs((x, "float64", self.n, "x"), (y, "float64", self.n, "y"))
        _disjoint(x, y, "x and y")
        _check(lib().ddmgnn_spmv(self.ctx.h, self.h, xp, yp))

    # ---- training of DSS_theta
    def train_rhs(self, u, c_out):
        """c_out (device float32, sum_k values) = R_i r / |R_i r| per sub-mesh, r = b - A u."""
        up, cp = _devs((u, "float64", self.n, "u"), (c_out, "float32", self.sum_k, "c_out"))
        _check(lib().ddmgnn_train_rhs(self.ctx.h, self.h, up, cp))

    def train_grad(self, theta, subs, c, c_off, grad, kbar: int = 30, d: int = 10, alpha: float = 1e-3,
                   scale: float | None = None):
        """Loss and gradient of the training objective over samples (subs[s], c[c_off[s]:]).
        scale defaults to 1 / (total nodes). Returns (loss, |grad|)."""
        subs = np.ascontiguousarray(subs, np.int32)
        offs = np.ascontiguousarray(c_off, np.int64)
        if subs.shape != offs.shape:
            raise ValueError("subs and c_off differ in length")
        ptr = self.hp.sub_ptr
        if subs.size and (subs.min() < 0 or subs.max() >= self.K):
            raise ValueError(f"sub-mesh index out of range [0, {self.K})")
        ks = (ptr[subs + 1] - ptr[subs]) if subs.size else np.zeros(0, np.int64)
        if offs.size and (offs.min() < 0 or int((offs + ks).max()) > c.numel()):
            raise ValueError("a sample's right-hand side c[c_off : c_off + k_i] lies outside c")
        if scale is None:
            nodes = int(ks.sum())
            scale = 1.0 / nodes if nodes else 1.0
        nt = n_theta(kbar, d)
        desc = ModelDesc(kbar, d, alpha)
        loss, gn = _f64(), _f64()
        tp, cp, gp = _devs((theta, "float32", nt, "theta"), (c, "float32", None, "c"),
                           (grad, "float32", nt, "grad"))
        _check(lib().ddmgnn_train_grad(self.ctx.h, self.h, ctypes.byref(desc), tp,
                                       subs.ctypes.data_as(ctypes.POINTER(_i32)), subs.size, cp,
                                       offs.ctypes.data_as(ctypes.POINTER(_i64)), scale, gp,
                                       ctypes.byref(loss), ctypes.byref(gn)))
        return loss.value, gn.value


def adam_step(ctx: Context, theta, grad, m, v, gnorm: float, t: int, lr: float = 1e-2, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8, clip: float = 1e-2):
    """One Adam step on device float32 tensors (gradient clipped to norm `clip`)."""
    n = theta.numel()
    ptrs = _devs((theta, "float32", None, "theta"), (grad, "float32", n, "grad"), (m, "float32", n, "m"),
                 (v, "float32", n, "v"))
    _check(lib().ddmgnn_adam_step(ctx.h, *ptrs, n, gnorm, t, lr, beta1, beta2, eps, clip))


def solve_batch(ctx: Context, problems, u_outs, opts: SolveOpts | None = None, check=True):
    """Solve several problems of one context and model together; returns one Stats per problem."""
    o = opts or default_opts()
    n = len(problems)
    hs = (_p * n)(*[p.h for p in problems])
    if len(u_outs) != n:
        raise ValueError("one output vector per problem")
    outs = (_p * n)(*_devs(*[(u, "float64", p.n, f"u_outs[{i}]") for i, (p, u) in enumerate(zip(problems, u_outs))]))
    st = (Stats * n)()
    rc = lib().ddmgnn_solve_batch(ctx.h, hs, n, ctypes.byref(o), outs, st)
    if check:
        _check(rc)
    return list(st)


class Server:
    """Serving loop with continuous batching (owns the context while it runs)."""

    def __init__(self, ctx: Context, model: Model, hbm_budget: int, max_active: int = 64, setup_threads: int = 0):
        self.ctx = ctx
        self.model = model
        self._n = {}
        h = _p()
        _check(lib().ddmgnn_server_create(ctx.h, model.h, int(hbm_budget), max_active, setup_threads,
                                          ctypes.byref(h)))
        self.h = h

    def submit(self, hp: HostProblem, opts: SolveOpts | None = None) -> int:
        o = opts or default_opts()
        d = hp.desc()
        t = ctypes.c_uint64()
        _check(lib().ddmgnn_server_submit(self.h, ctypes.byref(d), ctypes.byref(o), ctypes.byref(t)))
        self._n[t.value] = hp.n
        return t.value

    def poll(self, ticket: int, with_solution: bool = True):
        """None while pending, else (status, Stats, u or None); a finished request is returned once."""
        if ticket not in self._n:
            raise KeyError(f"unknown or already collected ticket {ticket}")
        u = np.empty(self._n[ticket], np.float64) if with_solution else None
        st = Stats()
        rc = lib().ddmgnn_server_poll(self.h, ticket, u.ctypes.data_as(_p) if u is not None else None,
                                      ctypes.byref(st))
        if rc == -9:
            return None
        del self._n[ticket]
        return rc, st, u

    def drain(self):
        _check(lib().ddmgnn_server_drain(self.h))

    def close(self):
        if getattr(self, "h", None):
            lib().ddmgnn_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
