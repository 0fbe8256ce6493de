"""Thin ctypes binding of librcr.so (include/rcr.h): argument marshalling only.

Every step of the solve runs in the library's HIP kernels; this module only
checks shapes, passes device pointers and the stream, and turns status codes
into exceptions.  There is no CPU fallback: if the library is missing the
import of `lib()` raises.
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# the in-tree build; RCR_LIB names another build of the same library
LIB_PATH = os.environ.get("RCR_LIB") or os.path.join(HERE, "librcr.so")

ERR_INVALID_TREE, ERR_BAD_DIMS, ERR_NULL_ARG, ERR_NOT_PD, ERR_SINGULAR, ERR_NONFINITE = -1, -2, -3, -4, -5, -6
ERR_OOM, ERR_HIP_ERROR, ERR_BAD_OPTION, ERR_SMALL_WORKSPACE, ERR_NO_DEVICE = -7, -8, -9, -10, -11
FP64, MIXED32 = 0, 1
EXEC_LEVELS, EXEC_GRAPH = 0, 1
SELECT_GREEDY_INDEX, SELECT_LIST_RANK = 0, 1
KERNEL_CLASSES = ("condense", "quad_contract", "quad_expand", "local_factor", "tcompose", "rhs_init",
                  "aff_contract", "aff_expand", "local_affine", "state_contract", "state_expand",
                  "recover", "residual", "quad_tail", "aff_tail", "state_tail")
NUM_KERNEL_CLASSES = len(KERNEL_CLASSES)

_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)


class PlanOptions(ctypes.Structure):
    _fields_ = [("selection", ctypes.c_int32), ("single_thread", ctypes.c_int32), ("reserved", ctypes.c_int32 * 6)]


class PlanStats(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("n", ctypes.c_int32), ("m", ctypes.c_int32), ("root", ctypes.c_int64),
                ("height", ctypes.c_int64), ("leaves", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("rounds", ctypes.c_int64), ("levels", ctypes.c_int64), ("expand_levels", ctypes.c_int64),
                ("state_levels", ctypes.c_int64), ("sexp_levels", ctypes.c_int64),
                ("n_rake", ctypes.c_int64), ("n_compress", ctypes.c_int64), ("n_combine", ctypes.c_int64),
                ("n_absorb", ctypes.c_int64), ("depth_bound", ctypes.c_int64), ("crew_ok", ctypes.c_int64),
                ("workspace_bytes_fp64", ctypes.c_int64), ("workspace_bytes_mixed", ctypes.c_int64),
                ("n_trees", ctypes.c_int64), ("plan_device_bytes", ctypes.c_int64),
                ("graph_cache_entries", ctypes.c_int64)]

GRAPH_CACHE_CAP = 8


class Problem(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")]


class Solution(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("K", "P", "x", "u", "lam")]


class Rhs(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("q", "r", "c")]


class RhsSolution(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "u", "lam")]


class Gradient(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")]


class NativeProblem(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("Q", "q", "c", "Delta", "M", "R", "r", "A", "B")]


class NativeSolution(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("x", "v", "lam")]


LAUNCH_FIELDS = ("quad_tail_rounds", "vec_tail_rounds", "vec_tail_waves")


class LaunchConfig(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int32) for k in LAUNCH_FIELDS] + [("reserved", ctypes.c_int32 * 5)]


class SolveOptions(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("refine_steps", ctypes.c_int32), ("executor", ctypes.c_int32),
                ("check", ctypes.c_int32), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_int64),
                ("kkt_residual", ctypes.POINTER(ctypes.c_double)), ("kernel_ms", ctypes.POINTER(ctypes.c_float)),
                ("kernel_launches", ctypes.POINTER(ctypes.c_int32)), ("reserved", ctypes.c_int32 * 4)]


EXPORTED = ("rcr_plan_create", "rcr_plan_create_device", "rcr_plan_digest", "rcr_plan_info", "rcr_plan_device_bytes", "rcr_plan_export", "rcr_plan_destroy", "rcr_batch_plan_create",
            "rcr_plan_upload", "rcr_lift_plan_create", "rcr_lift_solve", "rcr_plan_set_launch",
            "rcr_plan_get_launch", "rcr_plan_tune",
            "rcr_workspace_size", "rcr_solve", "rcr_factor", "rcr_solve_rhs", "rcr_adjoint", "rcr_kkt_residual",
            "rcr_batch_solve", "rcr_batch_prepare", "rcr_batch_release", "rcr_batch_workspace_size",
            "rcr_solve_noalloc", "rcr_noalloc_scratch_bytes", "rcr_ragged_plan_create", "rcr_ragged_offsets",
            "rcr_ragged_solve", "rcr_status_string")

_lib = None
_lock = threading.Lock()


class RcrError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)})")


def lib():
    """Load librcr.so (fails loudly when it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() first")
            L = ctypes.CDLL(LIB_PATH)
            L.rcr_plan_create.restype = ctypes.c_int
            L.rcr_plan_create.argtypes = [_i64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(PlanOptions), ctypes.POINTER(ctypes.c_void_p)]
            L.rcr_plan_create_device.restype = ctypes.c_int
            L.rcr_plan_create_device.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                 ctypes.POINTER(PlanOptions), ctypes.c_void_p,
                                                 ctypes.POINTER(ctypes.c_void_p)]
            L.rcr_plan_digest.restype = ctypes.c_int
            L.rcr_plan_digest.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
            L.rcr_plan_info.restype = ctypes.c_int
            L.rcr_plan_info.argtypes = [ctypes.c_void_p, ctypes.POINTER(PlanStats)]
            L.rcr_plan_device_bytes.restype = ctypes.c_int64
            L.rcr_plan_device_bytes.argtypes = [ctypes.c_void_p]
            L.rcr_plan_export.restype = ctypes.c_int
            L.rcr_plan_export.argtypes = [ctypes.c_void_p, _i32p, ctypes.c_int64, _i64p]
            L.rcr_plan_destroy.restype = None
            L.rcr_plan_destroy.argtypes = [ctypes.c_void_p]
            L.rcr_batch_plan_create.restype = ctypes.c_int
            L.rcr_batch_plan_create.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_void_p)]
            L.rcr_lift_plan_create.restype = ctypes.c_int
            L.rcr_lift_plan_create.argtypes = [_i64p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                               ctypes.POINTER(PlanOptions), ctypes.POINTER(ctypes.c_void_p)]
            L.rcr_lift_solve.restype = ctypes.c_int
            L.rcr_lift_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(NativeProblem),
                                         ctypes.POINTER(NativeSolution), ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_plan_set_launch.restype = ctypes.c_int
            L.rcr_plan_set_launch.argtypes = [ctypes.c_void_p, ctypes.POINTER(LaunchConfig)]
            L.rcr_plan_get_launch.restype = ctypes.c_int
            L.rcr_plan_get_launch.argtypes = [ctypes.c_void_p, ctypes.POINTER(LaunchConfig)]
            L.rcr_plan_tune.restype = ctypes.c_int
            L.rcr_plan_tune.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                        ctypes.POINTER(SolveOptions), ctypes.c_void_p, ctypes.POINTER(LaunchConfig),
                                        ctypes.POINTER(ctypes.c_float)]
            L.rcr_plan_upload.restype = ctypes.c_int
            L.rcr_plan_upload.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            L.rcr_workspace_size.restype = ctypes.c_int64
            L.rcr_workspace_size.argtypes = [ctypes.c_void_p, ctypes.c_int32]
            L.rcr_solve.restype = ctypes.c_int
            L.rcr_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                    ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_factor.restype = ctypes.c_int
            L.rcr_factor.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                     ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_solve_rhs.restype = ctypes.c_int
            L.rcr_solve_rhs.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                        ctypes.c_int32, ctypes.POINTER(Rhs), ctypes.POINTER(RhsSolution),
                                        ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_adjoint.restype = ctypes.c_int
            L.rcr_adjoint.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                      ctypes.POINTER(Rhs), ctypes.POINTER(Gradient), ctypes.POINTER(SolveOptions),
                                      ctypes.c_void_p]
            L.rcr_kkt_residual.restype = ctypes.c_int
            L.rcr_kkt_residual.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                           ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_batch_solve.restype = ctypes.c_int
            L.rcr_batch_solve.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(Problem),
                                          ctypes.POINTER(Solution), ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_batch_prepare.restype = ctypes.c_int
            L.rcr_batch_prepare.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_void_p]
            L.rcr_batch_release.restype = None
            L.rcr_batch_release.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32]
            L.rcr_batch_workspace_size.restype = ctypes.c_int64
            L.rcr_batch_workspace_size.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.c_int32]
            L.rcr_solve_noalloc.restype = ctypes.c_int
            L.rcr_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                            ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_noalloc_scratch_bytes.restype = ctypes.c_int64
            L.rcr_noalloc_scratch_bytes.argtypes = []
            L.rcr_ragged_plan_create.restype = ctypes.c_int
            L.rcr_ragged_plan_create.argtypes = [_i64p, ctypes.c_int64, _i32p, _i32p, ctypes.POINTER(PlanOptions),
                                                 ctypes.POINTER(ctypes.c_void_p)]
            L.rcr_ragged_offsets.restype = ctypes.c_int
            L.rcr_ragged_offsets.argtypes = [ctypes.c_void_p, _i64p]
            L.rcr_ragged_solve.restype = ctypes.c_int
            L.rcr_ragged_solve.argtypes = [ctypes.c_void_p, ctypes.POINTER(Problem), ctypes.POINTER(Solution),
                                           ctypes.POINTER(SolveOptions), ctypes.c_void_p]
            L.rcr_status_string.restype = ctypes.c_char_p
            L.rcr_status_string.argtypes = [ctypes.c_int]
            _lib = L
    return _lib


def status_string(s: int) -> str:
    return lib().rcr_status_string(int(s)).decode()


class Plan:
    """Reusable topology plan (rcr_plan_create).  Host-only; no GPU needed."""

    @classmethod
    def batch(cls, plans) -> "Plan":
        """Batched plan of independent trees (rcr_batch_plan_create); tree t owns the
        nodes [offsets[t], offsets[t + 1]) of the concatenated problem."""
        L = lib()
        k = len(plans)
        arr = (ctypes.c_void_p * k)(*[p._h.value for p in plans])
        h = ctypes.c_void_p()
        rc = L.rcr_batch_plan_create(arr, k, ctypes.byref(h))
        if rc != 0:
            raise RcrError(rc, "rcr_batch_plan_create")
        self = cls.__new__(cls)
        self._h = h
        self.N = int(sum(p.N for p in plans))
        self.n, self.m = plans[0].n, plans[0].m
        self.offsets = np.cumsum([0] + [p.N for p in plans]).astype(np.int64)
        self._parent = np.concatenate([np.where(p._parent >= 0, p._parent + o, -1)
                                       for p, o in zip(plans, self.offsets[:-1])])
        return self

    @classmethod
    def lift(cls, parent, n: int, m: int, selection: int = SELECT_GREEDY_INDEX, single_thread: bool = False) -> "Plan":
        """Plan of the lifted tree of a node-control problem (rcr_lift_plan_create)
        on the native parent array, state n and control m; solve it with lift_solve."""
        L = lib()
        self = cls.__new__(cls)
        self._parent = np.ascontiguousarray(parent, dtype=np.int64)
        h = ctypes.c_void_p()
        opt = PlanOptions(selection=selection, single_thread=int(bool(single_thread)))
        rc = L.rcr_lift_plan_create(self._parent.ctypes.data_as(_i64p), int(self._parent.shape[0]), int(n), int(m),
                                    ctypes.byref(opt), ctypes.byref(h))
        if rc != 0:
            raise RcrError(rc, "rcr_lift_plan_create")
        self._h = h
        st = self.stats()
        self.N, self.n, self.m = st["N"], st["n"], st["m"]
        self.native_N, self.native_n = int(self._parent.shape[0]), int(n)
        return self

    @classmethod
    def ragged(cls, parent, n_node, m_edge, selection: int = SELECT_GREEDY_INDEX,
               single_thread: bool = False) -> "Plan":
        """Plan of a tree with per-node state and per-edge control dimensions
        (rcr_ragged_plan_create); solve it with ragged_solve on packed arrays."""
        L = lib()
        self = cls.__new__(cls)
        self._parent = np.ascontiguousarray(parent, dtype=np.int64)
        nn = np.ascontiguousarray(n_node, dtype=np.int32)
        mm = np.ascontiguousarray(m_edge, dtype=np.int32)
        self.N = int(self._parent.shape[0])
        if nn.shape != (self.N,) or mm.shape != (self.N,):
            raise ValueError("n_node and m_edge need one entry per node")
        h = ctypes.c_void_p()
        opt = PlanOptions(selection=selection, single_thread=int(bool(single_thread)))
        rc = L.rcr_ragged_plan_create(self._parent.ctypes.data_as(_i64p), self.N, nn.ctypes.data_as(_i32p),
                                      mm.ctypes.data_as(_i32p), ctypes.byref(opt), ctypes.byref(h))
        if rc != 0:
            raise RcrError(rc, "rcr_ragged_plan_create")
        self._h = h
        st = self.stats()
        self.n, self.m = st["n"], st["m"]
        off = np.zeros(RAGGED_FIELDS_COUNT * (self.N + 1), dtype=np.int64)
        rc = L.rcr_ragged_offsets(self._h, off.ctypes.data_as(_i64p))
        if rc != 0:
            raise RcrError(rc, "rcr_ragged_offsets")
        self.ragged_offsets = {f: off[i * (self.N + 1):(i + 1) * (self.N + 1)] for i, f in enumerate(RAGGED_FIELDS)}
        return self

    def __init__(self, parent, n: int, m: int, selection: int = SELECT_GREEDY_INDEX, single_thread: bool = False):
        L = lib()
        self._parent = np.ascontiguousarray(parent, dtype=np.int64)
        self.N = int(self._parent.shape[0])
        self.n, self.m = int(n), int(m)
        h = ctypes.c_void_p()
        opt = PlanOptions(selection=selection, single_thread=int(bool(single_thread)))
        rc = L.rcr_plan_create(self._parent.ctypes.data_as(_i64p), self.N, self.n, self.m, ctypes.byref(opt),
                               ctypes.byref(h))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_create")
        self._h = h

    @classmethod
    def from_device(cls, parent, n: int, m: int, stream=None) -> "Plan":
        """rcr_plan_create_device: the plan built on the GPU from a device int64
        parent tensor (list-rank selection; identical to
        Plan(parent, n, m, selection=SELECT_LIST_RANK))."""
        import torch
        if not isinstance(parent, torch.Tensor) or not parent.is_cuda or parent.dtype != torch.int64 \
                or not parent.is_contiguous() or parent.dim() != 1:
            raise TypeError("parent must be a contiguous 1-D int64 CUDA tensor")
        L = lib()
        self = cls.__new__(cls)
        self.N = int(parent.shape[0])
        self.n, self.m = int(n), int(m)
        st = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        opt = PlanOptions(selection=SELECT_LIST_RANK)
        rc = L.rcr_plan_create_device(ctypes.c_void_p(parent.data_ptr()), self.N, self.n, self.m, ctypes.byref(opt),
                                      ctypes.c_void_p(st.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_create_device")
        self._h = h
        return self

    def digest(self) -> int:
        """rcr_plan_digest: a hash of every array and statistic of the plan."""
        d = ctypes.c_uint64()
        rc = lib().rcr_plan_digest(self._h, ctypes.byref(d))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_digest")
        return int(d.value)

    def stats(self) -> dict:
        s = PlanStats()
        rc = lib().rcr_plan_info(self._h, ctypes.byref(s))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_info")
        return {k: int(getattr(s, k)) for k, _ in PlanStats._fields_}

    def device_bytes(self) -> int:
        """rcr_plan_device_bytes: bytes of the plan's device copy (cheap; no CREW check)."""
        return int(lib().rcr_plan_device_bytes(self._h))

    def export_ops(self) -> np.ndarray:
        cnt = ctypes.c_int64()
        L = lib()
        rc = L.rcr_plan_export(self._h, None, 0, ctypes.byref(cnt))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_export")
        ops = np.zeros((cnt.value, 8), dtype=np.int32)
        rc = L.rcr_plan_export(self._h, ops.ctypes.data_as(_i32p), cnt.value, ctypes.byref(cnt))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_export")
        return ops

    def upload(self, stream=None):
        """rcr_plan_upload: make the device copy now, in the order of `stream`."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream()
        rc = lib().rcr_plan_upload(self._h, ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_upload")

    def set_launch(self, cfg: dict | None = None):
        """rcr_plan_set_launch (None: defaults).  Keys: LAUNCH_FIELDS."""
        c = None
        if cfg is not None:
            c = LaunchConfig(**{k: int(v) for k, v in cfg.items()})
        rc = lib().rcr_plan_set_launch(self._h, ctypes.byref(c) if c is not None else None)
        if rc != 0:
            raise RcrError(rc, "rcr_plan_set_launch")

    def get_launch(self) -> dict:
        c = LaunchConfig()
        rc = lib().rcr_plan_get_launch(self._h, ctypes.byref(c))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_get_launch")
        return {k: int(getattr(c, k)) for k in LAUNCH_FIELDS}

    def tune(self, prob: dict, out: dict | None = None, precision: int = FP64, refine_steps: int = -1,
             stream=None) -> tuple[dict, float]:
        """rcr_plan_tune: time the candidate launch mappings on this problem and keep
        the fastest.  Returns (config, ms per solve)."""
        import torch
        sh = _shapes(self.N, self.n, self.m)
        for k in PROBLEM_FIELDS:
            _check(prob[k], k, sh[k])
        if out is None:
            out = alloc_solution(self, prob["Q"].device)
        p = Problem(**{k: prob[k].data_ptr() for k in PROBLEM_FIELDS})
        s_ = Solution(**{k: out[k].data_ptr() for k in SOLUTION_FIELDS})
        o = SolveOptions(precision=precision, refine_steps=refine_steps, executor=EXEC_LEVELS)
        best = LaunchConfig()
        ms = ctypes.c_float(0.0)
        st = stream if stream is not None else torch.cuda.current_stream(prob["Q"].device)
        rc = lib().rcr_plan_tune(self._h, ctypes.byref(p), ctypes.byref(s_), ctypes.byref(o),
                                 ctypes.c_void_p(st.cuda_stream), ctypes.byref(best), ctypes.byref(ms))
        if rc != 0:
            raise RcrError(rc, "rcr_plan_tune")
        return {k: int(getattr(best, k)) for k in LAUNCH_FIELDS}, ms.value

    def workspace_size(self, precision: int = FP64) -> int:
        return int(lib().rcr_workspace_size(self._h, precision))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().rcr_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PROBLEM_FIELDS = ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")
SOLUTION_FIELDS = ("K", "P", "x", "u", "lam")
RAGGED_FIELDS = PROBLEM_FIELDS + SOLUTION_FIELDS  # the order of rcr_ragged_offsets
RAGGED_FIELDS_COUNT = len(RAGGED_FIELDS)


def _shapes(N, n, m):
    return {"Q": (N, n, n), "q": (N, n), "c": (N, n), "Delta": (N, n, n), "R": (N, m, m), "S": (N, n, m),
            "r": (N, m), "A": (N, n, n), "B": (N, n, m), "K": (N, m, n), "P": (N, n, n), "x": (N, n),
            "u": (N, m), "lam": (N, n)}


def _check(t, name, shape):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {shape}")


def solution_shapes(N: int, n: int, m: int) -> dict:
    """Shapes of the rcr_solution fields of an N-node problem."""
    sh = _shapes(N, n, m)
    return {k: sh[k] for k in SOLUTION_FIELDS}


def alloc_solution(plan: Plan, device="cuda"):
    import torch
    sh = _shapes(plan.N, plan.n, plan.m)
    return {k: torch.empty(sh[k], dtype=torch.float64, device=device) for k in SOLUTION_FIELDS}


def solve(plan: Plan, prob: dict, out: dict | None = None, precision: int = FP64, executor: int = EXEC_LEVELS,
          check: bool = False, kkt_residual: bool = False, kernel_ms: bool = False, refine_steps: int = -1,
          workspace=None, stream=None) -> dict:
    """rcr_solve on device tensors.  Returns the solution dict, plus 'kkt_residual'
    and 'kernel_ms' entries when requested."""
    import torch
    sh = _shapes(plan.N, plan.n, plan.m)
    for k in PROBLEM_FIELDS:
        _check(prob[k], k, sh[k])
    if out is None:
        out = alloc_solution(plan, prob["Q"].device)
    for k in SOLUTION_FIELDS:
        _check(out[k], k, sh[k])
    p = Problem(**{k: prob[k].data_ptr() for k in PROBLEM_FIELDS})
    s = Solution(**{k: out[k].data_ptr() for k in SOLUTION_FIELDS})
    o = SolveOptions(precision=precision, refine_steps=refine_steps, executor=executor, check=int(check))
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    res = ctypes.c_double(-1.0)
    if kkt_residual:
        o.kkt_residual = ctypes.pointer(res)
    kms = (ctypes.c_float * NUM_KERNEL_CLASSES)()
    kln = (ctypes.c_int32 * NUM_KERNEL_CLASSES)()
    if kernel_ms:
        o.kernel_ms = ctypes.cast(kms, ctypes.POINTER(ctypes.c_float))
        o.kernel_launches = ctypes.cast(kln, ctypes.POINTER(ctypes.c_int32))
    st = stream if stream is not None else torch.cuda.current_stream(prob["Q"].device)
    rc = lib().rcr_solve(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o), ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_solve")
    result = dict(out)
    if kkt_residual:
        result["kkt_residual"] = res.value
    if kernel_ms:
        result["kernel_ms"] = {KERNEL_CLASSES[i]: float(kms[i]) for i in range(NUM_KERNEL_CLASSES)}
        result["kernel_launches"] = {KERNEL_CLASSES[i]: int(kln[i]) for i in range(NUM_KERNEL_CLASSES)}
    return result


def _options(precision, executor, check, refine_steps, workspace, kkt_residual, kernel_ms):
    """SolveOptions plus the host cells the library writes into."""
    o = SolveOptions(precision=precision, refine_steps=refine_steps, executor=executor, check=int(check))
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    res = ctypes.c_double(-1.0)
    if kkt_residual:
        o.kkt_residual = ctypes.pointer(res)
    kms = (ctypes.c_float * NUM_KERNEL_CLASSES)()
    kln = (ctypes.c_int32 * NUM_KERNEL_CLASSES)()
    if kernel_ms:
        o.kernel_ms = ctypes.cast(kms, ctypes.POINTER(ctypes.c_float))
        o.kernel_launches = ctypes.cast(kln, ctypes.POINTER(ctypes.c_int32))
    return o, res, kms, kln


def _extras(result, kkt_residual, kernel_ms, res, kms, kln):
    if kkt_residual:
        result["kkt_residual"] = res.value
    if kernel_ms:
        result["kernel_ms"] = {KERNEL_CLASSES[i]: float(kms[i]) for i in range(NUM_KERNEL_CLASSES)}
        result["kernel_launches"] = {KERNEL_CLASSES[i]: int(kln[i]) for i in range(NUM_KERNEL_CLASSES)}
    return result


def _stream(stream, device):
    import torch
    return stream if stream is not None else torch.cuda.current_stream(device)


RHS_FIELDS = ("q", "r", "c")
RHS_SOLUTION_FIELDS = ("x", "u", "lam")
MATRIX_FIELDS = ("Q", "Delta", "R", "S", "A", "B")


def factor(plan: Plan, prob: dict, out: dict | None = None, precision: int = FP64, executor: int = EXEC_LEVELS,
           check: bool = False, kernel_ms: bool = False, workspace=None, stream=None) -> dict:
    """rcr_factor: Algorithm 1, Steps 2-3 on the matrices of `prob` (q, r, c not
    read).  Returns {'K', 'P'}; the rest of the factor stays in the workspace."""
    import torch
    sh = _shapes(plan.N, plan.n, plan.m)
    for k in MATRIX_FIELDS:
        _check(prob[k], k, sh[k])
    dev = prob["Q"].device
    if out is None:
        out = {k: torch.empty(sh[k], dtype=torch.float64, device=dev) for k in ("K", "P")}
    for k in ("K", "P"):
        _check(out[k], k, sh[k])
    p = Problem(**{k: (prob[k].data_ptr() if k in prob else None) for k in PROBLEM_FIELDS})
    s = Solution(K=out["K"].data_ptr(), P=out["P"].data_ptr())
    o, res, kms, kln = _options(precision, executor, check, -1, workspace, False, kernel_ms)
    rc = lib().rcr_factor(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                          ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_factor")
    return _extras({"K": out["K"], "P": out["P"]}, False, kernel_ms, res, kms, kln)


def solve_rhs(plan: Plan, prob: dict, fac: dict, rhs: list, outs: list | None = None, precision: int = FP64,
              executor: int = EXEC_LEVELS, check: bool = False, kkt_residual: bool = False,
              kernel_ms: bool = False, refine_steps: int = -1, workspace=None, stream=None) -> dict:
    """rcr_solve_rhs: Steps 4-6 for each right-hand side dict (q, r, c) of `rhs`
    on the factor of rcr_factor (fac holds its K, P; an rcr_solve in between on
    the same workspace leaves none, and the plan-owned workspace then raises
    RcrError ERR_BAD_OPTION).  Returns {'solutions': [...]} with x, u, lam per
    right-hand side."""
    import torch
    sh = _shapes(plan.N, plan.n, plan.m)
    for k in MATRIX_FIELDS:
        _check(prob[k], k, sh[k])
    for k in ("K", "P"):
        _check(fac[k], k, sh[k])
    dev = prob["Q"].device
    if outs is None:
        outs = [{k: torch.empty(sh[k], dtype=torch.float64, device=dev) for k in RHS_SOLUTION_FIELDS} for _ in rhs]
    if len(outs) != len(rhs) or not rhs:
        raise ValueError("one solution dict per right-hand side, at least one")
    for r_, o_ in zip(rhs, outs):
        for k in RHS_FIELDS:
            _check(r_[k], k, sh[k])
        for k in RHS_SOLUTION_FIELDS:
            _check(o_[k], k, sh[k])
    kk = len(rhs)
    ra = (Rhs * kk)(*[Rhs(**{k: r_[k].data_ptr() for k in RHS_FIELDS}) for r_ in rhs])
    sa = (RhsSolution * kk)(*[RhsSolution(**{k: o_[k].data_ptr() for k in RHS_SOLUTION_FIELDS}) for o_ in outs])
    p = Problem(**{k: (prob[k].data_ptr() if k in prob else None) for k in PROBLEM_FIELDS})
    f = Solution(K=fac["K"].data_ptr(), P=fac["P"].data_ptr())
    o, res, kms, kln = _options(precision, executor, check, refine_steps, workspace, kkt_residual, kernel_ms)
    rc = lib().rcr_solve_rhs(plan._h, ctypes.byref(p), ctypes.byref(f), kk, ra, sa, ctypes.byref(o),
                             ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_solve_rhs")
    return _extras({"solutions": outs}, kkt_residual, kernel_ms, res, kms, kln)


GRADIENT_FIELDS = PROBLEM_FIELDS


def adjoint(plan: Plan, prob: dict, fwd: dict, seed: dict, grads: dict | None = None, want=GRADIENT_FIELDS,
            precision: int = FP64, executor: int = EXEC_LEVELS, check: bool = False, refine_steps: int = -1,
            workspace=None, stream=None) -> dict:
    """rcr_adjoint: gradients of L with respect to the problem data from the seeds
    seed = {'x': dL/dx, 'u': dL/du, 'lam': dL/dlam}; fwd holds the factor's K, P
    and the forward x, u, lam.  Returns the gradient dict (fields of `want`; q, r,
    c always)."""
    import torch
    sh = _shapes(plan.N, plan.n, plan.m)
    dev = prob["Q"].device
    for k in MATRIX_FIELDS:
        _check(prob[k], k, sh[k])
    for k in SOLUTION_FIELDS:
        _check(fwd[k], k, sh[k])
    for k, f_ in (("x", "q"), ("u", "r"), ("lam", "c")):
        _check(seed[k], k, sh[f_])
    want = set(want) | {"q", "r", "c"}
    if grads is None:
        grads = {k: torch.empty(sh[k], dtype=torch.float64, device=dev) for k in GRADIENT_FIELDS if k in want}
    for k, v in grads.items():
        _check(v, k, sh[k])
    g = Gradient(**{k: (grads[k].data_ptr() if k in grads else None) for k in GRADIENT_FIELDS})
    sd = Rhs(q=seed["x"].data_ptr(), r=seed["u"].data_ptr(), c=seed["lam"].data_ptr())
    p = Problem(**{k: (prob[k].data_ptr() if k in prob else None) for k in PROBLEM_FIELDS})
    f = Solution(**{k: fwd[k].data_ptr() for k in SOLUTION_FIELDS})
    o, res, kms, kln = _options(precision, executor, check, refine_steps, workspace, False, False)
    rc = lib().rcr_adjoint(plan._h, ctypes.byref(p), ctypes.byref(f), ctypes.byref(sd), ctypes.byref(g),
                           ctypes.byref(o), ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_adjoint")
    return grads


def kkt_residual(plan: Plan, prob: dict, sol: dict, workspace=None, stream=None) -> float:
    """rcr_kkt_residual: max-abs residual of eq. (kkt) of the iterate sol (x, u, lam)."""
    sh = _shapes(plan.N, plan.n, plan.m)
    for k in PROBLEM_FIELDS:
        _check(prob[k], k, sh[k])
    for k in RHS_SOLUTION_FIELDS:
        _check(sol[k], k, sh[k])
    dev = prob["Q"].device
    p = Problem(**{k: prob[k].data_ptr() for k in PROBLEM_FIELDS})
    s = Solution(**{k: (sol[k].data_ptr() if k in sol else None) for k in SOLUTION_FIELDS})
    o, res, _, _ = _options(FP64, EXEC_LEVELS, False, -1, workspace, True, False)
    rc = lib().rcr_kkt_residual(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                                ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_kkt_residual")
    return res.value


def noalloc_scratch_bytes() -> int:
    return int(lib().rcr_noalloc_scratch_bytes())


def solve_noalloc(plan: Plan, prob: dict, out: dict, precision: int = FP64, check: bool = False,
                  kkt_residual: bool = False, refine_steps: int = -1, stream=None) -> dict:
    """rcr_solve_noalloc: rcr_solve on the library's static per-GPU scratch array.
    The plan must be uploaded (Plan.upload) and `out` preallocated."""
    sh = _shapes(plan.N, plan.n, plan.m)
    for k in PROBLEM_FIELDS:
        _check(prob[k], k, sh[k])
    for k in SOLUTION_FIELDS:
        _check(out[k], k, sh[k])
    p = Problem(**{k: prob[k].data_ptr() for k in PROBLEM_FIELDS})
    s = Solution(**{k: out[k].data_ptr() for k in SOLUTION_FIELDS})
    o, res, kms, kln = _options(precision, EXEC_LEVELS, check, refine_steps, None, kkt_residual, False)
    rc = lib().rcr_solve_noalloc(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                                 ctypes.c_void_p(_stream(stream, prob["Q"].device).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_solve_noalloc")
    return _extras(dict(out), kkt_residual, False, res, kms, kln)


def ragged_solve(plan: Plan, prob: dict, out: dict | None = None, precision: int = FP64, executor: int = EXEC_LEVELS,
                 check: bool = False, kkt_residual: bool = False, refine_steps: int = -1, workspace=None,
                 stream=None) -> dict:
    """rcr_ragged_solve: packed 1-D float64 device tensors (lengths from
    plan.ragged_offsets) for the problem fields; returns the packed solution."""
    import torch
    off = getattr(plan, "ragged_offsets", None)
    if off is None:
        raise ValueError("ragged_solve needs a plan from Plan.ragged")
    for k in PROBLEM_FIELDS:
        _check(prob[k], k, (int(off[k][-1]),))
    dev = prob["Q"].device
    if out is None:
        out = {k: torch.empty(max(int(off[k][-1]), 1), dtype=torch.float64, device=dev)[:int(off[k][-1])]
               for k in SOLUTION_FIELDS}
    for k in SOLUTION_FIELDS:
        _check(out[k], k, (int(off[k][-1]),))
    p = Problem(**{k: prob[k].data_ptr() for k in PROBLEM_FIELDS})
    s = Solution(**{k: out[k].data_ptr() for k in SOLUTION_FIELDS})
    o, res, kms, kln = _options(precision, executor, check, refine_steps, workspace, kkt_residual, False)
    rc = lib().rcr_ragged_solve(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                                ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_ragged_solve")
    return _extras(dict(out), kkt_residual, False, res, kms, kln)


def _plan_array(plans):
    return (ctypes.c_void_p * len(plans))(*[p._h.value for p in plans])


def batch_prepare(plans, stream=None):
    """rcr_batch_prepare: build, cache and upload the merged plan of these plans."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib().rcr_batch_prepare(_plan_array(plans), len(plans), ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_batch_prepare")


def batch_release(plans):
    """rcr_batch_release: drop the library's cached merged plan of these plans."""
    lib().rcr_batch_release(_plan_array(plans), len(plans))


def batch_workspace_size(plans, precision: int = FP64) -> int:
    return int(lib().rcr_batch_workspace_size(_plan_array(plans), len(plans), precision))


def batch_solve(plans, probs: list, outs: list | None = None, precision: int = FP64, executor: int = EXEC_LEVELS,
                check: bool = False, kkt_residual: bool = False, refine_steps: int = -1, workspace=None,
                stream=None) -> dict:
    """rcr_batch_solve: tree t (plans[t]) with its own problem probs[t] and solution
    outs[t] (device tensors), all solved in one merged launch sequence.  Returns
    {'solutions': outs} (plus 'kkt_residual', the largest over the trees)."""
    import torch
    if not plans or len(probs) != len(plans):
        raise ValueError("one problem per plan, at least one plan")
    dev = probs[0]["Q"].device
    if outs is None:
        outs = [alloc_solution(p_, dev) for p_ in plans]
    if len(outs) != len(plans):
        raise ValueError("one solution per plan")
    for p_, pr, ou in zip(plans, probs, outs):
        sh = _shapes(p_.N, p_.n, p_.m)
        for k in PROBLEM_FIELDS:
            _check(pr[k], k, sh[k])
        for k in SOLUTION_FIELDS:
            _check(ou[k], k, sh[k])
    kk = len(plans)
    pa = (Problem * kk)(*[Problem(**{k: pr[k].data_ptr() for k in PROBLEM_FIELDS}) for pr in probs])
    sa = (Solution * kk)(*[Solution(**{k: ou[k].data_ptr() for k in SOLUTION_FIELDS}) for ou in outs])
    o, res, kms, kln = _options(precision, executor, check, refine_steps, workspace, kkt_residual, False)
    rc = lib().rcr_batch_solve(_plan_array(plans), kk, pa, sa, ctypes.byref(o),
                               ctypes.c_void_p(_stream(stream, dev).cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_batch_solve")
    return _extras({"solutions": outs}, kkt_residual, False, res, kms, kln)


NATIVE_FIELDS = ("Q", "q", "c", "Delta", "M", "R", "r", "A", "B")
NATIVE_SOLUTION_FIELDS = ("x", "v", "lam")


def _native_shapes(N, n, m):
    return {"Q": (N, n, n), "q": (N, n), "c": (N, n), "Delta": (N, n, n), "M": (N, n, m), "R": (N, m, m),
            "r": (N, m), "A": (N, n, n), "B": (N, n, m), "x": (N, n), "v": (N, m), "lam": (N, n)}


def lift_solve(plan: Plan, prob: dict, out: dict | None = None, precision: int = FP64, executor: int = EXEC_LEVELS,
               check: bool = False, kkt_residual: bool = False, refine_steps: int = -1, workspace=None,
               stream=None) -> dict:
    """rcr_lift_solve: a node-control problem (device tensors, NATIVE_FIELDS) through
    the exact lifting.  Returns x, v, lam (and 'kkt_residual' of the lifted system)."""
    import torch
    if getattr(plan, "native_N", None) is None:
        raise ValueError("lift_solve needs a plan from Plan.lift")
    sh = _native_shapes(plan.native_N, plan.native_n, plan.m)
    for k in NATIVE_FIELDS:
        _check(prob[k], k, sh[k])
    if out is None:
        out = {k: torch.empty(sh[k], dtype=torch.float64, device=prob["Q"].device) for k in NATIVE_SOLUTION_FIELDS}
    for k in NATIVE_SOLUTION_FIELDS:
        _check(out[k], k, sh[k])
    p = NativeProblem(**{k: prob[k].data_ptr() for k in NATIVE_FIELDS})
    s = NativeSolution(**{k: out[k].data_ptr() for k in NATIVE_SOLUTION_FIELDS})
    o = SolveOptions(precision=precision, refine_steps=refine_steps, executor=executor, check=int(check))
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    res = ctypes.c_double(-1.0)
    if kkt_residual:
        o.kkt_residual = ctypes.pointer(res)
    st = stream if stream is not None else torch.cuda.current_stream(prob["Q"].device)
    rc = lib().rcr_lift_solve(plan._h, ctypes.byref(p), ctypes.byref(s), ctypes.byref(o),
                              ctypes.c_void_p(st.cuda_stream))
    if rc != 0:
        raise RcrError(rc, "rcr_lift_solve")
    result = dict(out)
    if kkt_residual:
        result["kkt_residual"] = res.value
    return result


def concat_problems(datas) -> dict:
    """Concatenate host problems of independent trees in the node order of a
    batched plan (Plan.batch)."""
    return {k: np.concatenate([np.ascontiguousarray(d[k]) for d in datas], axis=0) for k in PROBLEM_FIELDS}


def to_device(data: dict, device="cuda", fields=PROBLEM_FIELDS) -> dict:
    """Copy a host problem dict (numpy float64) to device tensors."""
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(data[k], dtype=np.float64)).to(device) for k in fields}
