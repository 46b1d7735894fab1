"""Thin Python binding of the hsolve C ABI (include/hsolve.h).

Argument marshalling only: every step of the factorization and of the solve runs in the
HIP library ``libhsolve.so`` built from ``csrc/`` (``python -m paper_1611_03189_amd.build``).
PyTorch provides device memory and the stream: the factorization runs in an arena, a
``torch.uint8`` tensor of the size ``hsolve_analyze`` bounds (or one the caller passes). If
the library is missing, importing the functions that need it raises ``RuntimeError``; there
is no fallback.
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhsolve.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "hsolve.h")

LORASP = 0
GC = 1
GC_PROJ1 = 2
KRYLOV = {"pcg": 0, "fpcg": 1, "gmres": 2, "stationary": 3}
EPS_SCHEDULE = {"constant": 0, "shrink": 1, "grow": 2}
ORDER = {"index": 0, "waiting": 1}

STATUS = {
    0: "HSOLVE_OK", 1: "HSOLVE_NOT_CONVERGED", -1: "HSOLVE_ERR_INVALID",
    -2: "HSOLVE_ERR_NOT_SYMMETRIC", -3: "HSOLVE_ERR_NOT_SPD", -4: "HSOLVE_ERR_OOM",
    -5: "HSOLVE_ERR_DEVICE", -6: "HSOLVE_ERR_STATE", -7: "HSOLVE_ERR_TOO_LARGE",
}


class HSolveError(RuntimeError):
    def __init__(self, status: int, where: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}")
        self.status = status


class NotSPD(HSolveError):
    pass


class Options(ctypes.Structure):
    _fields_ = [
        ("leaf_size", c_int), ("eps", c_double), ("variant", c_int), ("nvec", c_int),
        ("phi", POINTER(c_double)), ("dim", c_int), ("coords", POINTER(c_double)),
        ("tol", c_double), ("max_iter", c_int), ("krylov", c_int), ("stream", c_void_p),
        ("apply_prec", c_int), ("restart", c_int), ("overlap_pivots", c_int),
        ("factor_prec", c_int), ("max_super", c_int), ("max_nrhs", c_int), ("eps_schedule", c_int),
        ("cmp_lpe", c_int), ("cmp_vectors", c_int), ("apply_graph", c_int), ("neighbours", c_int),
        ("eps1", c_double), ("cmp_ritz", c_int), ("order", c_int),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("iterations", c_int), ("rel_residual", c_double), ("t_analyze", c_double),
        ("t_factor", c_double), ("t_solve", c_double), ("levels", c_int), ("colours", c_int),
        ("max_rank", c_int), ("factor_bytes", c_int64), ("factor_flops", c_double),
        ("apply_bytes", c_double), ("fail_level", c_int), ("fail_node", c_int),
        ("device_bytes", c_int64), ("arena_bound", c_int64),
    ]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None


def exported_names() -> list[str]:
    """Function names declared in include/hsolve.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(hsolve_[a-z_]+)\s*\(", text)))


def load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1611_03189_amd.build`")
    try:        # the library links the HIP runtime PyTorch ships: load that copy first
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(LIB_PATH)
    P = c_void_p
    sig = {
        "hsolve_default_options": (None, [POINTER(Options)]),
        "hsolve_analyze": (c_int, [c_int, POINTER(c_int64), POINTER(c_int32), POINTER(Options), POINTER(P),
                                   POINTER(ctypes.c_size_t)]),
        "hsolve_factor": (c_int, [P, P, P, ctypes.c_size_t]),
        "hsolve_apply": (c_int, [P, c_int, P, c_int, P, c_int]),
        "hsolve_apply_static": (c_int, [P, c_int, P, c_int, P, c_int]),
        "hsolve_solve": (c_int, [P, c_int, P, c_int, P, c_int, POINTER(Stats)]),
        "hsolve_spmv": (c_int, [P, P, P]),
        "hsolve_get_stats": (c_int, [P, POINTER(Stats)]),
        "hsolve_set_stream": (c_int, [P, P]),
        "hsolve_tune_workspace_bytes": (ctypes.c_size_t, []),
        "hsolve_tune_gemm": (c_int, [P, ctypes.c_size_t, P, POINTER(c_int32), POINTER(c_double)]),
        "hsolve_set_gemm_choice": (c_int, [POINTER(c_int32)]),
        "hsolve_destroy": (c_int, [P]),
        "hsolve_status_string": (ctypes.c_char_p, [c_int]),
        "hsolve_depth": (c_int, [P]),
        "hsolve_last_error": (ctypes.c_char_p, [P]),
        "hsolve_leaf_order": (c_int, [P, POINTER(c_int32), POINTER(c_int32)]),
        "hsolve_level_colours": (c_int, [P, c_int, POINTER(c_int32), POINTER(c_int32)]),
        "hsolve_node_sets": (c_int, [P, c_int, c_int, POINTER(c_int32), POINTER(c_int32),
                                     POINTER(c_int32), POINTER(c_int32), c_int]),
        "hsolve_ranks": (c_int, [P, c_int, POINTER(c_int32)]),
        "hsolve_node_factor": (c_int, [P, c_int, c_int, POINTER(c_int32), POINTER(c_double), c_int64]),
        "hsolve_profile_begin": (c_int, [P]),
        "hsolve_profile_only": (c_int, [P, ctypes.c_char_p]),
        "hsolve_profile_end": (c_int, [P, POINTER(c_int32)]),
        "hsolve_profile_entry": (c_int, [P, c_int, ctypes.c_char_p, c_int, POINTER(c_double),
                                         POINTER(c_int64), POINTER(c_double)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str, lib=None, handle=None):
    if status in (0, 1):
        return status
    if lib is not None and handle:
        msg = lib.hsolve_last_error(handle)
        if msg:
            where = f"{where} ({msg.decode()})"
    if status == -3:
        raise NotSPD(status, where)
    raise HSolveError(status, where)


def _i32p(a):
    return a.ctypes.data_as(POINTER(c_int32))


def _dev(t, torch):
    """A contiguous float64 tensor on the current GPU (copies numpy / host input)."""
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.asarray(t, dtype=np.float64))
    if not t.is_cuda:
        t = t.cuda()
    if t.dtype != torch.float64:
        raise TypeError("hsolve works on float64 data")
    return t.contiguous()


def _cols(t, n, torch, what):
    """A float64 CUDA tensor of n rows as (nrhs, n) row-major = n x nrhs column-major."""
    t = _dev(t, torch)
    if t.dim() not in (1, 2) or t.shape[0] != n or t.numel() == 0:
        raise ValueError(f"{what}: expected a vector of {n} entries or an {n} x nrhs matrix, got "
                         f"shape {tuple(t.shape)}")
    vec = t.dim() == 1
    M = t.reshape(n, -1) if vec else t
    return M.t().contiguous(), vec


# (tile rows, tile columns, K step, persistent grid)
GEMM_SHAPES = [(64, 64, 16, 0), (64, 64, 32, 0), (128, 64, 16, 0), (128, 128, 16, 0), (32, 32, 64, 0),
               (32, 32, 128, 0), (64, 64, 16, 1), (32, 32, 64, 1)]
GEMM_BUCKETS = 12


def tune_gemm(stream=None) -> dict:
    """Time every tile shape of the grouped GEMM on each size bucket (hsolve_tune_gemm) and
    keep the fastest for the process; returns the choice and the timings."""
    import torch
    lib = load()
    work = torch.empty(int(lib.hsolve_tune_workspace_bytes()), dtype=torch.uint8, device="cuda")
    choice = np.zeros(2 * GEMM_BUCKETS, dtype=np.int32)
    ms = np.zeros(2 * GEMM_BUCKETS * len(GEMM_SHAPES))
    _check(lib.hsolve_tune_gemm(c_void_p(work.data_ptr()), work.numel(),
                                c_void_p(stream.cuda_stream) if stream is not None else None,
                                _i32p(choice), ms.ctypes.data_as(POINTER(c_double))), "hsolve_tune_gemm")
    torch.cuda.synchronize()
    del work
    return {"choice": choice[:GEMM_BUCKETS].tolist(), "choice_f32": choice[GEMM_BUCKETS:].tolist(),
            "shapes": [list(x) for x in GEMM_SHAPES],
            "ms": ms[:GEMM_BUCKETS * len(GEMM_SHAPES)].reshape(GEMM_BUCKETS, len(GEMM_SHAPES)).round(4).tolist(),
            "ms_f32": ms[GEMM_BUCKETS * len(GEMM_SHAPES):].reshape(GEMM_BUCKETS, len(GEMM_SHAPES)).round(4).tolist()}


def set_gemm_choice(choice, choice_f32=None) -> None:
    """Install a tile-shape choice per bucket (e.g. one saved from tune_gemm) for the FP64
    GEMMs and, given or else the same, the FP32 ones."""
    c = np.ascontiguousarray(list(choice) + list(choice if choice_f32 is None else choice_f32), dtype=np.int32)
    if c.shape != (2 * GEMM_BUCKETS,):
        raise ValueError(f"expected {GEMM_BUCKETS} entries")
    _check(load().hsolve_set_gemm_choice(_i32p(c)), "hsolve_set_gemm_choice")


class HSolver:
    """One analysed sparse SPD pattern with (after :meth:`factor`) its hierarchical factor.

    ``row_ptr``/``col_idx``: CSR pattern (host arrays, symmetric, sorted rows);
    ``coords`` (n x dim) drive the bisection; ``variant`` is ``"gc"`` (default) or
    ``"lorasp"``; ``phi`` (n x p) are the vectors GC preserves (default: constant).
    ``arena_bound`` is the device memory a factorization of this pattern can need.
    """

    def __init__(self, row_ptr, col_idx, coords=None, leaf: int = 16, eps: float = 1e-2,
                 variant: str = "gc", phi=None, tol: float = 1e-10, max_iter: int = 1000,
                 stream=None, krylov: str = "pcg", apply_prec: int = 64, restart: int = 200,
                 overlap_pivots: bool = True, factor_prec: int = 64, max_super: int = 512,
                 max_nrhs: int = 32, eps_schedule: str = "constant", cmp_lpe: int = 0,
                 cmp_vectors: int = 0, apply_graph: bool = True, neighbours: str = "footprint",
                 eps1: float = 0.0, cmp_ritz: bool = True, order: str = "waiting"):
        lib = load()
        self._lib = lib
        self.row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
        self.col_idx = np.ascontiguousarray(col_idx, dtype=np.int32)
        self.n = len(self.row_ptr) - 1
        self.nnz = int(self.row_ptr[-1])
        opt = Options()
        lib.hsolve_default_options(ctypes.byref(opt))
        opt.leaf_size = int(leaf)
        opt.eps = float(eps)
        opt.variant = ({"gc": GC, "lorasp": LORASP, "gc_proj1": GC_PROJ1}[variant] if isinstance(variant, str)
                       else int(variant))
        opt.eps1 = float(eps1)
        opt.tol = float(tol)
        opt.max_iter = int(max_iter)
        opt.krylov = KRYLOV[krylov] if isinstance(krylov, str) else int(krylov)
        opt.apply_prec = int(apply_prec)
        opt.restart = int(restart)
        opt.overlap_pivots = 1 if overlap_pivots else 0
        opt.factor_prec = int(factor_prec)
        opt.max_super = int(max_super)
        opt.max_nrhs = int(max_nrhs)
        opt.eps_schedule = EPS_SCHEDULE[eps_schedule] if isinstance(eps_schedule, str) else int(eps_schedule)
        opt.cmp_lpe = int(cmp_lpe)
        opt.cmp_vectors = int(cmp_vectors)
        opt.apply_graph = 1 if apply_graph else 0
        opt.cmp_ritz = int(cmp_ritz)
        opt.order = ORDER[order] if isinstance(order, str) else int(order)
        opt.neighbours = {"footprint": 0, "geometric": 1}[neighbours] if isinstance(neighbours, str) else int(neighbours)
        self._keep = []
        if coords is not None:
            c = np.ascontiguousarray(np.asarray(coords, dtype=np.float64).reshape(self.n, -1))
            self._keep.append(c)
            opt.dim = c.shape[1]
            opt.coords = c.ctypes.data_as(POINTER(c_double))
        if phi is not None:
            ph = np.asfortranarray(np.asarray(phi, dtype=np.float64).reshape(self.n, -1))
            self._keep.append(ph)
            opt.nvec = ph.shape[1]
            opt.phi = ph.ctypes.data_as(POINTER(c_double))
        self.stream = stream
        opt.stream = c_void_p(stream.cuda_stream) if stream is not None else None
        h = c_void_p()
        bound = ctypes.c_size_t()
        _check(lib.hsolve_analyze(self.n, self.row_ptr.ctypes.data_as(POINTER(c_int64)),
                                  _i32p(self.col_idx), ctypes.byref(opt), ctypes.byref(h),
                                  ctypes.byref(bound)),
               "hsolve_analyze")
        self._h = h
        self.arena_bound = int(bound.value)
        self._keep.clear()          # analyze copied coordinates and phi
        self.values = None
        self.arena = None

    # -- lifecycle -----------------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._lib.hsolve_destroy(self._h)
            self._h = None
        self.arena = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # -- numeric -------------------------------------------------------------------
    def factor(self, values, arena=None):
        """Factor with the CSR values (nnz float64, host or device). ``arena`` is a CUDA
        uint8 tensor the plan works in (kept until the next factor or close); by default one
        of ``arena_bound`` bytes is made once and reused."""
        import torch
        if isinstance(values, torch.Tensor) and values.is_cuda:
            v = values
            if v.dtype != torch.float64:
                raise TypeError("hsolve works on float64 data")
            v = v.contiguous()
        else:
            v = np.ascontiguousarray(values, dtype=np.float64)
        if v.reshape(-1).shape[0] != self.nnz:
            raise ValueError(f"values: expected {self.nnz} entries, got {v.reshape(-1).shape[0]}")
        if arena is None:
            arena = self.arena
            if arena is None or arena.numel() < self.arena_bound:
                self.arena = None
                arena = torch.empty(max(self.arena_bound, 256), dtype=torch.uint8, device="cuda")
        elif not (isinstance(arena, torch.Tensor) and arena.is_cuda and arena.dtype == torch.uint8
                  and arena.is_contiguous()):
            raise TypeError("arena must be a contiguous CUDA uint8 tensor")
        self.arena = arena
        self.values = v
        ptr = c_void_p(v.data_ptr()) if isinstance(v, torch.Tensor) else v.ctypes.data_as(c_void_p)
        _check(self._lib.hsolve_factor(self._h, ptr, c_void_p(arena.data_ptr()), arena.numel()),
               "hsolve_factor", self._lib, self._h)
        return self

    def apply(self, r, out=None):
        import torch
        Rc, vec = _cols(r, self.n, torch, "apply")
        Z = torch.empty_like(Rc) if out is None else out
        if Z.shape != Rc.shape or not Z.is_contiguous() or Z.dtype != torch.float64 or not Z.is_cuda:
            raise ValueError("apply: out must be a contiguous float64 CUDA tensor of shape (nrhs, n)")
        _check(self._lib.hsolve_apply(self._h, Rc.shape[0], c_void_p(Rc.data_ptr()), self.n,
                                      c_void_p(Z.data_ptr()), self.n), "hsolve_apply",
               self._lib, self._h)
        Z = Z.t()
        return Z.reshape(-1) if vec else Z

    def apply_static(self, r, out=None):
        """As :meth:`apply`, through hsolve_apply_static (solve vectors in the library's static
        device scratch; nothing allocated by the library)."""
        import torch
        Rc, vec = _cols(r, self.n, torch, "apply_static")
        Z = torch.empty_like(Rc) if out is None else out
        if Z.shape != Rc.shape or not Z.is_contiguous() or Z.dtype != torch.float64 or not Z.is_cuda:
            raise ValueError("apply_static: out must be a contiguous float64 CUDA tensor of shape (nrhs, n)")
        _check(self._lib.hsolve_apply_static(self._h, Rc.shape[0], c_void_p(Rc.data_ptr()), self.n,
                                             c_void_p(Z.data_ptr()), self.n), "hsolve_apply_static",
               self._lib, self._h)
        Z = Z.t()
        return Z.reshape(-1) if vec else Z

    def solve(self, b):
        import torch
        Bc, vec = _cols(b, self.n, torch, "solve")
        X = torch.empty_like(Bc)
        st = Stats()
        status = _check(self._lib.hsolve_solve(self._h, Bc.shape[0], c_void_p(Bc.data_ptr()), self.n,
                                               c_void_p(X.data_ptr()), self.n, ctypes.byref(st)),
                        "hsolve_solve", self._lib, self._h)
        X = X.t()
        d = st.as_dict()
        d["converged"] = status == 0
        return (X.reshape(-1) if vec else X), d

    def spmv(self, x):
        import torch
        x = _dev(x, torch)
        if x.numel() != self.n:
            raise ValueError(f"spmv: expected {self.n} entries, got {x.numel()}")
        x = x.reshape(-1)
        y = torch.empty_like(x)
        _check(self._lib.hsolve_spmv(self._h, c_void_p(x.data_ptr()), c_void_p(y.data_ptr())),
               "hsolve_spmv", self._lib, self._h)
        return y

    def set_stream(self, stream):
        """Run the plan's later GPU work on `stream` (a torch.cuda.Stream or None)."""
        self.stream = stream
        _check(self._lib.hsolve_set_stream(self._h, c_void_p(stream.cuda_stream) if stream is not None else None),
               "hsolve_set_stream")

    # -- kernel timing ---------------------------------------------------------------
    def profile_begin(self, only: str | None = None):
        """Start recording kernel times; with `only`, launches of that kernel alone."""
        _check(self._lib.hsolve_profile_only(self._h, only.encode() if only else None), "hsolve_profile_only")
        _check(self._lib.hsolve_profile_begin(self._h), "hsolve_profile_begin")

    def profile_end(self) -> list[dict]:
        """Per-kernel totals since profile_begin: name, ms, launches, work (flops or bytes)."""
        nk = c_int32()
        _check(self._lib.hsolve_profile_end(self._h, ctypes.byref(nk)), "hsolve_profile_end",
               self._lib, self._h)
        out = []
        for i in range(nk.value):
            name = ctypes.create_string_buffer(64)
            ms, work, launches = c_double(), c_double(), c_int64()
            _check(self._lib.hsolve_profile_entry(self._h, i, name, 64, ctypes.byref(ms),
                                                  ctypes.byref(launches), ctypes.byref(work)),
                   "hsolve_profile_entry")
            out.append(dict(name=name.value.decode(), ms=ms.value, launches=launches.value,
                            work=work.value))
        return out

    # -- introspection -------------------------------------------------------------
    def stats(self) -> dict:
        st = Stats()
        _check(self._lib.hsolve_get_stats(self._h, ctypes.byref(st)), "hsolve_get_stats")
        return st.as_dict()

    @property
    def depth(self) -> int:
        return self._lib.hsolve_depth(self._h)

    def leaf_order(self):
        L = self.depth
        perm = np.empty(self.n, dtype=np.int32)
        off = np.empty((1 << L) + 1, dtype=np.int32)
        _check(self._lib.hsolve_leaf_order(self._h, _i32p(perm), _i32p(off)), "hsolve_leaf_order")
        return perm, off

    def colours(self, depth: int):
        col = np.empty(1 << depth, dtype=np.int32)
        nc = c_int32()
        _check(self._lib.hsolve_level_colours(self._h, depth, _i32p(col), ctypes.byref(nc)),
               "hsolve_level_colours")
        return col, nc.value

    def node_sets(self, depth: int, node: int, cap: int = 4096):
        nb = np.empty(cap, dtype=np.int32)
        ws = np.empty(cap, dtype=np.int32)
        nn, nw = c_int32(), c_int32()
        _check(self._lib.hsolve_node_sets(self._h, depth, node, _i32p(nb), ctypes.byref(nn),
                                          _i32p(ws), ctypes.byref(nw), cap), "hsolve_node_sets")
        return nb[:nn.value].copy(), ws[:nw.value].copy()

    def node_factor(self, depth: int, node: int):
        """(M_ss, A_Ns M_ss, P_ss) of one eliminated super node, copied to the host."""
        dims = np.zeros(3, dtype=np.int32)
        _check(self._lib.hsolve_node_factor(self._h, depth, node, _i32p(dims), None, 0),
               "hsolve_node_factor", self._lib, self._h)
        m, ntot, k = (int(x) for x in dims)
        if m == 0:
            return None
        G = np.zeros((m + ntot + k) * m)
        _check(self._lib.hsolve_node_factor(self._h, depth, node, _i32p(dims),
                                            G.ctypes.data_as(POINTER(c_double)), G.size),
               "hsolve_node_factor", self._lib, self._h)
        G = G.reshape(m, m + ntot + k).T
        return G[:m], G[m:m + ntot], G[m + ntot:]

    def ranks(self, depth: int):
        out = np.empty(1 << depth, dtype=np.int32)
        _check(self._lib.hsolve_ranks(self._h, depth, _i32p(out)), "hsolve_ranks")
        return out
