"""Python face of libpodcg: one object per context, torch tensors in and out.

Every method marshals arguments and calls the C ABI of the same name; all
arithmetic runs in the library's HIP kernels.  Tensors must be contiguous
float64 (int32 for CSR indices) on the GPU the context was created on.
"""

from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L


class PodCGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"podcg error {code}: {msg}")
        self.code = code


def _ptr(t: torch.Tensor | None, dtype) -> C.c_void_p | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"tensor must be contiguous {dtype}")
    return C.c_void_p(t.data_ptr())


class PodCG:
    """Context for a sequence of SPD systems of size n (include/podcg.h)."""

    def __init__(self, n: int, omega: int = 20, rank_max: int = 10, maxit: int = 10000,
                 check_every: int = 16, weights: str = "idw", timing: int = 0,
                 rank_rtol: float = 1e-12, energy: float = 1.0, precision: str = "fp64",
                 max_refine: int = 20, inner_rtol: float = 1e-6, spmv_grid: int = 0,
                 update_grid: int = 0, dir_grid: int = 0, projection: str = "implicit",
                 lds_solve: bool = True, stream=None):
        self._L = L.load()
        opt = L.Options()
        self._L.podcg_default_options(C.byref(opt))
        opt.omega, opt.rank_max, opt.maxit = omega, rank_max, maxit
        opt.check_every, opt.timing = check_every, timing
        opt.weights = {"idw": 0, "unit": 1}[weights]
        opt.rank_rtol, opt.energy = rank_rtol, energy
        opt.precision = {"fp64": 0, "mixed": 1}[precision]
        opt.max_refine, opt.inner_rtol = max_refine, inner_rtol
        opt.spmv_grid, opt.update_grid, opt.dir_grid = spmv_grid, update_grid, dir_grid
        opt.projection = {"explicit": 0, "implicit": 1}[projection]
        opt.lds_solve = 1 if lds_solve else 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.n = int(n)
        self.omega, self.rank_max = omega, rank_max
        h = C.c_void_p()
        rc = self._L.podcg_create(C.byref(h), self.n, C.byref(opt), C.c_void_p(stream.cuda_stream))
        if rc != 0:
            raise PodCGError(rc, self._L.podcg_strerror(rc).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.podcg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise PodCGError(rc, self._L.podcg_last_error(self._h).decode())
        return rc

    # ---------------------------------------------------------------- the four calls
    def set_matrix(self, vals: torch.Tensor, rowptr: torch.Tensor | None = None,
                   colind: torch.Tensor | None = None):
        """A_j from CSR (rowptr/colind None: same pattern as before)."""
        self._check(self._L.podcg_set_matrix(self._h, vals.numel(), _ptr(rowptr, torch.int32),
                                             _ptr(colind, torch.int32), _ptr(vals, torch.float64)))

    def push_snapshot(self, s: torch.Tensor):
        self._check(self._L.podcg_push_snapshot(self._h, _ptr(s, torch.float64)))

    def build_pod(self, wait: bool = True) -> int | None:
        """Build the next basis; returns its rank, or None with wait=False (the
        call then returns without waiting for the GPU)."""
        if not wait:
            self._check(self._L.podcg_build_pod(self._h, None))
            return None
        y = C.c_int32()
        self._check(self._L.podcg_build_pod(self._h, C.byref(y)))
        return y.value

    def solve(self, b: torch.Tensor, x: torch.Tensor, rtol: float) -> L.Stats:
        """x holds xbar on entry and the solution on return."""
        st = L.Stats()
        self._check(self._L.podcg_solve(self._h, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                        float(rtol), C.byref(st)))
        return st

    # ---------------------------------------------------------------- the rest
    def solve_noalloc(self, b: torch.Tensor, x: torch.Tensor, rtol: float) -> L.Stats:
        """podcg_solve_noalloc: the small-system solve with no allocation in the call."""
        st = L.Stats()
        self._check(self._L.podcg_solve_noalloc(self._h, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                                float(rtol), C.byref(st)))
        return st

    def solve_plain(self, b: torch.Tensor, x: torch.Tensor, rtol: float) -> L.Stats:
        st = L.Stats()
        self._check(self._L.podcg_solve_plain(self._h, _ptr(b, torch.float64),
                                              _ptr(x, torch.float64), float(rtol), C.byref(st)))
        return st

    def reset_snapshots(self):
        self._check(self._L.podcg_reset_snapshots(self._h))

    def set_basis(self, W: torch.Tensor | None):
        """W: (n, y) tensor (stored column-major by the library) or None."""
        if W is None or W.numel() == 0:
            self._check(self._L.podcg_set_basis(self._h, None, 0))
            return
        Wc = W.t().contiguous()
        self._check(self._L.podcg_set_basis(self._h, _ptr(Wc, torch.float64), Wc.shape[0]))

    def get_basis(self) -> torch.Tensor:
        out = torch.empty((max(self.rank_max, 1), self.n), dtype=torch.float64, device="cuda")
        y = C.c_int32()
        self._check(self._L.podcg_get_basis(self._h, _ptr(out, torch.float64), C.byref(y)))
        return out[: y.value].t()

    def get_reduced(self):
        """(G, G^{-1}) of the current basis as NumPy arrays."""
        G = np.zeros(L.MAX_BASIS * L.MAX_BASIS)
        Gi = np.zeros(L.MAX_BASIS * L.MAX_BASIS)
        y = C.c_int32()
        self._check(self._L.podcg_get_reduced(self._h, G.ctypes.data_as(C.c_void_p),
                                              Gi.ctypes.data_as(C.c_void_p), C.byref(y)))
        k = y.value
        return G[: k * k].reshape(k, k), Gi[: k * k].reshape(k, k)

    def pod_spectrum(self) -> np.ndarray:
        lam = np.zeros(L.MAX_BASIS)
        c = C.c_int32()
        self._check(self._L.podcg_get_pod_spectrum(self._h, lam.ctypes.data_as(C.c_void_p),
                                                   C.byref(c)))
        return lam[: c.value].copy()

    def format_info(self) -> dict:
        """Slices of the stored pattern by column storage (int32, 16-bit offsets, offset
        table), stored value slots and the column bytes one product reads."""
        c = np.zeros(5, dtype=np.int64)
        self._check(self._L.podcg_get_format(self._h, c.ctypes.data_as(C.c_void_p)))
        return {"int32": int(c[0]), "offset16": int(c[1]), "table": int(c[2]), "slots": int(c[3]),
                "column_bytes": int(c[4])}

    def format_counts(self) -> dict:
        """Slices of the stored pattern by column storage (int32, 16-bit offsets, offset table)."""
        f = self.format_info()
        return {k: f[k] for k in ("int32", "offset16", "table")}

    def matvec(self, x: torch.Tensor, y: torch.Tensor):
        self._check(self._L.podcg_matvec(self._h, _ptr(x, torch.float64), _ptr(y, torch.float64)))

    def pattern_outer(self, u: torch.Tensor, v: torch.Tensor, scale: float,
                      out: torch.Tensor) -> torch.Tensor:
        """out[e] = scale * u[row(e)] * v[col(e)] on the stored CSR pattern."""
        self._check(self._L.podcg_pattern_outer(self._h, _ptr(u, torch.float64),
                                                _ptr(v, torch.float64), float(scale),
                                                _ptr(out, torch.float64)))
        return out

    # ------------------------------------------------------- three-stage method
    def ts_enable(self, **kw) -> dict:
        """Three-stage mode (Alg. 3); keyword options as in podcg_ts_options."""
        opt = L.TsOptions()
        self._L.podcg_ts_default_options(C.byref(opt))
        for k, v in kw.items():
            if k in ("weights",) and isinstance(v, str):
                v = {"rbf": 0, "previous": 1}[v]
            if k in ("stage3_gram",) and isinstance(v, str):
                v = {"blockdiag": 0, "exact": 1}[v]
            setattr(opt, k, v)
        self._check(self._L.podcg_ts_enable(self._h, C.byref(opt)))
        return opt.as_dict()

    def ts_solve(self, b: torch.Tensor, x: torch.Tensor, rtol: float) -> L.TsStats:
        st = L.TsStats()
        self._check(self._L.podcg_ts_solve(self._h, _ptr(b, torch.float64), _ptr(x, torch.float64),
                                           float(rtol), C.byref(st)))
        return st

    def ts_state(self):
        """(Y (n, m) tensor, stage-1 column list)."""
        m, w = C.c_int32(), C.c_int32()
        self._check(self._L.podcg_ts_get_state(self._h, None, C.byref(m), None, C.byref(w)))
        Y = torch.empty((max(m.value, 1), self.n), dtype=torch.float64, device="cuda")
        sel = (C.c_int32 * max(w.value, 1))()
        self._check(self._L.podcg_ts_get_state(self._h, _ptr(Y, torch.float64), C.byref(m), sel,
                                               C.byref(w)))
        return Y[:m.value].T, [sel[i] for i in range(w.value)]

    def ts_set_state(self, Y: torch.Tensor | None, sel, eta_acc=None):
        m = 0 if Y is None else Y.shape[1]
        Yc = None if Y is None else Y.T.contiguous()
        arr = (C.c_int32 * max(len(sel), 1))(*sel)
        eta = None
        if eta_acc is not None:
            eta = (C.c_double * m)(*[float(v) for v in eta_acc])
        self._check(self._L.podcg_ts_set_state(self._h, None if Yc is None else _ptr(Yc, torch.float64),
                                               m, arr, len(sel), eta))

    def stream_triad(self, a, b, c, s: float = 3.0, reps: int = 20) -> float:
        ms = C.c_double()
        self._check(self._L.podcg_stream_triad(self._h, _ptr(a, torch.float64),
                                               _ptr(b, torch.float64), _ptr(c, torch.float64),
                                               a.numel(), float(s), int(reps), C.byref(ms)))
        return ms.value


class PodCGBatch:
    """Independent sequences advanced together (podcg_batch_* of include/podcg.h).

    `members` are PodCG contexts (FP64); each keeps its own matrix, snapshots
    and basis and is still driven with set_matrix / push_snapshot / build_pod,
    or all at once with set_values / push_build.  solve() runs one system of
    every member in one batched loop."""

    def __init__(self, members, slices_per_item: int | None = None, rows_per_item: int | None = None,
                 grid: int | None = None, graph_iters: int | None = None,
                 check_every: int | None = None):
        self._L = L.load()
        self.members = list(members)
        opt = L.BatchOptions()
        self._L.podcg_batch_default_options(C.byref(opt))
        for k, v in (("slices_per_item", slices_per_item), ("rows_per_item", rows_per_item),
                     ("grid", grid), ("graph_iters", graph_iters), ("check_every", check_every)):
            if v is not None:
                setattr(opt, k, int(v))
        arr = (C.c_void_p * len(self.members))(*[m._h for m in self.members])
        h = C.c_void_p()
        rc = self._L.podcg_batch_create(C.byref(h), len(self.members), arr, C.byref(opt))
        if rc != 0:
            raise PodCGError(rc, self._L.podcg_strerror(rc).decode())
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.podcg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int) -> int:
        if rc < 0:
            raise PodCGError(rc, self._L.podcg_batch_last_error(self._h).decode())
        return rc

    def _arrays(self, bs, xs):
        if len(bs) != len(self.members) or len(xs) != len(self.members):
            raise ValueError("one b and one x per member")
        for m, b, x in zip(self.members, bs, xs):
            if b.numel() != m.n or x.numel() != m.n:
                raise ValueError("vector length differs from the member size")
        pb = (C.c_void_p * len(bs))(*[_ptr(b, torch.float64).value for b in bs])
        px = (C.c_void_p * len(xs))(*[_ptr(x, torch.float64).value for x in xs])
        return pb, px

    @property
    def options(self) -> dict:
        opt = L.BatchOptions()
        self._check(self._L.podcg_batch_get_options(self._h, C.byref(opt)))
        return opt.as_dict()

    def set_options(self, **kw):
        opt = L.BatchOptions()
        self._check(self._L.podcg_batch_get_options(self._h, C.byref(opt)))
        for k, v in kw.items():
            setattr(opt, k, int(v))
        self._check(self._L.podcg_batch_set_options(self._h, C.byref(opt)))

    def solve(self, bs, xs, rtol, plain: bool = False):
        """One system per member; returns (code, [Stats per member])."""
        pb, px = self._arrays(bs, xs)
        tol = rtol if hasattr(rtol, "__len__") else [rtol] * len(self.members)
        ptol = (C.c_double * len(self.members))(*[float(t) for t in tol])
        stats = (L.Stats * len(self.members))()
        rc = self._check(self._L.podcg_batch_solve(self._h, pb, px, ptol, 1 if plain else 0, stats))
        return rc, list(stats)

    def set_values(self, vals):
        """New CSR values for every member (same patterns), one batched ingest."""
        if len(vals) != len(self.members):
            raise ValueError("one value array per member")
        pv = (C.c_void_p * len(vals))(*[_ptr(v, torch.float64).value for v in vals])
        nz = (C.c_int64 * len(vals))(*[v.numel() for v in vals])
        return self._check(self._L.podcg_batch_set_values(self._h, nz, pv))

    def push_build(self, xs):
        """Push xs[m] as member m's newest snapshot and build every member's next
        basis, batched (returns without waiting for the GPU)."""
        if len(xs) != len(self.members):
            raise ValueError("one snapshot per member")
        for m, x in zip(self.members, xs):
            if x.numel() != m.n:
                raise ValueError("snapshot length differs from the member size")
        px = (C.c_void_p * len(xs))(*[_ptr(x, torch.float64).value for x in xs])
        return self._check(self._L.podcg_batch_push_build(self._h, px))

    def tune(self, bs, xs, iters: int = 32):
        """Autotune work-item sizes and grid; x is overwritten.  Returns (options, ms)."""
        pb, px = self._arrays(bs, xs)
        opt = L.BatchOptions()
        ms = C.c_double()
        self._check(self._L.podcg_batch_tune(self._h, pb, px, int(iters), C.byref(opt), C.byref(ms)))
        return opt.as_dict(), ms.value
