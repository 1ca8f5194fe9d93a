"""Python binding of libkry: argument marshalling only.

Every numerical step runs in the HIP library (libkry.so, built in-tree by
``paper_1707_00023_amd.build``).  PyTorch supplies device memory and the
current stream; this module only converts tensors to raw pointers, checks
shapes and dtypes, and turns status codes into exceptions.  There is no
fallback: if the library is missing, loading fails with an error.

Vector layout: a state vector has n = 6 nx ny nz entries, six planes
[Hx, Hy, Hz, Ex, Ey, Ez] each nz x ny x nx in C order.  Several vectors are
passed as a contiguous tensor of shape (ncols, n).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkry.so")

KRY_OK, KRY_EINVAL, KRY_ENOMEM, KRY_EHIP, KRY_ENOCONV = 0, -1, -2, -3, -4
_CODES = {KRY_EINVAL: "KRY_EINVAL", KRY_ENOMEM: "KRY_ENOMEM", KRY_EHIP: "KRY_EHIP",
          KRY_ENOCONV: "KRY_ENOCONV"}

EXPORTED = ("kry_create", "kry_destroy", "kry_last_error", "kry_size", "kry_apply",
            "kry_apply_f32", "kry_arnoldi", "kry_expv", "kry_solve_multifreq",
            "kry_stationary", "kry_grad", "kry_block_arnoldi", "kry_autotune",
            "kry_set_tune", "kry_arnoldi_noalloc", "kry_solve_restarted", "kry_solve_split2",
            "kry_autotune_sstep", "kry_grad_transient", "kry_column_stats", "kry_norm_series")


class KryGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("boundary", ctypes.c_int32)]


class KryOpts(ctypes.Structure):
    _fields_ = [("storage", ctypes.c_int32), ("krylov_dim", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("tol", ctypes.c_double),
                ("block_width", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("inner_product", ctypes.c_int32), ("stream", ctypes.c_void_p),
                ("timing", ctypes.c_int32), ("block_steps", ctypes.c_int32),
                ("block_steps_transient", ctypes.c_int32), ("verbose", ctypes.c_int32),
                ("orth", ctypes.c_int32), ("s_step", ctypes.c_int32),
                ("omega_continuation", ctypes.c_int32), ("transient_continuation", ctypes.c_int32),
                ("host_blocks", ctypes.c_int32)]


class KryStats(ctypes.Structure):
    _fields_ = [("matvecs_stationary", ctypes.c_int64), ("matvecs_transient", ctypes.c_int64),
                ("cycles_stationary", ctypes.c_int64), ("steps_transient", ctypes.c_int64),
                ("max_residual", ctypes.c_double), ("max_err_estimate", ctypes.c_double),
                ("ms_stationary", ctypes.c_double), ("ms_transient", ctypes.c_double),
                ("ms_total", ctypes.c_double), ("converged", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double * 6), ("kernel_launches", ctypes.c_int64 * 6),
                ("kernel_bytes", ctypes.c_double * 6), ("kernel_flops", ctypes.c_double * 6),
                ("kernel_launches_all", ctypes.c_int64 * 6), ("kernel_bytes_all", ctypes.c_double * 6)]

    def as_dict(self):
        out = {}
        for f, _ in self._fields_:
            v = getattr(self, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out


class KryColStats(ctypes.Structure):
    _fields_ = [("omega", ctypes.c_double), ("source", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("matvecs_stationary", ctypes.c_int64), ("matvecs_transient", ctypes.c_int64),
                ("steps_transient", ctypes.c_int64), ("residual", ctypes.c_double),
                ("err_estimate", ctypes.c_double), ("harmonic_norm", ctypes.c_double),
                ("ms_transient", ctypes.c_double), ("series_len", ctypes.c_int32),
                ("pad_", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "pad_"}


DEFAULT_S_STEP = 16

# operator: the Yee stencil (fused with the first Gram-Schmidt dots in the
# one-step Arnoldi, the polynomial-basis stencil in the s-step Arnoldi)
KERNEL_CLASSES = ("operator", "gs_update", "gs_dots", "combine", "block_gram", "block_gemm")


class KryTune(ctypes.Structure):
    _fields_ = [("cpt_stencil", ctypes.c_int32), ("cpt_update", ctypes.c_int32),
                ("cpt_dots", ctypes.c_int32), ("us_stencil", ctypes.c_double * 3),
                ("us_update", ctypes.c_double * 3), ("us_dots", ctypes.c_double * 3),
                ("zm_stencil", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("us_stencil_zm", ctypes.c_double * 3)]


class KryError(RuntimeError):
    def __init__(self, code, msg, stats=None):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code
        self.stats = stats


class NotConverged(KryError):
    """KRY_ENOCONV: a restart limit was reached.  The outputs of the call hold
    the library's best estimate; ``stats`` holds its residual statistics.
    Pass allow_noconv=True to a solver method to get the estimate back
    instead of this exception."""


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libkry.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libkry.so not found at {path}; build it with "
                           f"`python -m paper_1707_00023_amd.build`")
    lib = ctypes.CDLL(path)
    P, I32, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    lib.kry_create.argtypes = [ctypes.POINTER(KryGrid), P, P, P, ctypes.POINTER(KryOpts),
                               ctypes.POINTER(P)]
    lib.kry_create.restype = ctypes.c_int
    lib.kry_destroy.argtypes = [P]
    lib.kry_destroy.restype = None
    lib.kry_last_error.argtypes = [P]
    lib.kry_last_error.restype = ctypes.c_char_p
    lib.kry_size.argtypes = [P]
    lib.kry_size.restype = ctypes.c_int64
    lib.kry_apply.argtypes = [P, P, P, I32]
    lib.kry_apply_f32.argtypes = [P, P, P, I32]
    lib.kry_arnoldi.argtypes = [P, P, I32, P, P, ctypes.POINTER(D)]
    lib.kry_arnoldi_noalloc.argtypes = [P, P, I32, P, P, ctypes.POINTER(D)]
    lib.kry_arnoldi_noalloc.restype = ctypes.c_int
    lib.kry_expv.argtypes = [P, D, P, P, I32, ctypes.POINTER(KryStats)]
    lib.kry_solve_multifreq.argtypes = [P, P, I32, I32, P, I32, D, P, ctypes.POINTER(KryStats)]
    lib.kry_stationary.argtypes = [P, P, I32, I32, P, I32, P, ctypes.POINTER(KryStats)]
    lib.kry_solve_restarted.argtypes = [P, P, I32, I32, P, I32, D, P, ctypes.POINTER(KryStats)]
    lib.kry_solve_split2.argtypes = [P, P, I32, I32, P, I32, D, I32, P, ctypes.POINTER(KryStats)]
    lib.kry_grad.argtypes = [P, P, I32, P, I32, I32, ctypes.POINTER(D), P,
                             ctypes.POINTER(KryStats)]
    lib.kry_grad_transient.argtypes = [P, P, I32, P, I32, I32, D, ctypes.POINTER(D), P,
                                       ctypes.POINTER(KryStats)]
    lib.kry_column_stats.argtypes = [P, I32, ctypes.POINTER(KryColStats)]
    lib.kry_column_stats.restype = ctypes.c_int
    lib.kry_norm_series.argtypes = [P, I32, P, P, P, I32]
    lib.kry_norm_series.restype = ctypes.c_int
    lib.kry_block_arnoldi.argtypes = [P, P, I32, I32, P, P]
    lib.kry_block_arnoldi.restype = ctypes.c_int
    lib.kry_autotune.argtypes = [P, I32, ctypes.POINTER(KryTune)]
    lib.kry_autotune.restype = ctypes.c_int
    lib.kry_set_tune.argtypes = [P, ctypes.POINTER(KryTune)]
    lib.kry_set_tune.restype = ctypes.c_int
    lib.kry_autotune_sstep.argtypes = [P, P, I32, ctypes.POINTER(I32), P]
    lib.kry_autotune_sstep.restype = ctypes.c_int
    for name in ("kry_apply", "kry_apply_f32", "kry_arnoldi", "kry_expv",
                 "kry_solve_multifreq", "kry_stationary", "kry_grad", "kry_solve_restarted",
                 "kry_solve_split2", "kry_grad_transient"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class Options:
    storage: str = "f64"        # "f64" or "f32"
    krylov_dim: int = 30
    max_restarts: int = 0
    tol: float = 1e-8
    timing: int = 0  # 1 (or True): every launch timed; N > 1: one launch in N
    orth: str = "delayed"       # "delayed" (two basis sweeps per step) or "cgs2"
    block_width: int = 0        # > 1: batched form, groups of block_width/2 columns
    use_graph: bool = False     # replay captured Arnoldi cycles (HIP graphs)
    verbose: bool = False       # progress lines on stderr during long solves
    block_steps: int = 0        # batched shifted solves: block steps per restart (0 auto)
    block_steps_transient: int = 0  # batched exponential: block steps per restart (0 auto)
    # s-step Arnoldi block size (Chebyshev block orthogonalised as one
    # tall-skinny block; the block is FP64 with either storage); None: 16
    s_step: Optional[int] = None
    # per-frequency sources: start each shifted solve from the extrapolation
    # of the same source's solutions at earlier frequencies of the call
    omega_continuation: bool = False
    # continue each column's transient from the previous column of the same
    # source: e^{-TA} is applied to the difference of the two Im z only
    transient_continuation: bool = False
    # s-step blocks finished on the host (one synchronisation per
    # Gram-Schmidt pass) instead of on the device (one per restart cycle)
    host_blocks: bool = False


class Solver:
    """One libkry context: a grid with its materials on the current device."""

    def __init__(self, eps, mu=None, sigma=None, opts: Optional[Options] = None):
        import torch
        lib = load_library()
        opts = opts or Options()
        if eps.dim() != 3:
            raise ValueError("eps must be (nz, ny, nx)")
        nz, ny, nx = eps.shape
        dev = eps.device
        if dev.type != "cuda":
            raise ValueError("materials must be device tensors")
        keep = []
        def prep(t):
            if t is None:
                return None
            if tuple(t.shape) != (nz, ny, nx):
                raise ValueError("material shapes differ")
            t = t.to(device=dev, dtype=torch.float64).contiguous()
            keep.append(t)
            return t
        e, m, s = prep(eps), prep(mu), prep(sigma)
        self.grid = KryGrid(nx, ny, nz, 0)
        self.opts = KryOpts(1 if opts.storage == "f32" else 0, opts.krylov_dim,
                            opts.max_restarts, opts.tol, opts.block_width,
                            int(bool(opts.use_graph)), 0,
                            _stream_ptr().value,
                            int(opts.timing), opts.block_steps,
                            opts.block_steps_transient, int(bool(opts.verbose)),
                            1 if opts.orth == "cgs2" else 0,
                            int(opts.s_step if opts.s_step is not None else DEFAULT_S_STEP),
                            int(bool(opts.omega_continuation)),
                            int(bool(opts.transient_continuation)),
                            int(bool(opts.host_blocks)))
        self.storage = opts.storage
        ctx = ctypes.c_void_p()
        rc = lib.kry_create(ctypes.byref(self.grid), _ptr(e),
                            _ptr(m) if m is not None else None,
                            _ptr(s) if s is not None else None,
                            ctypes.byref(self.opts), ctypes.byref(ctx))
        if rc != KRY_OK:
            raise KryError(rc, lib.kry_last_error(None).decode())
        self._ctx = ctx
        self._lib = lib
        self.n = int(lib.kry_size(ctx))
        self.device = dev
        self.last_stats = None

    def close(self):
        if getattr(self, "_ctx", None):
            self._lib.kry_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow_noconv=False, stats=None):
        if rc == KRY_OK or (allow_noconv and rc == KRY_ENOCONV):
            return rc
        msg = self._lib.kry_last_error(self._ctx).decode()
        if rc == KRY_ENOCONV:
            raise NotConverged(rc, msg or "restart limit reached", stats)
        raise KryError(rc, msg, stats)

    def _vecs(self, x, dtype):
        import torch
        if x.dim() == 1:
            x = x.unsqueeze(0)
        if x.shape[-1] != self.n:
            raise ValueError(f"expected vectors of length {self.n}")
        if x.device != self.device:
            raise ValueError("tensor on the wrong device")
        return x.to(dtype).contiguous()

    def apply(self, v):
        """w = A v; v: (ncols, n) or (n,) float64 (float32 via apply_f32)."""
        import torch
        v = self._vecs(v, torch.float64)
        w = torch.empty_like(v)
        self._check(self._lib.kry_apply(self._ctx, _ptr(v), _ptr(w), v.shape[0]))
        return w

    def apply_f32(self, v):
        import torch
        v = self._vecs(v, torch.float32)
        w = torch.empty_like(v)
        self._check(self._lib.kry_apply_f32(self._ctx, _ptr(v), _ptr(w), v.shape[0]))
        return w

    def arnoldi(self, v, m: int):
        """(V (m+1, n), H (m+1, m) numpy, beta, steps) of m Arnoldi steps from v."""
        import numpy as np
        import torch
        v = self._vecs(v, torch.float64)[0]
        dt = torch.float32 if self.storage == "f32" else torch.float64
        V = torch.empty((m + 1, self.n), dtype=dt, device=self.device)
        H = np.zeros((m, m + 1))  # column-major (m+1) x m
        beta = ctypes.c_double()
        rc = self._lib.kry_arnoldi(self._ctx, _ptr(v), m, _ptr(V),
                                   H.ctypes.data_as(ctypes.c_void_p), ctypes.byref(beta))
        if rc < 0:
            self._check(rc)
        return V, H.T.copy(), beta.value, rc

    def autotune(self, cache: Optional[str] = None, cnt: int = 0,
                 s_candidates: Optional[Sequence[int]] = None):
        """Choose the kernels' launch shapes, and with `s_candidates` the
        s-step block size, by timing them on this grid.

        With `cache` (a JSON path) a measured choice is reused for the same
        grid, storage, Krylov dimension, block width and GPU architecture,
        and new measurements are added to it.  Returns the choice as a dict.
        """
        import json
        import numpy as np
        import torch
        arch = getattr(torch.cuda.get_device_properties(self.device), "gcnArchName", "gpu")
        key = (f"{self.grid.nx}x{self.grid.ny}x{self.grid.nz}-{self.storage}-"
               f"m{self.opts.krylov_dim}-p{self.opts.block_width}-c{cnt}-{arch}")
        table = {}
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)

        def tune_s(cands):
            cand = np.ascontiguousarray(np.asarray(cands, dtype=np.int32))
            us = np.zeros(cand.size)
            best = ctypes.c_int32()
            self._check(self._lib.kry_autotune_sstep(self._ctx, cand.ctypes.data_as(ctypes.c_void_p),
                                                      int(cand.size), ctypes.byref(best),
                                                      us.ctypes.data_as(ctypes.c_void_p)))
            return int(best.value), [float(x) for x in us]

        t = KryTune()
        if key in table and (s_candidates is None or "s_step" in table[key]):
            e = table[key]
            t.cpt_stencil, t.cpt_update, t.cpt_dots = e["cpt_stencil"], e["cpt_update"], e["cpt_dots"]
            t.zm_stencil = e.get("zm_stencil", 0)
            self._check(self._lib.kry_set_tune(self._ctx, ctypes.byref(t)))
            if s_candidates is not None:
                tune_s([e["s_step"]])  # applies the cached block size
            return dict(e, cached=True)
        self._check(self._lib.kry_autotune(self._ctx, int(cnt), ctypes.byref(t)))
        e = {"cpt_stencil": t.cpt_stencil, "cpt_update": t.cpt_update, "cpt_dots": t.cpt_dots,
             "us_stencil": list(t.us_stencil), "us_update": list(t.us_update),
             "us_dots": list(t.us_dots), "zm_stencil": t.zm_stencil,
             "us_stencil_zm": list(t.us_stencil_zm)}
        if s_candidates is not None:
            e["s_step"], e["us_cycle"] = tune_s(s_candidates)
            e["s_candidates"] = [int(x) for x in s_candidates]
        if cache:
            table[key] = e
            d = os.path.dirname(os.path.abspath(cache))
            os.makedirs(d, exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return dict(e, cached=False)

    def set_tune(self, cpt_stencil: int = 1, cpt_update: int = 1, cpt_dots: int = 1,
                 zm_stencil: int = 0):
        """Apply launch shapes: cells per thread of the operator, update and
        dot kernels (1, 2 or 4), and the z-marching form of the s-step basis
        stencil (planes per workgroup 4, 8 or 16; 0: cell-parallel)."""
        t = KryTune()
        t.cpt_stencil, t.cpt_update, t.cpt_dots, t.zm_stencil = cpt_stencil, cpt_update, cpt_dots, zm_stencil
        self._check(self._lib.kry_set_tune(self._ctx, ctypes.byref(t)))

    def block_arnoldi(self, V0, mb: int):
        """(V ((mb+1) p, n), H ((mb+1) p, mb p) numpy, block steps) from the block V0 (p, n)."""
        import numpy as np
        import torch
        V0 = self._vecs(V0, torch.float64)
        p = V0.shape[0]
        dt = torch.float32 if self.storage == "f32" else torch.float64
        V = torch.empty(((mb + 1) * p, self.n), dtype=dt, device=self.device)
        H = np.zeros((mb * p, (mb + 1) * p))  # column-major ((mb+1)p) x (mb p)
        rc = self._lib.kry_block_arnoldi(self._ctx, _ptr(V0), p, mb, _ptr(V),
                                         H.ctypes.data_as(ctypes.c_void_p))
        if rc < 0:
            self._check(rc)
        return V, H.T.copy(), rc

    def expv(self, t: float, v, allow_noconv: bool = False):
        """e^{-tA} v for each row of v."""
        import torch
        v = self._vecs(v, torch.float64)
        y = torch.empty_like(v)
        st = KryStats()
        rc = self._lib.kry_expv(self._ctx, float(t), _ptr(v), _ptr(y), v.shape[0], ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return y

    def _omega_b(self, omegas, b, b_per_omega):
        import numpy as np
        import torch
        om = np.ascontiguousarray(np.asarray(omegas, dtype=np.float64).reshape(-1))
        b = self._vecs(b, torch.complex128)
        nw = om.size
        if b_per_omega:
            if b.shape[0] % nw:
                raise ValueError("b rows must be n_omega * n_src")
            nsrc = b.shape[0] // nw
        else:
            nsrc = b.shape[0]
        return om, b, nw, nsrc

    def stationary(self, omegas: Sequence[float], b, b_per_omega: bool = False,
                   allow_noconv: bool = False):
        """z = (A + i w I)^-1 b; returns complex128 (n_omega * n_src, n)."""
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        z = torch.empty((nw * nsrc, self.n), dtype=torch.complex128, device=self.device)
        st = KryStats()
        rc = self._lib.kry_stationary(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, nsrc,
                                      _ptr(b), int(bool(b_per_omega)), _ptr(z), ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return z

    def solve_multifreq(self, omegas: Sequence[float], b, T: float, b_per_omega: bool = False,
                        allow_noconv: bool = False):
        """y(T) for every (omega, source) column; float64 (n_omega * n_src, n)."""
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        y = torch.empty((nw * nsrc, self.n), dtype=torch.float64, device=self.device)
        st = KryStats()
        rc = self._lib.kry_solve_multifreq(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, nsrc,
                                           _ptr(b), int(bool(b_per_omega)), float(T), _ptr(y),
                                           ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return y

    def solve_restarted(self, omegas: Sequence[float], b, T: float, b_per_omega: bool = False,
                        allow_noconv: bool = False):
        """y(T) for every (omega, source) column by the residual-restarted
        Krylov method (no shifted solve); same conventions as solve_multifreq."""
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        y = torch.empty((nw * nsrc, self.n), dtype=torch.float64, device=self.device)
        st = KryStats()
        rc = self._lib.kry_solve_restarted(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, nsrc,
                                           _ptr(b), int(bool(b_per_omega)), float(T), _ptr(y),
                                           ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return y

    def solve_split2(self, omegas: Sequence[float], b, T: float, periods: int = 1,
                     b_per_omega: bool = False, allow_noconv: bool = False):
        """y(T) for every (omega, source) column by source splitting over
        subintervals of `periods` source periods; conventions as solve_multifreq."""
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        y = torch.empty((nw * nsrc, self.n), dtype=torch.float64, device=self.device)
        st = KryStats()
        rc = self._lib.kry_solve_split2(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, nsrc,
                                        _ptr(b), int(bool(b_per_omega)), float(T), int(periods),
                                        _ptr(y), ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return y

    def grad(self, omegas: Sequence[float], b, plane_k: int, b_per_omega: bool = False,
             loss_only: bool = False, allow_noconv: bool = False):
        """(L, dL/d eps) of the period-averaged flux through plane z = plane_k.

        b: complex128 (1, n) shared source or (n_omega, n) per-omega sources.
        Returns the loss (float) and dL/d eps as a float64 (nz, ny, nx) tensor.
        """
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        if nsrc != 1:
            raise ValueError("one source per frequency (or one shared source)")
        g = None if loss_only else torch.empty((self.grid.nz, self.grid.ny, self.grid.nx),
                                               dtype=torch.float64, device=self.device)
        loss = ctypes.c_double()
        st = KryStats()
        rc = self._lib.kry_grad(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, _ptr(b),
                                int(bool(b_per_omega)), int(plane_k), ctypes.byref(loss),
                                None if g is None else _ptr(g), ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return loss.value, g

    def column_stats(self, col: int):
        """Per-column record of the last solve_multifreq call (single-vector
        path): frequency, source, operator applications of its shifted-solve
        group and of its transient, restarts in time, true shifted residual,
        transient error estimate, |Im(e^{iwT} z)|_M, wall time."""
        out = KryColStats()
        self._check(self._lib.kry_column_stats(self._ctx, int(col), ctypes.byref(out)))
        return out.as_dict()

    def norm_series(self, col: int):
        """(t, |y_hat(t)|_M, ms per restart) of column col's transient in the
        last solve_multifreq call, as numpy arrays (the last sample is T)."""
        import numpy as np
        n = self._lib.kry_norm_series(self._ctx, int(col), None, None, None, 0)
        if n < 0:
            self._check(n)
        t, nrm, ms = (np.zeros(n) for _ in range(3))
        self._lib.kry_norm_series(self._ctx, int(col), t.ctypes.data_as(ctypes.c_void_p),
                                  nrm.ctypes.data_as(ctypes.c_void_p), ms.ctypes.data_as(ctypes.c_void_p), n)
        return t, nrm, ms

    def grad_transient(self, omegas: Sequence[float], b, plane_k: int, T: float,
                       b_per_omega: bool = False, loss_only: bool = False,
                       allow_noconv: bool = False):
        """(L, dL/d eps) of the instantaneous flux through plane z = plane_k of
        the whole field at time T (time-harmonic part minus the transient).

        b: complex128 (1, n) shared source or (n_omega, n) per-omega sources.
        Returns the loss (float) and dL/d eps as a float64 (nz, ny, nx) tensor.
        """
        import torch
        om, b, nw, nsrc = self._omega_b(omegas, b, b_per_omega)
        if nsrc != 1:
            raise ValueError("one source per frequency (or one shared source)")
        g = None if loss_only else torch.empty((self.grid.nz, self.grid.ny, self.grid.nx),
                                               dtype=torch.float64, device=self.device)
        loss = ctypes.c_double()
        st = KryStats()
        rc = self._lib.kry_grad_transient(self._ctx, om.ctypes.data_as(ctypes.c_void_p), nw, _ptr(b),
                                          int(bool(b_per_omega)), int(plane_k), float(T),
                                          ctypes.byref(loss), None if g is None else _ptr(g),
                                          ctypes.byref(st))
        self.last_stats = st.as_dict()
        self._check(rc, allow_noconv, self.last_stats)
        return loss.value, g


def _flux_function():
    import torch

    class FluxLoss(torch.autograd.Function):
        """L(eps) = transmitted period-averaged power; backward by the adjoint."""

        @staticmethod
        def forward(ctx, eps, sigma, b, omegas, plane_k, opts, b_per_omega):
            # the forward and adjoint solves must both converge: an
            # unconverged adjoint would hand autograd a wrong gradient, so
            # KRY_ENOCONV raises NotConverged here
            solver = Solver(eps.detach(), None, sigma, opts)
            try:
                L, g = solver.grad(omegas, b, plane_k, b_per_omega)
            finally:
                solver.close()
            ctx.save_for_backward(g)
            return torch.tensor(L, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None, None, None, None, None

    return FluxLoss


def flux_loss(eps, sigma, b, omegas, plane_k, opts: Optional[Options] = None,
              b_per_omega: bool = False):
    """Differentiable transmitted power (torch.autograd) w.r.t. per-cell eps."""
    return _flux_function().apply(eps, sigma, b, omegas, plane_k, opts or Options(),
                                  b_per_omega)


def _flux_at_function():
    import torch

    class FluxAtT(torch.autograd.Function):
        """L(eps) = instantaneous flux of the field at time T; backward by the
        adjoint of the shifted solves and of the exponential."""

        @staticmethod
        def forward(ctx, eps, sigma, b, omegas, plane_k, T, opts, b_per_omega):
            solver = Solver(eps.detach(), None, sigma, opts)
            try:
                L, g = solver.grad_transient(omegas, b, plane_k, T, b_per_omega)
            finally:
                solver.close()
            ctx.save_for_backward(g)
            return torch.tensor(L, dtype=torch.float64, device=eps.device)

        @staticmethod
        def backward(ctx, grad_out):
            (g,) = ctx.saved_tensors
            return grad_out * g, None, None, None, None, None, None, None

    return FluxAtT


def flux_loss_at(eps, sigma, b, omegas, plane_k, T, opts: Optional[Options] = None,
                 b_per_omega: bool = False):
    """Differentiable flux of the field at time T (transient included),
    w.r.t. per-cell eps."""
    return _flux_at_function().apply(eps, sigma, b, omegas, plane_k, T, opts or Options(),
                                     b_per_omega)
