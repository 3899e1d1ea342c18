"""Thin ctypes binding of liblsw.so (the C ABI declared in include/lsw.h).

PyTorch provides device memory and the stream; every step of the setup, the
preconditioner and the Krylov solve runs in the library's HIP kernels and C++ runtime.
There is no CPU fallback: importing this module without the built library, or calling
it without a GPU, raises.

    Solver(m_ext, omega, h, n, n_pml, q, r, ...)   lsw_setup  (Setup + Factorise, Sec. 3)
    Solver.apply(r)                                 lsw_apply  (z = M^-1 r, Alg. Scenario3 / scenario 4)
    Solver.solve(f)                                 lsw_solve  (FGMRES, Sec. 3 Phase 3)
    Solver.adjoint(g)                               lsw_adjoint (A^H v = g via A = A^T)
    Solver.matvec(x)                                lsw_matvec (y = A x)
    HelmholtzSolve.apply(m_bulk, f, ...)           autograd: u = A(m)^-1 f with the adjoint gradient
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "liblsw.so")

LSW_OK, LSW_EINVAL, LSW_ENOMEM, LSW_EHIP, LSW_ESINGULAR, LSW_ENAN, LSW_ENOCONV = 0, -1, -2, -3, -4, -5, -6
LSW_FP64, LSW_MIXED = 0, 1
LSW_SWEEP_COMPRESSED, LSW_SWEEP_CHAIN = 0, 1
_NAMES = {0: "LSW_OK", -1: "LSW_EINVAL", -2: "LSW_ENOMEM", -3: "LSW_EHIP", -4: "LSW_ESINGULAR",
          -5: "LSW_ENAN", -6: "LSW_ENOCONV"}
EXPORTS = ("lsw_setup", "lsw_apply", "lsw_apply_noalloc", "lsw_solve", "lsw_adjoint", "lsw_matvec",
           "lsw_mass_gradient", "lsw_query", "lsw_last_error", "lsw_destroy")
NOALLOC_SCRATCH_BYTES = 64 << 20   # LSW_NOALLOC_SCRATCH_BYTES


class lsw_grid_t(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("n", ctypes.c_int * 3), ("n_pml", ctypes.c_int * 3)]


class lsw_cdd_t(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("r", ctypes.c_int), ("windows", ctypes.c_int), ("shift", ctypes.c_int * 2)]


class lsw_pml_t(ctypes.Structure):
    _fields_ = [("C", ctypes.c_double), ("n_pml_local", ctypes.c_int)]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
RELEASE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)


class lsw_opts_t(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("restart", ctypes.c_int), ("maxit", ctypes.c_int),
                ("tol", ctypes.c_double), ("nrhs_max", ctypes.c_int), ("stream", ctypes.c_void_p),
                ("sweep_mode", ctypes.c_int), ("alloc", ALLOC_FN), ("release", RELEASE_FN),
                ("alloc_ctx", ctypes.c_void_p)]


class lsw_rhs_info_t(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int), ("converged", ctypes.c_int), ("relres", ctypes.c_double)]


class lsw_info_t(ctypes.Structure):
    _fields_ = [("h_rhs", ctypes.POINTER(lsw_rhs_info_t)), ("h_history", ctypes.POINTER(ctypes.c_double)),
                ("history_len", ctypes.c_int), ("t_solve_ms", ctypes.c_double), ("applies", ctypes.c_int)]


class lsw_stats_t(ctypes.Structure):
    _fields_ = [("q", ctypes.c_int), ("r", ctypes.c_int), ("n_subdomains", ctypes.c_int),
                ("W_max", ctypes.c_int), ("H_max", ctypes.c_int), ("N", ctypes.c_longlong),
                ("factor_elems", ctypes.c_longlong), ("factor_elem_bytes", ctypes.c_int),
                ("solves_per_apply", ctypes.c_int), ("fronts_per_apply", ctypes.c_int),
                ("apply_chain_bytes", ctypes.c_double), ("apply_gemv_bytes", ctypes.c_double),
                ("chain_launches", ctypes.c_int), ("gemv_launches", ctypes.c_int), ("q_elems", ctypes.c_longlong),
                ("factor_flops", ctypes.c_double), ("t_setup_ms", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("t_q_ms", ctypes.c_double), ("last_apply_ms", ctypes.c_double),
                ("last_chain_ms", ctypes.c_double), ("last_gemv_ms", ctypes.c_double),
                ("apply_stage1_bytes", ctypes.c_double), ("apply_final_bytes", ctypes.c_double),
                ("last_stage1_ms", ctypes.c_double), ("last_final_ms", ctypes.c_double),
                ("last_final_rhs_ms", ctypes.c_double), ("rhs_per_workgroup", ctypes.c_int),
                ("tune_ms", ctypes.c_double * 5), ("symmetric_factors", ctypes.c_int),
                ("packed_factor_elems", ctypes.c_longlong), ("gemv_items", ctypes.c_int),
                ("gemv_max_inputs", ctypes.c_int), ("cdd_count", ctypes.c_int), ("window_shift", ctypes.c_int * 2),
                ("last_dom_ms", ctypes.c_double), ("dom_launches", ctypes.c_int), ("dom_bytes", ctypes.c_double),
                ("noalloc_bytes", ctypes.c_longlong), ("sym_threads", ctypes.c_int),
                ("sym_tiles_per_lane", ctypes.c_int), ("sym_ring", ctypes.c_int), ("sym_lanes_per_row", ctypes.c_int),
                ("sym_shapes_timed", ctypes.c_int), ("sym_tune_best_ms", ctypes.c_double),
                ("sym_tune_worst_ms", ctypes.c_double), ("apply_stage1_full_bytes", ctypes.c_double),
                ("apply_final_full_bytes", ctypes.c_double), ("gemv_mma", ctypes.c_int),
                ("gemv_tune_ms", ctypes.c_double * 2)]


_lib = None


def library_path() -> str:
    return _LIB_PATH


def load_library() -> ctypes.CDLL:
    """Loads liblsw.so (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with `python -m paper_1909_01467_amd.build`")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, dp, ip = ctypes.c_void_p, ctypes.c_double, ctypes.c_int
    lib.lsw_setup.argtypes = [ctypes.POINTER(vp), vp, dp, dp, ctypes.POINTER(lsw_grid_t),
                              ctypes.POINTER(lsw_cdd_t), ctypes.POINTER(lsw_pml_t), ctypes.POINTER(lsw_opts_t)]
    lib.lsw_apply.argtypes = [vp, vp, vp, ip]
    lib.lsw_apply_noalloc.argtypes = [vp, vp, vp, ip]
    lib.lsw_solve.argtypes = [vp, vp, vp, ip, ctypes.POINTER(lsw_info_t)]
    lib.lsw_adjoint.argtypes = [vp, vp, vp, ip, ctypes.POINTER(lsw_info_t)]
    lib.lsw_matvec.argtypes = [vp, vp, vp, ip]
    lib.lsw_mass_gradient.argtypes = [vp, vp, vp, ip, vp]
    lib.lsw_query.argtypes = [vp, ctypes.POINTER(lsw_stats_t)]
    lib.lsw_last_error.argtypes = [vp]
    lib.lsw_last_error.restype = ctypes.c_char_p
    lib.lsw_destroy.argtypes = [vp]
    for name in EXPORTS:
        if name != "lsw_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class LswError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def extend_medium(m_bulk: torch.Tensor, n_pml) -> torch.Tensor:
    """Normal (constant) extension of the squared slowness into the PML (Sec. 1.1), as a
    differentiable gather: every PML point copies its nearest bulk point.  m_bulk is [y, x]
    or [z, y, x]; n_pml is one width or one per physical axis (x, y[, z])."""
    d = m_bulk.dim()
    ps = (n_pml,) * d if isinstance(n_pml, int) else tuple(n_pml)
    out = m_bulk
    for axis in range(d):                      # array axis; physical axis d - 1 - axis
        n, p = m_bulk.shape[axis], ps[d - 1 - axis]
        idx = torch.clamp(torch.arange(n + 2 * p, device=m_bulk.device) - p, 0, n - 1)
        out = torch.index_select(out, axis, idx)
    return out


def _dptr(t: torch.Tensor) -> int:
    if not t.is_cuda:
        raise ValueError("device tensor required")
    if t.is_conj() or t.is_neg():
        raise ValueError("lazy conjugate/negative views must be resolved before passing raw pointers")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor required")
    return t.data_ptr()


class Solver:
    """A set-up and factorised L-sweeps preconditioner with its GMRES solver (one lsw handle).

    windows=True selects scenario 4 (Sec. 2.1): the CDD and three shifted copies, each sweeping
    the right-hand side times its window of a partition of unity; `shift` is then the shift of
    the copies along (x, y) ((0, 0): half of the smallest group).  Without windows `shift`
    shifts this CDD's own interior boundaries.

    torch_allocator=True places the handle's whole device workspace in PyTorch's caching
    allocator (on the solver's stream) instead of hipMalloc."""

    def __init__(self, m_ext: torch.Tensor, omega: float, h: float, n, n_pml, q: int, r: int | None = None,
                 C: float | None = None, n_pml_local: int | None = None, precision: str = "fp64",
                 restart: int = 50, maxit: int = 500, tol: float = 1e-6, nrhs_max: int = 1,
                 sweep_mode: str = "compressed", windows: bool = False, shift=(0, 0),
                 torch_allocator: bool = False):
        lib = load_library()
        if not torch.cuda.is_available():
            raise RuntimeError("the L-sweeps library needs a GPU")
        dim = m_ext.dim()
        if dim not in (2, 3):
            raise ValueError("m must be a 2D [y, x] or 3D [z, y, x] array on the extended grid")
        ns = (n,) * dim if isinstance(n, int) else tuple(n)
        ps = (n_pml,) * dim if isinstance(n_pml, int) else tuple(n_pml)
        r = q if r is None else r
        m_ext = m_ext.to(device="cuda", dtype=torch.float64).contiguous()
        expect = tuple(ns[k] + 2 * ps[k] for k in reversed(range(dim)))
        if tuple(m_ext.shape) != expect:
            raise ValueError(f"m must be on the extended grid {expect}, got {tuple(m_ext.shape)}")
        self.dim = dim
        self.shape = tuple(m_ext.shape)
        self.N = m_ext.numel()
        self.omega, self.h, self.n, self.n_pml, self.q, self.r = omega, h, ns, ps, q, r
        self.nrhs_max = nrhs_max
        self.C = 16.0 * math.log(omega) if C is None else C
        self.precision = precision
        grid = lsw_grid_t(dim, (ctypes.c_int * 3)(*ns, *([0] * (3 - dim))), (ctypes.c_int * 3)(*ps, *([0] * (3 - dim))))
        cdd = lsw_cdd_t(q, r, 1 if windows else 0, (ctypes.c_int * 2)(*shift))
        pml = lsw_pml_t(self.C, -1 if n_pml_local is None else n_pml_local)
        self.stream = torch.cuda.current_stream()
        if sweep_mode not in ("compressed", "chain"):
            raise ValueError("sweep_mode is 'compressed' or 'chain'")
        opts = lsw_opts_t(LSW_MIXED if precision == "mixed" else LSW_FP64, restart, maxit, tol, nrhs_max,
                          ctypes.c_void_p(self.stream.cuda_stream),
                          LSW_SWEEP_CHAIN if sweep_mode == "chain" else LSW_SWEEP_COMPRESSED)
        if torch_allocator:
            stream = self.stream

            def _alloc(nbytes, _ctx):
                try:
                    return torch.cuda.caching_allocator_alloc(nbytes, stream=stream)
                except Exception:   # out of memory: the library reports LSW_ENOMEM
                    return None

            def _release(ptr, _ctx):
                try:
                    torch.cuda.caching_allocator_delete(ptr)
                except Exception:
                    pass

            # the callbacks must outlive the handle (lsw_destroy calls release)
            self._callbacks = (ALLOC_FN(_alloc), RELEASE_FN(_release))
            opts.alloc, opts.release = self._callbacks
        handle = ctypes.c_void_p()
        torch.cuda.synchronize()
        rc = lib.lsw_setup(ctypes.byref(handle), ctypes.c_void_p(_dptr(m_ext)), omega, h, ctypes.byref(grid),
                           ctypes.byref(cdd), ctypes.byref(pml), ctypes.byref(opts))
        if rc != LSW_OK:
            raise LswError(rc, lib.lsw_last_error(None).decode())
        self._h = handle
        self._lib = lib

    # ------------------------------------------------------------------ helpers
    def _check(self, rc: int, allow_noconv: bool = False):
        if rc == LSW_OK or (allow_noconv and rc == LSW_ENOCONV):
            return
        raise LswError(rc, self._lib.lsw_last_error(self._h).decode())

    def _handle(self):
        if not getattr(self, "_h", None):
            raise RuntimeError("this Solver was closed")
        return self._h

    def _vec(self, x: torch.Tensor) -> tuple[torch.Tensor, int, bool]:
        single = x.dim() == 1 or tuple(x.shape) == self.shape
        x = x.to(device="cuda", dtype=torch.complex128).resolve_conj().resolve_neg()
        x = x.reshape(-1 if single else x.shape[0], self.N).contiguous()
        if single:
            x = x.reshape(1, self.N)
        if x.shape[0] > self.nrhs_max:
            raise ValueError(f"at most nrhs_max={self.nrhs_max} right-hand sides")
        return x, x.shape[0], single

    def _out(self, y: torch.Tensor, single: bool) -> torch.Tensor:
        return y.reshape(self.shape) if single else y.reshape(y.shape[0], *self.shape)

    # ------------------------------------------------------------------ API
    def apply(self, r: torch.Tensor) -> torch.Tensor:
        r, k, single = self._vec(r)
        z = torch.empty_like(r)
        self._check(self._lib.lsw_apply(self._handle(), ctypes.c_void_p(_dptr(r)), ctypes.c_void_p(_dptr(z)), k))
        return self._out(z, single)

    def apply_noalloc(self, r: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """lsw_apply_noalloc: the same z = M^-1 r with the library's scratch in its per-GPU static
        array (no device allocation inside the call); queued on the solver's stream.  `out`, when
        given, receives z (complex128, contiguous, the shape of r)."""
        r, k, single = self._vec(r)
        z = torch.empty_like(r) if out is None else out.reshape(k, self.N)
        self._check(self._lib.lsw_apply_noalloc(self._handle(), ctypes.c_void_p(_dptr(r)), ctypes.c_void_p(_dptr(z)), k))
        return self._out(z, single)

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        x, k, single = self._vec(x)
        y = torch.empty_like(x)
        self._check(self._lib.lsw_matvec(self._handle(), ctypes.c_void_p(_dptr(x)), ctypes.c_void_p(_dptr(y)), k))
        return self._out(y, single)

    def _krylov(self, fn, b, u0, history):
        b, k, single = self._vec(b)
        u = torch.zeros_like(b) if u0 is None else self._vec(u0)[0].clone()
        rhs = (lsw_rhs_info_t * k)()
        hist = (ctypes.c_double * (k * history))() if history else None
        info = lsw_info_t(rhs, hist, history, 0.0, 0)
        rc = fn(self._handle(), ctypes.c_void_p(_dptr(b)), ctypes.c_void_p(_dptr(u)), k, ctypes.byref(info))
        self._check(rc, allow_noconv=True)
        out = {"iterations": [rhs[s].iterations for s in range(k)],
               "converged": [bool(rhs[s].converged) for s in range(k)],
               "relres": [rhs[s].relres for s in range(k)],
               "t_solve_ms": info.t_solve_ms, "applies": info.applies}
        if history:
            out["history"] = [[hist[s * history + t] for t in range(history)] for s in range(k)]
        return self._out(u, single), out

    def solve(self, f: torch.Tensor, u0: torch.Tensor | None = None, history: int = 0):
        """u = A^-1 f by FGMRES + L-sweeps; returns (u, info)."""
        return self._krylov(self._lib.lsw_solve, f, u0, history)

    def adjoint(self, g: torch.Tensor, v0: torch.Tensor | None = None, history: int = 0):
        """v = A^-H g with the same factorisation (A = A^T); returns (v, info)."""
        return self._krylov(self._lib.lsw_adjoint, g, v0, history)

    def mass_gradient(self, lam: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
        """omega^2 Re(sum_s lam_s * u_s / (alpha_x alpha_y)) on the extended grid."""
        lam, k, _ = self._vec(lam)
        u, k2, _ = self._vec(u)
        assert k == k2
        g = torch.zeros(self.shape, dtype=torch.float64, device="cuda")
        self._check(self._lib.lsw_mass_gradient(self._handle(), ctypes.c_void_p(_dptr(lam)), ctypes.c_void_p(_dptr(u)),
                                                k, ctypes.c_void_p(_dptr(g))))
        return g

    def stats(self) -> dict:
        st = lsw_stats_t()
        self._check(self._lib.lsw_query(self._handle(), ctypes.byref(st)))
        out = {name: getattr(st, name) for name, _ in lsw_stats_t._fields_}
        out["tune_ms"] = list(out["tune_ms"])
        out["window_shift"] = list(out["window_shift"])
        out["gemv_tune_ms"] = list(out["gemv_tune_ms"])
        return out

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lsw_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _require_converged(solver: Solver, info: dict, what: str) -> None:
    """A gradient built from an unconverged state or adjoint field is wrong without any sign of it,
    so the autograd path refuses it (the plain Solver API reports LSW_ENOCONV through `info`)."""
    bad = [k for k, ok in enumerate(info["converged"]) if not ok]
    if bad:
        solver.close()
        raise LswError(LSW_ENOCONV, f"{what} did not reach tol for right-hand sides {bad} "
                                    f"(relative residuals {[info['relres'][k] for k in bad]})")


class HelmholtzSolve(torch.autograd.Function):
    """u = A(m)^-1 f on the extended grid, differentiable in the bulk squared slowness m
    and in f.  Backward (adjoint state, A = A^T): lam = A^-H g_u solved with the same
    factorisation; grad_f = lam; grad_m(ext) = omega^2 Re(conj(lam) * u / (alpha_x alpha_y))
    folded onto the bulk by the autograd of the normal extension."""

    @staticmethod
    def forward(ctx, m_ext, f, solver_kwargs):
        kw = dict(solver_kwargs)
        solver = Solver(m_ext.detach(), **kw)
        u, info = solver.solve(f.detach())
        _require_converged(solver, info, "forward solve")
        ctx.solver = solver
        ctx.f_shape = f.shape
        ctx.save_for_backward(u)
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, g_u):
        (u,) = ctx.saved_tensors
        solver = ctx.solver
        lam, info = solver.adjoint(g_u.contiguous())
        _require_converged(solver, info, "adjoint solve")
        grad_m = solver.mass_gradient(torch.conj_physical(lam), u) if ctx.needs_input_grad[0] else None
        grad_f = lam.reshape(ctx.f_shape) if ctx.needs_input_grad[1] else None
        # the handle stays open: a graph kept with retain_graph may be differentiated again; it is
        # released with the graph (Solver.__del__)
        return grad_m, grad_f, None
