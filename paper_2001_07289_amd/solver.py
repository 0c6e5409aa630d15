"""Python face of the BDDC-SO library: the same calls as the C ABI.

Every numeric step runs in the HIP library; this module only moves pointers,
sizes and streams.  PyTorch provides device memory and the current stream.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional, Sequence

import numpy as np
import torch

from . import _binding as B


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor) -> C.c_void_p:
    return C.c_void_p(t.data_ptr())


def _f64_cuda(t: torch.Tensor, name: str) -> torch.Tensor:
    if not (t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise TypeError(f"{name} must be a contiguous float64 CUDA tensor")
    return t


def copy_probe(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    """Streaming copy of src into dst (same byte size) by the library's copy kernel."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("src and dst sizes differ")
    B.check(B.load().bddcso_copy_probe(_ptr(src), _ptr(dst), nbytes, _stream(stream)))


def default_options(**kw) -> B.Options:
    o = B.Options()
    B.load().bddcso_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Problem:
    """Mesh, partitions and interface classification (bddcso_problem_create)."""

    def __init__(self, dim: int, n_el: Sequence[int], h: Sequence[float], elem_sub, elem_subsub):
        lib = B.load()
        ne = (C.c_int64 * 3)(*(list(n_el) + [1] * (3 - len(n_el))))
        hh = (C.c_double * 3)(*(list(h) + [1.0] * (3 - len(h))))
        es = np.ascontiguousarray(elem_sub, dtype=np.int32)
        ess = np.ascontiguousarray(elem_subsub, dtype=np.int32)
        n_elem = int(np.prod(n_el))
        if es.size != n_elem or ess.size != n_elem:
            raise ValueError("elem_sub / elem_subsub must have one entry per element")
        out = C.c_void_p()
        B.check(lib.bddcso_problem_create(dim, ne, hh, es.ctypes.data_as(C.POINTER(C.c_int32)),
                                          ess.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(out)))
        self._h = out
        self.dim = dim
        self.n_el = tuple(int(n) for n in n_el)
        self.n_elements = n_elem

    @classmethod
    def from_workload(cls, p) -> "Problem":
        return cls(p.dim, p.n_el, p.h, p.elem_sub, p.elem_subsub)

    def info(self, primal_mask: int = 7) -> dict:
        nf, ng, nc = C.c_int64(), C.c_int64(), C.c_int64()
        ns = C.c_int()
        cnt = (C.c_int64 * 3)()
        B.check(B.load().bddcso_problem_info(self._h, primal_mask, C.byref(nf), C.byref(ng), C.byref(nc),
                                             C.byref(ns), cnt))
        return {"n_free": nf.value, "n_gamma": ng.value, "n_coarse": nc.value, "n_sub": ns.value,
                "counts": {"v": cnt[0], "e": cnt[1], "f": cnt[2]}}

    @property
    def n_free(self) -> int:
        return self.info()["n_free"]

    def plan_stats(self, options: Optional[B.Options] = None, **kw) -> dict:
        o = options if options is not None else default_options(**kw)
        st = B.PlanStats()
        B.check(B.load().bddcso_plan_info(self._h, C.byref(o), C.byref(st)))
        return {name: getattr(st, name) for name, _ in B.PlanStats._fields_}

    def workspace_size(self, options: Optional[B.Options] = None, **kw) -> int:
        """Device bytes a setup with these options needs (bddcso_setup_workspace_size)."""
        o = options if options is not None else default_options(**kw)
        n = C.c_size_t()
        B.check(B.load().bddcso_setup_workspace_size(self._h, C.byref(o), C.byref(n)))
        return n.value

    def autotune(self, rho: torch.Tensor, b: torch.Tensor, options: Optional[B.Options] = None, stream=None,
                 **kw):
        """bddcso_autotune: the fastest launch-shape variant of the options for
        one step (numeric setup + solve of b) of this problem.  Returns the
        tuned options and the trials as a list of (knobs, ms, status)."""
        _f64_cuda(rho, "rho")
        _f64_cuda(b, "b")
        o = options if options is not None else default_options(**kw)
        nrhs = b.numel() // self.n_free
        best, rep = B.Options(), B.TuneReport()
        B.check(B.load().bddcso_autotune(self._h, _ptr(rho), C.byref(o), _ptr(b), nrhs, _stream(stream),
                                         C.byref(best), C.byref(rep)))
        knobs = ("update_tile", "slab_width", "slab_lookahead", "sweep_reg_rows", "block_target", "mr_min_rhs",
                 "graph")
        trials = [({k: getattr(rep.tried[t], k) for k in knobs}, rep.step_ms[t], B.STATUS.get(rep.status[t]))
                  for t in range(rep.n_trials)]
        return best, {"trials": trials, "best": rep.best}

    def coef_from_log(self, theta: torch.Tensor, stream=None) -> torch.Tensor:
        """rho = exp(F theta), F the 3^dim box mean (bddcso_coef_from_log)."""
        _f64_cuda(theta, "theta")
        out = torch.empty_like(theta)
        B.check(B.load().bddcso_coef_from_log(self._h, _ptr(theta), _ptr(out), _stream(stream)))
        return out

    def box_filter(self, x: torch.Tensor, transpose: bool = False, stream=None) -> torch.Tensor:
        _f64_cuda(x, "x")
        out = torch.empty_like(x)
        B.check(B.load().bddcso_box_filter(self._h, _ptr(x), _ptr(out), int(transpose), _stream(stream)))
        return out

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                B.load().bddcso_problem_destroy(h)
            except (TypeError, AttributeError):  # interpreter shutdown: the module is gone
                pass
            self._h = None


class Preconditioner:
    """Device factors of one setup (bddcso_setup / bddcso_refactor).

    The device memory is a PyTorch-owned workspace of
    ``bddcso_setup_workspace_size`` bytes on rho's device, kept alive with
    the preconditioner (``workspace=False`` lets the library allocate it).
    """

    def __init__(self, problem: Problem, rho: torch.Tensor, options: Optional[B.Options] = None,
                 stream=None, workspace: bool = True, **kw):
        self.problem = problem
        self.options = options if options is not None else default_options(**kw)
        _f64_cuda(rho, "rho")
        self._ws = None
        ws_ptr, ws_bytes = None, 0
        if workspace:
            ws_bytes = problem.workspace_size(self.options)
            # the caching allocator returns blocks aligned to at least 512 bytes
            self._ws = torch.empty(ws_bytes, dtype=torch.uint8, device=rho.device)
            ws_ptr = C.c_void_p(self._ws.data_ptr())
        out = C.c_void_p()
        B.check(B.load().bddcso_setup(problem._h, _ptr(rho), C.byref(self.options), ws_ptr, ws_bytes,
                                      _stream(stream), C.byref(out)))
        self._h = out
        self.n_free = problem.n_free

    @property
    def generation(self) -> int:
        """Numeric setups done so far (bddcso_precond_generation)."""
        g = C.c_int64()
        B.check(B.load().bddcso_precond_generation(self._h, C.byref(g)))
        return g.value

    def refactor(self, rho: torch.Tensor, stream=None) -> None:
        _f64_cuda(rho, "rho")
        B.check(B.load().bddcso_refactor(self._h, _ptr(rho), _stream(stream)))

    def check_pivots(self, stream=None) -> None:
        B.check(B.load().bddcso_check_pivots(self._h, _stream(stream)))

    def _nrhs(self, x: torch.Tensor) -> int:
        if x.numel() % self.n_free:
            raise ValueError("vector length must be a multiple of n_free")
        return x.numel() // self.n_free

    def operator(self, x: torch.Tensor, stream=None) -> torch.Tensor:
        _f64_cuda(x, "x")
        y = torch.empty_like(x)
        B.check(B.load().bddcso_operator_apply(self._h, _ptr(x), _ptr(y), self._nrhs(x), _stream(stream)))
        return y

    def apply(self, r: torch.Tensor, stream=None) -> torch.Tensor:
        _f64_cuda(r, "r")
        z = torch.empty_like(r)
        B.check(B.load().bddcso_apply(self._h, _ptr(r), _ptr(z), self._nrhs(r), _stream(stream)))
        return z

    def solve(self, b: torch.Tensor, stream=None, raise_on_noconv: bool = True):
        _f64_cuda(b, "b")
        x = torch.empty_like(b)
        st = B.Stats()
        status = B.load().bddcso_solve(self._h, _ptr(b), _ptr(x), self._nrhs(b), C.byref(st), _stream(stream))
        if status != 0 and (raise_on_noconv or status != -5):
            B.check(status)
        n = st.nrhs
        stats = {
            "iters": list(st.iters[:n]), "converged": list(st.converged[:n]),
            "relres": list(st.relres[:n]), "kappa": list(st.kappa[:n]),
            "lambda_min": list(st.lambda_min[:n]), "lambda_max": list(st.lambda_max[:n]),
            "n_coarse": st.n_coarse, "t_solve_ms": st.t_solve_ms, "status": B.STATUS.get(status, status),
        }
        return x, stats

    def solve_noalloc(self, b: torch.Tensor, x: torch.Tensor, stream=None, raise_on_noconv: bool = True):
        """bddcso_solve_noalloc into the caller's x (same shape as b); allocates nothing."""
        _f64_cuda(b, "b")
        _f64_cuda(x, "x")
        if x.shape != b.shape:
            raise ValueError("x must have the shape of b")
        st = B.Stats()
        status = B.load().bddcso_solve_noalloc(self._h, _ptr(b), _ptr(x), self._nrhs(b), C.byref(st),
                                               _stream(stream))
        if status != 0 and (raise_on_noconv or status != -5):
            B.check(status)
        n = st.nrhs
        return {"iters": list(st.iters[:n]), "converged": list(st.converged[:n]), "relres": list(st.relres[:n]),
                "kappa": list(st.kappa[:n]), "status": B.STATUS.get(status, status)}

    def element_grad(self, u: torch.Tensor, lam: torch.Tensor, stream=None) -> torch.Tensor:
        _f64_cuda(u, "u")
        _f64_cuda(lam, "lam")
        g = torch.empty(self.problem.n_elements, dtype=torch.float64, device=u.device)
        B.check(B.load().bddcso_element_grad(self._h, _ptr(u), _ptr(lam), _ptr(g), self._nrhs(u),
                                             _stream(stream)))
        return g

    def info(self) -> dict:
        nc, nf, nb, ce = C.c_int64(), C.c_int64(), C.c_int64(), C.c_int64()
        B.check(B.load().bddcso_precond_info(self._h, C.byref(nc), C.byref(nf), C.byref(nb), C.byref(ce)))
        return {"n_coarse": nc.value, "n_fronts": nf.value, "device_bytes": nb.value,
                "coarse_factor_entries": ce.value}

    KERNEL_CLASSES = {"sweep_update": 1, "block_solve": 2, "gemm": 3, "sweep_panel": 4, "sweep_small": 5,
                      "schur_couple": 6, "couple_multi": 7, "q1_apply": 8}

    def profile(self, classes=None) -> None:
        """Start event timing of the named kernel classes (all when None); [] stops it."""
        names = list(self.KERNEL_CLASSES) if classes is None else list(classes)
        mask = 0
        for c in names:
            mask |= 1 << self.KERNEL_CLASSES[c]
        B.check(B.load().bddcso_profile(self._h, mask))

    def profile_read(self) -> dict:
        out = {}
        for name, c in self.KERNEL_CLASSES.items():
            n, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
            B.check(B.load().bddcso_profile_read(self._h, c, C.byref(n), C.byref(ms), C.byref(fl), C.byref(by)))
            rf, rb = C.c_double(), C.c_double()
            B.check(B.load().bddcso_profile_reference(self._h, c, C.byref(rf), C.byref(rb)))
            out[name] = {"launches": n.value, "total_ms": ms.value, "flops": fl.value, "bytes": by.value,
                         "ref_flops": rf.value, "ref_bytes": rb.value}
        return out

    def local_coarse(self, sub: int, cap: int = 4096, stream=None):
        kc = np.zeros(cap * cap)
        ids = np.zeros(cap, dtype=np.int64)
        nc = C.c_int64()
        B.check(B.load().bddcso_local_coarse(self._h, sub, kc.ctypes.data_as(C.POINTER(C.c_double)),
                                             ids.ctypes.data_as(C.POINTER(C.c_int64)), cap, C.byref(nc),
                                             _stream(stream)))
        n = nc.value
        return kc[: n * n].reshape(n, n, order="F").copy(), ids[:n].copy()

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                B.load().bddcso_precond_destroy(h)
            except (TypeError, AttributeError):  # interpreter shutdown: the module is gone
                pass
            self._h = None
        self._ws = None  # released only after the library has let go of it


class BDDCSOSolve(torch.autograd.Function):
    """u = A(rho(theta))^{-1} f with rho = exp(F theta) (F: 3^dim box mean).

    Backward: the adjoint solve A lambda = dL/du with the same BDDC-SO
    preconditioner (A is symmetric), then dL/dtheta = F^T (rho * g) with
    g_e = -lambda_e^T K^_e u_e from the element kernel.  The forward's rho
    is kept: when the preconditioner has been refactored since (another
    forward on it), the backward refactors it from that rho first, so the
    gradient always belongs to its own forward.
    """

    @staticmethod
    def forward(ctx, theta, f, pc: Preconditioner):
        rho = pc.problem.coef_from_log(theta.detach().contiguous())
        pc.refactor(rho)
        u, st = pc.solve(f.contiguous())
        ctx.pc = pc
        ctx.stats = st
        ctx.generation = pc.generation
        ctx.save_for_backward(u, rho)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        u, rho = ctx.saved_tensors
        pc = ctx.pc
        if pc.generation != ctx.generation:
            pc.refactor(rho)
            ctx.generation = pc.generation
        lam, _ = pc.solve(grad_u.contiguous())
        g = pc.element_grad(u, lam)           # -rho_e lam_e^T K^_e u_e = dL/dtheta~_e
        return pc.problem.box_filter(g, transpose=True), None, None
