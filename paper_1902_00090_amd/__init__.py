"""MI355X (gfx950) data-driven GMRES for 2D FDFD Maxwell problems.

Python binding of libddgmres.so: argument marshalling only.  torch tensors
provide device memory and the current HIP stream; every arithmetic step of the
solver, the principal-component basis and the convolutional predictor runs in
the library's HIP kernels.  The names follow the C ABI in include/ddgmres.h.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import DD_C64, DD_C128, DDError, check, ptr_array

__all__ = ["FdfdOp", "Solver", "autotune", "workspace_bytes", "gmres_solve", "gmres_solve_batched",
           "pca_build",
           "local_pca_targets", "proj_loss_batched", "Cnn", "Predictor", "save_pca", "DDError",
           "lib_path"]


def lib_path() -> str:
    return _lib.LIB_PATH


def _torch():
    import torch
    return torch


def _stream():
    torch = _torch()
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _stream_if_gpu():
    """The current stream, or the null stream where no GPU is visible (host-side
    argument checks of the library run before any device call)."""
    torch = _torch()
    return _stream() if torch.cuda.is_available() else None


DD_MAX_K = 64  # largest number of augmenting vectors the library accepts


def _check_lengths(nb, **lists):
    """Every per-problem list (None allowed) must hold exactly nb entries: the
    library reads nb pointers from each array it is given."""
    for name, v in lists.items():
        if v is not None and len(v) != nb:
            raise ValueError(f"{name} has {len(v)} entries, expected one per problem ({nb})")


def _check_subspace(U, D, what="U"):
    """U must be a 2-D [k, D] array with 0 <= k <= DD_MAX_K (checked before any
    pointer reaches the library, which reads k * D elements)."""
    if U is None:
        return 0
    if U.dim() != 2 or U.shape[1] != D:
        raise ValueError(f"{what} must be [k, D={D}], got {tuple(U.shape)}")
    if U.shape[0] > DD_MAX_K:
        raise ValueError(f"{what} has {U.shape[0]} vectors, at most {DD_MAX_K} are supported")
    return int(U.shape[0])


def _dev(t, dtype=None, numel=None, what="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{what} must have dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what} must have {numel} elements, got {t.numel()}")
    return C.c_void_p(t.data_ptr())


class FdfdOp:
    """A = -(Dxb Dxf + Dyb Dyf) - omega^2 diag(eps) on an nx x ny Yee grid (Eq. 1)."""

    def __init__(self, eps, omega, dx, npml, grade=3, ln_R=-16.0, npml_y=None):
        eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float32))
        if eps.ndim != 2:
            raise ValueError("eps must be [ny, nx]")
        self.ny, self.nx = eps.shape
        self.D = self.nx * self.ny
        self.omega, self.dx, self.npml = float(omega), float(dx), int(npml)
        pml = _lib.dd_pml(int(npml), int(npml if npml_y is None else npml_y), int(grade),
                          float(ln_R))
        h = C.c_void_p()
        check(_lib.lib().fdfd_op_create(eps.ctypes.data_as(C.POINTER(C.c_float)), self.nx,
                                        self.ny, self.omega, self.dx, C.byref(pml),
                                        _stream_if_gpu(), C.byref(h)), "fdfd_op_create")
        self._h = h

    @classmethod
    def from_instance(cls, inst):
        return cls(inst.eps, inst.omega, inst.dx, inst.npml)

    @property
    def handle(self):
        return self._h

    def apply(self, x, out=None):
        torch = _torch()
        prec = DD_C64 if x.dtype == torch.complex64 else DD_C128
        if x.dtype not in (torch.complex64, torch.complex128):
            raise TypeError("x must be complex64 or complex128")
        if out is None:
            out = torch.empty_like(x)
        check(_lib.lib().fdfd_op_apply(self._h, _dev(x, numel=self.D, what="x"),
                                       _dev(out, x.dtype, self.D, "out"), prec, _stream()),
              "fdfd_op_apply")
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().fdfd_op_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


PRECONDS = {None: 0, "none": 0, "jacobi": 1, "pml": 2}


def _opts(restart=100, kmax=0, inner="c64", cgs_passes=2, elems_per_thread=0, hist_cap=0,
          check_every=4, select_reorth=True, use_graph=False, precond=None, workspace=None,
          fused=False):
    o = _lib.dd_solver_opts()
    _lib.lib().dd_solver_opts_default(C.byref(o))
    o.inner = DD_C64 if inner == "c64" else DD_C128
    o.cgs_passes = int(cgs_passes)
    o.restart = int(restart)
    o.kmax = int(kmax)
    o.elems_per_thread = int(elems_per_thread)
    o.hist_cap = int(hist_cap)
    o.check_every = int(check_every)
    o.select_reorth = int(bool(select_reorth))
    o.use_graph = int(bool(use_graph))
    o.precond = PRECONDS[precond]
    o.fused = int(bool(fused))
    if workspace is not None:
        o.workspace = C.c_void_p(_dev(workspace, what="workspace").value)
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def workspace_bytes(ops, restart=100, kmax=0, inner="c64", cgs_passes=2, elems_per_thread=0,
                    hist_cap=0, precond=None, fused=False):
    """Device bytes a Solver with these operators and options needs (no device
    memory is touched)."""
    o = _opts(restart, kmax, inner, cgs_passes, elems_per_thread, hist_cap, 4, True, False,
              precond, None, fused)
    n = C.c_size_t()
    check(_lib.lib().dd_solver_workspace_bytes(ptr_array([op.handle for op in ops]), len(ops),
                                               C.byref(o), C.byref(n)),
          "dd_solver_workspace_bytes")
    return n.value


def autotune(ops, restart=100, inner="c64", cgs_passes=2, select_reorth=True):
    """Fastest elements-per-thread value for these operators, and the timings
    (ms per Arnoldi step) of the candidates 1, 2, 4, 8."""
    o = _opts(restart, 0, inner, cgs_passes, 0, 0, 4, select_reorth)
    best = C.c_int()
    ms = (C.c_double * 4)()
    check(_lib.lib().dd_solver_autotune(ptr_array([op.handle for op in ops]), len(ops), C.byref(o),
                                        C.byref(best), ms), "dd_solver_autotune")
    return best.value, list(ms)


class Solver:
    """Batched data-driven GMRES over a list of operators (lockstep cycles)."""

    def __init__(self, ops, restart=100, kmax=0, inner="c64", cgs_passes=2,
                 elems_per_thread=0, hist_cap=0, check_every=4, select_reorth=True,
                 use_graph=False, precond=None, workspace=None, fused=False):
        """precond: None, "jacobi" or "pml" (diagonal preconditioners, see the C header).
        fused: one sweep per Arnoldi step where it applies (cgs_passes=1,
        kmax + restart + 1 <= 128); off by default (faster for one problem
        alone, slower for batches).
        workspace: an optional device tensor (at least workspace_bytes(...) bytes,
        256-byte aligned) that holds all of the solver's device arrays; the
        solver then allocates no device memory and keeps a reference to it."""
        self.ops = list(ops)
        self.nb = len(self.ops)
        self._workspace = workspace
        self.opts = _opts(restart, kmax, inner, cgs_passes, elems_per_thread, hist_cap,
                          check_every, select_reorth, use_graph, precond, workspace, fused)
        self.inner = inner
        self.restart, self.kmax = int(restart), int(kmax)
        h = C.c_void_p()
        check(_lib.lib().dd_solver_create(ptr_array([o.handle for o in self.ops]), self.nb,
                                          C.byref(self.opts), C.byref(h)), "dd_solver_create")
        self._h = h
        self._U = None
        self.k = [0] * self.nb

    def bind(self, ops):
        ops = list(ops)
        check(_lib.lib().dd_solver_bind(self._h, ptr_array([o.handle for o in ops])),
              "dd_solver_bind")
        self.ops = ops
        self.k = [0] * self.nb

    def set_subspace(self, U):
        """U: list (one per problem) of [k, D] tensors in the inner precision, or None."""
        torch = _torch()
        if U is None:
            check(_lib.lib().dd_solver_set_subspace(self._h, None, None, _stream()),
                  "dd_solver_set_subspace")
            self.k = [0] * self.nb
            return
        dt = torch.complex64 if self.inner == "c64" else torch.complex128
        _check_lengths(self.nb, U=U)
        ptrs, ks = [], (C.c_int * self.nb)()
        for p, u in enumerate(U):
            if u is None or u.numel() == 0:
                ptrs.append(None)
                ks[p] = 0
                continue
            if _check_subspace(u, self.ops[p].D, f"U[{p}]") > self.kmax:
                raise ValueError(f"U[{p}] has {u.shape[0]} vectors, the solver's kmax is "
                                 f"{self.kmax}")
            ptrs.append(_dev(u, dt, what=f"U[{p}]").value)
            ks[p] = u.shape[0]
        check(_lib.lib().dd_solver_set_subspace(self._h, ptr_array(ptrs), ks, _stream()),
              "dd_solver_set_subspace")
        self.k = list(ks)

    def solve(self, b, x0=None, tol=1e-6, maxit=20000, x=None):
        """b: list of [D] complex128 tensors.  Returns (x list, list of info dicts, status)."""
        torch = _torch()
        _check_lengths(self.nb, b=b, x=x, x0=x0)
        if x is None:
            x = [torch.empty_like(bb) for bb in b]
        bp = ptr_array([_dev(bb, torch.complex128, self.ops[p].D, f"b[{p}]").value
                        for p, bb in enumerate(b)])
        xp = ptr_array([_dev(xx, torch.complex128, self.ops[p].D, f"x[{p}]").value
                        for p, xx in enumerate(x)])
        x0p = None
        if x0 is not None:
            x0p = ptr_array([None if v is None else
                             _dev(v, torch.complex128, self.ops[p].D, f"x0[{p}]").value
                             for p, v in enumerate(x0)])
        info = (_lib.dd_info * self.nb)()
        st = check(_lib.lib().dd_solver_solve(self._h, bp, x0p, float(tol), int(maxit), xp, info,
                                              _stream()), "dd_solver_solve")
        return x, [i.as_dict() for i in info], st

    def history(self, p):
        cap = self.opts.hist_cap
        out = np.zeros(max(cap, 1), np.float64)
        n = C.c_int()
        check(_lib.lib().dd_solver_history(self._h, p, out.ctypes.data_as(C.POINTER(C.c_double)),
                                           cap, C.byref(n)), "dd_solver_history")
        return out[:n.value].copy()

    def debug(self, p, what):
        """Internal arrays of problem p: 'C', 'Q', 'H', 'B', 'Rinv' (see the C header)."""
        D = self.ops[p].D
        k, m = self.k[p], self.restart
        cdt = np.complex64 if self.inner == "c64" else np.complex128
        shapes = {"C": (0, (k, D), cdt), "Q": (1, (m + 1, D), cdt),
                  "H": (2, (m, m + 1), np.complex128), "B": (3, (m, k), np.complex128),
                  "Rinv": (4, (k, k), np.complex128)}
        code, shape, dt = shapes[what]
        out = np.zeros(shape, dt)
        check(_lib.lib().dd_solver_debug_copy(self._h, p, code, out.ctypes.data_as(C.c_void_p),
                                              out.nbytes), "dd_solver_debug_copy")
        return out

    def profile(self, enable=True):
        """Turn on live HIP-event timing of the streaming sweeps (resets stats)."""
        check(_lib.lib().dd_solver_profile(self._h, int(bool(enable))), "dd_solver_profile")

    def recycle(self, kr):
        """Harmonic Ritz vectors of each problem's last cycle (subspace
        recycling, Sec. 1; supplement Sec. 1): returns (Y, theta) with Y a
        list of [kout_p, D] tensors in the inner precision (for set_subspace
        of the next system) and theta an [nb, kr] complex array of their
        harmonic Ritz values (zero past kout_p)."""
        torch = _torch()
        if not 1 <= int(kr) <= 64:
            raise ValueError(f"kr = {kr} outside 1..64")
        kr = int(kr)
        dt = torch.complex64 if self.inner == "c64" else torch.complex128
        Y = [torch.empty((kr, op.D), dtype=dt, device="cuda") for op in self.ops]
        kout = (C.c_int * self.nb)()
        th = np.zeros((self.nb, kr, 2), np.float64)
        check(_lib.lib().dd_solver_recycle(self._h, kr, ptr_array([y.data_ptr() for y in Y]), kout,
                                           th.ctypes.data_as(C.POINTER(C.c_double)), _stream()),
              "dd_solver_recycle")
        return [Y[p][:kout[p]] for p in range(self.nb)], th[..., 0] + 1j * th[..., 1]

    def kernel_stats(self):
        """{'matvec_dots'|'second_pass'|'update_norm'|'fused_sweep': (ms, launches, bytes)}."""
        ks = _lib.dd_kernel_stats()
        check(_lib.lib().dd_solver_kernel_stats(self._h, C.byref(ks)), "dd_solver_kernel_stats")
        names = ["matvec_dots", "second_pass", "update_norm", "fused_sweep"]
        return {n: (ks.ms[i], ks.launches[i], ks.bytes[i]) for i, n in enumerate(names)}

    @property
    def elems_per_thread(self):
        """The tile width the solver runs with (the rule's or the autotuner's)."""
        return _lib.lib().dd_solver_elems_per_thread(self._h)

    @property
    def device_bytes(self):
        return _lib.lib().dd_solver_device_bytes(self._h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().dd_solver_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gmres_solve(op, b, U=None, tol=1e-6, restart=100, maxit=20000, x0=None, inner="c64",
                cgs_passes=2, x=None):
    """One problem: returns (x, info dict, status)."""
    torch = _torch()
    if x is None:
        x = torch.empty_like(b)
    o = _opts(restart, 0, inner, cgs_passes)
    info = _lib.dd_info()
    k = _check_subspace(U, op.D)
    dt = torch.complex64 if inner == "c64" else torch.complex128
    st = check(_lib.lib().gmres_solve(
        op.handle, _dev(b, torch.complex128, op.D, "b"),
        None if x0 is None else _dev(x0, torch.complex128, op.D, "x0"),
        None if U is None else _dev(U, dt, what="U"), k, float(tol), int(restart), int(maxit),
        C.byref(o), _dev(x, torch.complex128, op.D, "x"), C.byref(info), _stream()),
        "gmres_solve")
    return x, info.as_dict(), st


def gmres_solve_batched(ops, b, U=None, tol=1e-6, restart=100, maxit=20000, inner="c64",
                        cgs_passes=2):
    s = Solver(ops, restart=restart, kmax=max([0] + [u.shape[0] for u in (U or []) if u is not None]),
               inner=inner, cgs_passes=cgs_passes)
    try:
        if U is not None:
            s.set_subspace(U)
        return s.solve(b, tol=tol, maxit=maxit)
    finally:
        s.close()


def pca_build(S, k):
    """S: [M, D] complex64 snapshots (device).  Returns (U [k, D] complex64, sigma [k])."""
    torch = _torch()
    M, D = S.shape
    U = torch.empty((k, D), dtype=torch.complex64, device=S.device)
    sig = np.zeros(k, np.float64)
    check(_lib.lib().pca_build(_dev(S, torch.complex64, what="S"), M, D, k, _dev(U),
                               sig.ctypes.data_as(C.POINTER(C.c_double)), _stream()), "pca_build")
    return U, sig


def local_pca_targets(F, window, k):
    """F: [S, D] complex64 solution fields of one trajectory (device).
    Returns T [S, k, D] complex64: target j of step s is u_j (u_j^H f_s)."""
    torch = _torch()
    S, D = F.shape
    T = torch.empty((S, k, D), dtype=torch.complex64, device=F.device)
    check(_lib.lib().local_pca_targets(_dev(F, torch.complex64, what="F"), S, D, int(window), int(k),
                                       _dev(T), _stream()), "local_pca_targets")
    return T


def proj_loss_batched(V, f):
    """V: [nb, k, D] complex64, f: [nb, D] complex128 (device).  Returns numpy [nb]."""
    torch = _torch()
    nb, k, D = V.shape
    out = np.zeros(nb, np.float64)
    check(_lib.lib().proj_loss_batched(_dev(V, torch.complex64, what="V"),
                                       _dev(f, torch.complex128, nb * D, "f"), nb, k, D,
                                       out.ctypes.data_as(C.POINTER(C.c_double)), _stream()),
          "proj_loss_batched")
    return out


def eim_field(ops, b, out=None):
    """Effective-index fields (the CNN's second input) of the problems
    (ops[p], b[p]); b: list of [D] complex128 device tensors.  Returns a list
    of [D] complex64 tensors, or fills the rows of out ([nb, D] complex64)."""
    torch = _torch()
    nb = len(ops)
    if len(b) != nb:
        raise ValueError("one right-hand side per operator")
    if out is None:
        F = [torch.empty(op.D, dtype=torch.complex64, device=bb.device) for op, bb in zip(ops, b)]
    else:
        _dev(out, torch.complex64, what="out")
        F = [out[p, :ops[p].D] for p in range(nb)]
    opp = ptr_array([op._h.value for op in ops])
    bp = ptr_array([_dev(bb, torch.complex128, ops[p].D, f"b[{p}]").value for p, bb in enumerate(b)])
    fp = ptr_array([f.data_ptr() for f in F])
    check(_lib.lib().eim_field(opp, nb, bp, fp, _stream()), "eim_field")
    return F if out is None else out


def eim_field_noalloc(ops, b, F):
    """eim_field into caller-provided outputs F (list of [D] complex64 device
    tensors) with no device allocation: the library's fixed scratch array
    holds the work (batches up to DD_EIM_NOALLOC_BYTES of scratch)."""
    torch = _torch()
    nb = len(ops)
    _check_lengths(nb, b=b, F=F)
    opp = ptr_array([op._h.value for op in ops])
    bp = ptr_array([_dev(bb, torch.complex128, ops[p].D, f"b[{p}]").value for p, bb in enumerate(b)])
    fp = ptr_array([_dev(f, torch.complex64, ops[p].D, f"F[{p}]").value for p, f in enumerate(F)])
    check(_lib.lib().eim_field_noalloc(opp, nb, bp, fp, _stream()), "eim_field_noalloc")
    return F


def res_loss_batched(ops, b, V):
    """Residual loss (eq:res_loss) of V[p] ([k, D] complex64) for the problems
    (ops[p], b[p] [D] complex128), all device tensors.  Returns numpy [nb]."""
    torch = _torch()
    nb = len(ops)
    k = V[0].shape[0]
    out = np.zeros(nb, np.float64)
    opp = ptr_array([op._h.value for op in ops])
    bp = ptr_array([_dev(bb, torch.complex128, ops[p].D, f"b[{p}]").value for p, bb in enumerate(b)])
    vp = ptr_array([_dev(v, torch.complex64, k * ops[p].D, f"V[{p}]").value for p, v in enumerate(V)])
    check(_lib.lib().res_loss_batched(opp, bp, vp, nb, k, out.ctypes.data_as(C.POINTER(C.c_double)),
                                      _stream()), "res_loss_batched")
    return out


def res_loss_grad_batched(ops, b, V):
    """Residual loss and its conjugate gradient G = -(A^H r) c^H / ||b||^2 with
    respect to V[p] ([k, D] complex64), for the problems (ops[p], b[p]).
    Returns (numpy [nb] losses, list of [k, D] complex64 gradients)."""
    torch = _torch()
    nb = len(ops)
    _check_lengths(nb, b=b, V=V)
    k = V[0].shape[0]
    out = np.zeros(nb, np.float64)
    G = [torch.empty((k, op.D), dtype=torch.complex64, device=v.device) for op, v in zip(ops, V)]
    opp = ptr_array([op._h.value for op in ops])
    bp = ptr_array([_dev(bb, torch.complex128, ops[p].D, f"b[{p}]").value for p, bb in enumerate(b)])
    vp = ptr_array([_dev(v, torch.complex64, k * ops[p].D, f"V[{p}]").value for p, v in enumerate(V)])
    gp = ptr_array([g.data_ptr() for g in G])
    check(_lib.lib().res_loss_grad_batched(opp, bp, vp, nb, k,
                                           out.ctypes.data_as(C.POINTER(C.c_double)), gp,
                                           _stream()), "res_loss_grad_batched")
    return out, G


def save_pca(path, U, nx, ny):
    """Write a PCA basis U ([k, D] complex64, device) as a predictor file."""
    torch = _torch()
    k = U.shape[0]
    _check_subspace(U, int(nx) * int(ny))
    check(_lib.lib().predictor_save_pca(str(path).encode(), _dev(U, torch.complex64, what="U"), k,
                                        int(nx), int(ny), _stream()), "predictor_save_pca")


class Predictor:
    """A subspace predictor loaded from a file: a PCA basis or a CNN (the
    C ABI's predictor_load / predict_subspace / predictor_destroy)."""

    KINDS = {1: "pca", 2: "cnn"}

    def __init__(self, path, max_batch=1):
        h = C.c_void_p()
        check(_lib.lib().predictor_load(str(path).encode(), int(max_batch), C.byref(h)),
              "predictor_load")
        self._h = h
        v = [C.c_int() for _ in range(5)]
        check(_lib.lib().predictor_info(h, *[C.byref(x) for x in v]), "predictor_info")
        kind, self.nx, self.ny, self.k, self.in_channels = (x.value for x in v)
        self.kind = self.KINDS[kind]
        self.D = self.nx * self.ny
        self.max_batch = int(max_batch)

    def predict(self, B, eps=None, ops=None, b=None, U=None):
        """U [B, k, D] complex64: the subspaces of B problems.  eps [B, ny, nx]
        float32 for a CNN; ops and b (lists) for a three-plane CNN."""
        torch = _torch()
        if U is None:
            U = torch.empty((B, self.k, self.D), dtype=torch.complex64, device="cuda")
        _dev(U, torch.complex64, B * self.k * self.D, "U")
        _check_lengths(B, ops=ops, b=b)
        opp = None if ops is None else ptr_array([op._h.value for op in ops])
        bp = None if b is None else ptr_array(
            [_dev(bb, torch.complex128, self.D, f"b[{i}]").value for i, bb in enumerate(b)])
        ep = None if eps is None else _dev(eps, torch.float32, B * self.D, "eps")
        check(_lib.lib().predict_subspace(self._h, opp, bp, ep, int(B), _dev(U), _stream()),
              "predict_subspace")
        return U

    def close(self):
        if getattr(self, "_h", None):
            _lib.lib().predictor_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


from .cnn import Cnn  # noqa: E402


def harmonic_ritz_host(G, M, kr):
    """The host-side small eigenproblem of Solver.recycle: G, M are nw x ns
    complex arrays (A S = W G, M = W^H S); returns (Z [ns, kr], theta [kr])."""
    G = np.ascontiguousarray(G, np.complex128)
    M = np.ascontiguousarray(M, np.complex128)
    nw, ns = G.shape
    if M.shape != G.shape:
        raise ValueError("G and M must have the same shape")
    Z = np.zeros((ns, kr), np.complex128)
    th = np.zeros(kr, np.complex128)
    dp = C.POINTER(C.c_double)
    check(_lib.lib().dd_harmonic_ritz_host(ns, nw, G.ctypes.data_as(dp), M.ctypes.data_as(dp),
                                           int(kr), Z.ctypes.data_as(dp), th.ctypes.data_as(dp)),
          "dd_harmonic_ritz_host")
    return Z, th
