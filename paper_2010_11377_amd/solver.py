"""Python face of libirk: ``IRKSolver`` wraps one ``irk_solver`` handle.

PyTorch supplies device memory (float64 CUDA tensors on ROCm) and the HIP
stream; every computation happens in the library.  Nothing here falls back to
a CPU implementation: without the built library or a GPU the constructor
raises.
"""
import ctypes
import time

import numpy as np
import torch

from . import binding as B


def _csr_struct(indptr, indices, data):
    indptr = np.ascontiguousarray(indptr, dtype=np.int32)
    indices = np.ascontiguousarray(indices, dtype=np.int32)
    data = np.ascontiguousarray(data, dtype=np.float64)
    n = indptr.size - 1
    st = B.CSR(n, int(indices.size), indptr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
               indices.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), B.dptr(data))
    return st, (indptr, indices, data)


def _dev(t, numel, name):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA tensor" % name)
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != numel:
        raise ValueError("%s must be a contiguous float64 tensor with %d elements" % (name, numel))
    return ctypes.c_void_p(t.data_ptr())


class IRKSolver:
    """Solver for the IRK stage system ``(I + h A (x) K) k = 1 (x) (g - K u)``
    preconditioned by ``P = I + h A~ (x) K`` (``A~ = LD`` by default) with one
    AMG V-cycle per stage block.

    Parameters: Butcher ``(A, b, c)``; ``K`` as CSR ``(indptr, indices, data)``
    on the ``grid = (nx, ny)``; timestep ``h_t``; options of ``irk_options``;
    ``M`` the mass matrix as CSR on the same grid (None: ``M = I``).
    """

    def __init__(self, A, b, c, K, h_t, grid, precision="fp64", precond="LD", restart=40,
                 max_iter=200, nu_pre=2, nu_post=2, coarse_max=64, rtol=1e-8, true_resid=True,
                 reorth=0, side="right", M=None, interp="linear", graphs=None,
                 coarse_ratio=None, smoother="rbgs", jacobi_omega=0.8, fuse_levels=True,
                 device=None):
        if not torch.cuda.is_available():
            raise RuntimeError("IRKSolver needs a ROCm GPU (torch.cuda.is_available() is False)")
        self.lib = B.lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        A = np.ascontiguousarray(A, dtype=np.float64)
        self._b = np.ascontiguousarray(b, dtype=np.float64)
        self._c = np.ascontiguousarray(c, dtype=np.float64)
        self.A = A
        self.s = A.shape[0]
        nx, ny = grid
        self.nx, self.ny = int(nx), int(ny)
        self.N = self.nx * self.ny
        self.h_t = float(h_t)
        opt = B.default_options()
        opt.precision = B.IRK_MIXED if precision == "mixed" else B.IRK_FP64
        opt.precond = B.PRECOND[precond]
        opt.restart, opt.max_iter = int(restart), int(max_iter)
        opt.nu_pre, opt.nu_post = int(nu_pre), int(nu_post)
        opt.coarse_max = int(coarse_max)
        opt.rtol = float(rtol)
        opt.true_resid = 1 if true_resid else 0
        opt.reorth = int(reorth)
        opt.side = {"right": B.IRK_RIGHT, "left": B.IRK_LEFT}[side]
        opt.interp = {"linear": B.IRK_INTERP_LINEAR, "constant": B.IRK_INTERP_CONSTANT}[interp]
        if graphs is not None:
            opt.graphs = 1 if graphs else 0
        if coarse_ratio is not None:
            opt.coarse_ratio = float(coarse_ratio)
        opt.smoother = B.SMOOTHER[smoother]
        opt.jacobi_omega = float(jacobi_omega)
        opt.fuse_levels = 1 if fuse_levels else 0
        self.options = opt
        tab = B.Butcher(self.s, B.dptr(self.A), B.dptr(self._b), B.dptr(self._c))
        csr, keep = _csr_struct(*K)
        mcsr = None
        if M is not None:
            mcsr, mkeep = _csr_struct(*M)
        g = B.Grid(self.nx, self.ny)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            self._stream = stream
            st = self.lib.irk_setup(ctypes.byref(handle), ctypes.byref(tab),
                                    ctypes.byref(mcsr) if mcsr is not None else None,
                                    ctypes.byref(csr),
                                    self.h_t, ctypes.byref(g), ctypes.byref(opt),
                                    ctypes.c_void_p(stream.cuda_stream))
        if st != B.IRK_OK:
            raise B.IRKError(st, self.lib.irk_last_error(None).decode())
        self._h = handle
        self.last_stats = None
        self.last_status = None
        self._source = None
        self.op_version = 0  # bumped by every update_operator

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self.lib.irk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, allow_not_converged=False):
        if st == B.IRK_OK or (allow_not_converged and st == B.IRK_E_NOT_CONVERGED):
            return st
        raise B.IRKError(st, self.lib.irk_last_error(self._h).decode())

    def info(self):
        N, s, lev, cc = (ctypes.c_int() for _ in range(4))
        self._check(self.lib.irk_info(self._h, ctypes.byref(N), ctypes.byref(s), ctypes.byref(lev),
                                      ctypes.byref(cc)))
        return {"N": N.value, "s": s.value, "levels": lev.value, "constant_coeff": bool(cc.value)}

    def graph_stats(self):
        """(captured preconditioner graphs, replays since setup)."""
        g, r = ctypes.c_int(), ctypes.c_longlong()
        self._check(self.lib.irk_graph_stats(self._h, ctypes.byref(g), ctypes.byref(r)))
        return g.value, r.value

    # -- problem data ----------------------------------------------------------
    def set_source(self, g):
        if g is None:
            self._check(self.lib.irk_set_source(self._h, None))
            self._source = None
            return
        gt = torch.as_tensor(g, dtype=torch.float64, device=self.device).contiguous()
        self._check(self.lib.irk_set_source(self._h, _dev(gt, self.N, "g")))
        self._source = gt

    def update_operator(self, K):
        """Replace K (same grid and structure); returns the new operator
        version (``op_version``)."""
        csr, keep = _csr_struct(*K)
        self._check(self.lib.irk_update_operator(self._h, ctypes.byref(csr)))
        self.op_version += 1
        return self.op_version

    # -- steps -------------------------------------------------------------------
    def step(self, u, out=None, allow_not_converged=False):
        """One IRK step ``u -> u + h sum b_i k_i`` (returns ``out``)."""
        if out is None:
            out = torch.empty_like(u)
        stats = B.Stats()
        st = self.lib.irk_step(self._h, _dev(u, self.N, "u"), _dev(out, self.N, "out"),
                               ctypes.byref(stats))
        self.last_stats = stats
        self.last_status = st
        self._check(st, allow_not_converged)
        return out

    def step_noalloc(self, u, out):
        """``irk_step_noalloc``: the step on the library's static scratch (no
        device allocation in the call; ``out`` must be given)."""
        stats = B.Stats()
        st = self.lib.irk_step_noalloc(self._h, _dev(u, self.N, "u"), _dev(out, self.N, "out"),
                                       ctypes.byref(stats))
        self.last_stats = stats
        self.last_status = st
        self._check(st)
        return out

    def step_stages(self, u):
        """One step that also returns the stage vectors k, shape (s, N)."""
        out = torch.empty_like(u)
        k = torch.empty(self.s * self.N, dtype=torch.float64, device=u.device)
        stats = B.Stats()
        st = self.lib.irk_step_stages(self._h, _dev(u, self.N, "u"), _dev(out, self.N, "out"),
                                      _dev(k, self.s * self.N, "k"), ctypes.byref(stats))
        self.last_stats = stats
        self._check(st)
        return out, k.view(self.s, self.N)

    def adjoint_step(self, u_n, lam_np1):
        """Discrete adjoint step: returns ``(lam_n, psi, U)`` (psi, U of shape
        (s, N))."""
        lam_n = torch.empty_like(lam_np1)
        psi = torch.empty(self.s * self.N, dtype=torch.float64, device=u_n.device)
        U = torch.empty_like(psi)
        stats = B.Stats()
        st = self.lib.irk_adjoint_step(self._h, _dev(u_n, self.N, "u_n"),
                                       _dev(lam_np1, self.N, "lam"), _dev(lam_n, self.N, "lam_n"),
                                       _dev(psi, self.s * self.N, "psi"), _dev(U, self.s * self.N, "U"),
                                       ctypes.byref(stats))
        self.last_stats = stats
        self._check(st)
        return lam_n, psi.view(self.s, self.N), U.view(self.s, self.N)

    def grad_diffusion_nodes(self, psi, U, h_x, gnode):
        self._check(self.lib.irk_grad_diffusion_nodes(
            self._h, _dev(psi.reshape(-1), self.s * self.N, "psi"),
            _dev(U.reshape(-1), self.s * self.N, "U"), float(h_x),
            _dev(gnode.reshape(-1), (self.nx + 2) * (self.ny + 2), "gnode")))

    def grad_diffusion_faces(self, psi, U, h_x, gface):
        """Accumulate dJ/dkappa_f into ``gface``: x faces (ny x (nx+1)) then
        y faces ((ny+1) x nx), flattened."""
        nf = self.ny * (self.nx + 1) + (self.ny + 1) * self.nx
        self._check(self.lib.irk_grad_diffusion_faces(
            self._h, _dev(psi.reshape(-1), self.s * self.N, "psi"),
            _dev(U.reshape(-1), self.s * self.N, "U"), float(h_x),
            _dev(gface.reshape(-1), nf, "gface")))

    def apply_operator(self, x):
        y = torch.empty_like(x)
        self._check(self.lib.irk_apply_operator(self._h, _dev(x, self.s * self.N, "x"),
                                                _dev(y, self.s * self.N, "y")))
        return y

    def apply_preconditioner(self, v):
        z = torch.empty_like(v)
        self._check(self.lib.irk_apply_preconditioner(self._h, _dev(v, self.s * self.N, "v"),
                                                      _dev(z, self.s * self.N, "z")))
        return z

    def profile_select(self, kernel_class):
        """Time every launch of one kernel class with HIP events (None stops)."""
        kc = -1 if kernel_class is None else B.KERNEL_CLASSES.index(kernel_class)
        self._check(self.lib.irk_profile_select(self._h, kc))

    def profile_read(self):
        n, ms, by = ctypes.c_longlong(), ctypes.c_double(), ctypes.c_double()
        self._check(self.lib.irk_profile_read(self._h, ctypes.byref(n), ctypes.byref(ms),
                                              ctypes.byref(by)))
        return {"launches": n.value, "ms": ms.value, "bytes": by.value}

    def stats_dict(self):
        s = self.last_stats
        if s is None:
            return None
        return {"iters": s.iters, "restarts": s.restarts, "rel_resid_est": s.rel_resid_est,
                "rel_resid_true": s.rel_resid_true, "seconds": s.seconds}
