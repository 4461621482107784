"""Python binding over the C ABI: a Plan owns a libphi plan and its workspace.

PyTorch provides device memory (the workspace and the caller's vectors) and
the stream; every step of Phi, Phi^dagger and the dual step runs in the HIP
kernels of libphi.so.
"""
import ctypes

import numpy as np

from . import _lib as L


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _dptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(torch, device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """Phi = Theta G F Z for L channels of an Ny x Nx image with data blocks.

    base: int32 [M_tot, 2] window origins (user order, blocks concatenated);
    stencil: [M_tot] window sizes; n_blocks: [L]; n_vis: [sum B];
    theta: [sum B] or None; scale_y/scale_x: FP64 Z scales.
    """

    def __init__(self, ny, nx, n_blocks, n_vis, base, stencil, scale_y, scale_x, theta=None,
                 g_prec="c64", flags=0, tile=0, persist_blocks=0, device="cuda:0", bind=True):
        self._lib = L.load()
        self.ny, self.nx = int(ny), int(nx)
        self._n_blocks = np.ascontiguousarray(n_blocks, dtype=np.int32)
        self._n_vis = np.ascontiguousarray(n_vis, dtype=np.int64)
        self._base = np.ascontiguousarray(base, dtype=np.int32).reshape(-1, 2)
        self._stencil = np.ascontiguousarray(stencil, dtype=np.uint8)
        self._sy = np.ascontiguousarray(scale_y, dtype=np.float64)
        self._sx = np.ascontiguousarray(scale_x, dtype=np.float64)
        self._theta = None if theta is None else np.ascontiguousarray(theta, dtype=np.float64)
        self.L = len(self._n_blocks)
        self.nblk = int(self._n_blocks.sum())
        self.M = int(self._n_vis.sum())
        self.g_prec = g_prec
        d = L.Desc()
        d.n_channels, d.ny, d.nx = self.L, self.ny, self.nx
        d.h_n_blocks = self._n_blocks.ctypes.data
        d.h_n_vis = self._n_vis.ctypes.data
        d.h_base = self._base.ctypes.data if self.M else None
        d.h_stencil = self._stencil.ctypes.data if self.M else None
        d.h_theta = self._theta.ctypes.data if self._theta is not None else None
        d.h_scale_y = self._sy.ctypes.data
        d.h_scale_x = self._sx.ctypes.data
        d.g_prec = L.G_PREC[g_prec] if isinstance(g_prec, str) else int(g_prec)
        d.flags, d.tile, d.persist_blocks = int(flags), int(tile), int(persist_blocks)
        self._h = ctypes.c_void_p()
        L.check(self._lib.phi_plan_create(ctypes.byref(d), ctypes.byref(self._h)), "phi_plan_create")
        self.device = device
        self.ws = None
        if bind:
            self.bind()

    # ---------------------------------------------------------------- setup
    def info(self):
        i = L.Info()
        L.check(self._lib.phi_plan_get_info(self._h, ctypes.byref(i)), "phi_plan_get_info")
        return {k: getattr(i, k) for k, _ in L.Info._fields_}

    def workspace_size(self):
        n = ctypes.c_size_t()
        L.check(self._lib.phi_plan_workspace_size(self._h, ctypes.byref(n)), "phi_plan_workspace_size")
        return n.value

    def bind(self):
        import torch
        n = self.workspace_size()
        self.ws = torch.empty(n, dtype=torch.uint8, device=self.device)
        L.check(self._lib.phi_plan_bind(self._h, _dptr(self.ws), n, _stream(torch, self.device)),
                "phi_plan_bind")

    def load_g(self, block, windows):
        """Upload block `block`'s windows (user order, S*S row-major each)."""
        import torch
        w = np.ascontiguousarray(windows)
        if w.dtype == np.complex128:
            kind = L.HOST_C128
        elif w.dtype == np.complex64:
            kind = L.HOST_C64
        else:
            raise TypeError("windows must be complex128 or complex64")
        L.check(self._lib.phi_plan_load_g(self._h, int(block), _ptr(w), kind, _stream(torch, self.device)),
                "phi_plan_load_g")

    def load_kb(self, block, kappa):
        """Kaiser-Bessel mode: continuous grid coordinates [n, 2] (FP64, user order)."""
        import torch
        k = np.ascontiguousarray(kappa, dtype=np.float64).reshape(-1, 2)
        L.check(self._lib.phi_plan_load_kb(self._h, int(block), _ptr(k), _stream(torch, self.device)),
                "phi_plan_load_kb")

    def set_flags(self, flags):
        L.check(self._lib.phi_plan_set_flags(self._h, int(flags)), "phi_plan_set_flags")

    def set_tuning(self, tile, persist_blocks=0):
        import torch
        L.check(self._lib.phi_plan_set_tuning(self._h, int(tile), int(persist_blocks), _stream(torch, self.device)),
                "phi_plan_set_tuning")

    def set_theta(self, theta):
        import torch
        t = np.ascontiguousarray(theta, dtype=np.float64)
        L.check(self._lib.phi_plan_set_theta(self._h, _ptr(t), _stream(torch, self.device)),
                "phi_plan_set_theta")

    # ---------------------------------------------------------------- order
    def to_plan(self, v_user, out=None):
        import torch
        out = torch.empty_like(v_user) if out is None else out
        L.check(self._lib.phi_to_plan_order(self._h, _dptr(v_user), _dptr(out), _stream(torch, self.device)),
                "phi_to_plan_order")
        return out

    def from_plan(self, v_plan, out=None):
        import torch
        out = torch.empty_like(v_plan) if out is None else out
        L.check(self._lib.phi_from_plan_order(self._h, _dptr(v_plan), _dptr(out), _stream(torch, self.device)),
                "phi_from_plan_order")
        return out

    # ------------------------------------------------------------ operators
    def _check_img(self, x):
        import torch
        if x.dtype != torch.float32 or not x.is_contiguous() or x.numel() != self.L * self.ny * self.nx:
            raise ValueError("image must be contiguous float32 [L, Ny, Nx]")

    def _check_vis(self, v):
        import torch
        if v.dtype != torch.complex64 or not v.is_contiguous() or v.numel() != self.M:
            raise ValueError("visibilities must be contiguous complex64 [M_tot]")

    def forward(self, x, out=None):
        """y = Phi x (plan order)."""
        import torch
        self._check_img(x)
        y = torch.empty(self.M, dtype=torch.complex64, device=self.device) if out is None else out
        self._check_vis(y)
        L.check(self._lib.phi_forward(self._h, _dptr(x), _dptr(y), _stream(torch, self.device)), "phi_forward")
        return y

    def adjoint(self, v, out=None):
        """x = Re Phi^dagger v (v in plan order)."""
        import torch
        self._check_vis(v)
        x = torch.empty((self.L, self.ny, self.nx), dtype=torch.float32, device=self.device) if out is None else out
        self._check_img(x)
        L.check(self._lib.phi_adjoint(self._h, _dptr(v), _dptr(x), _stream(torch, self.device)), "phi_adjoint")
        return x

    def dual_step(self, xt, v, y, eps, sigma=None, grad=None, rho=None, res=None):
        """In-place l2-ball dual step on v; returns (grad, rho, res)."""
        import torch
        self._check_img(xt)
        self._check_vis(v)
        self._check_vis(y)
        dev = self.device
        grad = torch.empty((self.L, self.ny, self.nx), dtype=torch.float32, device=dev) if grad is None else grad
        rho = torch.empty(self.nblk, dtype=torch.float64, device=dev) if rho is None else rho
        res = torch.empty(self.nblk, dtype=torch.float64, device=dev) if res is None else res
        for t in (eps,) + ((sigma,) if sigma is not None else ()):
            if t.dtype != torch.float64 or t.numel() != self.nblk:
                raise ValueError("eps / sigma must be float64 [sum B]")
        L.check(self._lib.l2ball_dual_step(self._h, _dptr(xt), _dptr(v), _dptr(y), _dptr(eps), _dptr(sigma),
                                           _dptr(grad), _dptr(rho), _dptr(res), _stream(torch, dev)),
                "l2ball_dual_step")
        return grad, rho, res

    def psf(self, out=None):
        """(PSF images [L][Ny][Nx], peaks [L] float64): Phi_l^dagger Phi_l delta
        and its value at the phase centre (eta_l = 1 / peak)."""
        import torch
        x = out if out is not None else torch.empty((self.L, self.ny, self.nx), dtype=torch.float32,
                                                      device=self.device)
        self._check_img(x)
        peak = torch.empty(self.L, dtype=torch.float64, device=self.device)
        L.check(self._lib.phi_psf(self._h, _dptr(x), _dptr(peak), _stream(torch, self.device)), "phi_psf")
        return x, peak

    def residual_image(self, x, y, eta=None, out=None):
        """eta_l Re Phi_l^dagger (y_l - Phi_l x_l); y in plan order."""
        import torch
        self._check_img(x)
        self._check_vis(y)
        r = out if out is not None else torch.empty_like(x)
        if eta is not None:
            assert eta.dtype == torch.float64 and eta.numel() == self.L
        L.check(self._lib.phi_residual_image(self._h, _dptr(x), _dptr(y), _dptr(eta), _dptr(r),
                                             _stream(torch, self.device)), "phi_residual_image")
        return r

    def power_iteration(self, x, n_iter, tmp=None):
        """||Phi_l||^2 estimates (float64 [L]) after n_iter power steps; x (float32
        [L][Ny][Nx], nonzero per channel) is replaced by the last unit iterate."""
        import torch
        self._check_img(x)
        t = tmp if tmp is not None else torch.empty_like(x)
        nu = torch.empty(self.L, dtype=torch.float64, device=self.device)
        L.check(self._lib.phi_power_iteration(self._h, _dptr(x), _dptr(t), int(n_iter), _dptr(nu),
                                              _stream(torch, self.device)), "phi_power_iteration")
        return nu

    def power_iteration_static(self, x, n_iter):
        """power_iteration without a scratch image (phi_power_iteration_static:
        the library's fixed per-GPU scratch array, no allocation)."""
        import torch
        self._check_img(x)
        nu = torch.empty(self.L, dtype=torch.float64, device=self.device)
        L.check(self._lib.phi_power_iteration_static(self._h, _dptr(x), int(n_iter), _dptr(nu),
                                                     _stream(torch, self.device)), "phi_power_iteration_static")
        return nu

    # ------------------------------------------------------------- G builder
    def build_g(self, block, kappa, h, a, ant=None, dde=None, J=7):
        """Compute block `block`'s rows of G on the device (phi_plan_build_g).
        kappa: float64 [n, 2]; h: int32 [n]; a: float64 [n]; ant: int32
        [n, 2] or None; dde: complex128 [n_ant, sa, sa] or None (device
        tensors, user order of the block)."""
        import torch
        d = L.GBuild()
        d.J = int(J)
        d.n_ant = int(dde.shape[0]) if dde is not None else 0
        d.sa = int(dde.shape[1]) if dde is not None else 1
        for t, dt in ((kappa, torch.float64), (h, torch.int32), (a, torch.float64)):
            if t.dtype != dt or not t.is_contiguous():
                raise ValueError("kappa float64 [n, 2], h int32 [n], a float64 [n], contiguous")
        if (ant is None) != (dde is None):
            raise ValueError("ant and dde go together")
        if ant is not None and (ant.dtype != torch.int32 or dde.dtype != torch.complex128):
            raise ValueError("ant int32 [n, 2], dde complex128 [n_ant, sa, sa]")
        L.check(self._lib.phi_plan_build_g(self._h, int(block), ctypes.byref(d), _dptr(kappa), _dptr(h), _dptr(a),
                                           _dptr(ant), _dptr(dde), _stream(torch, self.device)),
                "phi_plan_build_g")

    def read_g(self, block, n_taps):
        """Block `block`'s stored G in user order (complex128, n_taps = sum of
        its S^2), converted exactly from the stored precision."""
        import torch
        out = np.empty(int(n_taps), dtype=np.complex128)
        L.check(self._lib.phi_plan_read_g(self._h, int(block), _ptr(out), L.HOST_C128,
                                          _stream(torch, self.device)), "phi_plan_read_g")
        return out

    # ------------------------------------------------------------ PDFB loop
    @staticmethod
    def eps_rule(lambda_lo=0.99, lambda_hi=1.01, lambda_mix=0.618, var_tol=1e-3, min_gap=10, freeze=True):
        """The adaptive l2-bound rule as the C struct (defaults as in the
        header's example values)."""
        r = L.EpsRule()
        r.lambda_lo, r.lambda_hi, r.lambda_mix, r.var_tol = lambda_lo, lambda_hi, lambda_mix, var_tol
        r.min_gap, r.freeze = int(min_gap), 1 if freeze else 0
        return r

    def _f64(self, t, n, what):
        import torch
        if t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous():
            raise ValueError("%s must be contiguous float64 [%d]" % (what, n))

    def pdfb_primal(self, x, xt, grad, tau, var=None):
        """x <- max(x - tau_l grad_l, 0), xt <- 2 x+ - x (in place); returns
        var float64 [L][2] = (||x+ - x||^2, ||x+||^2)."""
        import torch
        for t in (x, xt, grad):
            self._check_img(t)
        self._f64(tau, self.L, "tau")
        var = torch.empty((self.L, 2), dtype=torch.float64, device=self.device) if var is None else var
        self._f64(var, 2 * self.L, "var")
        L.check(self._lib.phi_pdfb_primal(self._h, _dptr(x), _dptr(xt), _dptr(grad), _dptr(tau), _dptr(var),
                                          _stream(torch, self.device)), "phi_pdfb_primal")
        return var

    def eps_update(self, res, var, eps, state, rule):
        """One application of the adaptive rule (eps, state updated in place)."""
        import torch
        self._f64(res, self.nblk, "res")
        self._f64(eps, self.nblk, "eps")
        self._f64(var, 2 * self.L, "var")
        if state.dtype != torch.int32 or state.numel() != 3 * self.nblk:
            raise ValueError("state must be int32 [sum B][3]")
        L.check(self._lib.phi_eps_update(self._h, _dptr(res), _dptr(var), ctypes.byref(rule), _dptr(eps),
                                         _dptr(state), _stream(torch, self.device)), "phi_eps_update")

    def pdfb_run(self, x, xt, v, y, eps, tau, n_iter, sigma=None, rule=None, state=None, grad=None, rho=None,
                 res=None, var=None):
        """n_iter PDFB iterations in place on x, xt, v (and eps, state with a
        rule).  Returns (grad, rho, res, var, state) of the last iteration."""
        import torch
        dev = self.device
        self._check_img(x)
        self._check_img(xt)
        self._check_vis(v)
        self._check_vis(y)
        self._f64(eps, self.nblk, "eps")
        self._f64(tau, self.L, "tau")
        if sigma is not None:
            self._f64(sigma, self.nblk, "sigma")
        grad = torch.empty_like(x) if grad is None else grad
        rho = torch.empty(self.nblk, dtype=torch.float64, device=dev) if rho is None else rho
        res = torch.empty(self.nblk, dtype=torch.float64, device=dev) if res is None else res
        var = torch.empty((self.L, 2), dtype=torch.float64, device=dev) if var is None else var
        self._f64(var, 2 * self.L, "var")
        if rule is not None and state is None:
            state = torch.zeros((self.nblk, 3), dtype=torch.int32, device=dev)
        L.check(self._lib.phi_pdfb_run(self._h, _dptr(x), _dptr(xt), _dptr(v), _dptr(y), _dptr(eps),
                                       _dptr(sigma), _dptr(tau), int(n_iter),
                                       ctypes.byref(rule) if rule is not None else None, _dptr(state),
                                       _dptr(grad), _dptr(rho), _dptr(res), _dptr(var), _stream(torch, dev)),
                "phi_pdfb_run")
        return grad, rho, res, var, state

    def check(self):
        import torch
        L.check(self._lib.phi_plan_check(self._h, _stream(torch, self.device)), "phi_plan_check")

    # --------------------------------------------------------------- timing
    def set_timing(self, on):
        L.check(self._lib.phi_plan_set_timing(self._h, 1 if on else 0), "phi_plan_set_timing")

    def get_timing(self):
        ms = (ctypes.c_double * 16)()
        names = (ctypes.c_char_p * 16)()
        n = ctypes.c_int32()
        calls = ctypes.c_int64()
        L.check(self._lib.phi_plan_get_timing(self._h, 16, ms, names, ctypes.byref(n), ctypes.byref(calls)),
                "phi_plan_get_timing")
        return {names[i].decode(): ms[i] for i in range(n.value)}, calls.value

    def autotune(self, reps=3):
        import torch
        return self._lib.phi_plan_autotune(self._h, _stream(torch, self.device), int(reps))

    # ------------------------------------------- gridding reduction (PHI_DR)
    def dr_rows(self):
        """(cells [M'] int64, window origins [M', 2] int32, edges [M'] uint8) of
        the reduced rows, in reduced order (host, available before binding)."""
        m = int(self.info()["dr_rows"])
        cells = np.empty(m, np.int64)
        base = np.empty((m, 2), np.int32)
        sten = np.empty(m, np.uint8)
        L.check(self._lib.phi_dr_rows(self._h, _ptr(cells), _ptr(base), _ptr(sten)), "phi_dr_rows")
        return cells, base, sten

    def dr_setup(self, y=None, out=None):
        """Device set-up of the reduction from the loaded G: returns (y' complex64
        [M'] in reduced order, M'_b int64 [sum B]); y in plan order or None."""
        import torch
        m = int(self.info()["dr_rows"])
        yred = torch.empty(m, dtype=torch.complex64, device=self.device) if out is None else out
        if y is not None:
            self._check_vis(y)
        m_red = np.empty(self.nblk, np.int64)
        L.check(self._lib.phi_dr_setup(self._h, _dptr(y), _dptr(yred), _ptr(m_red), _stream(torch, self.device)),
                "phi_dr_setup")
        return yred, m_red

    def dual_step_dr(self, xt, vred, yred, eps_red, sigma=None, grad=None, rho=None, res=None):
        """l2ball_dual_step_dr: the reduced dual step in place on vred; returns (grad, rho, res)."""
        import torch
        self._check_img(xt)
        dev = self.device
        m = int(self.info()["dr_rows"])
        for t in (vred, yred):
            if t.dtype != torch.complex64 or not t.is_contiguous() or t.numel() != m:
                raise ValueError("reduced vectors must be contiguous complex64 [M']")
        grad = torch.empty((self.L, self.ny, self.nx), dtype=torch.float32, device=dev) if grad is None else grad
        rho = torch.empty(self.nblk, dtype=torch.float64, device=dev) if rho is None else rho
        res = torch.empty(self.nblk, dtype=torch.float64, device=dev) if res is None else res
        self._f64(eps_red, self.nblk, "eps_red")
        L.check(self._lib.l2ball_dual_step_dr(self._h, _dptr(xt), _dptr(vred), _dptr(yred), _dptr(eps_red),
                                              _dptr(sigma), _dptr(grad), _dptr(rho), _dptr(res),
                                              _stream(torch, dev)), "l2ball_dual_step_dr")
        return grad, rho, res

    def reduced(self):
        """The reduced plan (phi_dr_plan) as a Plan object borrowing this plan's
        handle: forward is Phi', adjoint Re Phi'^dagger, dual_step the reduced
        step; it lives as long as this plan."""
        h = ctypes.c_void_p()
        L.check(self._lib.phi_dr_plan(self._h, ctypes.byref(h)), "phi_dr_plan")
        r = Plan.__new__(Plan)
        r._lib, r._h, r._owner, r.device = self._lib, h, self, self.device
        r.ny, r.nx, r.L, r.nblk = self.ny, self.nx, self.L, self.nblk
        r._n_blocks = self._n_blocks
        r.g_prec = self.g_prec
        r.M = int(r.info()["n_vis_total"])
        r.ws = None
        return r

    def close(self):
        if getattr(self, "_owner", None) is not None:   # a reduced plan goes with its plan
            self._h = ctypes.c_void_p()
            return
        if getattr(self, "_h", None) and self._h.value:
            self._lib.phi_plan_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
