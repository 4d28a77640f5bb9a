"""PyTorch-facing wrapper of the radiation step library.

PyTorch provides device memory and the stream; the C ABI of libemma_rt.so does
all the work.  Fields are torch tensors on the context's device:
    N  [G, nz, ny, nx]      float32 (mixed) or float64 (fp64)   photons cm^-3
    F  [G, 3, nz, ny, nx]   same dtype as N                      photons cm^-2 s^-1
    x  [nz, ny, nx]         float64   ionised fraction x_HII
    T  [nz, ny, nx]         float64   K
    n0 [nz, ny, nx]         float64   total hydrogen density n_H, cm^-3
    src_cell [n_src] int64 (flat cell index), src_rate [n_src] float64 (photons/s)
"""
import ctypes

import torch

from . import _lib

C_LIGHT = 2.99792458e10


def group_constants(T_bb, edges_eV):
    """Black-body group constants computed by the library (host quadrature)."""
    return _lib.emma_rt_group_constants(T_bb, list(edges_eV))


class EmmaRT:
    """One radiation context: a fixed grid, group set and precision.

    Calls run on the torch stream that is current on ``device`` when the
    context is created.
    """

    def __init__(self, shape, n_groups, dx, c_red, precision="mixed", groups=None, T_bb=1e5,
                 edges_eV=None, otsa=True, isothermal=False, max_substeps=100000,
                 adjoint_max_steps=0, path="split", device="cuda:0", bc=None, inflow=None,
                 flux="glf"):
        nz, ny, nx = shape
        self.shape = (nz, ny, nx)
        self.G = int(n_groups)
        self.dx = float(dx)
        self.c_red = float(c_red)
        self.precision = precision
        if precision not in ("mixed", "fp64"):
            raise ValueError("precision must be 'mixed' or 'fp64'")
        self.dtype = torch.float32 if precision == "mixed" else torch.float64
        self.device = torch.device(device)
        if groups is None:
            if edges_eV is None:
                raise ValueError("give either groups or edges_eV")
            groups = group_constants(T_bb, edges_eV)
        self.groups = {k: [float(v) for v in groups[k]][: self.G]
                       for k in ("sigma_N", "sigma_E", "mean_E", "frac")}
        cfg = _lib.emma_rt_config()
        cfg.nx, cfg.ny, cfg.nz, cfg.n_groups = nx, ny, nz, self.G
        cfg.dx, cfg.c_red = self.dx, self.c_red
        cfg.precision = _lib.EMMA_RT_MIXED if precision == "mixed" else _lib.EMMA_RT_FP64
        cfg.otsa, cfg.isothermal = int(bool(otsa)), int(bool(isothermal))
        cfg.max_substeps = int(max_substeps)
        cfg.adjoint_max_steps = int(adjoint_max_steps)
        if path not in _lib.PATHS:
            raise ValueError(f"path must be one of {sorted(_lib.PATHS)}")
        cfg.path = _lib.PATHS[path]
        self.path = path
        # faces x-, x+, y-, y+, z-, z+: names of _lib.BCS; inflow in photons cm^-2 s^-1
        bc = ["periodic"] * 6 if bc is None else list(bc)
        inflow = [0.0] * 6 if inflow is None else [float(v) for v in inflow]
        if len(bc) != 6 or len(inflow) != 6:
            raise ValueError("bc and inflow need one entry per face (x-, x+, y-, y+, z-, z+)")
        for f in range(6):
            cfg.bc[f] = _lib.BCS[bc[f]] if isinstance(bc[f], str) else int(bc[f])
            cfg.inflow[f] = inflow[f]
        if flux not in _lib.FLUXES:
            raise ValueError(f"flux must be one of {sorted(_lib.FLUXES)}")
        cfg.flux = _lib.FLUXES[flux]
        self.bc, self.inflow, self.flux = bc, inflow, flux
        for g in range(self.G):
            cfg.sigma_N[g] = self.groups["sigma_N"][g]
            cfg.sigma_E[g] = self.groups["sigma_E"][g]
            cfg.mean_E[g] = self.groups["mean_E"][g]
            cfg.src_frac[g] = self.groups["frac"][g]
        self.cfg = cfg
        self.adjoint_max_steps = int(adjoint_max_steps)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            self._ctx = _lib.emma_rt_init(cfg, self.stream.cuda_stream)

    # ---------------------------------------------------------------- helpers
    def close(self):
        if getattr(self, "_ctx", None):
            _lib.emma_rt_free(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, t, name, dtype, shape):
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.device != self.device:
            raise ValueError(f"{name} is on {t.device}, context is on {self.device}")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
        return t.data_ptr()

    def _fields(self, N, F, x, T, n0):
        G, s = self.G, self.shape
        return (self._check(N, "N", self.dtype, (G,) + s),
                self._check(F, "F", self.dtype, (G, 3) + s),
                self._check(x, "x", torch.float64, s),
                self._check(T, "T", torch.float64, s),
                self._check(n0, "n0", torch.float64, s))

    def _sources(self, src_cell, src_rate):
        n = int(src_cell.numel())
        if n == 0:
            return 0, 0, 0
        pc = self._check(src_cell, "src_cell", torch.int64, (n,))
        pr = self._check(src_rate, "src_rate", torch.float64, (n,))
        return n, pc, pr

    def new_state(self, x0=1.2e-3, T0=100.0):
        G, s = self.G, self.shape
        N = torch.zeros((G,) + s, dtype=self.dtype, device=self.device)
        F = torch.zeros((G, 3) + s, dtype=self.dtype, device=self.device)
        x = torch.full(s, x0, dtype=torch.float64, device=self.device)
        T = torch.full(s, T0, dtype=torch.float64, device=self.device)
        return N, F, x, T

    def profile(self, enable=True):
        """Turn per-kernel event timing on or off."""
        _lib.emma_rt_profile_enable(self._ctx, enable)

    def profile_read(self):
        """{kernel name: (launches, total ms)} since the last read (waits)."""
        return _lib.emma_rt_profile_read(self._ctx)

    def max_dt(self):
        return self.dx / (3.0 * self.c_red)

    # ------------------------------------------------------------------ calls
    def step(self, N, F, x, T, n0, src_cell, src_rate, dt, n_steps=1, diag=False,
             raise_on_status=True):
        """Advance the state in place; returns the diagnostics dict if asked."""
        pN, pF, px, pT, pn = self._fields(N, F, x, T, n0)
        n, pc, pr = self._sources(src_cell, src_rate)
        d = _lib.emma_rt_diag() if diag else None
        rc = _lib.emma_rt_step(self._ctx, pN, pF, px, pT, pn, pc, pr, n, dt, n_steps, d)
        if rc != _lib.EMMA_RT_OK and raise_on_status:
            raise _lib.EmmaError(rc, _lib.emma_rt_last_error(self._ctx))
        if diag:
            out = d.as_dict(self.G)
            out["status"] = rc
            return out
        return rc

    def step_noalloc(self, N, F, x, T, n0, src_cell, src_rate, dt, n_steps=1, raise_on_status=True):
        """The same steps through emma_rt_step_noalloc: this context's
        configuration and stream, the library's fixed scratch instead of the
        context's (no device allocation in the call; no diagnostics)."""
        pN, pF, px, pT, pn = self._fields(N, F, x, T, n0)
        n, pc, pr = self._sources(src_cell, src_rate)
        rc = _lib.emma_rt_step_noalloc(self.cfg, self.stream.cuda_stream, pN, pF, px, pT, pn, pc, pr, n, dt,
                                       n_steps)
        if rc != _lib.EMMA_RT_OK and raise_on_status:
            raise _lib.EmmaError(rc, _lib.emma_rt_last_error(None))
        return rc

    def step_crta(self, N, F, x, T, n0, src_cell, src_rate, dt, ref_cell, ratio, x_fine, T_fine, n_fine,
                  n_steps=1, src_child=None, diag=False, raise_on_status=True):
        """Steps with static refinement (coarse transport, chemistry on the
        children of the refined cells; Sec. 5).  ref_cell int64 [n_ref];
        x_fine, T_fine (updated in place), n_fine float64 [n_ref, ratio^3];
        src_child int32 [n_src] (child of each source in a refined cell)."""
        pN, pF, px, pT, pn = self._fields(N, F, x, T, n0)
        n, pc, pr = self._sources(src_cell, src_rate)
        pch = self._check(src_child, "src_child", torch.int32, (n,)) if (n and src_child is not None) else 0
        n_ref = int(ref_cell.numel())
        nc = int(ratio) ** 3
        if n_ref:
            pref = self._check(ref_cell, "ref_cell", torch.int64, (n_ref,))
            pxf = self._check(x_fine, "x_fine", torch.float64, (n_ref, nc))
            pTf = self._check(T_fine, "T_fine", torch.float64, (n_ref, nc))
            pnf = self._check(n_fine, "n_fine", torch.float64, (n_ref, nc))
        else:
            pref = pxf = pTf = pnf = 0
        d = _lib.emma_rt_diag() if diag else None
        rc = _lib.emma_rt_step_crta(self._ctx, pN, pF, px, pT, pn, pc, pr, pch, n, dt, n_steps, pref, n_ref,
                                    int(ratio), pxf, pTf, pnf, d)
        if rc != _lib.EMMA_RT_OK and raise_on_status:
            raise _lib.EmmaError(rc, _lib.emma_rt_last_error(self._ctx))
        if diag:
            out = d.as_dict(self.G)
            out["status"] = rc
            return out
        return rc

    def step_adjoint(self, N0, F0, x0, T0, n0, src_cell, src_rate, dt, n_steps, gN, gF, gx, gT,
                     g_n0, g_rate):
        """In place: (gN, gF, gx, gT) from dL/d(end state) to dL/d(start state);
        g_n0 and g_rate are accumulated."""
        pN, pF, px, pT, pn = self._fields(N0, F0, x0, T0, n0)
        qN, qF, qx, qT, qn = self._fields(gN, gF, gx, gT, g_n0)
        n, pc, pr = self._sources(src_cell, src_rate)
        qr = self._check(g_rate, "g_rate", torch.float64, (n,)) if n else 0
        rc = _lib.emma_rt_step_adjoint(self._ctx, pN, pF, px, pT, pn, pc, pr, n, dt, n_steps,
                                       qN, qF, qx, qT, qn, qr)
        if rc != _lib.EMMA_RT_OK:
            raise _lib.EmmaError(rc, _lib.emma_rt_last_error(self._ctx))

    def step_crta_adjoint(self, N0, F0, x0, T0, n0, src_cell, src_rate, dt, n_steps, ref_cell, ratio,
                          x_fine0, T_fine0, n_fine, gN, gF, gx, gT, g_n0, g_rate, g_x_fine, g_T_fine,
                          g_n_fine, src_child=None, work=None):
        """The adjoint of step_crta, in place as step_adjoint; (g_x_fine,
        g_T_fine) go from dL/d(children's end state) to dL/d(start state) and
        g_n_fine is accumulated.  work: a device tensor of at least
        crta_adjoint_work_bytes(n_steps, n_ref, ratio) bytes (allocated here
        when None)."""
        pN, pF, px, pT, pn = self._fields(N0, F0, x0, T0, n0)
        qN, qF, qx, qT, qn = self._fields(gN, gF, gx, gT, g_n0)
        n, pc, pr = self._sources(src_cell, src_rate)
        qr = self._check(g_rate, "g_rate", torch.float64, (n,)) if n else 0
        pch = self._check(src_child, "src_child", torch.int32, (n,)) if (n and src_child is not None) else 0
        n_ref = int(ref_cell.numel())
        nc = int(ratio) ** 3
        if n_ref:
            pref = self._check(ref_cell, "ref_cell", torch.int64, (n_ref,))
            f = [self._check(t, name, torch.float64, (n_ref, nc)) for t, name in
                 ((x_fine0, "x_fine0"), (T_fine0, "T_fine0"), (n_fine, "n_fine"), (g_x_fine, "g_x_fine"),
                  (g_T_fine, "g_T_fine"), (g_n_fine, "g_n_fine"))]
        else:
            pref, f = 0, [0] * 6
        need = _lib.emma_rt_crta_adjoint_work_bytes(n_steps, n_ref, ratio)
        if need < 0:
            raise ValueError("n_steps must be >= 1 and ratio 2 or 4")
        if work is None and need > 0:
            work = torch.empty(need, dtype=torch.uint8, device=self.device)
        pw, wb = 0, 0
        if work is not None:
            if work.device != self.device or not work.is_contiguous():
                raise ValueError("work must be a contiguous tensor on the context's device")
            pw, wb = work.data_ptr(), work.numel() * work.element_size()
        rc = _lib.emma_rt_step_crta_adjoint(self._ctx, pN, pF, px, pT, pn, pc, pr, pch, n, dt, n_steps, pref,
                                            n_ref, int(ratio), f[0], f[1], f[2], pw, wb, qN, qF, qx, qT, qn,
                                            qr, f[3], f[4], f[5])
        if rc != _lib.EMMA_RT_OK:
            raise _lib.EmmaError(rc, _lib.emma_rt_last_error(self._ctx))


class RTStep(torch.autograd.Function):
    """n_steps radiation steps as a differentiable map of (n0, src_rate, N, F, x, T).

    Forward: the state is kept every K steps (checkpoints).  Backward: each
    K-step segment is recomputed from its checkpoint inside the library (its
    tape) and run backwards with emma_rt_step_adjoint, last segment first.
    The context must have adjoint_max_steps >= K.

        N1, F1, x1, T1 = RTStep.apply(n0, src_rate, N, F, x, T, rt, src_cell, dt, n_steps, K)
    """

    @staticmethod
    def forward(ctx, n0, src_rate, N, F, x, T, rt, src_cell, dt, n_steps, K):
        if K < 1 or K > rt.adjoint_max_steps:
            raise ValueError(f"K must be in 1..{rt.adjoint_max_steps} (the context's adjoint_max_steps)")
        N, F, x, T = N.detach().clone(), F.detach().clone(), x.detach().clone(), T.detach().clone()
        n0d, rated = n0.detach(), src_rate.detach()
        ckpts = []
        done = 0
        while done < n_steps:
            k = min(K, n_steps - done)
            ckpts.append((N.clone(), F.clone(), x.clone(), T.clone(), k))
            rt.step(N, F, x, T, n0d, src_cell, rated, dt, n_steps=k)
            done += k
        ctx.rt, ctx.src_cell, ctx.dt, ctx.ckpts = rt, src_cell, dt, ckpts
        ctx.save_for_backward(n0d, rated)
        return N, F, x, T

    @staticmethod
    def backward(ctx, gN, gF, gx, gT):
        n0, rate = ctx.saved_tensors
        rt = ctx.rt
        like = ctx.ckpts[0]

        def grad_or_zero(g, ref):
            return g.detach().to(ref.dtype).contiguous().clone() if g is not None else torch.zeros_like(ref)

        gN, gF = grad_or_zero(gN, like[0]), grad_or_zero(gF, like[1])
        gx, gT = grad_or_zero(gx, like[2]), grad_or_zero(gT, like[3])
        g_n0 = torch.zeros_like(n0)
        g_rate = torch.zeros_like(rate)
        for (N0, F0, x0, T0, k) in reversed(ctx.ckpts):
            rt.step_adjoint(N0, F0, x0, T0, n0, ctx.src_cell, rate, ctx.dt, k, gN, gF, gx, gT, g_n0,
                            g_rate)
        ctx.ckpts = None
        return g_n0, g_rate, gN, gF, gx, gT, None, None, None, None, None
