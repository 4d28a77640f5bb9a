"""The hand-written adjoint (emma_rt_step_adjoint and RTStep) on the GPU.

1. Dot-product test against the oracle's dual-number tangent:
   <w, J v> (oracle, FP64) = <J^T w, v> (library), relative 1e-9, on random
   ragged grids with sources, several steps, through the C ABI.
2. Central differences of the FP64 forward (h = 1e-6 relative) for the
   gradient of a loss on x_HII with respect to the source rates and n_H, on
   the 64^3 two-group workload with checkpoints every 10 steps; directions
   whose +h and -h runs take different chemistry decisions (substep or attempt
   totals differ) straddle a kink of the discrete map and are reported, not
   compared.  Agreement 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import emma_inputs as E
import oracle
from gpu_helpers import DEV, groups_for, to_dev

pytestmark = pytest.mark.gpu


def _rt(shape, G, dx, c, K, precision="fp64", **kw):
    from paper_1508_07888_amd import EmmaRT
    return EmmaRT(shape, G, dx, c, precision=precision, groups=groups_for(G), adjoint_max_steps=K,
                  device=DEV, **kw)


@pytest.mark.parametrize("shape,G,seed,steps,otsa", [((7, 9, 11), 2, 1, 3, 1), ((12, 10, 70), 3, 2, 4, 1),
                                                     ((6, 6, 6), 1, 3, 5, 1), ((8, 7, 9), 3, 4, 3, 0)])
def test_adjoint_dot_product_against_oracle_tangent(shape, G, seed, steps, otsa):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-2, f_max=0.6, p_full=0.0,
                                    p_dark=0.0)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    cells = rng.integers(0, V, 4).astype(np.int64)
    cells[1] = cells[0]
    rates = 10 ** rng.uniform(48, 50, 4)
    g = groups_for(G)
    # tangent direction: relative perturbations of every input
    dN = N * rng.standard_normal(N.shape)
    dF = F * rng.standard_normal(F.shape)
    dxh = x * (1 - x) * rng.standard_normal(x.shape)
    dT = T * rng.standard_normal(T.shape)
    dn0 = n0 * rng.standard_normal(n0.shape)
    dr = rates * rng.standard_normal(rates.shape)
    kw = dict(dx=dx, c_red=c, dt=dt, n_steps=steps, groups=g, otsa=otsa)
    (oN, oF, ox, oT), (tN, tF, tx, tT), cnt = oracle.run_tangent(
        N, F, x, T, n0, cells, rates, dN, dF, dxh, dT, dn0, dr, **kw)
    # weights scaled by the output magnitudes so every field contributes
    wN = rng.standard_normal(N.shape) / (np.abs(oN).max() + 1e-300)
    wF = rng.standard_normal(F.shape) / (np.abs(oF).max() + 1e-300)
    wx = rng.standard_normal(x.shape)
    wT = rng.standard_normal(T.shape) / np.abs(oT).max()
    lhs = (wN * tN).sum() + (wF * tF).sum() + (wx * tx).sum() + (wT * tT).sum()

    rt = _rt(shape, G, dx, c, steps, otsa=otsa)
    gN, gF, gx, gT = to_dev(wN), to_dev(wF), to_dev(wx), to_dev(wT)
    g_n0 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    g_rate = torch.zeros(4, dtype=torch.float64, device=DEV)
    rt.step_adjoint(to_dev(N), to_dev(F), to_dev(x), to_dev(T), to_dev(n0), to_dev(cells, torch.int64),
                    to_dev(rates), dt, steps, gN, gF, gx, gT, g_n0, g_rate)
    torch.cuda.synchronize()
    parts = [(gN.cpu().numpy() * dN).sum(), (gF.cpu().numpy() * dF).sum(),
             (gx.cpu().numpy() * dxh).sum(), (gT.cpu().numpy() * dT).sum(),
             (g_n0.cpu().numpy() * dn0).sum(), (g_rate.cpu().numpy() * dr).sum()]
    rhs = sum(parts)
    scale = sum(abs(p) for p in parts)
    print(f"{shape} G={G}: <w,Jv> {lhs:.14e} <J^T w,v> {rhs:.14e} parts {parts}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * max(scale, abs(lhs))
    rt.close()


@pytest.mark.parametrize("shape,G,seed,steps", [((9, 8, 10), 2, 11, 1), ((7, 12, 66), 3, 12, 1)])
def test_adjoint_dot_product_through_floor_limiter_and_clip(shape, G, seed, steps):
    """Inputs that make the floor, the limiter and the closure clip fire by a
    margin (no decision near its threshold, so the oracle's tangent and the
    library's forward take the same branches): 15 % of the cells with
    |F| = (1.05..1.5) c N (unrealisable: clipped closure, limited after the
    update), 5 % dark (N = F = 0), 5 % with N < 0 (floored).  The reverse of
    the floor and the limiter follows the forward's own decisions.  One step:
    a limited cell leaves the step at f = 1 to rounding, where the next step's
    closure sits on its kink and the two implementations may legitimately
    take different sides."""
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-2, f_max=0.6, p_full=0.0,
                                    p_dark=0.0)
    rng = np.random.default_rng(seed)
    hi = rng.random(N.shape) < 0.15
    F[:, :, :, :, :] = np.where(hi[:, None], F / np.maximum(np.linalg.norm(F, axis=1, keepdims=True), 1e-300)
                                * c * N[:, None] * rng.uniform(1.05, 1.5, N.shape)[:, None], F)
    dark = (rng.random(N.shape) < 0.05) & ~hi
    N[dark] = 0.0
    F[np.broadcast_to(dark[:, None], F.shape)] = 0.0
    neg = (rng.random(N.shape) < 0.05) & ~hi & ~dark
    N[neg] = -0.3 * N[neg]
    V = int(np.prod(shape))
    cells = rng.integers(0, V, 4).astype(np.int64)
    rates = 10 ** rng.uniform(48, 50, 4)
    g = groups_for(G)
    dN = N * rng.standard_normal(N.shape)
    dF = F * rng.standard_normal(F.shape)
    dxh = x * (1 - x) * rng.standard_normal(x.shape)
    dT = T * rng.standard_normal(T.shape)
    dn0 = n0 * rng.standard_normal(n0.shape)
    dr = rates * rng.standard_normal(rates.shape)
    kw = dict(dx=dx, c_red=c, dt=dt, n_steps=steps, groups=g)
    (oN, oF, ox, oT), (tN, tF, tx, tT), cnt = oracle.run_tangent(
        N, F, x, T, n0, cells, rates, dN, dF, dxh, dT, dn0, dr, **kw)
    assert cnt["limiter"] > 0 and cnt["neg_clamp"] > 0, cnt
    wN = rng.standard_normal(N.shape) / (np.abs(oN).max() + 1e-300)
    wF = rng.standard_normal(F.shape) / (np.abs(oF).max() + 1e-300)
    wx = rng.standard_normal(x.shape)
    wT = rng.standard_normal(T.shape) / np.abs(oT).max()
    lhs = (wN * tN).sum() + (wF * tF).sum() + (wx * tx).sum() + (wT * tT).sum()
    rt = _rt(shape, G, dx, c, steps)
    gN, gF, gx, gT = to_dev(wN), to_dev(wF), to_dev(wx), to_dev(wT)
    g_n0 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    g_rate = torch.zeros(4, dtype=torch.float64, device=DEV)
    rt.step_adjoint(to_dev(N), to_dev(F), to_dev(x), to_dev(T), to_dev(n0), to_dev(cells, torch.int64),
                    to_dev(rates), dt, steps, gN, gF, gx, gT, g_n0, g_rate)
    torch.cuda.synchronize()
    parts = [(gN.cpu().numpy() * dN).sum(), (gF.cpu().numpy() * dF).sum(),
             (gx.cpu().numpy() * dxh).sum(), (gT.cpu().numpy() * dT).sum(),
             (g_n0.cpu().numpy() * dn0).sum(), (g_rate.cpu().numpy() * dr).sum()]
    rhs = sum(parts)
    scale = sum(abs(p) for p in parts)
    print(f"{shape} G={G} limiter {cnt['limiter']} floor {cnt['neg_clamp']}: <w,Jv> {lhs:.14e} "
          f"<J^T w,v> {rhs:.14e}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * max(scale, abs(lhs))
    rt.close()


def _loss_setup(precision="fp64"):
    w = E.make_workload("adjoint64")
    G, shape = w["G"], w["shape"]
    rt = _rt(shape, G, w["dx"], w["c_red"], w["K"], precision=precision)
    fdt = rt.dtype
    st = dict(N=to_dev(w["N"], fdt), F=to_dev(w["F"], fdt), x=to_dev(w["x"]), T=to_dev(w["T"]),
              n0=to_dev(w["n0"]), cells=to_dev(w["src_cell"], torch.int64), rates=to_dev(w["src_rate"]))
    sub = (slice(24, 40),) * 3
    return w, rt, st, sub


def _forward_loss(w, rt, st, sub, n0, rates, diag=False):
    N, F, x, T = st["N"].clone(), st["F"].clone(), st["x"].clone(), st["T"].clone()
    d = rt.step(N, F, x, T, n0, st["cells"], rates, w["dt"], n_steps=w["steps"], diag=diag,
                raise_on_status=False)
    return float(x[sub].sum()), d


def test_adjoint64_gradient_matches_central_differences():
    from paper_1508_07888_amd import RTStep
    w, rt, st, sub = _loss_setup()
    n0 = st["n0"].clone().requires_grad_(True)
    rates = st["rates"].clone().requires_grad_(True)
    N1, F1, x1, T1 = RTStep.apply(n0, rates, st["N"], st["F"], st["x"], st["T"], rt, st["cells"],
                                  w["dt"], w["steps"], w["K"])
    loss = x1[sub].sum()
    loss.backward()
    g_rate = rates.grad.cpu().numpy()
    g_n0 = n0.grad
    base, d0 = _forward_loss(w, rt, st, sub, st["n0"], st["rates"], diag=True)
    assert abs(base - float(loss.detach())) <= 1e-12 * abs(base)
    h = 1e-6
    r0 = st["rates"]
    stable = 0
    for s in range(r0.numel()):
        rp, rm = r0.clone(), r0.clone()
        rp[s] *= 1 + h
        rm[s] *= 1 - h
        lp, dp = _forward_loss(w, rt, st, sub, st["n0"], rp, diag=True)
        lm, dm = _forward_loss(w, rt, st, sub, st["n0"], rm, diag=True)
        fd = (lp - lm) / (2 * h * float(r0[s]))
        same = dp["substeps"] == dm["substeps"] and dp["attempts"] == dm["attempts"]
        rel = abs(fd - g_rate[s]) / max(abs(fd), 1e-300)
        print(f"rate {s}: adjoint {g_rate[s]:.10e} fd {fd:.10e} rel {rel:.2e} stable {same}", flush=True)
        if same:
            stable += 1
            assert rel <= 1e-5
    assert stable >= 6
    rng = np.random.default_rng(0)
    n_stable = 0
    # n0 directions: three over the whole grid, then five supported on 4^3
    # blocks inside the loss volume (fewer cells whose chemistry decisions a
    # perturbation can flip); at least two must be decision-stable
    for trial in range(8):
        d = rng.standard_normal(w["shape"])
        if trial >= 3:
            m = np.zeros(w["shape"])
            z, y, x = rng.integers(24, 36, 3)
            m[z:z + 4, y:y + 4, x:x + 4] = 1.0
            d *= m
        dn = st["n0"] * torch.tensor(d, device=DEV)
        lp, dp = _forward_loss(w, rt, st, sub, st["n0"] + h * dn, st["rates"], diag=True)
        lm, dm = _forward_loss(w, rt, st, sub, st["n0"] - h * dn, st["rates"], diag=True)
        fd = (lp - lm) / (2 * h)
        ad = float((g_n0 * dn).sum())
        same = dp["substeps"] == dm["substeps"] and dp["attempts"] == dm["attempts"]
        rel = abs(fd - ad) / max(abs(fd), 1e-300)
        print(f"n0 direction {trial}: adjoint {ad:.10e} fd {fd:.10e} rel {rel:.2e} stable {same}",
              flush=True)
        if same:
            n_stable += 1
            assert rel <= 1e-5
    assert n_stable >= 2
    rt.close()


def test_checkpoint_segmentation_does_not_change_the_gradient():
    from paper_1508_07888_amd import RTStep
    w = E.make_workload("adjoint64", n=16)
    G, shape = w["G"], w["shape"]
    grads = []
    for K in (3, 12):
        rt = _rt(shape, G, w["dx"], w["c_red"], K)
        n0 = to_dev(w["n0"]).requires_grad_(True)
        rates = to_dev(w["src_rate"]).requires_grad_(True)
        out = RTStep.apply(n0, rates, to_dev(w["N"]), to_dev(w["F"]), to_dev(w["x"]), to_dev(w["T"]), rt,
                           to_dev(w["src_cell"], torch.int64), w["dt"], 12, K)
        (out[2].sum() + 1e-3 * out[3].sum()).backward()
        grads.append((n0.grad.cpu().numpy(), rates.grad.cpu().numpy()))
        rt.close()
    for a, b in zip(grads[0], grads[1]):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


@pytest.mark.parametrize("flux", ["glf", "hll"])
def test_mixed_precision_adjoint_close_to_fp64(flux):
    from paper_1508_07888_amd import RTStep
    w = E.make_workload("adjoint64", n=24)
    G, shape = w["G"], w["shape"]
    res = {}
    for precision in ("fp64", "mixed"):
        rt = _rt(shape, G, w["dx"], w["c_red"], 5, precision=precision, flux=flux)
        fdt = rt.dtype
        n0 = to_dev(w["n0"]).requires_grad_(True)
        rates = to_dev(w["src_rate"]).requires_grad_(True)
        out = RTStep.apply(n0, rates, to_dev(w["N"], fdt), to_dev(w["F"], fdt), to_dev(w["x"]),
                           to_dev(w["T"]), rt, to_dev(w["src_cell"], torch.int64), w["dt"], 10, 5)
        out[2].sum().backward()
        res[precision] = (n0.grad.cpu().numpy(), rates.grad.cpu().numpy())
        rt.close()
    for a, b in zip(res["mixed"], res["fp64"]):
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print(f"{flux}: mixed vs fp64 gradient: normwise {err:.2e}", flush=True)
        assert err <= 1e-3


def test_adjoint_argument_errors():
    from paper_1508_07888_amd import EmmaRT, _lib
    n = 6
    rt = EmmaRT((n, n, n), 1, 1e20, 3e9, precision="fp64", groups=groups_for(1), device=DEV)
    N, F, x, T = rt.new_state()
    n0 = torch.full((n, n, n), 1e-3, dtype=torch.float64, device=DEV)
    e = torch.zeros(0, dtype=torch.int64, device=DEV)
    with pytest.raises(_lib.EmmaError):  # no adjoint scratch in this context
        rt.step_adjoint(N, F, x, T, n0, e, e.double(), rt.max_dt(), 1, N.clone(), F.clone(), x.clone(),
                        T.clone(), n0.clone(), e.double())
    rt.close()
    rt = EmmaRT((n, n, n), 1, 1e20, 3e9, precision="fp64", groups=groups_for(1), adjoint_max_steps=2,
                device=DEV)
    with pytest.raises(_lib.EmmaError):  # segment longer than the tape
        rt.step_adjoint(N, F, x, T, n0, e, e.double(), rt.max_dt(), 3, N.clone(), F.clone(), x.clone(),
                        T.clone(), n0.clone(), e.double())
    rt.close()


def test_kernel_timing_through_an_adjoint_call():
    # regression: the tape's forward steps were bracketed twice (an outer
    # bracket around the step's own per-kernel brackets), which left events
    # unrecorded and made the profile read fail.  Also: with timing off the
    # kept-state pass over the cells the segment's forward marked runs on a
    # second stream beside the single-substep pass; with timing on, on the
    # context's stream after it.  Both orders give the same bits.
    w = E.make_workload("adjoint64", n=16)
    G, shape = w["G"], w["shape"]
    K = 4
    rt = _rt(shape, G, w["dx"], w["c_red"], K)
    N0, F0, x0, T0 = to_dev(w["N"]), to_dev(w["F"]), to_dev(w["x"]), to_dev(w["T"])
    n0 = to_dev(w["n0"])
    cells, rates = to_dev(w["src_cell"], torch.int64), to_dev(w["src_rate"])

    def adjoint():
        gN, gF, gT = torch.zeros_like(N0), torch.zeros_like(F0), torch.zeros_like(T0)
        gx = torch.ones_like(x0)
        g_n0, g_rate = torch.zeros_like(n0), torch.zeros_like(rates)
        rt.step_adjoint(N0, F0, x0, T0, n0, cells, rates, w["dt"], K, gN, gF, gx, gT, g_n0, g_rate)
        torch.cuda.synchronize()
        return [t.cpu().numpy() for t in (gN, gF, gx, gT, g_n0, g_rate)]

    # more than one substep somewhere, so the marked-cell pass has work
    N, F, x, T = N0.clone(), F0.clone(), x0.clone(), T0.clone()
    d = rt.step(N, F, x, T, n0, cells, rates, w["dt"], n_steps=K - 1, diag=True, raise_on_status=False)
    assert d["max_sub"] > 1
    side = adjoint()
    rt.profile(True)
    rt.profile_read()
    serial = adjoint()
    kern = rt.profile_read()
    rt.profile(False)
    rt.close()
    for a, b in zip(side, serial):
        assert np.array_equal(a, b)
    assert np.all(np.isfinite(side[4])) and np.any(side[4] != 0)
    # the segment's transport (every step, kept on the tape) is timed as the
    # adjoint's forward; the marked-cell pass (steps 0..K-2) and the work-list
    # pass (every step) are both timed as the deferred chemistry adjoint
    assert "transport" not in kern
    for kind, launches in (("chemistry", K - 1), ("adj_forward", K), ("adj_chemistry", K),
                           ("adj_chemistry_deferred", 2 * K - 1), ("adj_transport", K), ("adj_sources", 1)):
        assert kern[kind][0] == launches, (kind, kern[kind])
        assert kern[kind][1] > 0.0
