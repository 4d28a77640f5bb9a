"""Global boundaries (transmissive, reflective, inflow faces) and the HLL
flux on the GPU, through the C ABI, against the oracle; the adjoint with
boundaries, and the adjoint of the HLL flux, against the oracle's
dual-number tangent; and the mirror symmetry of a reflective octant on the
device itself.

Tolerances as in the periodic parity tests: FP64 1e-12 normwise; mixed 1e-4
on N and F, 1e-6 absolute on x_HII, 1e-3 on T; dot products 1e-9.
"""
import numpy as np
import pytest
import torch

import emma_inputs as E
import oracle
from gpu_helpers import DEV, groups_for, normwise, run_gpu, to_dev

pytestmark = pytest.mark.gpu

P, TR, RF, IN = "periodic", "transmissive", "reflective", "inflow"

CASES = {
    # name: (shape, G, bc x- x+ y- y+ z- z+, inflow per face)
    "transmissive": ((9, 13, 70), 2, [TR] * 6, None),
    "reflective": ((12, 12, 12), 3, [RF] * 6, None),
    "inflow_x": ((5, 20, 66), 2, [IN, TR, P, P, RF, RF], [4e6, 0, 0, 0, 0, 0]),
    "inflow_yz": ((33, 7, 9), 1, [P, P, IN, TR, TR, IN], [0, 0, 2e6, 0, 0, 3e6]),
    "thin": ((1, 1, 64), 2, [TR, RF, RF, RF, RF, TR], None),
    "mixed_kinds": ((6, 5, 130), 4, [RF, TR, TR, RF, IN, TR], [0, 0, 0, 0, 1e6, 0]),
    "whole_tiles": ((6, 8, 128), 2, [TR, TR, P, P, RF, IN], [0, 0, 0, 0, 0, 2e6]),
}


def _case(name, seed):
    shape, G, bc, inflow = CASES[name]
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    cells = rng.integers(0, V, 4).astype(np.int64)
    rates = 10 ** rng.uniform(47, 50, 4)
    return dict(N=N, F=F, x=x, T=T, n0=n0, cells=cells, rates=rates, dx=dx, c=c, dt=dt, G=G,
                bc=bc, inflow=inflow)


def _compare(gpu, ora, precision, label):
    gN, gF, gx, gT = gpu[:4]
    oN, oF, ox, oT = ora[:4]
    eN = normwise(gN, oN, True)
    eF = normwise(gF, oF, True)
    ex = float(np.max(np.abs(gx - ox)))
    eT = normwise(gT, oT)
    print(f"{label} {precision}: N {eN} F {eF} x(abs) {ex:.3e} T {eT:.3e}", flush=True)
    if precision == "fp64":
        assert max(eN) <= 1e-12 and max(eF) <= 1e-12
        assert normwise(gx, ox) <= 1e-12 and eT <= 1e-12
    else:
        assert max(eN) <= 1e-4 and max(eF) <= 1e-4 and ex <= 1e-6 and eT <= 1e-3


@pytest.mark.parametrize("path", ["fused", "split", "reference"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_boundaries_match_oracle(name, precision, path):
    k = _case(name, 21)
    g = groups_for(k["G"])
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=4, groups=g, bc=k["bc"], inflow=k["inflow"])
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                  precision=precision, path=path, **kw)
    _compare(gpu, ora, precision, f"{name} {path}")
    if precision == "fp64":
        d, oc = gpu[4], ora[4]
        assert d["substeps"] == oc["substeps"] and d["limiter_hits"] == oc["limiter"]


@pytest.mark.parametrize("path", ["reference", "split", "fused"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("name", ["transmissive", "inflow_x", "inflow_yz", "thin", "periodic", "reflective",
                                  "mixed_kinds", "whole_tiles"])
def test_hll_matches_oracle(name, precision, path):
    if name == "periodic":
        k = _case("reflective", 22)
        k["bc"], k["inflow"] = None, None
    else:
        k = _case(name, 22)
    g = groups_for(k["G"])
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=4, groups=g, bc=k["bc"], inflow=k["inflow"],
              flux="hll")
    ora = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    gpu = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                  precision=precision, path=path, **kw)
    _compare(gpu, ora, precision, f"hll {name} {path}")


@pytest.mark.parametrize("name", ["transmissive", "reflective", "inflow_x", "mixed_kinds", "thin"])
def test_adjoint_with_boundaries_dot_product(name):
    from paper_1508_07888_amd import EmmaRT
    k = _case(name, 23)
    N, F, x, T, n0 = E.random_state(CASES[name][0], k["G"], k["c"], seed=23, n_scale=1e-2, f_max=0.6,
                                    p_full=0.0, p_dark=0.0)
    shape, G, steps = CASES[name][0], k["G"], 3
    rng = np.random.default_rng(5)
    dN = N * rng.standard_normal(N.shape)
    dF = F * rng.standard_normal(F.shape)
    dxh = x * (1 - x) * rng.standard_normal(x.shape)
    dT = T * rng.standard_normal(T.shape)
    dn0 = n0 * rng.standard_normal(n0.shape)
    dr = k["rates"] * rng.standard_normal(4)
    g = groups_for(G)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=steps, groups=g, bc=k["bc"], inflow=k["inflow"])
    (oN, oF, ox, oT), (tN, tF, tx, tT), _ = oracle.run_tangent(N, F, x, T, n0, k["cells"], k["rates"], dN, dF,
                                                               dxh, dT, dn0, dr, **kw)
    wN = rng.standard_normal(N.shape) / np.abs(oN).max()
    wF = rng.standard_normal(F.shape) / np.abs(oF).max()
    wx = rng.standard_normal(x.shape)
    wT = rng.standard_normal(T.shape) / np.abs(oT).max()
    lhs = (wN * tN).sum() + (wF * tF).sum() + (wx * tx).sum() + (wT * tT).sum()
    rt = EmmaRT(shape, G, k["dx"], k["c"], precision="fp64", groups=g, adjoint_max_steps=steps, device=DEV,
                bc=k["bc"], inflow=k["inflow"])
    gN, gF, gx, gT = to_dev(wN), to_dev(wF), to_dev(wx), to_dev(wT)
    g_n0 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    g_rate = torch.zeros(4, dtype=torch.float64, device=DEV)
    rt.step_adjoint(to_dev(N), to_dev(F), to_dev(x), to_dev(T), to_dev(n0), to_dev(k["cells"], torch.int64),
                    to_dev(k["rates"]), k["dt"], steps, gN, gF, gx, gT, g_n0, g_rate)
    torch.cuda.synchronize()
    parts = [(gN.cpu().numpy() * dN).sum(), (gF.cpu().numpy() * dF).sum(), (gx.cpu().numpy() * dxh).sum(),
             (gT.cpu().numpy() * dT).sum(), (g_n0.cpu().numpy() * dn0).sum(), (g_rate.cpu().numpy() * dr).sum()]
    rhs = sum(parts)
    scale = sum(abs(p) for p in parts)
    print(f"{name}: <w,Jv> {lhs:.14e} <J^T w,v> {rhs:.14e}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * max(scale, abs(lhs))
    rt.close()


@pytest.mark.parametrize("path", ["split", "reference"])
@pytest.mark.parametrize("name,edge", [("periodic", False), ("periodic", True), ("transmissive", False),
                                       ("reflective", True), ("inflow_x", False), ("inflow_yz", True),
                                       ("mixed_kinds", False), ("thin", True)])
def test_hll_adjoint_dot_product(name, edge, path):
    # The adjoint of the HLL flux with M1 wave speeds (speed derivatives,
    # the min/max selections of a+ and a-, ghost terms) against the oracle's
    # dual-number tangent of the same flux.  edge: one step from inputs that
    # make the closure clip, the speed clip, the floor and the limiter fire
    # by a margin, as in the periodic test of them: 15 % of the cells with
    # |F| = (1.05..1.5) c N, 5 % dark, 5 % with N < 0 (a cell limited to
    # f = 1 sits on the closure's kink at the next step, where the two
    # implementations may take different sides to rounding).
    from paper_1508_07888_amd import EmmaRT
    k = _case("reflective" if name == "periodic" else name, 24)
    if name == "periodic":
        k["bc"], k["inflow"] = None, None
    shape = CASES["reflective" if name == "periodic" else name][0]
    G, steps = k["G"], (1 if edge else 3)
    N, F, x, T, n0 = E.random_state(shape, G, k["c"], seed=24, n_scale=1e-2, f_max=0.6, p_full=0.0, p_dark=0.0)
    rng = np.random.default_rng(6)
    if edge:
        c = k["c"]
        hi = rng.random(N.shape) < 0.15
        F = np.where(hi[:, None], F / np.maximum(np.linalg.norm(F, axis=1, keepdims=True), 1e-300)
                     * c * N[:, None] * rng.uniform(1.05, 1.5, N.shape)[:, None], F)
        dark = (rng.random(N.shape) < 0.05) & ~hi
        N[dark] = 0.0
        F[np.broadcast_to(dark[:, None], F.shape)] = 0.0
        neg = (rng.random(N.shape) < 0.05) & ~hi & ~dark
        N[neg] = -0.3 * N[neg]
    dN = N * rng.standard_normal(N.shape)
    dF = F * rng.standard_normal(F.shape)
    dxh = x * (1 - x) * rng.standard_normal(x.shape)
    dT = T * rng.standard_normal(T.shape)
    dn0 = n0 * rng.standard_normal(n0.shape)
    dr = k["rates"] * rng.standard_normal(4)
    g = groups_for(G)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=steps, groups=g, bc=k["bc"], inflow=k["inflow"],
              flux="hll")
    (oN, oF, ox, oT), (tN, tF, tx, tT), _ = oracle.run_tangent(N, F, x, T, n0, k["cells"], k["rates"], dN, dF,
                                                               dxh, dT, dn0, dr, **kw)
    wN = rng.standard_normal(N.shape) / np.abs(oN).max()
    wF = rng.standard_normal(F.shape) / np.abs(oF).max()
    wx = rng.standard_normal(x.shape)
    wT = rng.standard_normal(T.shape) / np.abs(oT).max()
    lhs = (wN * tN).sum() + (wF * tF).sum() + (wx * tx).sum() + (wT * tT).sum()
    rt = EmmaRT(shape, G, k["dx"], k["c"], precision="fp64", groups=g, adjoint_max_steps=steps, device=DEV,
                bc=k["bc"], inflow=k["inflow"], flux="hll", path=path)
    gN, gF, gx, gT = to_dev(wN), to_dev(wF), to_dev(wx), to_dev(wT)
    g_n0 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    g_rate = torch.zeros(4, dtype=torch.float64, device=DEV)
    rt.step_adjoint(to_dev(N), to_dev(F), to_dev(x), to_dev(T), to_dev(n0), to_dev(k["cells"], torch.int64),
                    to_dev(k["rates"]), k["dt"], steps, gN, gF, gx, gT, g_n0, g_rate)
    torch.cuda.synchronize()
    parts = [(gN.cpu().numpy() * dN).sum(), (gF.cpu().numpy() * dF).sum(), (gx.cpu().numpy() * dxh).sum(),
             (gT.cpu().numpy() * dT).sum(), (g_n0.cpu().numpy() * dn0).sum(), (g_rate.cpu().numpy() * dr).sum()]
    rhs = sum(parts)
    scale = sum(abs(p) for p in parts)
    print(f"hll {name} edge={edge} {path}: <w,Jv> {lhs:.14e} <J^T w,v> {rhs:.14e}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * max(scale, abs(lhs))
    rt.close()


def test_reflective_octant_equals_mirrored_periodic_run_on_device():
    # The Stromgren set-up (uniform 1e-3 cm^-3 gas at 1e4 K, frozen, one
    # 1e5 K black-body group) with the source split over the 8 cells around
    # the centre of a 64^3 periodic box is mirror symmetric about the three
    # central planes and the box faces, so a 32^3 box with reflective faces
    # and one of the 8 sources in its corner cell holds the same fields as
    # the octant [32, 64)^3.
    n = 32
    box = 13.2 * E.KPC
    dx = box / (2 * n)
    c = 0.01 * E.C_LIGHT
    dt = E.courant_dt(dx, c)
    g = groups_for(1)
    rate = 5e48 / 8
    steps = 300
    cells = np.array([((z * 2 * n) + y) * 2 * n + x for z in (n - 1, n) for y in (n - 1, n)
                      for x in (n - 1, n)], dtype=np.int64)
    kw = dict(dx=dx, c_red=c, dt=dt, n_steps=steps, groups=g, isothermal=1, precision="fp64")
    N, F, x, T = E.initial_state((2 * n,) * 3, 1, T0=1e4)
    full = run_gpu(N, F, x, T, np.full((2 * n,) * 3, 1e-3), cells, np.full(8, rate), **kw)
    N, F, x, T = E.initial_state((n,) * 3, 1, T0=1e4)
    octant = run_gpu(N, F, x, T, np.full((n,) * 3, 1e-3), np.array([0]), np.array([rate]),
                     bc=[RF] * 6, **kw)
    hi = slice(n, 2 * n)
    for a, b, name in ((full[0][:, hi, hi, hi], octant[0], "N"), (full[1][:, :, hi, hi, hi], octant[1], "F"),
                       (full[2][hi, hi, hi], octant[2], "x")):
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print(f"octant vs full {name}: {err:.2e}", flush=True)
        assert err <= 1e-12
    assert octant[2].max() > 0.5
