"""The adjoint of the refined-cell step (emma_rt_step_crta_adjoint, Sec. 5) on
the GPU.

1. Dot-product test against the oracle's dual-number tangent of its R19 step:
   <w, J v> (oracle, FP64) = <J^T w, v> (library), relative 1e-9, over the
   coarse state, the children's state, n_fine, n_H and the source rates, on
   ragged grids with sources in refined and plain cells, both ratios, both
   fluxes, on-the-spot and case A, several steps, through the C ABI.
2. With no refined cells the call is emma_rt_step_adjoint, bit for bit.
3. The mixed path's gradients against the FP64 path's, within 1e-3
   normwise (about 1e-7 measured).
4. Argument errors, repeated or out-of-grid parents included.
"""
import numpy as np
import pytest
import torch

import emma_inputs as E
import oracle
from gpu_helpers import DEV, groups_for, to_dev

pytestmark = pytest.mark.gpu


def _case(shape, G, ratio, seed, n_ref):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3, f_max=0.6, p_full=0.0, p_dark=0.0)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    nc = ratio ** 3
    ref = rng.choice(V, n_ref, replace=False).astype(np.int64)
    # sources: two in refined cells (one cell holding two), two elsewhere
    cells = np.concatenate([ref[:2], ref[:1], rng.integers(0, V, 2)]).astype(np.int64)
    rates = 10 ** rng.uniform(47, 49, cells.size)
    child = rng.integers(0, nc, cells.size).astype(np.int32)
    xf = rng.uniform(0.01, 0.9, (n_ref, nc))
    Tf = 10 ** rng.uniform(3, 4.5, (n_ref, nc))
    nf = 10 ** rng.uniform(-3.5, -2.5, (n_ref, nc))
    return dict(N=N, F=F, x=x, T=T, n0=n0, ref=ref, cells=cells, rates=rates, child=child, xf=xf, Tf=Tf,
                nf=nf, dx=dx, c=c, dt=dt, G=G, ratio=ratio, shape=shape)


def _rt(k, K, precision="fp64", **kw):
    from paper_1508_07888_amd import EmmaRT
    return EmmaRT(k["shape"], k["G"], k["dx"], k["c"], precision=precision, groups=groups_for(k["G"]),
                  adjoint_max_steps=K, device=DEV, **kw)


@pytest.mark.parametrize("shape,G,ratio,seed,n_ref,steps,opts", [
    ((5, 6, 7), 2, 2, 1, 12, 3, {}),
    ((4, 5, 66), 3, 2, 2, 40, 2, {"path": "reference"}),
    ((3, 4, 5), 1, 4, 3, 5, 2, {}),
    ((6, 5, 4), 2, 4, 4, 6, 3, {"flux": "hll"}),
    ((5, 5, 9), 2, 2, 5, 20, 3, {"otsa": 0}),
    ((1, 1, 8), 4, 2, 6, 8, 1, {}),
])
def test_crta_adjoint_dot_product_against_oracle_tangent(shape, G, ratio, seed, n_ref, steps, opts):
    k = _case(shape, G, ratio, seed, n_ref)
    rng = np.random.default_rng(100 + seed)
    g = groups_for(G)
    otsa = opts.get("otsa", 1)
    flux = opts.get("flux", "glf")
    # tangent direction: relative perturbations of every input
    d = dict(N=k["N"] * rng.standard_normal(k["N"].shape), F=k["F"] * rng.standard_normal(k["F"].shape),
             x=k["x"] * (1 - k["x"]) * rng.standard_normal(k["x"].shape),
             T=k["T"] * rng.standard_normal(k["T"].shape), n0=k["n0"] * rng.standard_normal(k["n0"].shape),
             rates=k["rates"] * rng.standard_normal(k["rates"].shape),
             xf=k["xf"] * (1 - k["xf"]) * rng.standard_normal(k["xf"].shape),
             Tf=k["Tf"] * rng.standard_normal(k["Tf"].shape), nf=k["nf"] * rng.standard_normal(k["nf"].shape))
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=steps, groups=g, otsa=otsa, flux=flux)
    out, tan, _ = oracle.run_crta_tangent(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"],
                                          k["child"], k["ref"], ratio, k["xf"], k["Tf"], k["nf"], d["N"], d["F"],
                                          d["x"], d["T"], d["n0"], d["rates"], d["xf"], d["Tf"], d["nf"], **kw)
    # weights scaled by the output magnitudes so that every field contributes
    w = [rng.standard_normal(o.shape) / (np.abs(o).max() + 1e-300) for o in out]
    w[2] = rng.standard_normal(out[2].shape)
    w[4] = rng.standard_normal(out[4].shape)
    lhs = sum(float((wi * ti).sum()) for wi, ti in zip(w, tan))

    rt = _rt(k, steps, otsa=otsa, flux=flux, path=opts.get("path", "split"))
    gN, gF, gx, gT, gxf, gTf = (to_dev(a) for a in w)
    g_n0 = torch.zeros(shape, dtype=torch.float64, device=DEV)
    g_rate = torch.zeros(k["rates"].size, dtype=torch.float64, device=DEV)
    g_nf = torch.zeros(k["nf"].shape, dtype=torch.float64, device=DEV)
    rt.step_crta_adjoint(to_dev(k["N"]), to_dev(k["F"]), to_dev(k["x"]), to_dev(k["T"]), to_dev(k["n0"]),
                         to_dev(k["cells"], torch.int64), to_dev(k["rates"]), k["dt"], steps,
                         to_dev(k["ref"], torch.int64), ratio, to_dev(k["xf"]), to_dev(k["Tf"]), to_dev(k["nf"]),
                         gN, gF, gx, gT, g_n0, g_rate, gxf, gTf, g_nf, src_child=to_dev(k["child"], torch.int32))
    torch.cuda.synchronize()
    grads = [gN, gF, gx, gT, g_n0, g_rate, gxf, gTf, g_nf]
    dirs = [d["N"], d["F"], d["x"], d["T"], d["n0"], d["rates"], d["xf"], d["Tf"], d["nf"]]
    parts = [float((gi.cpu().numpy() * di).sum()) for gi, di in zip(grads, dirs)]
    rhs = sum(parts)
    scale = sum(abs(p) for p in parts)
    print(f"{shape} G={G} r={ratio} {opts}: <w,Jv> {lhs:.14e} <J^T w,v> {rhs:.14e} parts {parts}", flush=True)
    assert abs(lhs - rhs) <= 1e-9 * max(scale, abs(lhs))
    # refined parents' x_HII and T are overwritten by the children's means
    ref = k["ref"]
    assert np.all(gx.cpu().numpy().reshape(-1)[ref] == 0) and np.all(gT.cpu().numpy().reshape(-1)[ref] == 0)
    rt.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_crta_adjoint_without_refined_cells_is_the_plain_adjoint(precision):
    k = _case((6, 7, 9), 2, 2, 7, 4)
    rt = _rt(k, 3, precision=precision)
    fdt = rt.dtype
    rng = np.random.default_rng(7)
    w = [rng.standard_normal(a.shape) for a in (k["N"], k["F"], k["x"], k["T"])]
    args = (to_dev(k["N"], fdt), to_dev(k["F"], fdt), to_dev(k["x"]), to_dev(k["T"]), to_dev(k["n0"]),
            to_dev(k["cells"], torch.int64), to_dev(k["rates"]), k["dt"], 3)
    res = []
    for crta in (False, True):
        g = [to_dev(w[0], fdt), to_dev(w[1], fdt), to_dev(w[2]), to_dev(w[3]),
             torch.zeros(k["shape"], dtype=torch.float64, device=DEV),
             torch.zeros(k["rates"].size, dtype=torch.float64, device=DEV)]
        if crta:
            e = torch.zeros((0, 8), dtype=torch.float64, device=DEV)
            rt.step_crta_adjoint(*args, torch.zeros(0, dtype=torch.int64, device=DEV), 2, e, e, e, *g, e, e, e)
        else:
            rt.step_adjoint(*args, *g)
        torch.cuda.synchronize()
        res.append([t.cpu().numpy() for t in g])
    for a, b in zip(*res):
        assert np.array_equal(a, b)
    rt.close()


@pytest.mark.parametrize("ratio", [2, 4])
def test_mixed_crta_adjoint_close_to_fp64(ratio):
    """The mixed path's refined-cell adjoint (FP32 N, F and their gradients,
    FP64 chemistry) against the FP64 one on the same inputs: dL/dn_H, the
    rates, n_fine and the children's x_HII, T, where the loss weights the
    end state (x_HII of coarse and fine cells, T) within 1e-3 normwise."""
    k = _case((6, 7, 9), 2, ratio, 40 + ratio, 10)
    steps = 3
    rng = np.random.default_rng(ratio)
    wx = rng.standard_normal(k["x"].shape)
    wT = rng.standard_normal(k["T"].shape) / np.abs(k["T"]).max()
    wxf = rng.standard_normal(k["xf"].shape)
    wTf = rng.standard_normal(k["Tf"].shape) / np.abs(k["Tf"]).max()
    res = {}
    for precision in ("fp64", "mixed"):
        rt = _rt(k, steps, precision=precision)
        fdt = rt.dtype
        gN = torch.zeros(k["N"].shape, dtype=fdt, device=DEV)
        gF = torch.zeros(k["F"].shape, dtype=fdt, device=DEV)
        gx, gT, gxf, gTf = to_dev(wx), to_dev(wT), to_dev(wxf), to_dev(wTf)
        g_n0 = torch.zeros(k["shape"], dtype=torch.float64, device=DEV)
        g_rate = torch.zeros(k["rates"].size, dtype=torch.float64, device=DEV)
        g_nf = torch.zeros(k["nf"].shape, dtype=torch.float64, device=DEV)
        rt.step_crta_adjoint(to_dev(k["N"], fdt), to_dev(k["F"], fdt), to_dev(k["x"]), to_dev(k["T"]),
                             to_dev(k["n0"]), to_dev(k["cells"], torch.int64), to_dev(k["rates"]), k["dt"], steps,
                             to_dev(k["ref"], torch.int64), ratio, to_dev(k["xf"]), to_dev(k["Tf"]), to_dev(k["nf"]),
                             gN, gF, gx, gT, g_n0, g_rate, gxf, gTf, g_nf,
                             src_child=to_dev(k["child"], torch.int32))
        torch.cuda.synchronize()
        res[precision] = [t.double().cpu().numpy() for t in (g_n0, g_rate, g_nf, gxf, gTf, gx, gT)]
        rt.close()
    names = ("n_H", "rate", "n_fine", "x_fine", "T_fine", "x", "T")
    for name, a, b in zip(names, res["mixed"], res["fp64"]):
        err = np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)
        print(f"r={ratio} {name}: mixed vs fp64 gradient normwise {err:.2e}", flush=True)
        assert err <= 1e-3, name


def test_crta_adjoint_argument_errors():
    from paper_1508_07888_amd import _lib
    k = _case((4, 4, 4), 1, 2, 8, 3)
    rt = _rt(k, 2)
    N, F, x, T, n0 = (to_dev(k[a]) for a in ("N", "F", "x", "T", "n0"))
    xf, Tf, nf = to_dev(k["xf"]), to_dev(k["Tf"]), to_dev(k["nf"])
    cells, rates = to_dev(k["cells"], torch.int64), to_dev(k["rates"])

    def call(ref, ratio=2, steps=2, work=None, fine=(xf, Tf, nf)):
        g = [N.clone(), F.clone(), x.clone(), T.clone(), torch.zeros_like(n0), torch.zeros_like(rates)]
        gf = [torch.zeros_like(f) for f in fine]
        rt.step_crta_adjoint(N, F, x, T, n0, cells, rates, k["dt"], steps, ref, ratio, *fine, *g, *gf,
                             work=work)

    dup = to_dev(np.array([k["ref"][0], k["ref"][1], k["ref"][0]]), torch.int64)
    with pytest.raises(_lib.EmmaError, match="repeated"):
        call(dup)
    out = to_dev(np.array([k["ref"][0], k["ref"][1], 64]), torch.int64)
    with pytest.raises(_lib.EmmaError, match="outside the grid"):
        call(out)
    ref = to_dev(k["ref"], torch.int64)
    small = torch.empty(_lib.emma_rt_crta_adjoint_work_bytes(2, 3, 2) - 8, dtype=torch.uint8, device=DEV)
    with pytest.raises(_lib.EmmaError, match="work must hold"):
        call(ref, work=small)
    with pytest.raises(_lib.EmmaError, match="n_steps"):
        call(ref, steps=3)
    with pytest.raises(ValueError):
        call(ref, ratio=3)
    # a good call still works after the errors
    call(ref)
    torch.cuda.synchronize()
    rt.close()
