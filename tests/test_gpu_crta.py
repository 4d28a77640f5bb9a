"""Static refinement with the coarse radiative transport approximation
(emma_rt_step_crta, Sec. 5) on the GPU: parity with the oracle's R19 step on
ragged grids, both ratios, both precisions, every path; children equal to
their parent reproduce emma_rt_step on the split path bit for bit; argument
errors.  Tolerances as in the other parity tests (FP64 1e-12 normwise on
N, F, x, T and the children's x, T; mixed 1e-4 on N, F, 1e-6 absolute on x,
1e-3 on T)."""
import numpy as np
import pytest
import torch

import emma_inputs as E
import oracle
from gpu_helpers import DEV, groups_for, normwise, to_dev

pytestmark = pytest.mark.gpu


def _case(shape, G, ratio, seed, n_ref):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    nc = ratio ** 3
    ref = rng.choice(V, n_ref, replace=False).astype(np.int64)
    cells = np.concatenate([ref[:3], ref[:1], rng.integers(0, V, 3)]).astype(np.int64)
    rates = 10 ** rng.uniform(47, 50, cells.size)
    child = rng.integers(0, nc, cells.size).astype(np.int32)
    xf = rng.uniform(0.001, 0.95, (n_ref, nc))
    Tf = 10 ** rng.uniform(2, 4.7, (n_ref, nc))
    nf = 10 ** rng.uniform(-4, -2, (n_ref, nc))
    return dict(N=N, F=F, x=x, T=T, n0=n0, ref=ref, cells=cells, rates=rates, child=child, xf=xf, Tf=Tf, nf=nf,
                dx=dx, c=c, dt=dt, G=G, ratio=ratio)


def _gpu(k, precision, path, steps, groups, cells=None, rates=None, child=None, xf=None, Tf=None, nf=None,
         diag=True):
    from paper_1508_07888_amd import EmmaRT
    rt = EmmaRT(k["n0"].shape, k["G"], k["dx"], k["c"], precision=precision, groups=groups, path=path, device=DEV)
    fdt = rt.dtype
    N, F = to_dev(k["N"], fdt), to_dev(k["F"], fdt)
    x, T, n0 = to_dev(k["x"]), to_dev(k["T"]), to_dev(k["n0"])
    cells = k["cells"] if cells is None else cells
    rates = k["rates"] if rates is None else rates
    child = k["child"] if child is None else child
    gxf = to_dev(k["xf"] if xf is None else xf)
    gTf = to_dev(k["Tf"] if Tf is None else Tf)
    gnf = to_dev(k["nf"] if nf is None else nf)
    d = rt.step_crta(N, F, x, T, n0, to_dev(cells, torch.int64), to_dev(rates), k["dt"], to_dev(k["ref"], torch.int64),
                     k["ratio"], gxf, gTf, gnf, n_steps=steps, src_child=to_dev(child, torch.int32), diag=diag,
                     raise_on_status=False)
    torch.cuda.synchronize()
    out = (N.double().cpu().numpy(), F.double().cpu().numpy(), x.cpu().numpy(), T.cpu().numpy(),
           gxf.cpu().numpy(), gTf.cpu().numpy(), d)
    rt.close()
    return out


@pytest.mark.parametrize("path", ["split", "fused", "reference"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("shape,G,ratio,seed,n_ref", [((7, 9, 11), 2, 2, 1, 40), ((12, 10, 70), 3, 4, 2, 25),
                                                      ((5, 6, 130), 1, 2, 3, 300), ((1, 1, 8), 4, 2, 4, 8)])
def test_crta_matches_oracle(shape, G, ratio, seed, n_ref, precision, path):
    k = _case(shape, G, ratio, seed, n_ref)
    g = groups_for(G)
    steps = 3
    o = oracle.run_crta(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], k["child"], k["ref"],
                        ratio, k["xf"], k["Tf"], k["nf"], dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=steps,
                        groups=g)
    r = _gpu(k, precision, path, steps, g)
    eN, eF = normwise(r[0], o[0], True), normwise(r[1], o[1], True)
    ex, eT = normwise(r[2], o[2]), normwise(r[3], o[3])
    exf, eTf = normwise(r[4], o[4]), normwise(r[5], o[5])
    print(f"{shape} r={ratio} {precision} {path}: N {eN} F {eF} x {ex:.2e} T {eT:.2e} "
          f"children x {exf:.2e} T {eTf:.2e}", flush=True)
    assert r[6]["status"] == 0
    # the substep histogram counts the coarse cells and, for a refined cell,
    # its r^3 children instead, once per step
    n_ref_cells = len(k["ref"])
    assert sum(r[6]["substep_hist"]) == (k["n0"].size - n_ref_cells + n_ref_cells * ratio ** 3) * steps
    if precision == "fp64":
        assert max(eN) <= 1e-12 and max(eF) <= 1e-12
        assert max(ex, eT, exf, eTf) <= 1e-12
        assert r[6]["substeps"] == o[6]["substeps"] and r[6]["attempts"] == o[6]["attempts"]
    else:
        assert max(eN) <= 1e-4 and max(eF) <= 1e-4
        assert np.max(np.abs(r[2] - o[2])) <= 1e-6 and np.max(np.abs(r[4] - o[4])) <= 1e-6
        assert eT <= 1e-3 and eTf <= 1e-3


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("ratio", [2, 4])
def test_uniform_refinement_reproduces_the_coarse_step(precision, ratio):
    from gpu_helpers import run_gpu
    k = _case((9, 10, 66), 3, ratio, 7, 30)
    nc = ratio ** 3
    g = groups_for(3)
    flat = lambda a: a.reshape(-1)[k["ref"]]
    xf = np.repeat(flat(k["x"])[:, None], nc, axis=1)
    Tf = np.repeat(flat(k["T"])[:, None], nc, axis=1)
    nf = np.repeat(flat(k["n0"])[:, None], nc, axis=1)
    refset = set(k["ref"].tolist())
    cells, rates, child = [], [], []
    for cell, rate in zip(k["cells"], k["rates"]):
        if int(cell) in refset:
            cells += [cell] * nc; rates += [rate / nc] * nc; child += list(range(nc))
        else:
            cells.append(cell); rates.append(rate); child.append(0)
    steps = 3
    coarse = run_gpu(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], dx=k["dx"], c_red=k["c"],
                     dt=k["dt"], n_steps=steps, groups=g, precision=precision, path="split")
    r = _gpu(k, precision, "split", steps, g, cells=np.array(cells), rates=np.array(rates),
             child=np.array(child, np.int32), xf=xf, Tf=Tf, nf=nf)
    for a, b in zip(r[:4], coarse[:4]):
        assert np.array_equal(a, b)
    assert np.array_equal(r[4], np.repeat(flat(coarse[2])[:, None], nc, axis=1))


def test_crta_argument_errors():
    from paper_1508_07888_amd import EmmaRT, _lib
    k = _case((6, 6, 6), 1, 2, 9, 5)
    g = groups_for(1)
    rt = EmmaRT((6, 6, 6), 1, k["dx"], k["c"], precision="fp64", groups=g, device=DEV)
    N, F, x, T = rt.new_state()
    n0 = to_dev(k["n0"])
    e = torch.zeros(0, dtype=torch.int64, device=DEV)
    xf, Tf, nf = to_dev(k["xf"]), to_dev(k["Tf"]), to_dev(k["nf"])
    with pytest.raises(_lib.EmmaError):  # ratio
        rt.step_crta(N, F, x, T, n0, e, e.double(), k["dt"], to_dev(k["ref"], torch.int64), 3,
                     torch.zeros((5, 27), dtype=torch.float64, device=DEV),
                     torch.zeros((5, 27), dtype=torch.float64, device=DEV),
                     torch.zeros((5, 27), dtype=torch.float64, device=DEV))
    dup = to_dev(np.concatenate([k["ref"][:4], k["ref"][:1]]), torch.int64)
    d = rt.step_crta(N, F, x, T, n0, e, e.double(), k["dt"], dup, 2, xf, Tf, nf, diag=True, raise_on_status=False)
    assert d["status"] == _lib.EMMA_RT_EINVAL
    out = to_dev(np.array([0, 1, 2, 3, 6 ** 3]), torch.int64)
    d = rt.step_crta(N, F, x, T, n0, e, e.double(), k["dt"], out, 2, xf, Tf, nf, diag=True, raise_on_status=False)
    assert d["status"] == _lib.EMMA_RT_EINVAL
    rt.close()
