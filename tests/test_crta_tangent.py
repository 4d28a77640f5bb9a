"""The oracle's dual-number tangent of the refined-cell step (R19) against
central differences of the oracle's own step (h = 1e-6 relative along random
directions of the coarse state, the children's state, n_fine and the source
rates; directions whose +h and -h runs take different chemistry decisions are
reported, not compared).  The tangent is what the GPU adjoint of the step is
checked against."""
import numpy as np
import pytest

import emma_inputs as E
import oracle


def _case(shape, G, ratio, seed, n_ref):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state(shape, G, c, seed=seed, n_scale=1e-3, f_max=0.6, p_full=0.0, p_dark=0.0)
    rng = np.random.default_rng(seed)
    V = int(np.prod(shape))
    nc = ratio ** 3
    ref = rng.choice(V, n_ref, replace=False).astype(np.int64)
    cells = np.concatenate([ref[:2], rng.integers(0, V, 2)]).astype(np.int64)
    rates = 10 ** rng.uniform(47, 49, cells.size)
    child = rng.integers(0, nc, cells.size).astype(np.int32)
    xf = rng.uniform(0.01, 0.9, (n_ref, nc))
    Tf = 10 ** rng.uniform(3, 4.5, (n_ref, nc))
    nf = 10 ** rng.uniform(-3.5, -2.5, (n_ref, nc))
    return dict(N=N, F=F, x=x, T=T, n0=n0, ref=ref, cells=cells, rates=rates, child=child, xf=xf, Tf=Tf,
                nf=nf, dx=dx, c=c, dt=dt, G=G, ratio=ratio)


@pytest.mark.parametrize("ratio", [2, 4])
def test_crta_tangent_matches_central_differences(ratio):
    k = _case((3, 4, 5), 2, ratio, 3 + ratio, 4)
    g = oracle.group_constants(E.T_BB, E.EDGES[k["G"]])
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=2, groups=g)
    rng = np.random.default_rng(ratio)
    base = dict(N=k["N"], F=k["F"], x=k["x"], T=k["T"], n0=k["n0"], rates=k["rates"], xf=k["xf"], Tf=k["Tf"],
                nf=k["nf"])

    def run(st):
        o = oracle.run_crta(st["N"], st["F"], st["x"], st["T"], st["n0"], k["cells"], st["rates"], k["child"],
                            k["ref"], ratio, st["xf"], st["Tf"], st["nf"], **kw)
        return o

    def loss(o, w):
        return sum(float((wi * oi).sum()) for wi, oi in zip(w, o[:6]))

    o0 = run(base)
    w = [rng.standard_normal(a.shape) / max(np.abs(a).max(), 1e-300) for a in o0[:6]]
    stable = 0
    for trial in range(4):
        d = {key: base[key] * rng.standard_normal(np.shape(base[key])) for key in base}
        d["x"] = base["x"] * (1 - base["x"]) * rng.standard_normal(base["x"].shape)
        d["xf"] = base["xf"] * (1 - base["xf"]) * rng.standard_normal(base["xf"].shape)
        (_, tan, _) = oracle.run_crta_tangent(base["N"], base["F"], base["x"], base["T"], base["n0"], k["cells"],
                                              base["rates"], k["child"], k["ref"], ratio, base["xf"], base["Tf"],
                                              base["nf"], d["N"], d["F"], d["x"], d["T"], d["n0"], d["rates"],
                                              d["xf"], d["Tf"], d["nf"], **kw)
        jv = sum(float((wi * ti).sum()) for wi, ti in zip(w, tan))
        h = 1e-6
        plus = {key: base[key] + h * d[key] for key in base}
        minus = {key: base[key] - h * d[key] for key in base}
        op, om = run(plus), run(minus)
        fd = (loss(op, w) - loss(om, w)) / (2 * h)
        same = op[6]["substeps"] == om[6]["substeps"] and op[6]["attempts"] == om[6]["attempts"]
        rel = abs(fd - jv) / max(abs(fd), 1e-300)
        print(f"r={ratio} direction {trial}: tangent {jv:.10e} fd {fd:.10e} rel {rel:.2e} stable {same}",
              flush=True)
        if same:
            stable += 1
            assert rel <= 1e-5
    assert stable >= 2
