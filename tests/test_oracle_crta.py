"""Pins of the oracle's coarse radiative transport approximation with static
refined cells (Sec. 5; reading R19 in the oracle header): the transport on
the coarse grid, the chemistry of every child of a refined cell with its
parent's radiation injected, then the parent restricted from its children.

- A uniform refinement of a uniform field (children equal to the parent,
  each source split evenly over the children) gives the coarse run exactly.
- Without an absorber the radiation is the coarse run's whatever the
  children's gas and wherever the sources sit among them (the restriction
  conserves photons and the child volumes add up to the parent's).
- After one step each child holds what the one-cell chemistry gives for its
  parent's post-transport radiation and its own gas, and the parent holds
  the children's means.
"""
import numpy as np
import pytest

import emma_inputs as E
import oracle

C = E.C_LIGHT


def _setup(n=7, G=2, seed=3, n_ref=9, ratio=2):
    c = 0.1 * C
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state((n, n, n), G, c, seed=seed, n_scale=1e-3)
    rng = np.random.default_rng(seed)
    V = n ** 3
    ref = np.sort(rng.choice(V, n_ref, replace=False)).astype(np.int64)
    cells = np.concatenate([ref[:2], rng.integers(0, V, 3)]).astype(np.int64)
    rates = 10 ** rng.uniform(47, 50, cells.size)
    g = oracle.group_constants(E.T_BB, E.EDGES[G])
    return dict(N=N, F=F, x=x, T=T, n0=n0, ref=ref, cells=cells, rates=rates, dx=dx, c=c, dt=dt, g=g,
                ratio=ratio, rng=rng)


def _uniform_children(k):
    nc = k["ratio"] ** 3
    flat = lambda a: a.reshape(-1)[k["ref"]]
    return (np.repeat(flat(k["x"])[:, None], nc, axis=1), np.repeat(flat(k["T"])[:, None], nc, axis=1),
            np.repeat(flat(k["n0"])[:, None], nc, axis=1))


@pytest.mark.parametrize("ratio", [2, 4])
def test_uniform_refinement_equals_coarse_run(ratio):
    k = _setup(ratio=ratio)
    nc = ratio ** 3
    xf, Tf, nf = _uniform_children(k)
    # every source in a refined cell becomes nc sources of rate / nc, one per child
    refset = set(k["ref"].tolist())
    cells, rates, child = [], [], []
    for cell, rate in zip(k["cells"], k["rates"]):
        if int(cell) in refset:
            cells += [cell] * nc
            rates += [rate / nc] * nc
            child += list(range(nc))
        else:
            cells.append(cell); rates.append(rate); child.append(0)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=3, groups=k["g"])
    cN, cF, cx, cT, _ = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    rN, rF, rx, rT, rxf, rTf, _ = oracle.run_crta(k["N"], k["F"], k["x"], k["T"], k["n0"], np.array(cells),
                                                  np.array(rates), np.array(child), k["ref"], ratio, xf, Tf, nf,
                                                  **kw)
    assert np.array_equal(rN, cN) and np.array_equal(rF, cF)
    assert np.array_equal(rx, cx) and np.array_equal(rT, cT)
    assert np.array_equal(rxf, np.repeat(cx.reshape(-1)[k["ref"]][:, None], nc, axis=1))
    assert np.array_equal(rTf, np.repeat(cT.reshape(-1)[k["ref"]][:, None], nc, axis=1))


def test_without_absorber_radiation_is_the_coarse_runs():
    k = _setup()
    nc = 8
    rng = k["rng"]
    xf = rng.uniform(0.0, 1.0, (k["ref"].size, nc))
    Tf = 10 ** rng.uniform(2, 5, (k["ref"].size, nc))
    nf = 10 ** rng.uniform(-4, -2, (k["ref"].size, nc))
    child = rng.integers(0, nc, k["cells"].size).astype(np.int32)
    g = dict(k["g"], sigma_N=np.zeros(2), sigma_E=np.zeros(2))
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=4, groups=g)
    cN, cF, *_ = oracle.run(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"], **kw)
    rN, rF, rx, rT, rxf, rTf, _ = oracle.run_crta(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"],
                                                  k["rates"], child, k["ref"], 2, xf, Tf, nf, **kw)
    assert np.max(np.abs(rN - cN)) <= 1e-13 * np.max(cN)
    assert np.max(np.abs(rF - cF)) <= 1e-13 * np.max(np.abs(cF))
    # the parent's ionised atoms and internal energy are its children's
    w = nf / nf.sum(axis=1, keepdims=True)
    assert np.allclose(rx.reshape(-1)[k["ref"]], (rxf * w).sum(axis=1), rtol=1e-14, atol=0)
    m = (1 + rxf) * nf
    assert np.allclose(rT.reshape(-1)[k["ref"]], (rTf * m).sum(axis=1) / m.sum(axis=1), rtol=1e-14, atol=0)


def test_children_run_the_cell_chemistry_on_the_injected_radiation():
    k = _setup(G=3)
    nc = 8
    rng = k["rng"]
    xf = rng.uniform(0.001, 0.9, (k["ref"].size, nc))
    Tf = 10 ** rng.uniform(2, 4.5, (k["ref"].size, nc))
    nf = 10 ** rng.uniform(-4, -2, (k["ref"].size, nc))
    child = rng.integers(0, nc, k["cells"].size).astype(np.int32)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=1, groups=k["g"])
    rN, rF, rx, rT, rxf, rTf, _ = oracle.run_crta(k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"],
                                                  k["rates"], child, k["ref"], 2, xf, Tf, nf, **kw)
    Ns, Fs, _ = oracle.transport(k["N"], k["F"], dx=k["dx"], c_red=k["c"], dt=k["dt"])
    vf = (k["dx"] / 2) ** 3
    shape = k["n0"].shape
    for j, p in enumerate(k["ref"]):
        z, y, xx = np.unravel_index(p, shape)
        mN, mF = [], []
        for c in range(nc):
            S = np.zeros(3)
            for s in range(k["cells"].size):
                if k["cells"][s] == p and child[s] == c:
                    S += k["rates"][s] * np.asarray(k["g"]["frac"]) / vf
            N1, F1, x1, T1, _ = oracle.chem_cell(Ns[:, z, y, xx], Fs[:, :, z, y, xx], xf[j, c], Tf[j, c],
                                                 nf[j, c], S, dt=k["dt"], c_red=k["c"], groups=k["g"])
            assert x1 == rxf[j, c] and T1 == rTf[j, c]
            mN.append(N1); mF.append(F1)
        assert np.allclose(rN[:, z, y, xx], np.mean(mN, axis=0), rtol=1e-15, atol=0)
        assert np.allclose(rF[:, :, z, y, xx], np.mean(mF, axis=0), rtol=1e-14, atol=1e-300)


def test_crta_rejects_bad_arguments():
    k = _setup()
    xf, Tf, nf = _uniform_children(k)
    kw = dict(dx=k["dx"], c_red=k["c"], dt=k["dt"], n_steps=1, groups=k["g"])
    args = (k["N"], k["F"], k["x"], k["T"], k["n0"], k["cells"], k["rates"])
    with pytest.raises(ValueError):  # ratio
        oracle.run_crta(*args, None, k["ref"], 3, xf, Tf, nf, **kw)
    with pytest.raises(ValueError):  # repeated refined cell
        oracle.run_crta(*args, None, np.concatenate([k["ref"], k["ref"][:1]]), 2,
                        np.vstack([xf, xf[:1]]), np.vstack([Tf, Tf[:1]]), np.vstack([nf, nf[:1]]), **kw)
    with pytest.raises(ValueError):  # child index
        oracle.run_crta(*args, np.full(k["cells"].size, 8, np.int32), k["ref"], 2, xf, Tf, nf, **kw)
