"""The oracle's dual-number tangent against central differences of the oracle.

This pins the tangent machinery (every operation's derivative rule, the
branch handling of min/abs/clamps) on its own, before it is used as the
reference for the hand-written adjoint of the HIP library.
"""
import numpy as np
import pytest

import emma_inputs as E
import oracle


def _case(seed, G, isothermal):
    c = 0.1 * E.C_LIGHT
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    N, F, x, T, n0 = E.random_state((5, 4, 6), G, c, seed=seed, n_scale=1e-2, f_max=0.5,
                                     p_full=0.0, p_dark=0.0)
    rng = np.random.default_rng(seed + 7)
    cells = rng.integers(0, n0.size, 3).astype(np.int64)
    rates = 10 ** rng.uniform(48, 50, 3)
    g = oracle.group_constants(E.T_BB, E.EDGES[G])
    kw = dict(dx=dx, c_red=c, dt=dt, n_steps=3, groups=g, isothermal=isothermal)
    return (N, F, x, T, n0, cells, rates), kw


@pytest.mark.parametrize("seed,G,iso", [(11, 1, 1), (12, 2, 0), (13, 3, 0)])
def test_tangent_matches_central_differences(seed, G, iso):
    (N, F, x, T, n0, cells, rates), kw = _case(seed, G, iso)
    rng = np.random.default_rng(seed)
    # relative perturbation directions
    dN = N * rng.standard_normal(N.shape)
    dF = F * rng.standard_normal(F.shape)
    dxh = x * (1 - x) * rng.standard_normal(x.shape)
    dT = T * rng.standard_normal(T.shape)
    dn0 = n0 * rng.standard_normal(n0.shape)
    dr = rates * rng.standard_normal(rates.shape)
    (Ne, Fe, xe, Te), (tN, tF, tx, tT), cnt = oracle.run_tangent(
        N, F, x, T, n0, cells, rates, dN, dF, dxh, dT, dn0, dr, **kw)
    base = oracle.run(N, F, x, T, n0, cells, rates, **kw)
    assert np.array_equal(base[0], Ne) and np.array_equal(base[2], xe)
    h = 1e-6
    plus = oracle.run(N + h * dN, F + h * dF, x + h * dxh, T + h * dT, n0 + h * dn0, cells,
                      rates + h * dr, return_substeps=True, **kw)
    minus = oracle.run(N - h * dN, F - h * dF, x - h * dxh, T - h * dT, n0 - h * dn0, cells,
                       rates - h * dr, return_substeps=True, **kw)
    # only cells whose substep sequence is the same on both sides are smooth
    same = plus[5] == minus[5]
    assert same.mean() > 0.9
    for k, t in ((0, tN), (2, tx), (3, tT)):
        fd = (plus[k] - minus[k]) / (2 * h)
        if k == 0:
            m = np.broadcast_to(same, fd.shape)
        else:
            m = same
        scale = np.abs(t[m]).max() + 1e-300
        assert np.max(np.abs(fd[m] - t[m])) <= 2e-5 * scale
