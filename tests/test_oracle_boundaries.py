"""Pins of the oracle's global boundaries (transmissive, reflective, planar
inflow source: Sec. 4, gather step, and the tests of Sec. 6) and of the HLL
flux with M1 wave speeds (Sec. 2.2.3).

Each checks an exact property: mirror symmetry (a reflective octant equals the
mirrored periodic run), exact first-order upwinding of f = 1 beams (outflow
through a transmissive face, a constant beam entering through an inflow
face: binomial closed forms), the eigenvalues of the one-dimensional M1
Jacobian (computed here numerically from the closure), the consistency and
the free-streaming limit of the HLL flux, and a Fourier mode at f -> 0 whose
dissipation speed is c/sqrt(3).
"""
import math

import numpy as np
import pytest

import emma_inputs as E
import oracle

C = E.C_LIGHT


def _groups(G):
    return oracle.group_constants(E.T_BB, E.EDGES[G])


def _binom_cdf_tail(n, nu, m):
    """P(Binomial(n, nu) >= m)."""
    return sum(math.comb(n, k) * nu ** k * (1 - nu) ** (n - k) for k in range(max(m, 0), n + 1))


# ------------------------------------------------------------- reflective

def _mirror_index(n):
    # full periodic grid of 2n cells, mirror planes between n-1 | n and 2n-1 | 0:
    # full cell i holds octant cell m(i) (F component reversed where i < n)
    i = np.arange(2 * n)
    return np.where(i >= n, i - n, n - 1 - i), i < n


@pytest.mark.parametrize("flux", ["glf", "hll"])
def test_reflective_octant_equals_mirrored_periodic_run(flux):
    n, G, steps = 5, 2, 6
    c = 0.1 * C
    dx = 6.6 * E.KPC / 32
    dt = E.courant_dt(dx, c)
    No, Fo, xo, To, n0o = E.random_state((n, n, n), G, c, seed=11, n_scale=1e-3, f_max=0.6,
                                         p_full=0.0, p_dark=0.0)
    m, neg = _mirror_index(n)
    sel = np.ix_(m, m, m)
    Nf = No[(slice(None),) + sel]
    Ff = Fo[(slice(None), slice(None)) + sel].copy()
    for d, axis in ((0, 3), (1, 2), (2, 1)):  # F_x flips along x (last axis), ...
        shape = [1] * 4
        shape[axis] = 2 * n
        Ff[:, d] *= np.where(neg, -1.0, 1.0).reshape(shape)
    xf, Tf, n0f = xo[sel], To[sel], n0o[sel]
    rate = 3e49
    # the octant's corner cell and its seven mirror images each host the source
    cells = np.array([((z * 2 * n) + y) * 2 * n + x for z in (n - 1, n) for y in (n - 1, n)
                      for x in (n - 1, n)], dtype=np.int64)
    g = _groups(G)
    kw = dict(dx=dx, c_red=c, dt=dt, n_steps=steps, groups=g, flux=flux)
    fN, fF, fx, fT, _ = oracle.run(Nf, Ff, xf, Tf, n0f, cells, np.full(8, rate), **kw)
    oN, oF, ox, oT, _ = oracle.run(No, Fo, xo, To, n0o, np.array([0]), np.array([rate]),
                                   bc=["reflective"] * 6, **kw)
    hi = slice(n, 2 * n)
    for a, b in ((fN[:, hi, hi, hi], oN), (fF[:, :, hi, hi, hi], oF), (fx[hi, hi, hi], ox),
                 (fT[hi, hi, hi], oT)):
        assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))
    # the x-mirrored octant holds the same fields with F_x reversed
    lo = slice(n - 1, None, -1)
    assert np.max(np.abs(fN[:, hi, hi, lo] - oN)) <= 1e-12 * np.max(oN)
    assert np.max(np.abs(-fF[:, 0, hi, hi, lo] - oF[:, 0])) <= 1e-12 * np.max(np.abs(oF[:, 0]))
    assert np.max(np.abs(oF[:, 0])) > 0


def test_reflective_wall_keeps_photons_in():
    # sigma = 0 and reflective faces everywhere: no photon leaves the box
    n, G = 6, 1
    c = 0.1 * C
    dx = 1e20
    dt = E.courant_dt(dx, c)
    N, F, *_ = E.random_state((n, n + 1, n + 2), G, c, seed=4)
    tot0 = N.sum()
    for _ in range(8):
        N, F, cnt = oracle.transport(N, F, dx=dx, c_red=c, dt=dt, bc=["reflective"] * 6)
        assert cnt["neg_clamp"] == 0
    assert abs(N.sum() / tot0 - 1) < 1e-13


# ----------------------------------------------------------- transmissive

def _axis_beam(nx, axis, sign, c, N0):
    """A beam at f = 1 along +-axis, uniform across the other two axes (two
    cells each), profile N0 along the axis; returns N[1,...], F[1,3,...]."""
    shape = [2, 2, 2]
    shape[2 - axis] = nx
    prof_shape = [1, 1, 1]
    prof_shape[2 - axis] = nx
    N = np.broadcast_to(N0.reshape(prof_shape), shape).copy()[None]
    F = np.zeros((1, 3) + tuple(shape))
    F[0, axis] = sign * c * N[0]
    return N, F


def _profile(N, axis):
    idx = [0, 0, 0]
    idx[2 - axis] = slice(None)
    return N[0][tuple(idx)]


@pytest.mark.parametrize("flux", ["glf", "hll"])
@pytest.mark.parametrize("axis,sign", [(0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1)])
def test_transmissive_outflow_is_exact_upwind(axis, sign, flux):
    # a pulse at f = 1 leaving through a transmissive face: exact first-order
    # upwinding, nothing comes back in (no wrap), nothing reflects
    nx, nu, steps = 14, 0.8 / 3.0, 25
    c, dx = 0.1 * C, 1e20
    dt = nu * dx / c
    N0 = np.zeros(nx)
    src = [8, 9] if sign > 0 else [nx - 9, nx - 10]
    N0[src[0]], N0[src[1]] = 1.0, 0.5
    N, F = _axis_beam(nx, axis, sign, c, N0)
    for _ in range(steps):
        N, F, cnt = oracle.transport(N, F, dx=dx, c_red=c, dt=dt, bc=["transmissive"] * 6, flux=flux)
        # HLL: ahead of and behind the pulse f = 1 +- 1 ulp makes the empty
        # neighbour's flux +-1 ulp; the floor takes the negative ones
        if flux == "glf":
            assert cnt["neg_clamp"] == 0
    expect = np.zeros(nx)
    for k in range(steps + 1):
        w = math.comb(steps, k) * nu ** k * (1 - nu) ** (steps - k)
        shifted = np.zeros(nx)
        if sign > 0:
            shifted[k:] = N0[:nx - k] if k < nx else 0
        else:
            shifted[:nx - k] = N0[k:] if k < nx else 0
        expect += w * shifted
    got = _profile(N, axis)
    # HLL's weighted form (speeds c and -c/sqrt(3) at the pulse's edges) rounds
    # more than the flux of eq. (e:glf); both are exact up to that rounding
    tol = 1e-14 if flux == "glf" else 2e-12
    assert np.max(np.abs(got - expect)) < tol
    assert 0 < got.sum() < N0.sum() * 0.9  # part of the pulse has left
    assert np.max(np.abs(F[0, axis] - sign * c * N[0])) < tol * c


# ----------------------------------------------------------------- inflow

@pytest.mark.parametrize("flux", ["glf", "hll"])
@pytest.mark.parametrize("face", range(6))
def test_inflow_face_fills_with_exact_upwind_profile(face, flux):
    # a constant beam Phi enters an empty box through one face (the opposite
    # face transmissive): the profile after n steps is
    # N_j = (Phi_g / c) P(Binomial(n, nu) >= j + 1), j cells from the face
    axis, plus = face // 2, face % 2
    nx, nu, steps = 12, 0.8 / 3.0, 15
    c, dx = 0.1 * C, 1e20
    dt = nu * dx / c
    phi, frac = 2.5e6, (0.3, 0.7)
    shape = [2, 2, 2]
    shape[2 - axis] = nx
    N = np.zeros((2,) + tuple(shape))
    F = np.zeros((2, 3) + tuple(shape))
    bc = ["periodic"] * 6
    bc[2 * axis], bc[2 * axis + 1] = "transmissive", "transmissive"
    bc[face] = "inflow"
    inflow = [0.0] * 6
    inflow[face] = phi
    for _ in range(steps):
        N, F, cnt = oracle.transport(N, F, dx=dx, c_red=c, dt=dt, bc=bc, inflow=inflow,
                                     flux=flux, frac=frac)
        assert cnt["neg_clamp"] == 0  # (the limiter takes |F| = c N + 1 ulp)
    for g in range(2):
        prof = _profile(N[g:g + 1], axis)
        if plus:
            prof = prof[::-1]
        expect = np.array([phi * frac[g] / c * _binom_cdf_tail(steps, nu, j + 1) for j in range(nx)])
        tol = 1e-13 if flux == "glf" else 2e-12
        assert np.max(np.abs(prof - expect)) <= tol * phi * frac[g] / c
        sign = -1.0 if plus else 1.0
        assert np.max(np.abs(F[g, axis] - sign * c * N[g])) <= tol * phi
        assert np.max(np.abs(np.delete(F[g], axis, axis=0))) == 0.0


def test_boundary_arguments_rejected():
    N = np.zeros((1, 2, 2, 2))
    F = np.zeros((1, 3, 2, 2, 2))
    with pytest.raises(ValueError):  # one face periodic, the other not
        oracle.transport(N, F, dx=1.0, c_red=1.0, dt=0.1, bc=[0, 1, 0, 0, 0, 0])
    with pytest.raises(ValueError):
        oracle.transport(N, F, dx=1.0, c_red=1.0, dt=0.1, bc=[4, 4, 0, 0, 0, 0])
    with pytest.raises(ValueError):
        oracle.transport(N, F, dx=1.0, c_red=1.0, dt=0.1, flux=2)


# -------------------------------------------------------------- HLL speeds

def _flux_1d(N, Fd, c):
    # the one-dimensional M1 flux along x: (F_x, c^2 P_xx) for F = Fd x^
    P = oracle.pressure(N, [Fd, 0.0, 0.0], c)
    return np.array([Fd, c * c * P[0, 0]])


def test_m1_speeds_are_the_eigenvalues_of_the_1d_jacobian():
    c = 0.1 * C
    N = 3.0
    lm, lp = oracle.m1_speeds(N, [0.0, 0.0, 0.0], 0, c)
    assert abs(lm + c / math.sqrt(3)) < 1e-15 * c and abs(lp - c / math.sqrt(3)) < 1e-15 * c
    assert oracle.m1_speeds(0.0, [0.0, 0.0, 0.0], 1, c) == (lm, lp)
    lm, lp = oracle.m1_speeds(N, [0.0, 0.0, c * N], 2, c)
    assert abs(lm - c) < 1e-14 * c and abs(lp - c) < 1e-14 * c
    lm, lp = oracle.m1_speeds(N, [0.0, -c * N, 0.0], 1, c)
    assert abs(lm + c) < 1e-14 * c and abs(lp + c) < 1e-14 * c
    for f in (-0.9, -0.5, -0.1, 0.2, 0.45, 0.7, 0.95):
        Fd = f * c * N
        h = 1e-6
        J = np.zeros((2, 2))
        J[:, 0] = (_flux_1d(N * (1 + h), Fd, c) - _flux_1d(N * (1 - h), Fd, c)) / (2 * h * N)
        dF = h * c * N
        J[:, 1] = (_flux_1d(N, Fd + dF, c) - _flux_1d(N, Fd - dF, c)) / (2 * dF)
        ev = np.sort(np.linalg.eigvals(J).real)
        for d in range(3):
            F = [0.0, 0.0, 0.0]
            F[d] = Fd
            lm, lp = oracle.m1_speeds(N, F, d, c)
            assert abs(lm - ev[0]) < 1e-7 * c and abs(lp - ev[1]) < 1e-7 * c
            assert -c * (1 + 1e-15) <= lm <= lp <= c * (1 + 1e-15)


def test_hll_is_consistent_and_upwinds_beams():
    c = 0.1 * C
    rng = np.random.default_rng(2)
    for _ in range(20):
        N = rng.uniform(0.1, 2.0)
        F = rng.standard_normal(3)
        F *= rng.uniform(0, 1) * c * N / np.linalg.norm(F)
        for d in range(3):
            P = oracle.pressure(N, F, c)
            phys = np.concatenate([[F[d]], c * c * P[:, d]])
            assert np.allclose(oracle.hll_flux(N, F, N, F, d, c), phys, rtol=1e-13,
                               atol=1e-13 * c * c * N)
    for d in range(3):  # f = 1 beams along +d: the left state's flux; along -d: the right's
        e = np.eye(3)[d]
        NL, NR = 1.3, 0.4
        out = oracle.hll_flux(NL, c * NL * e, NR, c * NR * e, d, c)
        assert np.allclose(out, np.concatenate([[c * NL], c * c * NL * e]), rtol=1e-14, atol=0)
        out = oracle.hll_flux(NL, -c * NL * e, NR, -c * NR * e, d, c)
        assert np.allclose(out, np.concatenate([[-c * NR], c * c * NR * e]), rtol=1e-14, atol=0)


def test_hll_fourier_mode_dissipates_at_sound_speed():
    # F = 0 and a small cosine in N: the speeds are +-c/sqrt(3) up to O(eps), so
    # each mode evolves through
    #   G(th) = [[1 - mu (1 - cos th), -i nu sin th], [-i nu/3 sin th, 1 - mu (1 - cos th)]]
    # with mu = nu / sqrt(3) (the GLF flux has mu = nu)
    nx, nu, steps, eps = 32, 0.25, 12, 1e-7
    k = 3
    th = 2 * math.pi * k / nx
    dx, c = 1e20, 0.1 * C
    dt = nu * dx / c
    xs = np.arange(nx)
    N = np.ones((1, 2, 2, nx)) * (1.0 + eps * np.cos(th * xs))
    F = np.zeros((1, 3, 2, 2, nx))
    for _ in range(steps):
        N, F, _ = oracle.transport(N, F, dx=dx, c_red=c, dt=dt, flux="hll")
    mu = nu / math.sqrt(3)
    a = 1 - mu * (1 - math.cos(th))
    s = nu * math.sin(th)
    Gm = np.array([[a, -1j * s], [-1j * s / 3, a]])
    v = np.linalg.matrix_power(Gm, steps) @ np.array([eps, 0.0])
    expect_N = 1.0 + np.real(v[0] * np.exp(1j * th * xs))
    expect_F = c * np.real(v[1] * np.exp(1j * th * xs))
    assert np.max(np.abs(N[0, 0, 0] - expect_N)) < 10 * eps * eps + 1e-15
    assert np.max(np.abs(F[0, 0, 0, 0] - expect_F)) < c * (10 * eps * eps + 1e-15)


def test_hll_conserves_photons_and_stays_realisable():
    c = 0.1 * C
    dx = 1e20
    dt = E.courant_dt(dx, c)
    N, F, *_ = E.random_state((10, 9, 8), 2, c, seed=5)
    tot0 = N.reshape(2, -1).sum(axis=1)
    for _ in range(5):
        N, F, cnt = oracle.transport(N, F, dx=dx, c_red=c, dt=dt, flux="hll")
        assert cnt["neg_clamp"] == 0 and N.min() >= 0
        assert np.all(np.linalg.norm(F, axis=1) <= c * N * (1 + 1e-12) + 1e-300)
    assert np.allclose(N.reshape(2, -1).sum(axis=1), tot0, rtol=1e-13, atol=0)


def test_m1_speeds_equal_the_printed_eigenvalue_form_near_free_streaming():
    # c (chi' +- sqrt(chi'^2 + 4 (chi - f chi')))/2 evaluated with 60 digits
    # from Levermore's chi (R3) and its derivative, against the oracle's
    # cancellation-free form, down to |f| = 1 - 1e-12 where the printed
    # radicand is a difference of O(1) terms of size 1e-24
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    c = 0.1 * C
    N = 2.0
    for f in (0.0, 0.3, -0.77, 0.999, -0.999999, 1 - 1e-9, -(1 - 1e-12), 1.0):
        fd = Decimal(f)
        s = (4 - 3 * fd * fd).sqrt()
        den = 5 + 2 * s
        num = 3 + 4 * fd * fd
        chi = num / den
        dchi = (8 * fd * den + 6 * fd * num / s) / (den * den)
        root = (dchi * dchi + 4 * (chi - fd * dchi)).sqrt()
        want = [float(Decimal(c) * (dchi - root) / 2), float(Decimal(c) * (dchi + root) / 2)]
        got = oracle.m1_speeds(N, [f * c * N, 0.0, 0.0], 0, c)
        for g, w in zip(got, want):
            # f itself is rebuilt from F / (c N) (an ulp off), and the
            # speeds change by about 4.5 c per unit of f near |f| = 1
            assert abs(g - w) <= 2e-15 * c, (f, got, want)
