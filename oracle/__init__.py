"""ctypes shim over the serial FP64 oracle (``emma_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check and
by the benchmark's CPU-baseline leg, never by the library under
``paper_1508_07888_amd``.  It marshals numpy arrays and holds none of the
method's arithmetic.

Layouts (C order, x fastest): N[G,nz,ny,nx], F[G,3,nz,ny,nx], x/T/n0[nz,ny,nx].
Units CGS.  ``groups`` is the dict {"sigma_N", "sigma_E", "mean_E", "frac"}
of per-group constants (cm^2, cm^2, erg, dimensionless).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int)
_lp = ctypes.POINTER(ctypes.c_int64)

COUNTER_NAMES = ("limiter", "neg_clamp", "x_clamp", "cap_hits",
                 "substeps", "attempts", "max_sub")


def use_library(path):
    """Load the oracle from another build of the same source (the
    benchmark's -O3 timing build); call before anything else."""
    global _LIB_PATH, _lib
    _LIB_PATH, _lib = path, None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.oracle_run.restype = ctypes.c_int
        L.oracle_run.argtypes = [_ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                 _lp, _dp, ctypes.c_int, _lp, _lp]
        L.oracle_run_tangent.restype = ctypes.c_int
        L.oracle_run_tangent.argtypes = [_ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                         _lp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, _dp,
                                         _lp]
        L.oracle_run_crta.restype = ctypes.c_int
        L.oracle_run_crta.argtypes = [_ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                      _lp, _dp, _ip, ctypes.c_int, ctypes.c_int, _lp, ctypes.c_int,
                                      _dp, _dp, _dp, _lp]
        L.oracle_run_crta_tangent.restype = ctypes.c_int
        L.oracle_run_crta_tangent.argtypes = [_ip, _dp, _dp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp,
                                              _lp, _dp, _ip, ctypes.c_int, ctypes.c_int, _lp, ctypes.c_int,
                                              _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp,
                                              _lp]
        L.oracle_transport.restype = ctypes.c_int
        L.oracle_transport.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, _lp]
        L.oracle_chem_cell.restype = ctypes.c_int
        L.oracle_chem_cell.argtypes = [_ip, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_double,
                                       _dp, _lp]
        L.oracle_pressure.restype = None
        L.oracle_pressure.argtypes = [ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.oracle_face_flux.restype = None
        L.oracle_face_flux.argtypes = [ctypes.c_double, _dp, ctypes.c_double, _dp,
                                       ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_hll_flux.restype = None
        L.oracle_hll_flux.argtypes = [ctypes.c_double, _dp, ctypes.c_double, _dp,
                                      ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_m1_speeds.restype = None
        L.oracle_m1_speeds.argtypes = [ctypes.c_double, _dp, ctypes.c_int, ctypes.c_double, _dp]
        L.oracle_rates.restype = None
        L.oracle_rates.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_int, _dp]
        L.oracle_rate_coeffs.restype = None
        L.oracle_rate_coeffs.argtypes = [ctypes.c_double, _dp]
        L.oracle_cross_section.restype = ctypes.c_double
        L.oracle_cross_section.argtypes = [ctypes.c_double]
        L.oracle_group_constants.restype = None
        L.oracle_group_constants.argtypes = [ctypes.c_double, _dp, ctypes.c_int, ctypes.c_int,
                                             _dp, _dp, _dp, _dp]
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a


BC = {"periodic": 0, "transmissive": 1, "reflective": 2, "inflow": 3}
FLUX = {"glf": 0, "hll": 1}


def _pack(shape, G, dx, c_red, dt, groups, otsa=1, isothermal=0, max_substeps=100000,
          bc=None, inflow=None, flux="glf"):
    """``bc``: six face kinds (x-, x+, y-, y+, z-, z+), names of BC or ints;
    ``inflow``: six photon flux densities (photons cm^-2 s^-1) for inflow faces."""
    nz, ny, nx = shape
    bc = [0] * 6 if bc is None else [BC[b] if isinstance(b, str) else int(b) for b in bc]
    inflow = [0.0] * 6 if inflow is None else [float(v) for v in inflow]
    fl = FLUX[flux] if isinstance(flux, str) else int(flux)
    ints = np.array([nx, ny, nz, G, otsa, isothermal, max_substeps] + bc + [fl], dtype=np.int32)
    dbls = np.array([dx, c_red, dt] + inflow, dtype=np.float64)
    gr = np.zeros((4, 4), dtype=np.float64)
    for r, key in enumerate(("sigma_N", "sigma_E", "mean_E", "frac")):
        v = np.asarray(groups[key], dtype=np.float64)
        gr[r, :G] = v[:G]
    return ints, dbls, gr


def _counters(c):
    return {k: int(v) for k, v in zip(COUNTER_NAMES, c)}


def run(N, F, x, T, n0, src_cell, src_rate, *, dx, c_red, dt, n_steps, groups,
        otsa=1, isothermal=0, max_substeps=100000, return_substeps=False, bc=None, inflow=None,
        flux="glf"):
    """Advance (N, F, x, T) by ``n_steps`` steps of ``dt``; returns copies and
    the counter dict (and per-cell accepted-substep totals if asked)."""
    N = _f64(N).copy(); F = _f64(F).copy(); x = _f64(x).copy(); T = _f64(T).copy()
    n0 = _f64(n0)
    G = N.shape[0]
    ints, dbls, gr = _pack(n0.shape, G, dx, c_red, dt, groups, otsa, isothermal, max_substeps,
                           bc, inflow, flux)
    sc = np.ascontiguousarray(src_cell, dtype=np.int64)
    sr = _f64(src_rate)
    sub = np.zeros(n0.size, dtype=np.int64)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_run(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), int(n_steps),
                          _d(N), _d(F), _d(x), _d(T), _d(n0),
                          sc.ctypes.data_as(_lp), _d(sr), int(sc.size),
                          sub.ctypes.data_as(_lp), cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_run rejected its arguments")
    out = (N, F, x, T, _counters(cnt))
    if return_substeps:
        out = out + (sub.reshape(n0.shape),)
    return out


def run_tangent(N, F, x, T, n0, src_cell, src_rate, dN, dF, dxh, dT, dn0, drate, *,
                dx, c_red, dt, n_steps, groups, otsa=1, isothermal=0, max_substeps=100000,
                bc=None, inflow=None, flux="glf"):
    """Forward run carried in dual numbers: returns the end state, its
    directional derivative along (dN, dF, dxh, dT, dn0, drate), and counters."""
    N = _f64(N).copy(); F = _f64(F).copy(); x = _f64(x).copy(); T = _f64(T).copy()
    dN = _f64(dN).copy(); dF = _f64(dF).copy(); dxh = _f64(dxh).copy(); dT = _f64(dT).copy()
    n0 = _f64(n0); dn0 = _f64(dn0)
    sc = np.ascontiguousarray(src_cell, dtype=np.int64)
    sr = _f64(src_rate); dr = _f64(drate)
    G = N.shape[0]
    ints, dbls, gr = _pack(n0.shape, G, dx, c_red, dt, groups, otsa, isothermal, max_substeps,
                           bc, inflow, flux)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_run_tangent(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), int(n_steps),
                                  _d(N), _d(F), _d(x), _d(T), _d(n0),
                                  sc.ctypes.data_as(_lp), _d(sr), int(sc.size),
                                  _d(dN), _d(dF), _d(dxh), _d(dT), _d(dn0), _d(dr),
                                  cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_run_tangent rejected its arguments")
    return (N, F, x, T), (dN, dF, dxh, dT), _counters(cnt)


def run_crta(N, F, x, T, n0, src_cell, src_rate, src_child, ref_cell, ratio, x_fine, T_fine, n_fine, *,
             dx, c_red, dt, n_steps, groups, otsa=1, isothermal=0, max_substeps=100000, bc=None,
             inflow=None, flux="glf"):
    """Coarse transport with the chemistry of refined cells on their children
    (reading R19).  x_fine, T_fine, n_fine: [n_ref, r^3] (child index
    (cz r + cy) r + cx); src_child: child of each source in a refined cell.
    Returns (N, F, x, T, x_fine, T_fine, counters)."""
    N = _f64(N).copy(); F = _f64(F).copy(); x = _f64(x).copy(); T = _f64(T).copy()
    n0 = _f64(n0)
    xf = _f64(x_fine).copy(); Tf = _f64(T_fine).copy(); nf = _f64(n_fine)
    G = N.shape[0]
    ints, dbls, gr = _pack(n0.shape, G, dx, c_red, dt, groups, otsa, isothermal, max_substeps,
                           bc, inflow, flux)
    sc = np.ascontiguousarray(src_cell, dtype=np.int64)
    sr = _f64(src_rate)
    ch = np.ascontiguousarray(np.zeros(sc.size) if src_child is None else src_child, dtype=np.int32)
    rc_ = np.ascontiguousarray(ref_cell, dtype=np.int64)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_run_crta(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), int(n_steps),
                               _d(N), _d(F), _d(x), _d(T), _d(n0), sc.ctypes.data_as(_lp), _d(sr),
                               ch.ctypes.data_as(_ip), int(sc.size), int(rc_.size), rc_.ctypes.data_as(_lp),
                               int(ratio), _d(xf), _d(Tf), _d(nf), cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_run_crta rejected its arguments")
    return N, F, x, T, xf, Tf, _counters(cnt)


def run_crta_tangent(N, F, x, T, n0, src_cell, src_rate, src_child, ref_cell, ratio, x_fine, T_fine, n_fine,
                     dN, dF, dxh, dT, dn0, drate, dxf, dTf, dnf, *, dx, c_red, dt, n_steps, groups, otsa=1,
                     isothermal=0, max_substeps=100000, bc=None, inflow=None, flux="glf"):
    """run_crta carried in dual numbers: returns the end state
    (N, F, x, T, x_fine, T_fine), its directional derivative along the given
    directions of the coarse state, the children's state and n_fine, and the
    source rates, and the counters."""
    N = _f64(N).copy(); F = _f64(F).copy(); x = _f64(x).copy(); T = _f64(T).copy()
    n0 = _f64(n0)
    xf = _f64(x_fine).copy(); Tf = _f64(T_fine).copy(); nf = _f64(n_fine)
    dN = _f64(dN).copy(); dF = _f64(dF).copy(); dxh = _f64(dxh).copy(); dT = _f64(dT).copy()
    dn0 = _f64(dn0); dr = _f64(drate)
    dxf = _f64(dxf).copy(); dTf = _f64(dTf).copy(); dnf = _f64(dnf)
    G = N.shape[0]
    ints, dbls, gr = _pack(n0.shape, G, dx, c_red, dt, groups, otsa, isothermal, max_substeps,
                           bc, inflow, flux)
    sc = np.ascontiguousarray(src_cell, dtype=np.int64)
    sr = _f64(src_rate)
    ch = np.ascontiguousarray(np.zeros(sc.size) if src_child is None else src_child, dtype=np.int32)
    rc_ = np.ascontiguousarray(ref_cell, dtype=np.int64)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_run_crta_tangent(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), int(n_steps),
                                       _d(N), _d(F), _d(x), _d(T), _d(n0), sc.ctypes.data_as(_lp), _d(sr),
                                       ch.ctypes.data_as(_ip), int(sc.size), int(rc_.size),
                                       rc_.ctypes.data_as(_lp), int(ratio), _d(xf), _d(Tf), _d(nf),
                                       _d(dN), _d(dF), _d(dxh), _d(dT), _d(dn0), _d(dr), _d(dxf), _d(dTf),
                                       _d(dnf), cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_run_crta_tangent rejected its arguments")
    return (N, F, x, T, xf, Tf), (dN, dF, dxh, dT, dxf, dTf), _counters(cnt)


def transport(N, F, *, dx, c_red, dt, bc=None, inflow=None, flux="glf", frac=None):
    """One conservative transport update (no chemistry) of every group;
    ``frac`` splits an inflow face's photon flux over the groups."""
    N = _f64(N); F = _f64(F)
    G = N.shape[0]
    fr = [0.0] * 4 if frac is None else list(frac) + [0.0] * (4 - len(frac))
    dummy = {"sigma_N": [0] * 4, "sigma_E": [0] * 4, "mean_E": [0] * 4, "frac": fr}
    ints, dbls, gr = _pack(N.shape[1:], G, dx, c_red, dt, dummy, bc=bc, inflow=inflow, flux=flux)
    Ns = np.empty_like(N); Fs = np.empty_like(F)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_transport(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), _d(N), _d(F),
                                _d(Ns), _d(Fs), cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_transport rejected its arguments")
    return Ns, Fs, _counters(cnt)


def chem_cell(N, F, x, T, n0, S, *, dt, c_red, groups, otsa=1, isothermal=0,
              max_substeps=100000, dx=1.0):
    """Chemistry of one cell: N[G], F[G,3], scalars x, T, n0 and S[G]."""
    N = _f64(N).copy(); F = _f64(F).copy(); S = _f64(S)
    G = N.shape[0]
    ints, dbls, gr = _pack((1, 1, 1), G, dx, c_red, dt, groups, otsa, isothermal, max_substeps)
    xa = np.array([x], dtype=np.float64); Ta = np.array([T], dtype=np.float64)
    cnt = np.zeros(7, dtype=np.int64)
    rc = lib().oracle_chem_cell(ints.ctypes.data_as(_ip), _d(dbls), _d(gr), _d(N), _d(F),
                                _d(xa), _d(Ta), float(n0), _d(S), cnt.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle_chem_cell rejected its arguments")
    return N, F, float(xa[0]), float(Ta[0]), _counters(cnt)


def pressure(N, F, c):
    F = _f64(F); P = np.empty(9, dtype=np.float64)
    lib().oracle_pressure(float(N), _d(F), float(c), _d(P))
    return P.reshape(3, 3)


def face_flux(NL, FL, NR, FR, d, c):
    FL = _f64(FL); FR = _f64(FR); out = np.empty(4, dtype=np.float64)
    lib().oracle_face_flux(float(NL), _d(FL), float(NR), _d(FR), int(d), float(c), _d(out))
    return out


def hll_flux(NL, FL, NR, FR, d, c):
    FL = _f64(FL); FR = _f64(FR); out = np.empty(4, dtype=np.float64)
    lib().oracle_hll_flux(float(NL), _d(FL), float(NR), _d(FR), int(d), float(c), _d(out))
    return out


def m1_speeds(N, F, d, c):
    """(lambda-, lambda+) along axis d."""
    F = _f64(F); out = np.empty(2, dtype=np.float64)
    lib().oracle_m1_speeds(float(N), _d(F), int(d), float(c), _d(out))
    return float(out[0]), float(out[1])


def rates(T, n0=1.0, x=0.5, otsa=1):
    out = np.empty(4, dtype=np.float64)
    lib().oracle_rates(float(T), float(n0), float(x), int(otsa), _d(out))
    return {"alpha_A": out[0], "alpha_B": out[1], "beta": out[2], "Lambda": out[3]}


def rate_coeffs(T):
    """The individual fits at T: alpha_A, alpha_B, beta (cm^3/s), rec_A, rec_B
    (recombination cooling), cexc (collisional excitation), brems (erg cm^3/s)."""
    out = np.empty(7, dtype=np.float64)
    lib().oracle_rate_coeffs(float(T), _d(out))
    return dict(zip(("alpha_A", "alpha_B", "beta", "rec_A", "rec_B", "cexc", "brems"), out))


def cross_section(E_eV):
    return lib().oracle_cross_section(float(E_eV))


def group_constants(T_bb, edges_eV, panels=20000):
    e = _f64(edges_eV)
    G = e.size - 1
    sN = np.empty(G); sE = np.empty(G); mE = np.empty(G); fr = np.empty(G)
    lib().oracle_group_constants(float(T_bb), _d(e), G, int(panels), _d(sN), _d(sE), _d(mE),
                                 _d(fr))
    return {"sigma_N": sN, "sigma_E": sE, "mean_E": mE, "frac": fr}
