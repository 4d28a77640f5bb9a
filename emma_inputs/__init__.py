"""Seeded synthetic inputs for the M1 radiation step.

This module serves both the HIP library's tests/benchmark and the oracle.  It
holds none of the method's arithmetic: it draws density fields, source lists
and initial states, and it states the workload parameters.  The physical
scales follow the paper's tests: hydrogen density 1e-3 cm^-3 and 100 K gas
with x = 1.2e-3 (HII-region test, Sec. 6), a 1e5 K black-body source spectrum
and the group edges 13.6 / 24.6 / 54.4 / 1000 eV (Sec. 2.2.3 and the
reionisation runs of Sec. 6).

Layouts (C order, x fastest): N[G,nz,ny,nx], F[G,3,nz,ny,nx], x/T/n0[nz,ny,nx].
"""
import numpy as np

C_LIGHT = 2.99792458e10
KPC = 3.0856775814913673e21
YR = 3.15576e7
T_BB = 1e5
EDGES = {1: (13.6, 1000.0), 2: (13.6, 24.6, 1000.0), 3: (13.6, 24.6, 54.4, 1000.0),
         4: (13.6, 24.6, 54.4, 200.0, 1000.0)}
COURANT = 0.8


def courant_dt(dx, c_red, courant=COURANT):
    """dt = C dx / (3 c_red): the unsplit 3D explicit update is positive for
    c_red dt / dx <= 1/3."""
    return courant * dx / (3.0 * c_red)


def lognormal_n0(n, sigma_ln, mean=1e-3, seed=0):
    """Log-normal density on an n^3 periodic grid with a Gaussian log-field of
    power spectrum P(k) ~ k^-2 (amplitude k^-1), standardised, exponentiated
    and rescaled so that the sample mean is exactly ``mean``."""
    rng = np.random.default_rng(seed)
    w = rng.standard_normal((n, n, n))
    k1 = np.fft.fftfreq(n) * n
    kz, ky, kx = np.meshgrid(k1, k1, k1, indexing="ij")
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(k)
    amp[k > 0] = 1.0 / k[k > 0]
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    g = (g - g.mean()) / g.std()
    r = np.exp(sigma_ln * g)
    return np.ascontiguousarray(mean * r / r.mean())


def sources_peaks(n0, n_src, lo, hi, seed=0):
    """The n_src densest cells (stable sort, ties to the lower flat index)
    with log10 rates drawn uniformly in [lo, hi] (photons/s)."""
    rng = np.random.default_rng(seed + 1000)
    flat = n0.reshape(-1)
    order = np.argsort(-flat, kind="stable")[:n_src]
    rates = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n_src)
    return order.astype(np.int64), rates


def sources_random(n_cells, n_src, lo, hi, seed=0):
    """n_src host cells drawn uniformly (duplicates allowed), log-uniform rates."""
    rng = np.random.default_rng(seed + 1000)
    cells = rng.integers(0, n_cells, n_src).astype(np.int64)
    rates = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n_src)
    return cells, rates


def sources_peaks_in_box(n0, n_src, lo, hi, box_lo, box_hi, seed=0):
    """The n_src densest cells inside [box_lo, box_hi)^3 (stable sort, ties to
    the lower flat index), log-uniform rates in [lo, hi]."""
    rng = np.random.default_rng(seed + 1000)
    nz, ny, nx = n0.shape
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    inside = ((z >= box_lo) & (z < box_hi) & (y >= box_lo) & (y < box_hi)
              & (x >= box_lo) & (x < box_hi)).reshape(-1)
    cand = np.nonzero(inside)[0]
    order = cand[np.argsort(-n0.reshape(-1)[cand], kind="stable")[:n_src]]
    rates = 10.0 ** rng.uniform(np.log10(lo), np.log10(hi), n_src)
    return order.astype(np.int64), rates


def initial_state(shape, G, x0=1.2e-3, T0=100.0):
    """Dark, cold, nearly neutral gas: N = F = 0, x = x0, T = T0."""
    nz, ny, nx = shape
    N = np.zeros((G, nz, ny, nx))
    F = np.zeros((G, 3, nz, ny, nx))
    x = np.full((nz, ny, nx), x0)
    T = np.full((nz, ny, nx), T0)
    return N, F, x, T


def random_state(shape, G, c_red, seed=0, n_scale=1.0, T_range=(1e2, 3e4), f_max=1.0,
                 p_full=0.1, p_dark=0.05):
    """Random realisable radiation state (|F| <= c N; a fraction p_full of the
    cells at f = 1 and p_dark with N = 0) and random gas state."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    N = n_scale * 10.0 ** rng.uniform(-3, 0, (G, nz, ny, nx))
    N[rng.random((G, nz, ny, nx)) < p_dark] = 0.0
    d = rng.standard_normal((G, 3, nz, ny, nx))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    f = rng.uniform(0, f_max, (G, 1, nz, ny, nx))
    f[rng.random((G, 1, nz, ny, nx)) < p_full] = 1.0
    F = d * f * c_red * N[:, None]
    x = 10.0 ** rng.uniform(-4, 0, (nz, ny, nx))
    x = np.minimum(x, 1.0 - 1e-6)
    T = 10.0 ** rng.uniform(np.log10(T_range[0]), np.log10(T_range[1]), (nz, ny, nx))
    n0 = 1e-3 * 10.0 ** rng.uniform(-1, 1, (nz, ny, nx))
    return N, F, x, T, n0


# Workloads.  Box 6.6 kpc for every grid; 1e5 K black body; on-the-spot
# chemistry; periodic boundaries; initial state from initial_state().
WORKLOADS = {
    "stromgren32": dict(n=32, G=1, precision="fp64", c_frac=1.0, steps=200,
                        n0="uniform", sources=("centre", 5e48)),
    "lognormal128": dict(n=128, G=3, precision="mixed", c_frac=0.1, steps=100, sigma_ln=1.0,
                         seed=2, sources=("peaks", 16, 1e48, 1e50)),
    "throughput256": dict(n=256, G=3, precision="mixed", c_frac=0.1, steps=50, sigma_ln=1.0,
                          seed=3, sources=("random", 256, 1e47, 1e50)),
    "adjoint64": dict(n=64, G=2, precision="fp64", c_frac=0.1, steps=60, sigma_ln=0.8, seed=4,
                      sources=("box", 8, 1e48, 1e50, 16, 48), K=10),
    "large512": dict(n=512, G=3, precision="mixed", c_frac=0.05, steps=20, sigma_ln=1.2,
                     seed=5, sources=("random", 4096, 1e46, 1e50), K=10),
}


def make_workload(name, n=None, box_kpc=6.6):
    """Return a dict with the full input set of a named workload (``n``
    overrides the grid size, keeping dx from the box and the same recipe)."""
    w = dict(WORKLOADS[name])
    n = n or w["n"]
    shape = (n, n, n)
    dx = box_kpc * KPC / n
    c_red = w["c_frac"] * C_LIGHT
    dt = courant_dt(dx, c_red)
    G = w["G"]
    if w.get("n0") == "uniform":
        n0 = np.full(shape, 1e-3)
    else:
        n0 = lognormal_n0(n, w["sigma_ln"], 1e-3, w["seed"])
    src = w["sources"]
    if src[0] == "centre":
        c = n // 2
        cells = np.array([(c * n + c) * n + c], dtype=np.int64)
        rates = np.array([src[1]])
    elif src[0] == "peaks":
        cells, rates = sources_peaks(n0, src[1], src[2], src[3], w["seed"])
    elif src[0] == "random":
        cells, rates = sources_random(n ** 3, src[1], src[2], src[3], w["seed"])
    else:
        lo, hi = src[4] * n // 64, src[5] * n // 64
        cells, rates = sources_peaks_in_box(n0, src[1], src[2], src[3], lo, hi, w["seed"])
    N, F, x, T = initial_state(shape, G)
    return dict(name=name, shape=shape, G=G, dx=dx, c_red=c_red, dt=dt, steps=w["steps"],
                precision=w["precision"], n0=n0, src_cell=cells, src_rate=rates,
                N=N, F=F, x=x, T=T, T_bb=T_BB, edges=EDGES[G], K=w.get("K"))
