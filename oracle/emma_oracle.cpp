/*
 * emma_oracle.cpp -- serial, double-precision CPU oracle of one EMMA radiation
 * step (Aubert, Deparis & Ocvirk 2015, "EMMA: an AMR cosmological simulation
 * code with radiative transfer"): M1 transport on a uniform periodic grid
 * followed by the sub-cycled hydrogen thermochemistry.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the checker, not the product.  Only
 * the test-suite, the smoke check and the CPU-baseline leg of the benchmark
 * may load the library built from it.  It shares no source, header, helper or
 * table with the HIP library, and it includes nothing from it.
 *
 * It is written to be read against the paper: plain loops, one cell at a time,
 * every face flux evaluated twice (once for each cell it borders, as the paper's
 * own gather step does), and no blocking, fusion or reordering.  Every routine
 * is a template on the scalar type so that the same text, instantiated with the
 * forward-mode dual number below, yields exact tangents of the discrete map
 * (used to check the hand-written adjoint).
 *
 * Readings of the paper taken here (the paper is silent, garbled or
 * inconsistent on these; each is stated where it is used):
 *   R1  the intercell flux is the global Lax-Friedrichs flux of Sec. 2.2.3,
 *       eq. (e:glf); it equals HLL with signal speeds -c and +c.
 *   R2  Eddington tensor D = (1-chi)/2 I + (3chi-1)/2 n(x)n.  The printed
 *       form swaps the two coefficients (its trace would be 4chi-1, not 1).
 *   R3  chi(f) is Levermore's (3+4f^2)/(5+2 sqrt(4-3f^2)); the paper only
 *       gives its range [1/3, 1].
 *   R4  f = 0 when N <= 0, else min(1, |F|/(cN)); n = 0 when |F| = 0.
 *   R5  the scheme is the 3D unsplit version of the printed 1D update.
 *   R6  c means the reduced speed of light c_red everywhere.
 *   R7  the source term enters only in the chemistry N update, as printed.
 *   R8  the chemistry N and F updates divide by 1 + dtau c sigma (1-x) n0
 *       (the printed denominators lack dtau).
 *   R9  dtau0 = min(dt_rem, |e/(H-Lambda)|), dt_rem when H = Lambda; H and
 *       Lambda at the start-of-substep state; each halving restarts from
 *       the start-of-substep state with the same rate coefficients.
 *   R10 accept when |e' - e| <= 0.1 e.  At most MAX_HALVINGS halvings per
 *       substep; after max_substeps accepted substeps one last substep of
 *       length dt_rem is taken unconditionally.  Both count as cap hits.
 *       A cell whose energy is not positive and finite is left unchanged.
 *   R11 e = 3/2 (1+x) n0 k_B T (gamma = 5/3).
 *   R12 rates, cooling and cross-section are the fits written out below.
 *   R13 x is clamped to [0, 1] after its update; N* >= 0 after transport;
 *       |F*| <= c N* is enforced by rescaling F*.
 *   R14 on-the-spot: alpha = alpha_B and no recombination photons;
 *       otherwise alpha = alpha_A and (alpha_A - alpha_B) x^2 n0^2 photons
 *       go to group 1.
 *   R15 isothermal validation mode: one substep of dt, no energy update.
 *   R16 global boundaries (Sec. 4, gather step): periodic by default; a
 *       transmissive face takes the cell itself as its outside neighbour, a
 *       reflective face the cell with the face-normal flux component
 *       reversed (a mirror); both faces of an axis are periodic or neither.
 *   R17 planar source (photo-evaporation test of Sec. 6): an inflow face's
 *       outside neighbour is a beam entering the domain along the face
 *       normal, F = Phi_g n_in and N = Phi_g / c (f = 1), where Phi_g is the
 *       face's photon flux density times the group's photon fraction.
 *   R19 coarse radiative transport approximation (Sec. 5) with static
 *       refinement: a refined coarse cell is split into r^3 children
 *       (r = 2 or 4) that carry their own n0, x, T; each step the transport
 *       runs on the coarse grid, the unrefined cells run their chemistry as
 *       usual, every child runs the chemistry with its parent's N*, F*
 *       injected (piecewise constant) and its own sources (child volume
 *       (dx/r)^3), and the parent then holds the children's mean N, F, the
 *       n0-weighted mean x and the (1+x) n0-weighted mean T (so the parent's
 *       photons, ionised atoms and internal energy are the children's); the
 *       means are pairwise sums over the children in index order
 *       ((c0+c1)+(c2+c3))+... so that equal children give the parent exactly.
 *   R18 the HLL flux "on the way" in Sec. 2.2.3 takes as signal speeds along
 *       axis d the eigenvalues of the one-dimensional M1 system (N, F_d) at
 *       the normal reduced flux f_d = F_d/(c N) (clipped to [-1, 1], 0 when
 *       N <= 0): c (chi' +- sqrt(chi'^2 + 4 (chi - f_d chi')))/2, with chi
 *       and chi' = dchi/df at f_d, evaluated in the equal closed form
 *       c (f_d +- 2 (s - 1)/sqrt(3))/s, s = sqrt(4 - 3 f_d^2) (m1_speeds);
 *       left speed min over both states and 0, right speed max over both
 *       states and 0.
 */
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <vector>
#include <algorithm>

namespace {

/* ---------------------------------------------------------------- constants */
/* CGS.  13.6 eV is the hydrogen ionisation threshold used in Sec. 2.2.4. */
const double C_LIGHT = 2.99792458e10;     /* cm s^-1 */
const double K_B = 1.380649e-16;          /* erg K^-1 */
const double EV = 1.602176634e-12;        /* erg */
const double E_ION_EV = 13.6;             /* eV */
const double T_HI = 157807.0;             /* K, ionisation temperature of H */
const double PI = 3.14159265358979323846;
const int MAX_HALVINGS = 64;              /* R10 */

/* ------------------------------------------------------ forward-mode dual */
/* A value and one directional derivative.  Comparisons look at the value only,
 * so the branch taken is the one the plain double run takes and the tangent
 * is the derivative of the piecewise-smooth discrete map along that branch. */
struct Dual {
    double v, d;
    Dual() : v(0), d(0) {}
    Dual(double a) : v(a), d(0) {}
    Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
    double q = a.v / b.v;
    return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual &operator+=(Dual &a, Dual b) { a = a + b; return a; }
inline Dual &operator-=(Dual &a, Dual b) { a = a - b; return a; }
inline Dual &operator*=(Dual &a, Dual b) { a = a * b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }
inline Dual exp(Dual a) { double e = std::exp(a.v); return Dual(e, e * a.d); }
inline Dual log(Dual a) { return Dual(std::log(a.v), a.d / a.v); }
inline Dual sqrt(Dual a) { double s = std::sqrt(a.v); return Dual(s, a.d / (2.0 * s)); }
inline Dual pow(Dual a, double p) {
    double r = std::pow(a.v, p);
    return Dual(r, p * std::pow(a.v, p - 1.0) * a.d);
}
inline Dual fabs(Dual a) { return a.v < 0 ? -a : a; }

inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }

using std::exp;
using std::log;
using std::sqrt;
using std::pow;
using std::fabs;

template <class R> inline R rmin(R a, R b) { return (b < a) ? b : a; }
template <class R> inline R rmax(R a, R b) { return (a < b) ? b : a; }

/* --------------------------------------------------------------- parameters */
/* Boundary kinds of the faces x-, x+, y-, y+, z-, z+ (R16, R17) and the flux
 * functions (R1, R18). */
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3 };
enum { FLUX_GLF = 0, FLUX_HLL = 1 };

struct Params {
    int nx, ny, nz, G;
    double dx, c, dt;
    int otsa, isothermal, max_substeps;
    int bc[6], flux;
    double inflow[6]; /* photons cm^-2 s^-1 entering through an inflow face */
    double sigN[4], sigE[4], meanE[4], frac[4];
    double SigmaE[4]; /* sigma_E <E> - sigma_N E_13.6, Sec. 2.2.4 */
};

struct Counters {
    int64_t limiter = 0, neg_clamp = 0, x_clamp = 0, cap_hits = 0;
    int64_t substeps = 0, attempts = 0, max_sub = 0;
};

/* ------------------------------------------------------- atomic rate fits */
/* Sec. 2.2.4 names the rate compilation but prints none of it (R12).  These
 * are the Hui & Gnedin (1997) fits, lam = 2 T_HI / T, in cm^3 s^-1. */
template <class R> struct Rates {
    R alphaA, alphaB, beta;
    R recA, recB;     /* recombination cooling coefficients x T, erg cm^3 s^-1 */
    R cexc;           /* collisional excitation coefficient, erg cm^3 s^-1 */
    R brems;          /* bremsstrahlung coefficient, erg cm^3 s^-1 */
};

template <class R> Rates<R> rates_at(R T) {
    Rates<R> r;
    R lam = 2.0 * T_HI / T;
    r.alphaA = 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
    r.alphaB = 2.753e-14 * pow(lam, 1.500) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    r.beta = 21.11 * pow(T, -1.5) * exp(-lam / 2.0) * pow(lam, -1.089)
             / pow(1.0 + pow(lam / 0.354, 0.874), 1.101);
    r.recA = 1.778e-29 * T * pow(lam, 1.965) / pow(1.0 + pow(lam / 0.541, 0.502), 2.697);
    r.recB = 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720);
    r.cexc = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sqrt(T / 1e5));
    r.brems = 1.42e-27 * 1.3 * sqrt(T);
    return r;
}

/* Cooling rate Lambda(n0, x, T) in erg cm^-3 s^-1 (eq. e:therm4), with
 * n_e = n_p = x n0 and n_HI = (1-x) n0: recombination (case B on the spot,
 * case A otherwise), collisional ionisation, collisional excitation and
 * bremsstrahlung.  Compton cooling is off (no redshift). */
template <class R> R cooling(const Rates<R> &r, R n0, R x, int otsa) {
    R ne = x * n0, np = x * n0, nHI = (1.0 - x) * n0;
    R rec = (otsa ? r.recB : r.recA) * ne * np;
    R cion = K_B * T_HI * r.beta * ne * nHI;
    R cex = r.cexc * ne * nHI;
    R ff = r.brems * ne * np;
    return rec + cion + cex + ff;
}

/* ------------------------------------------------------------ M1 closure */
/* Sec. 2.2.3: P = D N with the Eddington tensor D (R2, R3, R4).  Output is the
 * full symmetric 3x3 tensor P[k][d]. */
template <class R> void m1_pressure(R N, const R F[3], double c, R P[3][3]) {
    R F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    R Fn = (F2 > R(0.0)) ? sqrt(F2) : R(0.0);
    R f = R(0.0);
    if (N > R(0.0)) f = rmin(R(1.0), Fn / (c * N));
    R chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
    R n[3];
    for (int k = 0; k < 3; ++k) n[k] = (Fn > R(0.0)) ? F[k] / Fn : R(0.0);
    R iso = (1.0 - chi) / 2.0, dir = (3.0 * chi - 1.0) / 2.0;
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d)
            P[k][d] = N * ((k == d ? iso : R(0.0)) + dir * n[k] * n[d]);
}

/* ------------------------------------------------------------ M1 transport */
inline int64_t cell_index(const Params &p, int x, int y, int z) {
    return ((int64_t)z * p.ny + y) * p.nx + x;
}

/* Intercell flux of eq. (e:glf) across a face normal to axis d between a left
 * state (NL, FL) and a right state (NR, FR):
 *   flux of N   = (F_d,L + F_d,R)/2       - c (N_R - N_L)/2
 *   flux of F_k = c^2 (P_kd,L + P_kd,R)/2 - c (F_k,R - F_k,L)/2         */
template <class R>
void glf_flux(R NL, const R FL[3], R NR, const R FR[3], int d, double c,
              R &fluxN, R fluxF[3]) {
    R PL[3][3], PR[3][3];
    m1_pressure(NL, FL, c, PL);
    m1_pressure(NR, FR, c, PR);
    fluxN = 0.5 * (FL[d] + FR[d]) - 0.5 * c * (NR - NL);
    for (int k = 0; k < 3; ++k)
        fluxF[k] = 0.5 * c * c * (PL[k][d] + PR[k][d]) - 0.5 * c * (FR[k] - FL[k]);
}

/* Signal speeds along axis d of one state (R18).  With s = sqrt(4 - 3 f^2),
 * chi = (3 + 4f^2)/(5 + 2s) gives chi' - 2f = 2f (1 - s)/s and
 * chi - f^2 = (1 - s)^2/3, so the radicand chi'^2 + 4(chi - f chi') is
 * 16 (s - 1)^2/(3 s^2) and the eigenvalues c (chi' +- sqrt(radicand))/2 are
 * c (f +- 2 (s - 1)/sqrt(3))/s, with s - 1 = 3 (1 - f)(1 + f)/(1 + s): the
 * same values without the cancellation of the radicand near |f| = 1. */
template <class R> void m1_speeds(R N, const R F[3], int d, double c, R &lmin, R &lmax) {
    R f = R(0.0);
    if (N > R(0.0)) f = rmax(R(-1.0), rmin(R(1.0), F[d] / (c * N)));
    const R s = sqrt(4.0 - 3.0 * f * f);
    const R w = 3.4641016151377544 * (1.0 - f) * (1.0 + f) / (1.0 + s); /* 2 (s - 1)/sqrt(3) */
    lmin = c * (f - w) / s;
    lmax = c * (f + w) / s;
}

/* HLL flux across a face normal to axis d (R18):
 *   flux = (a+ Ft(U_L) - a- Ft(U_R) + a+ a- (U_R - U_L)) / (a+ - a-),
 * Ft_d(U) = (F_d, c^2 P_.d), a- = min(0, speeds), a+ = max(0, speeds).
 * With a+- = +-c it is the flux of eq. (e:glf). */
template <class R>
void hll_flux(R NL, const R FL[3], R NR, const R FR[3], int d, double c, R &fluxN, R fluxF[3]) {
    R PL[3][3], PR[3][3];
    m1_pressure(NL, FL, c, PL);
    m1_pressure(NR, FR, c, PR);
    R lminL, lmaxL, lminR, lmaxR;
    m1_speeds(NL, FL, d, c, lminL, lmaxL);
    m1_speeds(NR, FR, d, c, lminR, lmaxR);
    R am = rmin(R(0.0), rmin(lminL, lminR));
    R ap = rmax(R(0.0), rmax(lmaxL, lmaxR));
    R inv = 1.0 / (ap - am);
    fluxN = (ap * FL[d] - am * FR[d] + ap * am * (NR - NL)) * inv;
    for (int k = 0; k < 3; ++k)
        fluxF[k] = (ap * c * c * PL[k][d] - am * c * c * PR[k][d] + ap * am * (FR[k] - FL[k])) * inv;
}

template <class R>
void face_flux(const Params &p, R NL, const R FL[3], R NR, const R FR[3], int d, R &fluxN, R fluxF[3]) {
    if (p.flux == FLUX_HLL) hll_flux(NL, FL, NR, FR, d, p.c, fluxN, fluxF);
    else glf_flux(NL, FL, NR, FR, d, p.c, fluxN, fluxF);
}

/* The neighbour of cell (x, y, z) of group g on side s (-1 or +1) of axis d:
 * the next cell, across a periodic face the cell on the far side of the grid,
 * and across any other face the outside state of R16/R17. */
template <class R>
void neighbour(const Params &p, const R *Ng, const R *Fg, int g, int x, int y, int z, int d, int s,
               R &Nn, R Fn[3]) {
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    int c3[3] = {x, y, z};
    const int n3[3] = {p.nx, p.ny, p.nz};
    const int face = 2 * d + (s > 0 ? 1 : 0);
    int q = c3[d] + s;
    int kind = BC_PERIODIC;
    if (q < 0 || q >= n3[d]) {
        kind = p.bc[face];
        q = (kind == BC_PERIODIC) ? (q + n3[d]) % n3[d] : c3[d];
    }
    c3[d] = q;
    const int64_t j = cell_index(p, c3[0], c3[1], c3[2]);
    Nn = Ng[j];
    for (int k = 0; k < 3; ++k) Fn[k] = Fg[k * V + j];
    if (kind == BC_REFLECTIVE) {
        Fn[d] = -Fn[d];
    } else if (kind == BC_INFLOW) {
        const double phi = p.inflow[face] * p.frac[g];
        Nn = R(phi / p.c);
        for (int k = 0; k < 3; ++k) Fn[k] = R(0.0);
        Fn[d] = R(s < 0 ? phi : -phi); /* pointing into the domain */
    }
}

/* One conservative transport update of every group (eq. e:uprt, 3D unsplit,
 * R5; boundaries R16, R17; flux R1 or R18), from the old state (N, F) into (Ns, Fs),
 * followed by the floor N* >= 0 and the limiter |F*| <= c N* (R13).
 * Layout: N[g][z][y][x], F[g][k][z][y][x]. */
template <class R>
void transport(const Params &p, const R *N, const R *F, R *Ns, R *Fs, Counters &cnt) {
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const double lam = p.dt / p.dx;
    for (int g = 0; g < p.G; ++g) {
        const R *Ng = N + g * V;
        const R *Fg = F + (int64_t)g * 3 * V;
        for (int z = 0; z < p.nz; ++z)
        for (int y = 0; y < p.ny; ++y)
        for (int x = 0; x < p.nx; ++x) {
            int64_t i = cell_index(p, x, y, z);
            R Fi[3] = {Fg[i], Fg[V + i], Fg[2 * V + i]};
            R accN = R(0.0);
            R accF[3] = {R(0.0), R(0.0), R(0.0)};
            for (int d = 0; d < 3; ++d) {
                R Nm, Fm[3], Np, Fp[3];
                neighbour(p, Ng, Fg, g, x, y, z, d, -1, Nm, Fm);
                neighbour(p, Ng, Fg, g, x, y, z, d, +1, Np, Fp);
                R lo_N, lo_F[3], hi_N, hi_F[3];
                face_flux(p, Nm, Fm, Ng[i], Fi, d, lo_N, lo_F);   /* face i-1/2 */
                face_flux(p, Ng[i], Fi, Np, Fp, d, hi_N, hi_F);   /* face i+1/2 */
                accN += lo_N - hi_N;
                for (int k = 0; k < 3; ++k) accF[k] += lo_F[k] - hi_F[k];
            }
            R n = Ng[i] + lam * accN;
            R f[3];
            for (int k = 0; k < 3; ++k) f[k] = Fi[k] + lam * accF[k];
            if (n < R(0.0)) { n = R(0.0); cnt.neg_clamp++; }
            R F2 = f[0] * f[0] + f[1] * f[1] + f[2] * f[2];
            if (F2 > R(0.0)) {
                R Fn = sqrt(F2);
                if (Fn > p.c * n) {
                    R s = p.c * n / Fn;
                    for (int k = 0; k < 3; ++k) f[k] = f[k] * s;
                    cnt.limiter++;
                }
            }
            Ns[g * V + i] = n;
            for (int k = 0; k < 3; ++k) Fs[((int64_t)g * 3 + k) * V + i] = f[k];
        }
    }
}

/* ---------------------------------------------------------- thermochemistry */
/* The sub-cycled update of Sec. 2.2.4 for one cell (eqs. e:therm1g, e:therm2g,
 * e:therm3, e:therm4 with the multigroup sums e:g2, e:g3), following the
 * printed discrete sequence N -> F -> x -> e with readings R6-R11, R13-R15.
 * N[g], F[g][3] are the post-transport values on entry and the final ones on
 * exit; S[g] is the source rate density of this cell (photons s^-1 cm^-3).
 * Returns the number of accepted substeps; *cap is set when R10's guard fired. */
template <class R>
int chem_cell(const Params &p, R *N, R (*F)[3], R &x, R &T, R n0, const R *S,
              int *attempts_out, int *cap_out, int *xclamp_out) {
    const int G = p.G;
    const double c = p.c;
    R e = 1.5 * (1.0 + x) * n0 * K_B * T;
    R rem = R(p.dt);
    int nsub = 0, attempts = 0, cap = 0, xclamp = 0;
    while (rem > R(0.0)) {
        /* R10: a cell whose energy is not a positive finite number (invalid
         * input) is left as it stands for the rest of the step. */
        if (!p.isothermal && !(val(e) > 0.0 && val(e) < HUGE_VAL)) break;
        bool last = nsub >= p.max_substeps;          /* R10 */
        R Tp = p.isothermal ? T : e / (1.5 * (1.0 + x) * n0 * K_B);
        Rates<R> r = rates_at(Tp);
        R alpha = p.otsa ? r.alphaB : r.alphaA;
        R dtau = rem;
        if (!p.isothermal && !last) {
            R sumH = R(0.0);
            for (int g = 0; g < G; ++g) sumH += p.SigmaE[g] * N[g];
            R H = c * (1.0 - x) * n0 * sumH;
            R Lam = cooling(r, n0, x, p.otsa);
            if (!(H == Lam)) dtau = rmin(rem, fabs(e / (H - Lam)));
        }
        R Nn[4], Fn[4][3], xn, en;
        int halvings = 0;
        for (;;) {
            attempts++;
            /* photons: sources, recombination photons, absorption (R7, R8, R14) */
            for (int g = 0; g < G; ++g) {
                R kappa = c * p.sigN[g] * (1.0 - x) * n0;
                R rec = R(0.0);
                if (g == 0 && !p.otsa) rec = (r.alphaA - r.alphaB) * x * x * n0 * n0;
                R den = 1.0 + dtau * kappa;
                Nn[g] = (N[g] + (S[g] + rec) * dtau) / den;
                for (int k = 0; k < 3; ++k) Fn[g][k] = F[g][k] / den;
            }
            /* ionised fraction, with the new photon densities */
            R Gam = R(0.0);
            for (int g = 0; g < G; ++g) Gam += c * p.sigN[g] * Nn[g];
            xn = 1.0 - (alpha * x * x * n0 * dtau + 1.0 - x)
                       / (1.0 + dtau * (r.beta * x * n0 + Gam));
            if (xn < R(0.0)) { xn = R(0.0); xclamp++; }
            if (xn > R(1.0)) { xn = R(1.0); xclamp++; }
            if (p.isothermal) { en = e; break; }
            /* internal energy: photo-heating with the new N and x, cooling at T^p */
            R sumH = R(0.0);
            for (int g = 0; g < G; ++g) sumH += p.SigmaE[g] * Nn[g];
            en = e + dtau * c * (1.0 - xn) * n0 * sumH
                   - dtau * cooling(r, n0, xn, p.otsa);
            if (last) break;
            if (fabs(en - e) <= 0.1 * e) break;                 /* R10 */
            if (halvings == MAX_HALVINGS) { cap = 1; break; }
            dtau = dtau / 2.0;
            halvings++;
        }
        for (int g = 0; g < G; ++g) {
            N[g] = Nn[g];
            for (int k = 0; k < 3; ++k) F[g][k] = Fn[g][k];
        }
        x = xn;
        e = en;
        rem = rem - dtau;
        nsub++;
        if (last) { cap = 1; break; }
        if (p.isothermal) break;
    }
    if (!p.isothermal) T = e / (1.5 * (1.0 + x) * n0 * K_B);
    *attempts_out = attempts;
    *cap_out = cap;
    *xclamp_out = xclamp;
    return nsub;
}

/* ----------------------------------------------------------- whole step */
/* S[i][g]: summed source rate density per cell (R7): every source adds
 * rate * frac_g / dx^3 to its host cell, in list order. */
template <class R>
void source_density(const Params &p, const int64_t *src_cell, const R *src_rate, int n_src,
                    std::vector<R> &S) {
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    S.assign((size_t)V * p.G, R(0.0));
    const double vol = p.dx * p.dx * p.dx;
    for (int s = 0; s < n_src; ++s)
        for (int g = 0; g < p.G; ++g)
            S[(size_t)src_cell[s] * p.G + g] += src_rate[s] * p.frac[g] / vol;
}

template <class R>
void run_steps(const Params &p, int n_steps, R *N, R *F, R *x, R *T, const R *n0,
               const std::vector<R> &S, int64_t *substeps_cell, Counters &cnt) {
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const int G = p.G;
    std::vector<R> Ns((size_t)G * V), Fs((size_t)G * 3 * V);
    for (int step = 0; step < n_steps; ++step) {
        transport(p, N, F, Ns.data(), Fs.data(), cnt);
        for (int64_t i = 0; i < V; ++i) {
            R Nc[4], Fc[4][3], Sc[4];
            for (int g = 0; g < G; ++g) {
                Nc[g] = Ns[g * V + i];
                for (int k = 0; k < 3; ++k) Fc[g][k] = Fs[((int64_t)g * 3 + k) * V + i];
                Sc[g] = S[(size_t)i * G + g];
            }
            int att = 0, cap = 0, xcl = 0;
            int ns = chem_cell(p, Nc, Fc, x[i], T[i], n0[i], Sc, &att, &cap, &xcl);
            cnt.substeps += ns;
            cnt.attempts += att;
            cnt.cap_hits += cap;
            cnt.x_clamp += xcl;
            if (ns > cnt.max_sub) cnt.max_sub = ns;
            if (substeps_cell) substeps_cell[i] += ns;
            for (int g = 0; g < G; ++g) {
                N[g * V + i] = Nc[g];
                for (int k = 0; k < 3; ++k) F[((int64_t)g * 3 + k) * V + i] = Fc[g][k];
            }
        }
    }
}

/* --------------------------------------- coarse transport, fine chemistry */
/* Pairwise sum of v[0..n) (n a power of two) in index order (R19). */
template <class R> R pair_sum(const R *v, int n) {
    if (n == 1) return v[0];
    return pair_sum(v, n / 2) + pair_sum(v + n / 2, n / 2);
}

/* n_steps steps of R19.  ref_cell[n_ref]: refined coarse cells (distinct);
 * xf, Tf, nf: [n_ref][r^3] child fields, child index (cz r + cy) r + cx;
 * Sc: coarse source densities (sources in unrefined cells), Sf: [n_ref r^3][G]
 * child source densities. */
template <class R>
void run_crta(const Params &p, int n_steps, R *N, R *F, R *x, R *T, const R *n0, const std::vector<R> &Sc,
              int n_ref, const int64_t *ref_cell, int ratio, R *xf, R *Tf, const R *nf, const std::vector<R> &Sf,
              Counters &cnt) {
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const int G = p.G;
    const int nc = ratio * ratio * ratio;
    std::vector<char> refined((size_t)V, 0);
    for (int j = 0; j < n_ref; ++j) refined[(size_t)ref_cell[j]] = 1;
    std::vector<R> Ns((size_t)G * V), Fs((size_t)G * 3 * V);
    std::vector<R> cN((size_t)nc), cF((size_t)nc), w((size_t)nc), tmp((size_t)nc);
    for (int step = 0; step < n_steps; ++step) {
        transport(p, N, F, Ns.data(), Fs.data(), cnt);
        /* unrefined coarse cells: the ordinary chemistry */
        for (int64_t i = 0; i < V; ++i) {
            if (refined[(size_t)i]) continue;
            R Nc[4], Fc[4][3], S[4];
            for (int g = 0; g < G; ++g) {
                Nc[g] = Ns[g * V + i];
                for (int k = 0; k < 3; ++k) Fc[g][k] = Fs[((int64_t)g * 3 + k) * V + i];
                S[g] = Sc[(size_t)i * G + g];
            }
            int att = 0, cap = 0, xcl = 0;
            int ns = chem_cell(p, Nc, Fc, x[i], T[i], n0[i], S, &att, &cap, &xcl);
            cnt.substeps += ns; cnt.attempts += att; cnt.cap_hits += cap; cnt.x_clamp += xcl;
            if (ns > cnt.max_sub) cnt.max_sub = ns;
            for (int g = 0; g < G; ++g) {
                N[g * V + i] = Nc[g];
                for (int k = 0; k < 3; ++k) F[((int64_t)g * 3 + k) * V + i] = Fc[g][k];
            }
        }
        /* refined cells: chemistry of every child with the parent's N*, F*, then restriction */
        for (int j = 0; j < n_ref; ++j) {
            const int64_t pi = ref_cell[j];
            std::vector<R> chN((size_t)nc * G), chF((size_t)nc * G * 3);
            for (int c = 0; c < nc; ++c) {
                const size_t f = (size_t)j * nc + c;
                R Nc[4], Fc[4][3], S[4];
                for (int g = 0; g < G; ++g) {
                    Nc[g] = Ns[g * V + pi];
                    for (int k = 0; k < 3; ++k) Fc[g][k] = Fs[((int64_t)g * 3 + k) * V + pi];
                    S[g] = Sf[f * G + g];
                }
                int att = 0, cap = 0, xcl = 0;
                int ns = chem_cell(p, Nc, Fc, xf[f], Tf[f], nf[f], S, &att, &cap, &xcl);
                cnt.substeps += ns; cnt.attempts += att; cnt.cap_hits += cap; cnt.x_clamp += xcl;
                if (ns > cnt.max_sub) cnt.max_sub = ns;
                for (int g = 0; g < G; ++g) {
                    chN[(size_t)c * G + g] = Nc[g];
                    for (int k = 0; k < 3; ++k) chF[((size_t)c * G + g) * 3 + k] = Fc[g][k];
                }
            }
            const R inv = R(1.0 / nc);
            for (int g = 0; g < G; ++g) {
                for (int c = 0; c < nc; ++c) cN[c] = chN[(size_t)c * G + g];
                N[g * V + pi] = pair_sum(cN.data(), nc) * inv;
                for (int k = 0; k < 3; ++k) {
                    for (int c = 0; c < nc; ++c) cF[c] = chF[((size_t)c * G + g) * 3 + k];
                    F[((int64_t)g * 3 + k) * V + pi] = pair_sum(cF.data(), nc) * inv;
                }
            }
            /* x: n0-weighted; T: (1+x) n0-weighted (internal energy e = 3/2 (1+x) n0 k_B T) */
            const size_t f0 = (size_t)j * nc;
            R nsum = pair_sum(nf + f0, nc);
            for (int c = 0; c < nc; ++c) tmp[c] = xf[f0 + c] * (nf[f0 + c] / nsum);
            x[pi] = pair_sum(tmp.data(), nc);
            for (int c = 0; c < nc; ++c) w[c] = (1.0 + xf[f0 + c]) * nf[f0 + c];
            R msum = pair_sum(w.data(), nc);
            for (int c = 0; c < nc; ++c) tmp[c] = Tf[f0 + c] * (w[c] / msum);
            T[pi] = pair_sum(tmp.data(), nc);
        }
    }
}

/* ------------------------------------------------------- photoionisation */
/* Hydrogen photoionisation cross-section (exact hydrogenic form, Osterbrock &
 * Ferland), the paper cites a fit for it without printing one (R12):
 *   sigma(nu) = 6.30e-18 (nu0/nu)^4 exp(4 - 4 atan(eps)/eps) / (1 - exp(-2 pi/eps)),
 *   eps = sqrt(nu/nu0 - 1), zero below threshold, 6.30e-18 at threshold. */
double cross_section(double E_eV) {
    if (E_eV < E_ION_EV) return 0.0;
    if (E_eV == E_ION_EV) return 6.30e-18;
    double r = E_eV / E_ION_EV;
    double eps = std::sqrt(r - 1.0);
    return 6.30e-18 * std::pow(1.0 / r, 4.0) * std::exp(4.0 - 4.0 * std::atan(eps) / eps)
           / (1.0 - std::exp(-2.0 * PI / eps));
}

/* Group constants of Sec. 2.2.3-2.2.4 (eqs. e:sgroup, e:siggroup and the
 * definitions of sigma_E and <E>) for a black body of temperature Tbb, whose
 * photon number spectrum per unit energy is E^2/(exp(E/kT)-1):
 *   sigma_N = int sigma N_E / int N_E,  <E> = int E N_E / int N_E,
 *   sigma_E = int sigma E N_E / (<E> int N_E),  frac = int_g N_E / int_all N_E.
 * Composite Simpson rule in ln E with n panels per group (plain, slow). */
void group_constants(double Tbb, const double *edges_eV, int G, int panels,
                     double *sigN, double *sigE, double *meanE_erg, double *frac) {
    const double kT = K_B * Tbb / EV; /* eV */
    if (panels % 2) panels++;             /* Simpson needs an even count */
    std::vector<double> n_int(G);
    double total = 0.0;
    for (int g = 0; g < G; ++g) {
        double a = std::log(edges_eV[g]), b = std::log(edges_eV[g + 1]);
        double h = (b - a) / panels;
        double I_n = 0, I_sn = 0, I_en = 0, I_sen = 0;
        for (int j = 0; j <= panels; ++j) {
            double w = (j == 0 || j == panels) ? 1.0 : ((j % 2) ? 4.0 : 2.0);
            double E = (j == 0) ? edges_eV[g]
                     : (j == panels) ? edges_eV[g + 1] : std::exp(a + j * h);
            /* dE = E dlnE */
            double nE = E * E / std::expm1(E / kT) * E;
            double s = cross_section(E);
            I_n += w * nE;
            I_sn += w * s * nE;
            I_en += w * E * nE;
            I_sen += w * s * E * nE;
        }
        sigN[g] = I_sn / I_n;
        double mE = I_en / I_n;
        meanE_erg[g] = mE * EV;
        sigE[g] = I_sen / (mE * I_n);
        n_int[g] = I_n * h / 3.0;
        total += n_int[g];
    }
    for (int g = 0; g < G; ++g) frac[g] = n_int[g] / total;
}

bool fill_params(Params &p, const int *ints, const double *dbls, const double *groups) {
    p.nx = ints[0]; p.ny = ints[1]; p.nz = ints[2]; p.G = ints[3];
    p.otsa = ints[4]; p.isothermal = ints[5]; p.max_substeps = ints[6];
    for (int f = 0; f < 6; ++f) p.bc[f] = ints[7 + f];
    p.flux = ints[13];
    p.dx = dbls[0]; p.c = dbls[1]; p.dt = dbls[2];
    for (int f = 0; f < 6; ++f) p.inflow[f] = dbls[3 + f];
    if (p.G < 1 || p.G > 4 || p.nx < 1 || p.ny < 1 || p.nz < 1) return false;
    if (p.flux != FLUX_GLF && p.flux != FLUX_HLL) return false;
    for (int d = 0; d < 3; ++d) {
        const int a = p.bc[2 * d], b = p.bc[2 * d + 1];
        if (a < BC_PERIODIC || a > BC_INFLOW || b < BC_PERIODIC || b > BC_INFLOW) return false;
        if ((a == BC_PERIODIC) != (b == BC_PERIODIC)) return false;
    }
    for (int g = 0; g < p.G; ++g) {
        p.sigN[g] = groups[0 * 4 + g];
        p.sigE[g] = groups[1 * 4 + g];
        p.meanE[g] = groups[2 * 4 + g];
        p.frac[g] = groups[3 * 4 + g];
        p.SigmaE[g] = p.sigE[g] * p.meanE[g] - p.sigN[g] * E_ION_EV * EV;
    }
    return true;
}

void export_counters(const Counters &c, int64_t *out) {
    if (!out) return;
    out[0] = c.limiter; out[1] = c.neg_clamp; out[2] = c.x_clamp; out[3] = c.cap_hits;
    out[4] = c.substeps; out[5] = c.attempts; out[6] = c.max_sub;
}

} /* namespace */

/* ===================================================================== C ABI */
/* ints:  [nx, ny, nz, G, otsa, isothermal, max_substeps, bc x- x+ y- y+ z- z+, flux]
 * dbls:  [dx (cm), c_red (cm/s), dt (s), inflow x- x+ y- y+ z- z+ (photons cm^-2 s^-1)]
 * groups: 4x4 row-major [sigma_N; sigma_E; <E> (erg); source fraction], first G used
 * counters (optional, 7): limiter, N<0 clamps, x clamps, cap hits,
 *                         accepted substeps, attempts, max substeps in a cell   */
extern "C" {

int oracle_run(const int *ints, const double *dbls, const double *groups, int n_steps,
               double *N, double *F, double *x, double *T, const double *n0,
               const int64_t *src_cell, const double *src_rate, int n_src,
               int64_t *substeps_cell, int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    std::vector<double> S;
    source_density(p, src_cell, src_rate, n_src, S);
    Counters cnt;
    run_steps<double>(p, n_steps, N, F, x, T, n0, S, substeps_cell, cnt);
    export_counters(cnt, counters);
    return 0;
}

/* Same map, carried in dual numbers: on entry dN, dF, dx_, dT hold a tangent
 * direction of the initial state and dn0, drate one of n0 and the source
 * rates; on exit (N, F, x, T) hold the end state and (dN, dF, dx_, dT) its
 * directional derivative. */
int oracle_run_tangent(const int *ints, const double *dbls, const double *groups, int n_steps,
                       double *N, double *F, double *x, double *T, const double *n0,
                       const int64_t *src_cell, const double *src_rate, int n_src,
                       double *dN, double *dF, double *dx_, double *dT,
                       const double *dn0, const double *drate, int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const int G = p.G;
    std::vector<Dual> dN_((size_t)G * V), dF_((size_t)G * 3 * V), dX(V), dTT(V), dn(V), dr(n_src);
    for (int64_t i = 0; i < (int64_t)G * V; ++i) dN_[i] = Dual(N[i], dN[i]);
    for (int64_t i = 0; i < (int64_t)G * 3 * V; ++i) dF_[i] = Dual(F[i], dF[i]);
    for (int64_t i = 0; i < V; ++i) {
        dX[i] = Dual(x[i], dx_[i]);
        dTT[i] = Dual(T[i], dT[i]);
        dn[i] = Dual(n0[i], dn0[i]);
    }
    for (int s = 0; s < n_src; ++s) dr[s] = Dual(src_rate[s], drate[s]);
    std::vector<Dual> S;
    source_density(p, src_cell, dr.data(), n_src, S);
    Counters cnt;
    run_steps<Dual>(p, n_steps, dN_.data(), dF_.data(), dX.data(), dTT.data(), dn.data(), S,
                    nullptr, cnt);
    for (int64_t i = 0; i < (int64_t)G * V; ++i) { N[i] = dN_[i].v; dN[i] = dN_[i].d; }
    for (int64_t i = 0; i < (int64_t)G * 3 * V; ++i) { F[i] = dF_[i].v; dF[i] = dF_[i].d; }
    for (int64_t i = 0; i < V; ++i) {
        x[i] = dX[i].v; dx_[i] = dX[i].d;
        T[i] = dTT[i].v; dT[i] = dTT[i].d;
    }
    export_counters(cnt, counters);
    return 0;
}

/* R19: n_steps steps with the coarse transport and the chemistry on the
 * children of the refined cells.  src_child[n_src]: child index of each source
 * whose host cell is refined (ignored otherwise).  Returns -1 for bad
 * arguments (ratio not 2 or 4, a refined cell out of range or repeated). */
int oracle_run_crta(const int *ints, const double *dbls, const double *groups, int n_steps,
                    double *N, double *F, double *x, double *T, const double *n0,
                    const int64_t *src_cell, const double *src_rate, const int *src_child, int n_src,
                    int n_ref, const int64_t *ref_cell, int ratio, double *xf, double *Tf, const double *nf,
                    int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    if (ratio != 2 && ratio != 4) return -1;
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const int nc = ratio * ratio * ratio;
    std::vector<int> which((size_t)V, -1);
    for (int j = 0; j < n_ref; ++j) {
        if (ref_cell[j] < 0 || ref_cell[j] >= V || which[(size_t)ref_cell[j]] >= 0) return -1;
        which[(size_t)ref_cell[j]] = j;
    }
    const int G = p.G;
    std::vector<double> Sc((size_t)V * G, 0.0), Sf((size_t)n_ref * nc * G, 0.0);
    const double vol = p.dx * p.dx * p.dx;
    const double hf = p.dx / ratio;
    const double volf = hf * hf * hf;
    for (int s = 0; s < n_src; ++s) {
        const int j = which[(size_t)src_cell[s]];
        if (j < 0) {
            for (int g = 0; g < G; ++g) Sc[(size_t)src_cell[s] * G + g] += src_rate[s] * p.frac[g] / vol;
        } else {
            const int c = src_child ? src_child[s] : 0;
            if (c < 0 || c >= nc) return -1;
            for (int g = 0; g < G; ++g) Sf[((size_t)j * nc + c) * G + g] += src_rate[s] * p.frac[g] / volf;
        }
    }
    Counters cnt;
    run_crta<double>(p, n_steps, N, F, x, T, n0, Sc, n_ref, ref_cell, ratio, xf, Tf, nf, Sf, cnt);
    export_counters(cnt, counters);
    return 0;
}

/* R19 carried in dual numbers: the end state (coarse and children) and its
 * directional derivative along (dN, dF, dx, dT, dn0) of the coarse state,
 * (dxf, dTf, dnf) of the children and drate of the source rates.  Source
 * densities as in oracle_run_crta. */
int oracle_run_crta_tangent(const int *ints, const double *dbls, const double *groups, int n_steps,
                            double *N, double *F, double *x, double *T, const double *n0,
                            const int64_t *src_cell, const double *src_rate, const int *src_child, int n_src,
                            int n_ref, const int64_t *ref_cell, int ratio, double *xf, double *Tf,
                            const double *nf, double *dN, double *dF, double *dx_, double *dT, const double *dn0,
                            const double *drate, double *dxf, double *dTf, const double *dnf, int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    if (ratio != 2 && ratio != 4) return -1;
    const int64_t V = (int64_t)p.nx * p.ny * p.nz;
    const int nc = ratio * ratio * ratio;
    std::vector<int> which((size_t)V, -1);
    for (int j = 0; j < n_ref; ++j) {
        if (ref_cell[j] < 0 || ref_cell[j] >= V || which[(size_t)ref_cell[j]] >= 0) return -1;
        which[(size_t)ref_cell[j]] = j;
    }
    const int G = p.G;
    const size_t nfine = (size_t)n_ref * nc;
    std::vector<Dual> dN_((size_t)G * V), dF_((size_t)G * 3 * V), dX(V), dTT(V), dn(V);
    std::vector<Dual> dXf(nfine), dTf_(nfine), dNf(nfine);
    for (int64_t i = 0; i < (int64_t)G * V; ++i) dN_[i] = Dual(N[i], dN[i]);
    for (int64_t i = 0; i < (int64_t)G * 3 * V; ++i) dF_[i] = Dual(F[i], dF[i]);
    for (int64_t i = 0; i < V; ++i) {
        dX[i] = Dual(x[i], dx_[i]);
        dTT[i] = Dual(T[i], dT[i]);
        dn[i] = Dual(n0[i], dn0[i]);
    }
    for (size_t f = 0; f < nfine; ++f) {
        dXf[f] = Dual(xf[f], dxf[f]);
        dTf_[f] = Dual(Tf[f], dTf[f]);
        dNf[f] = Dual(nf[f], dnf[f]);
    }
    std::vector<Dual> Sc((size_t)V * G, Dual(0.0)), Sf(nfine * G, Dual(0.0));
    const double vol = p.dx * p.dx * p.dx;
    const double hf = p.dx / ratio;
    const double volf = hf * hf * hf;
    for (int s = 0; s < n_src; ++s) {
        const Dual r(src_rate[s], drate[s]);
        const int j = which[(size_t)src_cell[s]];
        if (j < 0) {
            for (int g = 0; g < G; ++g) Sc[(size_t)src_cell[s] * G + g] += r * Dual(p.frac[g]) / Dual(vol);
        } else {
            const int c = src_child ? src_child[s] : 0;
            if (c < 0 || c >= nc) return -1;
            for (int g = 0; g < G; ++g) Sf[((size_t)j * nc + c) * G + g] += r * Dual(p.frac[g]) / Dual(volf);
        }
    }
    Counters cnt;
    run_crta<Dual>(p, n_steps, dN_.data(), dF_.data(), dX.data(), dTT.data(), dn.data(), Sc, n_ref, ref_cell,
                   ratio, dXf.data(), dTf_.data(), dNf.data(), Sf, cnt);
    for (int64_t i = 0; i < (int64_t)G * V; ++i) { N[i] = dN_[i].v; dN[i] = dN_[i].d; }
    for (int64_t i = 0; i < (int64_t)G * 3 * V; ++i) { F[i] = dF_[i].v; dF[i] = dF_[i].d; }
    for (int64_t i = 0; i < V; ++i) {
        x[i] = dX[i].v; dx_[i] = dX[i].d;
        T[i] = dTT[i].v; dT[i] = dTT[i].d;
    }
    for (size_t f = 0; f < nfine; ++f) {
        xf[f] = dXf[f].v; dxf[f] = dXf[f].d;
        Tf[f] = dTf_[f].v; dTf[f] = dTf_[f].d;
    }
    export_counters(cnt, counters);
    return 0;
}

/* Transport only (eq. e:uprt with the flux of eq. e:glf), one step. */
int oracle_transport(const int *ints, const double *dbls, const double *groups,
                     const double *N, const double *F, double *Ns, double *Fs,
                     int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    Counters cnt;
    transport<double>(p, N, F, Ns, Fs, cnt);
    export_counters(cnt, counters);
    return 0;
}

/* Chemistry of one cell (Sec. 2.2.4 sequence), in place. */
int oracle_chem_cell(const int *ints, const double *dbls, const double *groups,
                     double *N, double *F, double *x, double *T, double n0,
                     const double *S, int64_t *counters) {
    Params p;
    if (!fill_params(p, ints, dbls, groups)) return -1;
    double Fc[4][3];
    for (int g = 0; g < p.G; ++g)
        for (int k = 0; k < 3; ++k) Fc[g][k] = F[g * 3 + k];
    int att = 0, cap = 0, xcl = 0;
    int ns = chem_cell<double>(p, N, Fc, *x, *T, n0, S, &att, &cap, &xcl);
    for (int g = 0; g < p.G; ++g)
        for (int k = 0; k < 3; ++k) F[g * 3 + k] = Fc[g][k];
    Counters cnt;
    cnt.substeps = ns; cnt.attempts = att; cnt.cap_hits = cap; cnt.x_clamp = xcl; cnt.max_sub = ns;
    export_counters(cnt, counters);
    return 0;
}

/* M1 pressure tensor P[k][d] (row-major 3x3) for one state. */
void oracle_pressure(double N, const double *F, double c, double *P) {
    double Pm[3][3];
    double Fl[3] = {F[0], F[1], F[2]};
    m1_pressure<double>(N, Fl, c, Pm);
    for (int k = 0; k < 3; ++k)
        for (int d = 0; d < 3; ++d) P[k * 3 + d] = Pm[k][d];
}

/* Signal speeds of R18 along axis d: out[0] = lambda-, out[1] = lambda+. */
void oracle_m1_speeds(double N, const double *F, int d, double c, double *out) {
    double Fl[3] = {F[0], F[1], F[2]};
    m1_speeds<double>(N, Fl, d, c, out[0], out[1]);
}

/* HLL face flux of R18 along axis d: out[0] for N, out[1..3] for F. */
void oracle_hll_flux(double NL, const double *FL, double NR, const double *FR, int d,
                     double c, double *out) {
    double fl[3] = {FL[0], FL[1], FL[2]}, fr[3] = {FR[0], FR[1], FR[2]};
    double fN, fF[3];
    hll_flux<double>(NL, fl, NR, fr, d, c, fN, fF);
    out[0] = fN; out[1] = fF[0]; out[2] = fF[1]; out[3] = fF[2];
}

/* Face flux of eq. (e:glf) along axis d: out[0] for N, out[1..3] for F. */
void oracle_face_flux(double NL, const double *FL, double NR, const double *FR, int d,
                      double c, double *out) {
    double fl[3] = {FL[0], FL[1], FL[2]}, fr[3] = {FR[0], FR[1], FR[2]};
    double fN, fF[3];
    glf_flux<double>(NL, fl, NR, fr, d, c, fN, fF);
    out[0] = fN; out[1] = fF[0]; out[2] = fF[1]; out[3] = fF[2];
}

/* Rate coefficients at temperature T: alpha_A, alpha_B, beta, and the cooling
 * rate Lambda(n0, x, T) for on-the-spot (otsa=1) or case A. */
void oracle_rates(double T, double n0, double x, int otsa, double *out) {
    Rates<double> r = rates_at<double>(T);
    out[0] = r.alphaA;
    out[1] = r.alphaB;
    out[2] = r.beta;
    out[3] = cooling<double>(r, n0, x, otsa);
}

/* The seven rate coefficients at temperature T, in the order alpha_A,
 * alpha_B, beta (cm^3 s^-1), recombination cooling case A and case B,
 * collisional excitation, bremsstrahlung (erg cm^3 s^-1): read-only access
 * for the pins of the individual fits. */
void oracle_rate_coeffs(double T, double *out) {
    Rates<double> r = rates_at<double>(T);
    out[0] = r.alphaA;
    out[1] = r.alphaB;
    out[2] = r.beta;
    out[3] = r.recA;
    out[4] = r.recB;
    out[5] = r.cexc;
    out[6] = r.brems;
}

double oracle_cross_section(double E_eV) { return cross_section(E_eV); }

void oracle_group_constants(double Tbb, const double *edges_eV, int G, int panels,
                            double *sigN, double *sigE, double *meanE_erg, double *frac) {
    group_constants(Tbb, edges_eV, G, panels, sigN, sigE, meanE_erg, frac);
}

} /* extern "C" */
