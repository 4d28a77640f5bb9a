// physics.hpp -- device-side physics of the EMMA radiation step for gfx950.
//
// M1 closure (Sec. 2.2.3), atomic rates and cooling (Sec. 2.2.4), the
// per-cell thermochemistry subcycle (Sec. 2.2.4, eqs. e:therm1g, e:therm2g,
// e:therm3, e:therm4 with the group sums e:g2, e:g3).
//
// Readings of the paper used by the library (it is silent or garbled there):
//  * Eddington tensor D = (1-chi)/2 I + (3 chi - 1)/2 n n^T (the printed form
//    swaps the two coefficients, which would give tr D = 4 chi - 1);
//    chi(f) = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)) (Levermore), f = 0 when
//    N <= 0, f = min(1, |F| / (c N)) otherwise, n = 0 when F = 0.
//  * c is the reduced speed of light everywhere it appears.
//  * The chemistry N and F updates divide by 1 + dtau c sigma_N (1-x) n0
//    (the printed denominators miss dtau); sources enter only there.
//  * dtau0 = min(dt_rem, |e / (H - Lambda)|) from the start-of-substep state
//    (dt_rem when H = Lambda); a rejected attempt (|de| > 0.1 e) is redone from
//    the same start state with dtau / 2 and the same rate coefficients; at most
//    kMaxHalvings halvings, then the attempt is kept and the cell flagged.
//    After max_substeps accepted substeps one last substep of dt_rem is taken
//    unconditionally (flagged too).  A cell whose energy is not a positive
//    finite number is left as it stands.
//  * e = 3/2 (1 + x) n0 k_B T (gamma = 5/3; neutral + ion + electron).
//  * x is clamped to [0, 1] after its update.
//  * Rates: Hui & Gnedin (1997) fits (alpha_A, alpha_B, collisional
//    ionisation, recombination cooling), Cen (1992) collisional excitation,
//    bremsstrahlung with Gaunt factor 1.3; no Compton term.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace emma {

constexpr double kC = 2.99792458e10;        // cm/s
constexpr double kKB = 1.380649e-16;        // erg/K
constexpr double kEV = 1.602176634e-12;     // erg
constexpr double kE13 = 13.6 * kEV;         // hydrogen ionisation energy, erg
constexpr double kTHI = 157807.0;           // K
constexpr int kMaxHalvings = 64;

// ------------------------------------------------------------------ closure
// Pressure tensor P = N D (symmetric; xx, xy, xz, yy, yz, zz) of one state.
template <typename R> struct FastMath;
template <> struct FastMath<float> {
    __device__ static inline float sqrt(float a) { return __builtin_amdgcn_sqrtf(a); }
    __device__ static inline float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
    __device__ static inline float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};
template <> struct FastMath<double> {
    __device__ static inline double sqrt(double a) { return ::sqrt(a); }
    __device__ static inline double rcp(double a) { return 1.0 / a; }
    __device__ static inline double div(double a, double b) { return a / b; }
};

template <typename R>
__device__ inline void m1_pressure(R N, R Fx, R Fy, R Fz, R c, R P[6]) {
    using M = FastMath<R>;
    const R F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const R Fn = F2 > R(0) ? M::sqrt(F2) : R(0);
    R f = R(0);
    if (N > R(0)) {
        f = M::div(Fn, c * N);
        f = f < R(1) ? f : R(1);
    }
    const R f2 = f * f;
    const R chi = M::div(R(3) + R(4) * f2, R(5) + R(2) * M::sqrt(R(4) - R(3) * f2));
    const R a = R(0.5) * (R(1) - chi) * N;        // isotropic part
    const R b = R(0.5) * (R(3) * chi - R(1)) * N; // along n
    R nx = R(0), ny = R(0), nz = R(0);
    if (Fn > R(0)) {
        nx = M::div(Fx, Fn);
        ny = M::div(Fy, Fn);
        nz = M::div(Fz, Fn);
    }
    P[0] = a + b * nx * nx;
    P[1] = b * nx * ny;
    P[2] = b * nx * nz;
    P[3] = a + b * ny * ny;
    P[4] = b * ny * nz;
    P[5] = a + b * nz * nz;
}

// ------------------------------------------------------------------- rates
struct RateSet {
    double alpha;   // recombination coefficient used for x (B on the spot, else A)
    double dalpha;  // alpha_A - alpha_B (recombination photons, case A only)
    double beta;    // collisional ionisation, cm^3/s
    double crec;    // recombination cooling coefficient, erg cm^3/s
    double cci;     // k_B T_HI beta
    double cce;     // collisional excitation, erg cm^3/s
    double cff;     // bremsstrahlung, erg cm^3/s
};

__device__ inline RateSet rates_at(double T, bool otsa) {
    RateSet r;
    const double lam = 2.0 * kTHI / T;
    const double aB = 2.753e-14 * pow(lam, 1.500) / pow(1.0 + pow(lam / 2.740, 0.407), 2.242);
    double aA = 0.0;
    if (!otsa) aA = 1.269e-13 * pow(lam, 1.503) / pow(1.0 + pow(lam / 0.522, 0.470), 1.923);
    r.alpha = otsa ? aB : aA;
    r.dalpha = otsa ? 0.0 : aA - aB;
    r.beta = 21.11 * pow(T, -1.5) * exp(-lam / 2.0) * pow(lam, -1.089) /
             pow(1.0 + pow(lam / 0.354, 0.874), 1.101);
    r.crec = otsa ? 3.435e-30 * T * pow(lam, 1.970) / pow(1.0 + pow(lam / 2.250, 0.376), 3.720)
                  : 1.778e-29 * T * pow(lam, 1.965) / pow(1.0 + pow(lam / 0.541, 0.502), 2.697);
    r.cci = kKB * kTHI * r.beta;
    r.cce = 7.5e-19 * exp(-118348.0 / T) / (1.0 + sqrt(T / 1e5));
    r.cff = 1.42e-27 * 1.3 * sqrt(T);
    return r;
}

// Cooling rate Lambda(n0, x, T) (erg cm^-3 s^-1) with n_e = n_p = x n0 and
// n_HI = (1 - x) n0.
__device__ inline double cooling(const RateSet &r, double n0, double x) {
    const double ne = x * n0;
    const double nHI = (1.0 - x) * n0;
    return (r.crec + r.cff) * ne * ne + (r.cci + r.cce) * ne * nHI;
}

// --------------------------------------------------------------- chemistry
struct GroupConsts {
    double sigN[4];    // number-weighted cross-section, cm^2
    double SigE[4];    // sigma_E <E> - sigma_N E_13.6, erg cm^2 (heating)
    double frac[4];    // source photon fraction
};

struct ChemParams {
    double c;          // reduced speed of light
    double dt;
    int otsa, isothermal, max_substeps;
};

struct ChemStats {
    int substeps, attempts, cap, xclamp;
};

// The sub-cycled update of one cell over dt.  N[g], F[g][3] hold the
// post-transport values on entry and the end values on exit.
template <int G>
__device__ inline ChemStats chem_cell(const GroupConsts &gc, const ChemParams &p, double (&N)[G],
                                      double (&F)[G][3], double &x, double &T, double n0,
                                      const double (&S)[G]) {
    ChemStats st{0, 0, 0, 0};
    const double c = p.c;
    const double eunit = 1.5 * n0 * kKB;  // e = eunit (1 + x) T
    double e = eunit * (1.0 + x) * T;
    double rem = p.dt;
    while (rem > 0.0) {
        if (!p.isothermal && !(e > 0.0 && e < HUGE_VAL)) break;  // invalid input: leave the cell
        const bool last = st.substeps >= p.max_substeps;
        const double Tp = p.isothermal ? T : e / (eunit * (1.0 + x));
        const RateSet r = rates_at(Tp, p.otsa);
        double dtau = rem;
        if (!p.isothermal && !last) {
            double h = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) h += gc.SigE[g] * N[g];
            const double H = c * (1.0 - x) * n0 * h;
            const double L = cooling(r, n0, x);
            if (H != L) dtau = fmin(rem, fabs(e / (H - L)));
        }
        double Nn[G], inv[G], xn, en;
        int halvings = 0;
        for (;;) {
            st.attempts++;
            const double y0 = 1.0 - x;
            double gam = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double kap = c * gc.sigN[g] * y0 * n0;
                const double rec = (g == 0) ? r.dalpha * x * x * n0 * n0 : 0.0;
                const double den = 1.0 + dtau * kap;
                Nn[g] = (N[g] + (S[g] + rec) * dtau) / den;
                inv[g] = den;
                gam += c * gc.sigN[g] * Nn[g];
            }
            xn = 1.0 - (r.alpha * x * x * n0 * dtau + y0) / (1.0 + dtau * (r.beta * x * n0 + gam));
            if (xn < 0.0) { xn = 0.0; st.xclamp++; }
            if (xn > 1.0) { xn = 1.0; st.xclamp++; }
            if (p.isothermal) { en = e; break; }
            double h = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) h += gc.SigE[g] * Nn[g];
            en = e + dtau * c * (1.0 - xn) * n0 * h - dtau * cooling(r, n0, xn);
            if (last) break;
            if (fabs(en - e) <= 0.1 * e) break;
            if (halvings == kMaxHalvings) { st.cap = 1; break; }
            dtau = dtau * 0.5;
            halvings++;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            N[g] = Nn[g];
#pragma unroll
            for (int k = 0; k < 3; ++k) F[g][k] = F[g][k] / inv[g];
        }
        x = xn;
        e = en;
        rem = rem - dtau;
        st.substeps++;
        if (last) { st.cap = 1; break; }
        if (p.isothermal) break;
    }
    if (!p.isothermal) T = e / (eunit * (1.0 + x));
    return st;
}

}  // namespace emma
