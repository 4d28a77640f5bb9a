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

#include "fastmath.hpp"

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

// Eddington tensor closure (R2-R4 of the readings): P = D N with
// D = (1 - chi)/2 I + (3 chi - 1)/2 n n^T, f = |F|/(c N) clipped at 1.
// With s = sqrt(4 - 3 f^2), Levermore's chi = (3 + 4 f^2)/(5 + 2 s) equals
// (5 - 2 s)/3 exactly (multiply out (5 - 2s)(5 + 2s) = 9 + 12 f^2), so
//   (1 - chi)/2 = (s - 1)/3 = (1 - f^2)/(1 + s),
//   (3 chi - 1)/2 = 2 - s = 3 f^2/(2 + s),
// and with the reduced flux g = F/(c N) (|g| = f, an O(1) vector), q = |g|^2:
//   P = N [(1 - q)/(1 + s) I + 3/(2 + s) g g^T],
// both fractions from one reciprocal of (1 + s)(2 + s).  No square of a tiny
// |F| appears: for the faint fields ahead of a front |F|^2 underflows long
// before g does.  At the clip (q >= 1) chi = 1 and P = N g g^T / q: with q
// clamped to 1 inside s and (1 - q), and max(q, 1) folded into the
// reciprocal, the same expressions give exactly that (s = 1).  N <= 0: g = 0
// and D = I/3.  P comes out multiplied by `scale` (the transport asks for
// c^2 P, the flux's form).
template <typename R>
__device__ __forceinline__ void m1_pressure(R N, R Fx, R Fy, R Fz, R c, R P[6], R scale = R(1)) {
    using M = FastMath<R>;
    const R icn = N > R(0) ? M::rcp(c * N) : R(0);
    const R gx = Fx * icn, gy = Fy * icn, gz = Fz * icn;
    const R q = gx * gx + gy * gy + gz * gz;
    const R qc = q < R(1) ? q : R(1);
    const R s = M::sqrt(R(4) - R(3) * qc);
    const R r = M::rcp((R(1) + s) * (R(2) + s) * (q > R(1) ? q : R(1)));
    const R sN = scale * N;
    const R a = sN * (R(1) - qc) * (R(2) + s) * r;
    const R k = R(3) * sN * (R(1) + s) * r;
    const R kx = k * gx, ky = k * gy, kz = k * gz;
    P[0] = a + kx * gx;
    P[1] = kx * gy;
    P[2] = kx * gz;
    P[3] = a + ky * gy;
    P[4] = ky * gz;
    P[5] = a + kz * gz;
}

// The floor N* >= 0 and the limiter |F*| <= c N* after the transport update
// (reading R13), in the transport's own precision R.  Every forward kernel
// and the adjoint's replay of the forward call this one function, so the
// adjoint reverses the branch the forward took (bit 0: floored, bit 1:
// limited) and continues from the forward's own post-limiter values.
template <typename R>
__device__ __forceinline__ int floor_limit_fwd(R &n, R &fx, R &fy, R &fz, R c) {
#pragma clang fp contract(off)
    int taken = 0;
    if (n < R(0)) {
        n = R(0);
        taken = 1;
    }
    const R F2 = fx * fx + fy * fy + fz * fz;
    const R cn = c * n;
    if (F2 > cn * cn) {
        // scale F to |F| = c N.  The hardware single-precision square root
        // and reciprocal flush operands below the normal range to zero, so a
        // faint |F|^2 (possible ahead of a front, and with N floored to 0) is
        // first brought up by 2^100, exactly
        R sx = fx, sy = fy, sz = fz, sF2 = F2, scn = cn;
        if (sizeof(R) == 4 && F2 < R(0x1p-100)) {
            const R up = R(0x1p100);
            sx *= up;
            sy *= up;
            sz *= up;
            scn *= up;
            sF2 = sx * sx + sy * sy + sz * sz;
        }
        const R sc = scn * FastMath<R>::rcp(FastMath<R>::sqrt(sF2));
        fx *= sc;
        fy *= sc;
        fz *= sc;
        taken |= 2;
    }
    return taken;
}

// Signal speeds along one axis for the HLL flux: the eigenvalues of the
// one-dimensional M1 system (N, F_d) -> (F_d, c^2 chi(f) N) at the normal
// reduced flux f = F_d/(c N) in [-1, 1] (0 when N <= 0),
//   lambda = c (chi' -+ sqrt(chi'^2 + 4 (chi - f chi')))/2.
// With s = sqrt(4 - 3 f^2), chi' - 2f = 2f (1 - s)/s and chi - f^2 =
// (1 - s)^2/3, so the radicand is 16 (s - 1)^2/(3 s^2) and
//   lambda = c (f -+ 2 (s - 1)/sqrt(3))/s,  s - 1 = 3 (1 - f)(1 + f)/(1 + s):
// no cancellation near |f| = 1 (the radicand above is a difference of O(1)
// terms that vanishes there), so single precision is enough.
template <typename R>
__device__ __forceinline__ void m1_speeds(R N, R Fd, R c, R &lmin, R &lmax) {
    using M = FastMath<R>;
    R f = R(0);
    if (N > R(0)) {
        f = M::div(Fd, c * N);
        f = f < R(-1) ? R(-1) : (f > R(1) ? R(1) : f);
    }
    const R s = M::sqrt(R(4) - R(3) * f * f);
    const R is = M::rcp(s);
    const R w = R(3.4641016151377544) * (R(1) - f) * (R(1) + f) * M::rcp(R(1) + s);  // 2 (s - 1)/sqrt(3)
    lmin = c * (f - w) * is;
    lmax = c * (f + w) * is;
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

// All rate fits share the form A T^t lam^a / (1 + (lam/b)^c)^d with
// lam = 2 T_HI / T.  They are evaluated in the log domain from one
// L = ln(lam): A T^t exp(a L - d ln(1 + exp(c (L - ln b)))), i.e. two exp and
// one log per fit instead of four pow (same value to a few ulp; ln(1 + u)
// only needs a small ABSOLUTE error here since it is scaled by d inside exp).
// The FMA is explicit so that every caller (the per-cell rates, the
// cooperative rates of the long-subcycle pass, the adjoint) gets the same bits.
__host__ __device__ __forceinline__ double hg_fit(double L, double a, double lnb, double c, double d) {
    const double u = exp_fp64(c * (L - lnb));
    return fma(a, L, -(d * log_fp64(1.0 + u)));
}

// exp(-lam/2) T^-1.5 part of the collisional-ionisation fit's exponent
__host__ __device__ __forceinline__ double beta_pre(double lnT, double lam) { return fma(-0.5, lam, -1.5 * lnT); }

template <bool OTSA>
__host__ __device__ __forceinline__ RateSet rates_at(double T) {
    RateSet r;
    const double invT = recip_fp64(T);
    const double lam = 2.0 * kTHI * invT;
    const double L = log_fp64(lam);
    const double lnT = 12.662275226919286 - L;  // ln(2 T_HI) - L
    if (OTSA) {
        r.alpha = 2.753e-14 * exp_fp64(hg_fit(L, 1.500, 1.007957920399979, 0.407, 2.242));  // ln 2.740
        r.dalpha = 0.0;
        r.crec = 3.435e-30 * T * exp_fp64(hg_fit(L, 1.970, 0.8109302162163288, 0.376, 3.720));  // ln 2.250
    } else {
        const double aA = 1.269e-13 * exp_fp64(hg_fit(L, 1.503, -0.6500876910994983, 0.470, 1.923));  // ln 0.522
        const double aB = 2.753e-14 * exp_fp64(hg_fit(L, 1.500, 1.007957920399979, 0.407, 2.242));
        r.alpha = aA;
        r.dalpha = aA - aB;
        r.crec = 1.778e-29 * T * exp_fp64(hg_fit(L, 1.965, -0.6143360001356555, 0.502, 2.697));  // ln 0.541
    }
    // 21.11 T^-1.5 exp(-lam/2) lam^-1.089 / (1 + (lam/0.354)^0.874)^1.101
    r.beta = 21.11 * exp_fp64(beta_pre(lnT, lam) + hg_fit(L, -1.089, -1.0384583658483626, 0.874, 1.101));  // ln 0.354
    r.cci = kKB * kTHI * r.beta;
    const double sT = sqrt(T);
    // 118348 K: collisional excitation temperature; sqrt(T / 1e5) = sT / 316.2...
    r.cce = 7.5e-19 * exp_fp64(-118348.0 * invT) * recip_fp64(1.0 + sT * 0.003162277660168379);
    r.cff = 1.42e-27 * 1.3 * sT;
    return r;
}

__host__ __device__ __forceinline__ RateSet rates_at(double T, bool otsa) {
    return otsa ? rates_at<true>(T) : rates_at<false>(T);
}

// rates_at together with the temperature derivative of every coefficient
// (the adjoint needs both at the same temperature; dL/dT = -1/T): ln(lambda)
// and the inner u = exp(c (L - ln b)) of each fit serve both the value
// (same operations as rates_at, so the same bits) and the slope of its
// exponent, d/dL [a L - d ln(1 + u)] = a - d c u / (1 + u).
template <bool OTSA>
__host__ __device__ inline void rates_and_dT(double T, RateSet &r, RateSet &d) {
    const double invT = recip_fp64(T);
    const double lam = 2.0 * kTHI * invT;
    const double L = log_fp64(lam);
    const double lnT = 12.662275226919286 - L;  // ln(2 T_HI) - L
    // value exponent a L - d ln(1 + u) and slope a - d c u / (1 + u), u = exp(c (L - ln b))
    auto fit = [L](double a, double lnb, double c, double dd, double &slope) {
        const double u = exp_fp64(c * (L - lnb));
        slope = a - dd * c * u / (1.0 + u);
        return fma(a, L, -(dd * log_fp64(1.0 + u)));
    };
    double sa, sc, sb;
    if (OTSA) {
        r.alpha = 2.753e-14 * exp_fp64(fit(1.500, 1.007957920399979, 0.407, 2.242, sa));
        r.dalpha = 0.0;
        r.crec = 3.435e-30 * T * exp_fp64(fit(1.970, 0.8109302162163288, 0.376, 3.720, sc));
        d.alpha = -r.alpha * sa * invT;
        d.dalpha = 0.0;
        d.crec = r.crec * (1.0 - sc) * invT;
    } else {
        double sbB;
        const double aA = 1.269e-13 * exp_fp64(fit(1.503, -0.6500876910994983, 0.470, 1.923, sa));
        const double aB = 2.753e-14 * exp_fp64(fit(1.500, 1.007957920399979, 0.407, 2.242, sbB));
        r.alpha = aA;
        r.dalpha = aA - aB;
        r.crec = 1.778e-29 * T * exp_fp64(fit(1.965, -0.6143360001356555, 0.502, 2.697, sc));
        const double daA = -aA * sa * invT;
        const double daB = -(r.alpha - r.dalpha) * sbB * invT;
        d.alpha = daA;
        d.dalpha = daA - daB;
        d.crec = r.crec * (1.0 - sc) * invT;
    }
    r.beta = 21.11 * exp_fp64(beta_pre(lnT, lam) + fit(-1.089, -1.0384583658483626, 0.874, 1.101, sb));
    r.cci = kKB * kTHI * r.beta;
    const double sT = sqrt(T);
    r.cce = 7.5e-19 * exp_fp64(-118348.0 * invT) * recip_fp64(1.0 + sT * 0.003162277660168379);
    r.cff = 1.42e-27 * 1.3 * sT;
    d.beta = r.beta * (-1.5 + 0.5 * lam - sb) * invT;
    d.cci = kKB * kTHI * d.beta;
    const double k = 0.003162277660168379;
    d.cce = r.cce * (118348.0 * invT * invT - 0.5 * k / sT / (1.0 + k * sT));
    d.cff = 0.5 * r.cff * invT;
}

// Cooling rate Lambda(n0, x, T) (erg cm^-3 s^-1) with n_e = n_p = x n0 and
// n_HI = (1 - x) n0.
__host__ __device__ __forceinline__ double cooling(const RateSet &r, double n0, double x) {
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

// Decisions taken by one accepted substep (what the adjoint replays).
struct SubInfo {
    double Tp;     // temperature the rates were evaluated at
    double D;      // H - Lambda at the start of the substep
    int branch;    // 0: dtau0 = dt_rem, 1: dtau0 = |e / D|
    int h;         // number of halvings of dtau0
    int xclamp;    // 0: none, -1: x' clamped to 0, +1: x' clamped to 1
};

// One attempt of a substep with step dtau from the start state (N, x, e):
// N' (eq. e:therm1g), the factor inv[g] applied to F_g (eq. e:therm2g), x'
// clamped to [0, 1] (eq. e:therm3; xcl the side it was clamped to) and e'
// (eq. e:therm4; e itself in the isothermal mode).  This and first_dtau are
// the steps of substep() below written out for the cooperative pass, in the
// same operations; substep() keeps them inline (as calls they cost the
// per-cell chemistry kernel 20 more registers and a wave per SIMD).
template <int G>
__host__ __device__ __forceinline__ void attempt(const GroupConsts &gc, double c, bool iso, double n0,
                                                 const RateSet &r, const double (&S)[G], const double (&N)[G],
                                                 double x, double e, double dtau, double (&Nn)[G],
                                                 double (&inv)[G], double &xn, double &en, int &xcl) {
    const double y0 = 1.0 - x;
    double gam = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double kap = c * gc.sigN[g] * y0 * n0;
        const double rec = (g == 0) ? r.dalpha * x * x * n0 * n0 : 0.0;
        inv[g] = recip_fp64(1.0 + dtau * kap);
        Nn[g] = (N[g] + (S[g] + rec) * dtau) * inv[g];
        gam += c * gc.sigN[g] * Nn[g];
    }
    xn = 1.0 - (r.alpha * x * x * n0 * dtau + y0) * recip_fp64(1.0 + dtau * (r.beta * x * n0 + gam));
    xcl = 0;
    if (xn < 0.0) { xn = 0.0; xcl = -1; }
    if (xn > 1.0) { xn = 1.0; xcl = 1; }
    if (iso) { en = e; return; }
    double h = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) h += gc.SigE[g] * Nn[g];
    en = e + dtau * c * (1.0 - xn) * n0 * h - dtau * cooling(r, n0, xn);
}

// The first attempt's step of a substep: dt_rem, or |e / (H - Lambda)| when
// that is shorter (never on the guarded last substep).  D = H - Lambda.
template <int G>
__host__ __device__ __forceinline__ double first_dtau(const GroupConsts &gc, double c, bool iso, bool last,
                                                      double n0, const RateSet &r, const double (&N)[G], double x,
                                                      double e, double rem, double &D, int &branch) {
    double dtau = rem;
    D = 0.0;
    branch = 0;
    if (!iso && !last) {
        double h = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) h += gc.SigE[g] * N[g];
        const double H = c * (1.0 - x) * n0 * h;
        const double L = cooling(r, n0, x);
        D = H - L;
        if (H != L) {
            const double q = fabs(e * recip_fp64(D));
            if (q < rem) { dtau = q; branch = 1; }
        }
    }
    return dtau;
}

// One substep of the Sec. 2.2.4 sequence from the start state (N, x, e, rem):
// dtau0 = min(rem, |e / (H - Lambda)|) (rem on the last, guarded substep),
// halved until |e' - e| <= 0.1 e; returns false (state untouched) for an
// invalid energy.  On return (N, x, e, rem) is the new state and inv[g] the
// factor applied to F_g.  FAST = true compiles the default mode (on-the-spot,
// energy evolved) with those flags as constants; FAST = false reads them from p.
template <int G, bool FAST>
__host__ __device__ __forceinline__ bool substep(const GroupConsts &gc, const ChemParams &p, bool last, double n0,
                                        double eunit, double Tfix, const double (&S)[G], double (&N)[G],
                                        double &x, double &e, double &rem, double (&inv)[G], ChemStats &st,
                                        SubInfo *info) {
    const double c = p.c;
    const bool otsa = FAST ? true : (p.otsa != 0);
    const bool iso = FAST ? false : (p.isothermal != 0);
    if (!iso && !(e > 0.0 && e < HUGE_VAL)) return false;  // invalid input: leave the cell
    const double Tp = iso ? Tfix : e * recip_fp64(eunit * (1.0 + x));
    const RateSet r = FAST ? rates_at<true>(Tp) : rates_at(Tp, otsa);
    double dtau = rem, D = 0.0;
    int branch = 0;
    if (!iso && !last) {
        double h = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) h += gc.SigE[g] * N[g];
        const double H = c * (1.0 - x) * n0 * h;
        const double L = cooling(r, n0, x);
        D = H - L;
        if (H != L) {
            const double q = fabs(e * recip_fp64(D));
            if (q < rem) { dtau = q; branch = 1; }
        }
    }
    double Nn[G], xn, en;
    int halvings = 0, xcl = 0;
    for (;;) {
        st.attempts++;
        const double y0 = 1.0 - x;
        double gam = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double kap = c * gc.sigN[g] * y0 * n0;
            const double rec = (g == 0) ? r.dalpha * x * x * n0 * n0 : 0.0;
            inv[g] = recip_fp64(1.0 + dtau * kap);
            Nn[g] = (N[g] + (S[g] + rec) * dtau) * inv[g];
            gam += c * gc.sigN[g] * Nn[g];
        }
        xn = 1.0 - (r.alpha * x * x * n0 * dtau + y0) * recip_fp64(1.0 + dtau * (r.beta * x * n0 + gam));
        xcl = 0;
        if (xn < 0.0) { xn = 0.0; xcl = -1; }
        if (xn > 1.0) { xn = 1.0; xcl = 1; }
        if (iso) { en = e; break; }
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
    if (xcl) st.xclamp++;
#pragma unroll
    for (int g = 0; g < G; ++g) N[g] = Nn[g];
    if (info) {
        info->Tp = Tp;
        info->D = D;
        info->branch = branch;
        info->h = halvings;
        info->xclamp = xcl;
    }
    x = xn;
    e = en;
    rem = rem - dtau;
    st.substeps++;
    return true;
}

// A cell's subcycle between two substeps: everything the remaining substeps
// need, so that a later pass can continue it exactly where it stopped (the
// same arithmetic as an uninterrupted subcycle).  F enters only through Pf,
// the product of the substeps' factors applied to it so far.
template <int G> struct SubState {
    double N[G], Pf[G];
    double x, e, rem;
    ChemStats st;
};

// Start of a cell's subcycle over dt (e = 3/2 (1 + x) n0 k_B T).
template <int G>
__host__ __device__ __forceinline__ void sub_start(SubState<G> &s, const ChemParams &p, const double (&N)[G],
                                                   double x, double T, double n0) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        s.N[g] = N[g];
        s.Pf[g] = 1.0;
    }
    s.x = x;
    s.e = 1.5 * n0 * kKB * (1.0 + x) * T;
    s.rem = p.dt;
    s.st = ChemStats{0, 0, 0, 0};
}

// Substeps until dt is covered (true), or until `budget` substeps have been
// accepted with dt not covered yet (false: s holds the state to continue
// from).  Tfix: the cell's temperature, used only in isothermal mode.
template <int G, bool FAST>
__host__ __device__ __forceinline__ bool sub_run(SubState<G> &s, const GroupConsts &gc, const ChemParams &p,
                                                 double n0, double Tfix, const double (&S)[G], int budget) {
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double eunit = 1.5 * n0 * kKB;
    while (s.rem > 0.0) {
        if (s.st.substeps >= budget) return false;
        const bool last = s.st.substeps >= p.max_substeps;
        double inv[G];
        if (!substep<G, FAST>(gc, p, last, n0, eunit, Tfix, S, s.N, s.x, s.e, s.rem, inv, s.st, nullptr)) break;
#pragma unroll
        for (int g = 0; g < G; ++g) s.Pf[g] *= inv[g];
        if (last) { s.st.cap = 1; break; }
        if (iso) break;
    }
    return true;
}

// End-of-step temperature of a finished subcycle.
template <int G, bool FAST>
__host__ __device__ __forceinline__ double sub_T(const SubState<G> &s, const ChemParams &p, double n0, double Tfix) {
    const bool iso = FAST ? false : (p.isothermal != 0);
    return iso ? Tfix : s.e / (1.5 * n0 * kKB * (1.0 + s.x));
}

// The subcycle without F: F only ever gets multiplied by the substeps'
// factors, so the caller applies their product Pf[g] to F afterwards
// (F_out = F_in Pf).  Same budget semantics as chem_cell.
template <int G, bool FAST = false>
__host__ __device__ __forceinline__ ChemStats chem_cell_nxt(const GroupConsts &gc, const ChemParams &p,
                                                            double (&N)[G], double (&Pf)[G], double &x,
                                                            double &T, double n0, const double (&S)[G],
                                                            int budget = 0x7fffffff, bool *deferred = nullptr) {
    ChemStats st{0, 0, 0, 0};
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double eunit = 1.5 * n0 * kKB;  // e = eunit (1 + x) T
    double e = eunit * (1.0 + x) * T;
    double rem = p.dt;
#pragma unroll
    for (int g = 0; g < G; ++g) Pf[g] = 1.0;
    while (rem > 0.0) {
        if (st.substeps >= budget) {
            *deferred = true;
            return st;
        }
        const bool last = st.substeps >= p.max_substeps;
        double inv[G];
        if (!substep<G, FAST>(gc, p, last, n0, eunit, T, S, N, x, e, rem, inv, st, nullptr)) break;
#pragma unroll
        for (int g = 0; g < G; ++g) Pf[g] *= inv[g];
        if (last) { st.cap = 1; break; }
        if (iso) break;
    }
    if (!iso) T = e / (eunit * (1.0 + x));
    return st;
}

// The sub-cycled update of one cell over dt.  N[g], F[g][3] hold the
// post-transport values on entry and the end values on exit.  With a finite
// budget the cell gives up after that many accepted substeps if dt is not
// covered yet (*deferred = true; the outputs are then meaningless and the
// caller recomputes the cell later from its inputs).
template <int G, bool FAST = false>
__host__ __device__ __forceinline__ ChemStats chem_cell(const GroupConsts &gc, const ChemParams &p, double (&N)[G],
                                      double (&F)[G][3], double &x, double &T, double n0,
                                      const double (&S)[G], int budget = 0x7fffffff,
                                      bool *deferred = nullptr) {
    ChemStats st{0, 0, 0, 0};
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double eunit = 1.5 * n0 * kKB;  // e = eunit (1 + x) T
    double e = eunit * (1.0 + x) * T;
    double rem = p.dt;
    // F only ever gets multiplied by the substeps' factors: keep their product
    double Pf[G];
#pragma unroll
    for (int g = 0; g < G; ++g) Pf[g] = 1.0;
    while (rem > 0.0) {
        if (st.substeps >= budget) {
            *deferred = true;
            return st;
        }
        const bool last = st.substeps >= p.max_substeps;
        double inv[G];
        if (!substep<G, FAST>(gc, p, last, n0, eunit, T, S, N, x, e, rem, inv, st, nullptr)) break;
#pragma unroll
        for (int g = 0; g < G; ++g) Pf[g] *= inv[g];
        if (last) { st.cap = 1; break; }
        if (iso) break;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
#pragma unroll
        for (int k = 0; k < 3; ++k) F[g][k] = F[g][k] * Pf[g];
    }
    if (!iso) T = e / (eunit * (1.0 + x));
    return st;
}

}  // namespace emma
