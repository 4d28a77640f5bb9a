// adjoint.hpp -- reverse-mode derivative of the radiation step.
//
// The step is U -> transport (eq. e:uprt with the flux of eq. e:glf, then the
// floor N >= 0 and the limiter |F| <= c N) -> per-cell chemistry subcycle
// (Sec. 2.2.4).  Its exact derivative along the branches the forward run takes
// (dtau0 = rem or |e/(H - Lambda)|, the number of 10 % halvings, clamps) is
// applied in reverse:
//   k_chem_adj       per cell: replays the cell's substeps with the forward's
//                    own substep() (identical decisions), then runs them
//                    backwards; also reverses the floor and limiter.  Adds
//                    dL/dn0 and dL/dS (per source cell).
//   k_transport_adj  gather form (no atomics), z-marching columns: the
//                    transpose of the radius-1 stencil with the closure
//                    Jacobian dP/d(N, F).
//   k_transport_adj_hll  the same for the HLL flux with M1 wave speeds:
//                    transposed face Jacobians, speed derivatives included.
//   k_src_grad       dL/d(source rate) = sum_g frac_g / dx^3 dL/dS_g(host cell).
#pragma once

#include "kernels.hpp"
#include "../../include/emma_rt.h"

namespace emma {

struct AdjointScratch {
    void *tape;      // [K - 1][state]: N, F (storage type), x, T (double) at steps 1..K-1 of a
                     // segment (step 0 is the caller's start state)
    void *ustar;     // [K][4 G V] storage type: each step's transport output before the floor
                     // and the limiter; null when it did not fit (then recomputed)
    void *gU;        // [4 G][V] storage type: dL/d(pre-limiter transport output)
    double *gS;      // [EMMA_RT_MAX_SOURCES][G]: dL/dS per sorted source position
    int64_t tape_bytes_per_step;
    uint64_t *multi;       // [K][multi_words]: one bit per cell, set where the segment's
                           // forward subcycle of that step was not a single substep
    int64_t multi_words;
    uint32_t *list;        // [V]: the marked cells of one step, compacted
    uint32_t *list_count;  // [16]
    hipStream_t side;      // runs the kept-state pass beside the single-substep pass
    hipEvent_t ev_in, ev_out;
};

inline int64_t adjoint_state_bytes(const emma_rt_config &cfg) {
    const int64_t V = (int64_t)cfg.nx * cfg.ny * cfg.nz;
    const int64_t e = cfg.precision == EMMA_RT_FP64 ? 8 : 4;
    return V * (4 * cfg.n_groups * e + 16);
}

// Tape slots: the states after steps 1..K-1 of a segment (at least one slot).
inline int64_t adjoint_tape_slots(const emma_rt_config &cfg) {
    return cfg.adjoint_max_steps > 1 ? cfg.adjoint_max_steps - 1 : 1;
}

// 64-bit words of one step's bitmask: whole chemistry blocks of up to 256 cells.
inline int64_t adjoint_multi_words(int64_t V) { return (V + 255) / 256 * 4; }

// Transport tape: K steps of N*, F* in the storage precision.
inline int64_t adjoint_ustar_bytes(const emma_rt_config &cfg) {
    const int64_t V = (int64_t)cfg.nx * cfg.ny * cfg.nz;
    return (int64_t)cfg.adjoint_max_steps * 4 * cfg.n_groups * V * (cfg.precision == EMMA_RT_FP64 ? 8 : 4);
}

// Everything the adjoint allocates, the transport tape included.
inline int64_t adjoint_scratch_bytes(const emma_rt_config &cfg) {
    if (cfg.adjoint_max_steps < 1) return 0;
    const int64_t V = (int64_t)cfg.nx * cfg.ny * cfg.nz;
    const int64_t elem = cfg.precision == EMMA_RT_FP64 ? 8 : 4;
    return adjoint_tape_slots(cfg) * adjoint_state_bytes(cfg) + 4 * cfg.n_groups * V * elem +
           (int64_t)EMMA_RT_MAX_SOURCES * cfg.n_groups * 8 +
           (int64_t)cfg.adjoint_max_steps * adjoint_multi_words(V) * 8 + V * 4 + 64 + adjoint_ustar_bytes(cfg);
}

inline int adjoint_alloc(AdjointScratch &a, const emma_rt_config &cfg) {
    a = AdjointScratch{};
    a.tape_bytes_per_step = adjoint_state_bytes(cfg);
    if (cfg.adjoint_max_steps < 1) return 0;
    const int64_t V = (int64_t)cfg.nx * cfg.ny * cfg.nz;
    const int64_t elem = cfg.precision == EMMA_RT_FP64 ? 8 : 4;
    a.multi_words = adjoint_multi_words(V);
    if (hipMalloc(&a.tape, (size_t)(adjoint_tape_slots(cfg) * a.tape_bytes_per_step)) != hipSuccess) return -1;
    if (hipMalloc(&a.gU, (size_t)(4 * cfg.n_groups * V * elem)) != hipSuccess) return -1;
    if (hipMalloc((void **)&a.gS, (size_t)EMMA_RT_MAX_SOURCES * cfg.n_groups * 8) != hipSuccess) return -1;
    if (hipMalloc((void **)&a.multi, (size_t)(cfg.adjoint_max_steps * a.multi_words * 8)) != hipSuccess) return -1;
    if (hipMalloc((void **)&a.list, (size_t)V * 4) != hipSuccess) return -1;
    if (hipMalloc((void **)&a.list_count, 64) != hipSuccess) return -1;
    if (hipStreamCreateWithFlags(&a.side, hipStreamNonBlocking) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&a.ev_in, hipEventDisableTiming) != hipSuccess) return -1;
    if (hipEventCreateWithFlags(&a.ev_out, hipEventDisableTiming) != hipSuccess) return -1;
    // last, and optional: only while the device keeps the room of four more
    // states free beside it (for the caller's state and gradient arrays);
    // without it the reverse sweep recomputes each step's transport (same
    // bits, one more transport per step)
    size_t free_b = 0, total_b = 0;
    const int64_t need = adjoint_ustar_bytes(cfg) + 4 * adjoint_state_bytes(cfg);
    if (hipMemGetInfo(&free_b, &total_b) == hipSuccess && (int64_t)free_b >= need &&
        hipMalloc(&a.ustar, (size_t)adjoint_ustar_bytes(cfg)) != hipSuccess) {
        a.ustar = nullptr;
        (void)hipGetLastError();
    }
    return 0;
}

inline void adjoint_release(AdjointScratch &a) {
    if (a.tape) (void)hipFree(a.tape);
    if (a.ustar) (void)hipFree(a.ustar);
    if (a.gU) (void)hipFree(a.gU);
    if (a.gS) (void)hipFree(a.gS);
    if (a.multi) (void)hipFree(a.multi);
    if (a.list) (void)hipFree(a.list);
    if (a.list_count) (void)hipFree(a.list_count);
    if (a.ev_in) (void)hipEventDestroy(a.ev_in);
    if (a.ev_out) (void)hipEventDestroy(a.ev_out);
    if (a.side) (void)hipStreamDestroy(a.side);
    a = AdjointScratch{};
}

// ------------------------------------------------------- chemistry adjoint
struct RateAdj {
    double alpha, dalpha, beta, crec, cci, cce, cff;
};

// Lambda(n0, x) = (crec + cff) ne^2 + (cci + cce) ne nh, ne = x n0, nh = (1-x) n0:
// adds lam * dLambda/d(.) to the rate adjoints, x and n0.
__host__ __device__ __forceinline__ void cooling_adj(const RateSet &r, double n0, double x, double lam, RateAdj &ar,
                                            double &ax, double &an0) {
    const double ne = x * n0, nh = (1.0 - x) * n0;
    ar.crec += lam * ne * ne;
    ar.cff += lam * ne * ne;
    ar.cci += lam * ne * nh;
    ar.cce += lam * ne * nh;
    const double ane = lam * (2.0 * (r.crec + r.cff) * ne + (r.cci + r.cce) * nh);
    const double anh = lam * (r.cci + r.cce) * ne;
    ax += (ane - anh) * n0;
    an0 += ane * x + anh * (1.0 - x);
}

// Reverse of one chemistry substep that started from (N, x, e, rem) and took
// the decisions in info.  On entry aN, ax, ae, arem hold dL/d(end state of the
// substep); on exit dL/d(start state).  aF[g] = dL/d(factor applied to F_g)
// from outside (the F path).  Adds to an0, aS and aT (the temperature input,
// isothermal mode only).
template <int G, bool FAST>
__host__ __device__ inline void substep_adj(const GroupConsts &gc, const ChemParams &p, double n0, double eunit,
                                   const double (&S)[G], const double (&N)[G], double x, double e,
                                   double rem, const SubInfo &info, const double (&aFinv)[G], double (&aN)[G],
                                   double &ax, double &ae, double &arem, double &an0, double (&aS)[G],
                                   double &aT) {
    const double c = p.c;
    const bool otsa = FAST ? true : (p.otsa != 0);
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double Tp = info.Tp;
    // the rates at Tp and their temperature derivatives, in one evaluation
    RateSet r, dr;
    if (FAST || otsa) rates_and_dT<true>(Tp, r, dr);
    else rates_and_dT<false>(Tp, r, dr);
    // dtau of the accepted attempt
    double dtau0 = rem;
    if (info.branch) dtau0 = fabs(e * recip_fp64(info.D));
    const double dtau = ldexp(dtau0, -info.h);
    // forward intermediates of the accepted attempt
    const double y0 = 1.0 - x;
    double kap[G], inv[G], Nn[G], rec[G], gam = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        kap[g] = c * gc.sigN[g] * y0 * n0;
        rec[g] = (g == 0) ? r.dalpha * x * x * n0 * n0 : 0.0;
        inv[g] = recip_fp64(1.0 + dtau * kap[g]);
        Nn[g] = (N[g] + (S[g] + rec[g]) * dtau) * inv[g];
        gam += c * gc.sigN[g] * Nn[g];
    }
    const double num = r.alpha * x * x * n0 * dtau + y0;
    const double denx = 1.0 + dtau * (r.beta * x * n0 + gam);
    const double rdx = recip_fp64(denx);
    const double xn = info.xclamp ? (info.xclamp > 0 ? 1.0 : 0.0) : 1.0 - num * rdx;

    RateAdj ar{0, 0, 0, 0, 0, 0, 0};
    double adt = 0.0, axs = 0.0, aes = 0.0;
    double aNn[G];
#pragma unroll
    for (int g = 0; g < G; ++g) aNn[g] = aN[g];
    // rem' = rem - dtau
    const double arems = arem;
    adt -= arem;
    double axn = ax;
    if (!iso) {
        // e' = e + dtau (H' - Lambda'),  H' = c (1 - x') n0 sum_g SigE_g N'_g
        aes += ae;
        double hs = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) hs += gc.SigE[g] * Nn[g];
        const double Hn = c * (1.0 - xn) * n0 * hs;
        const double Ln = cooling(r, n0, xn);
        adt += ae * (Hn - Ln);
        const double aH = ae * dtau;
        axn -= aH * c * n0 * hs;
        an0 += aH * c * (1.0 - xn) * hs;
#pragma unroll
        for (int g = 0; g < G; ++g) aNn[g] += aH * c * (1.0 - xn) * n0 * gc.SigE[g];
        cooling_adj(r, n0, xn, -ae * dtau, ar, axn, an0);
    }
    // x' = 1 - num / denx (unless clamped)
    if (!info.xclamp) {
        const double anum = -axn * rdx;
        const double aden = axn * num * rdx * rdx;
        ar.alpha += anum * x * x * n0 * dtau;
        axs += anum * (2.0 * r.alpha * x * n0 * dtau - 1.0);
        an0 += anum * r.alpha * x * x * dtau;
        adt += anum * r.alpha * x * x * n0;
        adt += aden * (r.beta * x * n0 + gam);
        ar.beta += aden * dtau * x * n0;
        axs += aden * dtau * r.beta * n0;
        an0 += aden * dtau * r.beta * x;
        const double agam = aden * dtau;
#pragma unroll
        for (int g = 0; g < G; ++g) aNn[g] += agam * c * gc.sigN[g];
    }
    // N'_g = (N_g + (S_g + rec_g) dtau) inv_g,  inv_g = 1 / (1 + dtau kap_g)
#pragma unroll
    for (int g = 0; g < G; ++g) {
        aN[g] = aNn[g] * inv[g];
        aS[g] += aNn[g] * dtau * inv[g];
        const double arec = aNn[g] * dtau * inv[g];
        adt += aNn[g] * (S[g] + rec[g]) * inv[g];
        const double ainv = aNn[g] * (N[g] + (S[g] + rec[g]) * dtau) + aFinv[g];
        const double aden = -ainv * inv[g] * inv[g];
        adt += aden * kap[g];
        const double akap = aden * dtau;
        axs -= akap * c * gc.sigN[g] * n0;
        an0 += akap * c * gc.sigN[g] * y0;
        if (g == 0) {
            ar.dalpha += arec * x * x * n0 * n0;
            axs += arec * 2.0 * r.dalpha * x * n0 * n0;
            an0 += arec * 2.0 * r.dalpha * x * x * n0;
        }
    }
    // dtau = dtau0 / 2^h; dtau0 = rem or |e / D|, D = H - Lambda at the start
    const double adt0 = ldexp(adt, -info.h);
    double aremo = arems;
    if (!info.branch) {
        aremo += adt0;
    } else {
        const double D = info.D;
        const double sg = D < 0.0 ? -1.0 : 1.0;
        const double rD = recip_fp64(D);
        aes += adt0 * sg * rD;
        const double aD = -adt0 * e * sg * rD * rD;
        double hs0 = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) hs0 += gc.SigE[g] * N[g];
        axs -= aD * c * n0 * hs0;
        an0 += aD * c * (1.0 - x) * hs0;
#pragma unroll
        for (int g = 0; g < G; ++g) aN[g] += aD * c * (1.0 - x) * n0 * gc.SigE[g];
        cooling_adj(r, n0, x, -aD, ar, axs, an0);
    }
    // rates at Tp
    const double aTp = ar.alpha * dr.alpha + ar.dalpha * dr.dalpha + ar.beta * dr.beta + ar.crec * dr.crec +
                       ar.cci * dr.cci + ar.cce * dr.cce + ar.cff * dr.cff;
    if (iso) {
        aT += aTp;
    } else {
        // Tp = e / (eunit (1 + x)), eunit = 1.5 k_B n0
        aes += aTp / (eunit * (1.0 + x));
        axs -= aTp * Tp / (1.0 + x);
        an0 -= aTp * Tp / n0;
    }
    ax = axs;
    ae = aes;
    arem = aremo;
}

// Reverse of chem_cell: inputs (N, F, x, T) of the subcycle and dL/d(outputs)
// -> dL/d(inputs), dL/dn0, dL/dS.  The start state of each substep is
// recomputed with substep() (identical decisions): from the cell's start when
// M = 0 (cost quadratic in the cell's substep count K, which is 1 for almost
// every cell), else from the nearest of M kept states, one every
// s = ceil(K / M) substeps (kept by the counting pass when K <= M, else by a
// second forward pass; at most 3K + K s / 2 substeps in all).  Both give the
// same bits.  With a finite
// budget the cell gives up when K exceeds it (*deferred = true, outputs
// meaningless), so a caller can hand long subcycles to the kept-state form.
template <int G, bool FAST, int M = 0>
__host__ __device__ inline void chem_cell_adj(const GroupConsts &gc, const ChemParams &p, const double (&N0)[G],
                                     const double (&F0)[G][3], double x0, double T0, double n0,
                                     const double (&S)[G], const double (&aNo)[G], const double (&aFo)[G][3],
                                     double axo, double aTo, double (&aN)[G], double (&aF)[G][3], double &ax,
                                     double &aT, double &an0, double (&aS)[G], int budget = 0x7fffffff,
                                     bool *deferred = nullptr) {
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double eunit = 1.5 * n0 * kKB;
    const double e0 = eunit * (1.0 + x0) * T0;
    // forward pass: substep count, end state, product of the F factors
    double N[G], Pf[G];
#pragma unroll
    for (int g = 0; g < G; ++g) { N[g] = N0[g]; Pf[g] = 1.0; }
    double x = x0, e = e0, rem = p.dt;
    ChemStats st{0, 0, 0, 0};
    int K = 0;
    // kept start states (M > 0): substeps 0, s, 2s, ...; this pass keeps the
    // first M (s = 1), a second one is needed only when K > M
    constexpr int MK = M > 0 ? M : 1;
    double kN[MK][G], kx[MK], ke[MK], kr[MK];
    while (rem > 0.0) {
        if (K >= budget) {
            *deferred = true;
            return;
        }
        if (M > 0 && K < MK) {
#pragma unroll
            for (int g = 0; g < G; ++g) kN[K][g] = N[g];
            kx[K] = x;
            ke[K] = e;
            kr[K] = rem;
        }
        const bool last = K >= p.max_substeps;
        double inv[G];
        if (!substep<G, FAST>(gc, p, last, n0, eunit, T0, S, N, x, e, rem, inv, st, nullptr)) break;
#pragma unroll
        for (int g = 0; g < G; ++g) Pf[g] *= inv[g];
        K++;
        if (last || iso) break;
    }
    const int s = M > 0 ? (K + MK - 1) / MK : 0;
    if (M > 0 && K > MK) {
        double Ns[G];
#pragma unroll
        for (int g = 0; g < G; ++g) Ns[g] = N0[g];
        double xs = x0, es = e0, rs = p.dt;
        ChemStats st2{0, 0, 0, 0};
        double inv[G];
        for (int j = 0; j < K; ++j) {
            if (j % s == 0) {
                const int b = j / s;
#pragma unroll
                for (int g = 0; g < G; ++g) kN[b][g] = Ns[g];
                kx[b] = xs;
                ke[b] = es;
                kr[b] = rs;
            }
            substep<G, FAST>(gc, p, j >= p.max_substeps, n0, eunit, T0, S, Ns, xs, es, rs, inv, st2, nullptr);
        }
    }
    // F_out = F_in prod_k inv_k: dL/dinv_k (through F) = Phi_g / inv_k
    double Phi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        Phi[g] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            aF[g][k] = aFo[g][k] * Pf[g];
            Phi[g] += aFo[g][k] * F0[g][k] * Pf[g];
        }
        aN[g] = aNo[g];
        aS[g] = 0.0;
    }
    ax = axo;
    aT = 0.0;
    an0 = 0.0;
    double ae = 0.0, arem = 0.0;
    if (!iso) {
        // T_out = e / (eunit (1 + x))
        const double Tf = e / (eunit * (1.0 + x));
        ae += aTo / (eunit * (1.0 + x));
        ax -= aTo * Tf / (1.0 + x);
        an0 -= aTo * Tf / n0;
    } else {
        aT += aTo;
    }
    for (int k = K - 1; k >= 0; --k) {
        double Ns[G];
        double xs, es, rs;
        int j0;
        if (M > 0) {
            const int b = k / s;
#pragma unroll
            for (int g = 0; g < G; ++g) Ns[g] = kN[b][g];
            xs = kx[b];
            es = ke[b];
            rs = kr[b];
            j0 = b * s;
        } else {
#pragma unroll
            for (int g = 0; g < G; ++g) Ns[g] = N0[g];
            xs = x0;
            es = e0;
            rs = p.dt;
            j0 = 0;
        }
        ChemStats st2{0, 0, 0, 0};
        double inv[G];
        for (int j = j0; j < k; ++j)
            substep<G, FAST>(gc, p, j >= p.max_substeps, n0, eunit, T0, S, Ns, xs, es, rs, inv, st2, nullptr);
        // decisions of substep k from its start state
        double Nk[G];
#pragma unroll
        for (int g = 0; g < G; ++g) Nk[g] = Ns[g];
        double xk = xs, ek = es, rk = rs;
        SubInfo info;
        substep<G, FAST>(gc, p, k >= p.max_substeps, n0, eunit, T0, S, Nk, xk, ek, rk, inv, st2, &info);
        double aFinv[G];
#pragma unroll
        for (int g = 0; g < G; ++g) aFinv[g] = Phi[g] / inv[g];
        substep_adj<G, FAST>(gc, p, n0, eunit, S, Ns, xs, es, rs, info, aFinv, aN, ax, ae, arem, an0, aS, aT);
    }
    if (!iso) {
        // e0 = eunit (1 + x0) T0
        aT += ae * eunit * (1.0 + x0);
        ax += ae * eunit * T0;
        an0 += ae * 1.5 * kKB * (1.0 + x0) * T0;
    }
}

// chem_cell_adj for a subcycle of exactly one substep: the substep that
// counts it is the one the reverse replays, so its decisions and factors are
// kept instead of recomputed (same bits as chem_cell_adj).  Returns false,
// with nothing written, for any other subcycle.
template <int G, bool FAST>
__host__ __device__ inline bool chem_cell_adj1(const GroupConsts &gc, const ChemParams &p, const double (&N0)[G],
                                      const double (&F0)[G][3], double x0, double T0, double n0,
                                      const double (&S)[G], const double (&aNo)[G], const double (&aFo)[G][3],
                                      double axo, double aTo, double (&aN)[G], double (&aF)[G][3], double &ax,
                                      double &aT, double &an0, double (&aS)[G]) {
    const bool iso = FAST ? false : (p.isothermal != 0);
    const double eunit = 1.5 * n0 * kKB;
    const double e0 = eunit * (1.0 + x0) * T0;
    double N[G], inv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) N[g] = N0[g];
    double x = x0, e = e0, rem = p.dt;
    ChemStats st{0, 0, 0, 0};
    SubInfo info;
    if (!(rem > 0.0)) return false;
    if (!substep<G, FAST>(gc, p, 0 >= p.max_substeps, n0, eunit, T0, S, N, x, e, rem, inv, st, &info)) return false;
    if (rem > 0.0 && !iso && !(0 >= p.max_substeps)) return false;  // a second substep follows
    double Phi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        Phi[g] = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            aF[g][k] = aFo[g][k] * inv[g];
            Phi[g] += aFo[g][k] * F0[g][k] * inv[g];
        }
        aN[g] = aNo[g];
        aS[g] = 0.0;
    }
    ax = axo;
    aT = 0.0;
    an0 = 0.0;
    double ae = 0.0, arem = 0.0;
    if (!iso) {
        const double Tf = e / (eunit * (1.0 + x));
        ae += aTo / (eunit * (1.0 + x));
        ax -= aTo * Tf / (1.0 + x);
        an0 -= aTo * Tf / n0;
    } else {
        aT += aTo;
    }
    double aFinv[G];
#pragma unroll
    for (int g = 0; g < G; ++g) aFinv[g] = Phi[g] / inv[g];
    substep_adj<G, FAST>(gc, p, n0, eunit, S, N0, x0, e0, p.dt, info, aFinv, aN, ax, ae, arem, an0, aS, aT);
    if (!iso) {
        aT += ae * eunit * (1.0 + x0);
        ax += ae * eunit * T0;
        an0 += ae * 1.5 * kKB * (1.0 + x0) * T0;
    }
    return true;
}

// Reverse of the floor and limiter (floor_limit_fwd) along the branch the
// forward took (taken: bit 0 floored, bit 1 limited), given the PRE values
// (n, f) and dL/d(post values): N* = max(N~, 0); F* = F~ c N*/|F~| when
// limited.  The branch is the forward's own decision, never re-decided here.
__host__ __device__ __forceinline__ void floor_limit_adj(double n, double fx, double fy, double fz, double c,
                                                         int taken, double &an, double &afx, double &afy,
                                                         double &afz) {
    const bool floored = (taken & 1) != 0;
    const double np = floored ? 0.0 : n;
    if (taken & 2) {
        const double F2 = fx * fx + fy * fy + fz * fz;
        const double Fn = sqrt(F2);
        const double ux = fx / Fn, uy = fy / Fn, uz = fz / Fn;
        const double ud = ux * afx + uy * afy + uz * afz;
        an += c * ud;
        const double s = c * np / Fn;
        afx = s * (afx - ux * ud);
        afy = s * (afy - uy * ud);
        afz = s * (afz - uz * ud);
    }
    if (floored) an = 0.0;
}

// Kept start states of the deferred-cell chemistry adjoint, per lane (in
// scratch memory, 48 B each with three groups).  With at least as many as a
// subcycle has substeps every reverse substep restarts from its own start
// state and the second forward pass is not needed; the 256^3 benchmark's
// longest subcycles take ~100 substeps (0.51 ms per reverse step for this
// pass with 128, 0.72 with 64, 0.89 with 32).
#ifndef EMMA_ADJ_KEPT
#define EMMA_ADJ_KEPT 128
#endif

// The chemistry adjoint of cell i (and the reverse of the floor and limiter
// before it): M kept states (chem_cell_adj), or M < 0 for the single-substep
// form (chem_cell_adj1).  Returns false, with nothing written, when the
// cell's subcycle exceeds the budget (one substep for M < 0).
template <int G, typename S, bool FAST, int M>
__device__ inline bool chem_adj_cell(int64_t i, const S *__restrict__ Ut, const S *__restrict__ Ft,
                                     const double *__restrict__ xs, const double *__restrict__ Ts,
                                     const double *__restrict__ n0, int64_t V, const SrcTable &src,
                                     const GroupConsts &gc, const ChemParams &cp, const S *__restrict__ gN,
                                     const S *__restrict__ gF, double *__restrict__ gx, double *__restrict__ gT,
                                     double *__restrict__ g_n0, double *__restrict__ gS, S *__restrict__ gU,
                                     int budget, bool skip = false) {
    const double c = cp.c;
    double Npre[G], Fpre[G][3], Nst[G], Fst[G][3], aNo[G], aFo[G][3], Sc[G];
    int taken[G];
    // every group's values are loaded before any is used: the floor and the
    // limiter branch, and loads behind a branch would wait group by group
    S un[G], uf[G][3], gn[G], gf[G][3];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        un[g] = Ut[(int64_t)g * V + i];
        gn[g] = gN[(int64_t)g * V + i];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uf[g][k] = Ft[((int64_t)g * 3 + k) * V + i];
            gf[g][k] = gF[((int64_t)g * 3 + k) * V + i];
        }
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        // the forward's floor and limiter, in its own precision and arithmetic
        S n = un[g];
        S f[3] = {uf[g][0], uf[g][1], uf[g][2]};
        Npre[g] = (double)n;
#pragma unroll
        for (int k = 0; k < 3; ++k) Fpre[g][k] = (double)f[k];
        taken[g] = floor_limit_fwd<S>(n, f[0], f[1], f[2], (S)c);
        Nst[g] = (double)n;
#pragma unroll
        for (int k = 0; k < 3; ++k) Fst[g][k] = (double)f[k];
        aNo[g] = (double)gn[g];
#pragma unroll
        for (int k = 0; k < 3; ++k) aFo[g][k] = (double)gf[g][k];
    }
    source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
    double aN[G], aF[G][3], aS[G], ax, aT, an0;
    bool deferred = false;
    if (M < 0)
        deferred = !chem_cell_adj1<G, FAST>(gc, cp, Nst, Fst, xs[i], Ts[i], n0[i], Sc, aNo, aFo, gx[i], gT[i], aN,
                                            aF, ax, aT, an0, aS);
    else
        chem_cell_adj<G, FAST, (M < 0 ? 0 : M)>(gc, cp, Nst, Fst, xs[i], Ts[i], n0[i], Sc, aNo, aFo, gx[i], gT[i],
                                                aN, aF, ax, aT, an0, aS, budget, &deferred);
    // skip (the cell belongs to another pass) is tested only here, so that
    // its own load does not hold back the cell's loads: the lane computes
    // with its wave and writes nothing
    if (skip) return true;
    if (deferred) return false;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        floor_limit_adj(Npre[g], Fpre[g][0], Fpre[g][1], Fpre[g][2], c, taken[g], aN[g], aF[g][0], aF[g][1],
                        aF[g][2]);
        gU[(int64_t)(4 * g) * V + i] = (S)aN[g];
        gU[(int64_t)(4 * g + 1) * V + i] = (S)aF[g][0];
        gU[(int64_t)(4 * g + 2) * V + i] = (S)aF[g][1];
        gU[(int64_t)(4 * g + 3) * V + i] = (S)aF[g][2];
    }
    gx[i] = ax;
    gT[i] = aT;
    g_n0[i] += an0;
    if ((src.mask[i >> 5] >> (i & 31)) & 1u) {
        const int r = lower_bound_cell(src.sorted_cell, src.n, i);
#pragma unroll
        for (int g = 0; g < G; ++g) gS[(int64_t)r * G + g] += aS[g];
    }
    return true;
}

// First pass, one thread per cell: single-substep subcycles (about 98 % of
// the cell-steps of the 256^3 benchmark); the others go to the kept-state pass.
// With `multi` (the segment's forward marked the cells whose subcycle was not
// a single substep) the marked cells are left to that pass, which runs beside
// this one; without it, or for a cell the forward did not mark that needs
// more than one substep all the same, the cell is appended to the work list
// for a kept-state pass after this one.  Handing the first pass subcycles of
// up to 2 or 4 substeps (replayed from the cell's start) measured slower: 3.7
// and 4.3 ms per step at 256^3 against 2.4 ms for this split before the
// single-substep form.
// one wave per block, for the reason given at EMMA_CHEM_TB (1.21 ms against
// 1.29 ms with 256 threads at 256^3)
#ifndef EMMA_ADJ_TB
#define EMMA_ADJ_TB 64
#endif
// minimum waves per SIMD the register allocation of each adjoint kernel keeps
#ifndef EMMA_ADJ_CHEM_WAVES
#define EMMA_ADJ_CHEM_WAVES 1
#endif
#ifndef EMMA_ADJ_LIST_WAVES
#define EMMA_ADJ_LIST_WAVES 1
#endif
#ifndef EMMA_ADJ_TRANSPORT_WAVES
#define EMMA_ADJ_TRANSPORT_WAVES 3
#endif
template <int G, typename S, bool FAST>
__global__ __launch_bounds__(EMMA_ADJ_TB, EMMA_ADJ_CHEM_WAVES) void k_chem_adj(const S *__restrict__ Ut, const S *__restrict__ Ft,
                                                  const double *__restrict__ xs, const double *__restrict__ Ts,
                                                  const double *__restrict__ n0, int64_t V, SrcTable src,
                                                  GroupConsts gc, ChemParams cp, const S *__restrict__ gN,
                                                  const S *__restrict__ gF, double *__restrict__ gx,
                                                  double *__restrict__ gT, double *__restrict__ g_n0,
                                                  double *__restrict__ gS, S *__restrict__ gU, WorkList wl,
                                                  const uint64_t *__restrict__ multi,
                                                  const uint32_t *__restrict__ skip) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t mw = 0;
    if (multi) mw = multi[min(i, V - 1) >> 6];  // same branch for every lane
    const bool listed = (mw >> (i & 63)) & 1ull;
    // skip: refined cells, whose children's adjoint (k_crta_adj) takes them
    const bool refined = skip && i < V && ((skip[i >> 5] >> (i & 31)) & 1u);
    bool deferred = false;
    if (i < V && !refined)
        deferred = !chem_adj_cell<G, S, FAST, -1>(i, Ut, Ft, xs, Ts, n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, gS,
                                                  gU, 1, listed);
    defer_push(wl, deferred, (uint32_t)i);
}

// Compaction of one step's bitmask into a cell list: one thread per 64-bit
// word, one atomic per wave.  The order of the list is not fixed; no result
// depends on it (every cell's adjoint is computed on its own).
__global__ __launch_bounds__(256) void k_multi_list(const uint64_t *__restrict__ multi, int64_t words, int64_t V,
                                                    uint32_t *count, uint32_t *cells) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = (int)(threadIdx.x & 63);
    uint64_t w = j < words ? multi[j] : 0ull;
    if (j == words - 1 && (V & 63)) w &= (1ull << (V & 63)) - 1ull;  // no bits past the grid
    const uint32_t n = (uint32_t)__popcll(w);
    uint32_t incl = n;  // inclusive prefix sum over the wave
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = __shfl_up(incl, d, 64);
        if (lane >= d) incl += t;
    }
    const uint32_t total = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane == 63 && total) base = atomicAdd(count, total);
    base = __shfl(base, 63, 64);
    uint32_t k = base + incl - n;
    while (w) {
        const int b = __ffsll((unsigned long long)w) - 1;
        w &= w - 1ull;
        cells[k++] = (uint32_t)(j * 64 + b);
    }
}

// Second pass over the deferred cells (grid-stride over the list): every
// substep's start recomputed from the nearest of EMMA_ADJ_KEPT kept states.
template <int G, typename S, bool FAST>
__global__ __launch_bounds__(256, EMMA_ADJ_LIST_WAVES) void k_chem_adj_list(const S *__restrict__ Ut, const S *__restrict__ Ft,
                                                       const double *__restrict__ xs, const double *__restrict__ Ts,
                                                       const double *__restrict__ n0, int64_t V, SrcTable src,
                                                       GroupConsts gc, ChemParams cp, const S *__restrict__ gN,
                                                       const S *__restrict__ gF, double *__restrict__ gx,
                                                       double *__restrict__ gT, double *__restrict__ g_n0,
                                                       double *__restrict__ gS, S *__restrict__ gU,
                                                       WorkList wl) {
    const uint32_t n = *wl.count;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        chem_adj_cell<G, S, FAST, EMMA_ADJ_KEPT>((int64_t)wl.cells[k], Ut, Ft, xs, Ts, n0, V, src, gc, cp, gN, gF,
                                                 gx, gT, g_n0, gS, gU, 0x7fffffff);
}

// Reverse of the refined-cell chemistry (the step of emma_rt_step_crta after
// the coarse transport), one lane per child, NC consecutive lanes per parent
// as in k_crta_fine.  Each lane replays its child's subcycle to get the
// child's end state, forms the derivatives of the restriction (parent N, F:
// means over the children; x: n_fine-weighted; T: (1 + x) n_fine-weighted),
// adds them to dL/d(child's end state), runs the kept-state chemistry adjoint
// of the child, and writes dL/d(child's start state) over (gxf, gTf), adds
// dL/dn_fine to gnf and dL/d(rate) of its sources to g_rate.  The parent's
// dL/dU* is the sum over its children (the same lane tree as the forward's
// sums), taken through the reverse of the floor and the limiter; the parent's
// own x, T do not reach the step's end state (gx, gT of the parent become 0).
template <int G, typename S, bool FAST, int NC>
__global__ __launch_bounds__(256) void k_crta_adj(const S *__restrict__ Ut, const S *__restrict__ Ft, int64_t V,
                                                  const int64_t *__restrict__ ref_cell, int n_ref,
                                                  const double *__restrict__ xfi, const double *__restrict__ Tfi,
                                                  const double *__restrict__ nf,
                                                  const int64_t *__restrict__ sorted_cell,
                                                  const int32_t *__restrict__ sorted_idx,
                                                  const double *__restrict__ rate,
                                                  const int32_t *__restrict__ src_child, int n_src,
                                                  GroupConsts gc, ChemParams cp, double volf,
                                                  const S *__restrict__ gN, const S *__restrict__ gF,
                                                  double *__restrict__ gx, double *__restrict__ gT,
                                                  double *__restrict__ gxf, double *__restrict__ gTf,
                                                  double *__restrict__ gnf, double *__restrict__ g_rate,
                                                  S *__restrict__ gU) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = t / NC;
    const int ch = (int)(t % NC);
    const int64_t p = j < n_ref ? ref_cell[j] : -1;
    // every lane of a parent agrees on this, so the sums stay inside live lanes
    if (!(p >= 0 && p < V)) return;
    const double c = cp.c;
    double Npre[G], Fpre[G][3], Nst[G], Fst[G][3], Sc[G];
    int taken[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        S n = Ut[(int64_t)g * V + p];
        S f[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) f[k] = Ft[((int64_t)g * 3 + k) * V + p];
        Npre[g] = (double)n;
#pragma unroll
        for (int k = 0; k < 3; ++k) Fpre[g][k] = (double)f[k];
        taken[g] = floor_limit_fwd<S>(n, f[0], f[1], f[2], (S)c);
        Nst[g] = (double)n;
#pragma unroll
        for (int k = 0; k < 3; ++k) Fst[g][k] = (double)f[k];
        Sc[g] = 0.0;
    }
    // the child's sources, as in k_crta_fine
    const int r0 = n_src > 0 ? lower_bound_cell(sorted_cell, n_src, p) : 0;
    for (int r = r0; r < n_src && sorted_cell[r] == p; ++r) {
        const int s = sorted_idx[r];
        if ((src_child ? src_child[s] : 0) == ch) {
#pragma unroll
            for (int g = 0; g < G; ++g) Sc[g] += rate[s] * gc.frac[g] / volf;
        }
    }
    const int64_t f = j * NC + ch;
    const double xin = xfi[f], Tin = Tfi[f], nfc = nf[f];
    // the child's end state (x, T) and the restriction's sums, as the forward
    double Nc[G], Pf[G];
#pragma unroll
    for (int g = 0; g < G; ++g) Nc[g] = Nst[g];
    double xo = xin, To = Tin;
    chem_cell_nxt<G, FAST>(gc, cp, Nc, Pf, xo, To, nfc, Sc);
    const double nsum = child_sum<NC>(nfc);
    const double xp = child_sum<NC>(xo * (nfc / nsum));
    const double w = (1.0 + xo) * nfc;
    const double msum = child_sum<NC>(w);
    const double Tp = child_sum<NC>(To * (w / msum));
    // dL/d(parent's end state), read by every child before lane 0 rewrites it
    const double gxp = gx[p], gTp = gT[p];
    const double inv = 1.0 / NC;
    double aNo[G], aFo[G][3];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        aNo[g] = (double)gN[(int64_t)g * V + p] * inv;
#pragma unroll
        for (int k = 0; k < 3; ++k) aFo[g][k] = (double)gF[((int64_t)g * 3 + k) * V + p] * inv;
    }
    // x_p = sum x n / nsum, T_p = sum T w / msum with w = (1 + x) n
    const double dw = gTp * (To - Tp) / msum;
    const double axo = gxf[f] + gxp * nfc / nsum + dw * nfc;
    const double aTo = gTf[f] + gTp * w / msum;
    const double an_restr = gxp * (xo - xp) / nsum + dw * (1.0 + xo);
    double aN[G], aF[G][3], aS[G], ax, aT, an0;
    chem_cell_adj<G, FAST, EMMA_ADJ_KEPT>(gc, cp, Nst, Fst, xin, Tin, nfc, Sc, aNo, aFo, axo, aTo, aN, aF, ax, aT,
                                          an0, aS);
    gxf[f] = ax;
    gTf[f] = aT;
    gnf[f] += an0 + an_restr;
    for (int r = r0; r < n_src && sorted_cell[r] == p; ++r) {
        const int s = sorted_idx[r];
        if ((src_child ? src_child[s] : 0) == ch) {
            double d = 0.0;
#pragma unroll
            for (int g = 0; g < G; ++g) d += gc.frac[g] / volf * aS[g];
            g_rate[s] += d;
        }
    }
    // the parent's dL/dU*: the children's sum, then the floor and the limiter
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double an = child_sum<NC>(aN[g]);
        double af[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) af[k] = child_sum<NC>(aF[g][k]);
        if (ch == 0) {
            floor_limit_adj(Npre[g], Fpre[g][0], Fpre[g][1], Fpre[g][2], c, taken[g], an, af[0], af[1], af[2]);
            gU[(int64_t)(4 * g) * V + p] = (S)an;
#pragma unroll
            for (int k = 0; k < 3; ++k) gU[(int64_t)(4 * g + 1 + k) * V + p] = (S)af[k];
        }
    }
    if (ch == 0) {
        gx[p] = 0.0;
        gT[p] = 0.0;
    }
}

// ------------------------------------------------------- transport adjoint
// Closure derivatives in terms of the reduced flux g = F/(c N), q = |g|^2:
// P = a I + N K g g^T with a = (1 - chi)/2 N and K = h(q) below the clip,
// 1/q at it (chi = 1).  Then
//   dP/dN   = aN I + KN g g^T,
//   dP/dF_k = (1/c) [GA g_k I + GB g_k g g^T + K (e_k g^T + g e_k^T)],
// with only O(1) factors, so faint fields (|F|^2 or N^-4 out of range) are safe.
// Below the clip, with (3 chi - 1)/2 = q h, chi' = dchi/dq = 2 (h + q h')/3:
//   aN = (1 - chi)/2 + q chi',  KN = -(h + 2 q h'),  GA = -chi',  GB = 2 h';
// at the clip aN = GA = 0, KN = 1/q, GB = -2/q^2.
struct ClosureJac {
    double aN, GA, K, KN, GB;
    double g[3];
};

__host__ __device__ __forceinline__ ClosureJac closure_jac(double N, double Fx, double Fy, double Fz, double c) {
    ClosureJac j{1.0 / 3.0, 0.0, 0.0, 0.0, 0.0, {0.0, 0.0, 0.0}};
    if (!(N > 0.0)) return j;  // P = N/3 I: only dP/dN = I/3
    // reciprocals to about 1 ulp (recip_fp64) rather than correctly rounded
    // divisions: these factors only scale gradients
    const double icn = recip_fp64(c * N);
    j.g[0] = Fx * icn;
    j.g[1] = Fy * icn;
    j.g[2] = Fz * icn;
    const double q = j.g[0] * j.g[0] + j.g[1] * j.g[1] + j.g[2] * j.g[2];
    if (q >= 1.0) {
        const double rq = recip_fp64(q);
        j.aN = 0.0;
        j.K = rq;
        j.KN = rq;
        j.GB = -2.0 * rq * rq;
        return j;
    }
    const double s = sqrt(4.0 - 3.0 * q);
    const double den = 5.0 + 2.0 * s, t = 2.0 + s;
    const double rt = recip_fp64(t), rs = recip_fp64(s), rden = recip_fp64(den);
    const double u = 6.0 + 3.0 * rt;
    const double h = u * rden;
    const double hp = (1.5 * rs) * (3.0 * rt * rt * rden + 2.0 * u * rden * rden);
    const double chi = (1.0 + 2.0 * q * h) * (1.0 / 3.0);
    const double dchi = 2.0 * (h + q * hp) * (1.0 / 3.0);
    j.aN = 0.5 * (1.0 - chi) + dchi * q;
    j.GA = -dchi;
    j.K = h;
    j.KN = -(h + 2.0 * q * hp);
    j.GB = 2.0 * hp;
    return j;
}

// M_d(U)^T v for the flux Jacobian M_d = dFt_d/dU, Ft_d = (F_d, c^2 P_.d), of
// a state with closure Jacobian J; v = (v_N, w).
__host__ __device__ __forceinline__ void flux_jac_t(const ClosureJac &J, int d, double c, const double v[4],
                                                    double out[4]) {
    const double *g = J.g;
    const double w[3] = {v[1], v[2], v[3]};
    const double wg = w[0] * g[0] + w[1] * g[1] + w[2] * g[2];
    out[0] = c * c * (J.aN * w[d] + J.KN * wg * g[d]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double mk = c * (J.GA * g[k] * w[d] + J.GB * g[k] * wg * g[d] + J.K * w[k] * g[d]);
        if (k == d) mk += v[0] + c * J.K * wg;
        out[1 + k] = mk;
    }
}

// Transpose of the transport step at one cell and group.  U_i enters
// U*_{i+e_d} through A_d(U_i) and U*_{i-e_d} through B_d(U_i)
// (A = (Ft + c U)/2, B = (c U - Ft)/2), and U*_i through -c U_i per axis; at a
// non-periodic face, cell i also sees the ghost of itself (A_d(ghost) across
// its minus face, B_d(ghost) across its plus face): ghost = U_i
// (transmissive), U_i with F_d reversed (reflective, a symmetric map R, so
// the term is R A'(R U)^T g_i) or a constant (inflow).  gi = dL/dU*_i,
// vnb[d][s] = dL/dU* of the neighbour across face (d, s) (zero across a
// non-periodic face).
template <typename S>
__device__ __forceinline__ void transport_adj_cell(double n, const double (&Fv)[3], const double (&gi)[4],
                                                   const S (&vnb)[3][2][4], const Nbrs &nb, double c,
                                                   double lam, const Bounds<S> &bnd, double (&out)[4]) {
    const double hl = 0.5 * lam;
    const ClosureJac J = closure_jac(n, Fv[0], Fv[1], Fv[2], c);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = (1.0 - 3.0 * c * lam) * gi[q];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        // ordinary neighbours: (lam/2) [c (v+ + v-) + M_d(U)^T (v+ - v-)]
        double dv[4], m[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) dv[q] = (double)vnb[d][1][q] - (double)vnb[d][0][q];
        flux_jac_t(J, d, c, dv, m);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] += hl * (c * ((double)vnb[d][1][q] + (double)vnb[d][0][q]) + m[q]);
        // ghosts of this cell across its own non-periodic faces
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int face = nb.face[d][s];
            if (face < 0 || bnd.kind[face] == BC_INFLOW) continue;
            const bool refl = bnd.kind[face] == BC_REFLECTIVE;
            double Fg[3] = {Fv[0], Fv[1], Fv[2]};
            if (refl) Fg[d] = -Fg[d];
            const ClosureJac Jg = closure_jac(n, Fg[0], Fg[1], Fg[2], c);
            double mg[4];
            flux_jac_t(Jg, d, c, gi, mg);
            const double sg = s ? -1.0 : 1.0;  // A across the minus face, B across the plus face
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                double t = hl * (c * gi[q] + sg * mg[q]);
                if (refl && q == 1 + d) t = -t;
                out[q] += t;
            }
        }
    }
}

// Planes of a z chunk of the transport adjoint.
constexpr int kAdjLZ = 16;

// Gather form of the transport transpose for one group (blockIdx.y): blocks
// of 64 x 4 columns march up kAdjLZ-plane z chunks, keeping dL/dU* of the
// planes below, at and above the cell in registers, so the z neighbours are
// read from HBM once (cell-parallel, every cell read its six neighbours
// from memory: three times the algorithmic bytes); x and y neighbours come
// through the caches.  Blocks are renumbered per XCD like the forward tiles.
template <typename S>
__global__ __launch_bounds__(256, EMMA_ADJ_TRANSPORT_WAVES) void k_transport_adj(const S *__restrict__ N, const S *__restrict__ F,
                                                       const S *__restrict__ gU, S *__restrict__ gN,
                                                       S *__restrict__ gF, Grid gr, double c, double lam,
                                                       Bounds<S> bnd) {
    const int g = blockIdx.y;
    const int64_t V = gr.V;
    const int ntx = (gr.nx + 63) / 64, nty = (gr.ny + 3) / 4;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int x = (t % ntx) * 64 + (int)(threadIdx.x & 63);
    const int y = ((t / ntx) % nty) * 4 + (int)(threadIdx.x >> 6);
    const int z0 = (t / (ntx * nty)) * kAdjLZ;
    if (x >= gr.nx || y >= gr.ny || z0 >= gr.nz) return;  // no barriers below
    const int z1 = min(z0 + kAdjLZ, gr.nz);
    const int64_t plane = (int64_t)gr.nx * gr.ny;
    // restrict on the group's views too: the stores of one plane must not
    // hold back the loads of the next
    const S *__restrict__ gUg = gU + (int64_t)(4 * g) * V;
    const S *__restrict__ Ng = N + (int64_t)g * V;
    const S *__restrict__ Fg = F + (int64_t)(3 * g) * V;
    S *__restrict__ gNg = gN + (int64_t)g * V;
    S *__restrict__ gFg = gF + (int64_t)(3 * g) * V;
    int64_t i = (int64_t)z0 * plane + (int64_t)y * gr.nx + x;
    // dL/dU* values stay in the storage type until used.  Every neighbour
    // index is inside the grid (a cell's own index across a non-periodic
    // face), so the loads are unconditional and a ghost's value is selected
    // away afterwards: conditional loads each waited for their own data.
    S below[4], here[4], above[4];
    {
        const Nbrs nb = neighbours(gr, bnd, i, x, y, z0);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const S v = gUg[(int64_t)q * V + nb.idx[2][0]];
            below[q] = nb.face[2][0] < 0 ? v : S(0);
            here[q] = gUg[(int64_t)q * V + i];
        }
    }
    for (int z = z0; z < z1; ++z, i += plane) {
        const Nbrs nb = neighbours(gr, bnd, i, x, y, z);
        S vnb[3][2][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const S va = gUg[(int64_t)q * V + nb.idx[2][1]];
            above[q] = nb.face[2][1] < 0 ? va : S(0);
#pragma unroll
            for (int d = 0; d < 2; ++d)
#pragma unroll
                for (int s = 0; s < 2; ++s) {
                    const S v = gUg[(int64_t)q * V + nb.idx[d][s]];
                    vnb[d][s][q] = nb.face[d][s] < 0 ? v : S(0);
                }
            vnb[2][0][q] = below[q];
            vnb[2][1][q] = above[q];
        }
        const double n = (double)Ng[i];
        const double Fv[3] = {(double)Fg[i], (double)Fg[V + i], (double)Fg[2 * V + i]};
        const double hd[4] = {(double)here[0], (double)here[1], (double)here[2], (double)here[3]};
        double out[4];
        transport_adj_cell<S>(n, Fv, hd, vnb, nb, c, lam, bnd, out);
        gNg[i] = (S)out[0];
#pragma unroll
        for (int k = 0; k < 3; ++k) gFg[(int64_t)k * V + i] = (S)out[1 + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            below[q] = here[q];
            here[q] = above[q];
        }
    }
}

// ---------------------------------------------------- HLL transport adjoint
// Speeds of one state along axis d (m1_speeds in double) and their gradients
// with respect to (N, F_x, F_y, F_z).  f = F_d/(c N) clipped to [-1, 1], 0
// for N <= 0; where the clip or N <= 0 decides f, the gradients are zero
// (the same selections as the oracle's min/max).  With s = sqrt(4 - 3 f^2),
// ds/df = -3 f/s, w = 2 sqrt(3) (1 - f)(1 + f)/(1 + s) and
// lambda-+ = c (f -+ w)/s: dlambda-+/df = c ((1 -+ w') s - (f -+ w) s')/s^2.
struct SpeedJac {
    double lmin, lmax;
    double gmin[4], gmax[4];
};

__device__ inline SpeedJac speed_jac(const double (&u)[4], int d, double c) {
    SpeedJac r{0.0, 0.0, {0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    const double N = u[0];
    double f = 0.0;
    bool free_f = false;
    if (N > 0.0) {
        const double raw = u[1 + d] / (c * N);
        f = raw < 1.0 ? raw : 1.0;
        f = -1.0 < f ? f : -1.0;
        free_f = raw < 1.0 && -1.0 < raw;
    }
    // reciprocals to about 1 ulp: the speeds only weigh gradients here (the
    // selections above and in the face use them as well, like the forward's
    // own single-precision or FP64 speeds, and differ only at ties)
    const double s = sqrt(4.0 - 3.0 * f * f);
    const double is = recip_fp64(s), i1s = recip_fp64(1.0 + s);
    const double w = 3.4641016151377544 * (1.0 - f) * (1.0 + f) * i1s;
    r.lmin = c * (f - w) * is;
    r.lmax = c * (f + w) * is;
    if (free_f) {
        const double ds = -3.0 * f * is;
        const double dw = 3.4641016151377544 * (-2.0 * f * (1.0 + s) - (1.0 - f * f) * ds) * i1s * i1s;
        const double dmin = c * ((1.0 - dw) * s - (f - w) * ds) * is * is;
        const double dmax = c * ((1.0 + dw) * s - (f + w) * ds) * is * is;
        const double icn = recip_fp64(c * N);
        const double dfdN = -f * recip_fp64(N), dfdF = icn;
        r.gmin[0] = dmin * dfdN;
        r.gmin[1 + d] = dmin * dfdF;
        r.gmax[0] = dmax * dfdN;
        r.gmax[1 + d] = dmax * dfdF;
    }
    return r;
}

// One state's part of an HLL face along axis d: the state, its flux
// Ft_d = (F_d, c^2 P_.d) and its speeds (with their gradients when the
// state's own transpose is wanted).
struct SideData {
    double u[4], ft[4];
    SpeedJac sj;
};

__device__ inline SideData side_data(const double (&u)[4], int d, double c) {
    SideData sd;
    double P[6];
    m1_pressure<double>(u[0], u[1], u[2], u[3], c, P);
    const int i0 = d == 0 ? 0 : (d == 1 ? 1 : 2), i1 = d == 0 ? 1 : (d == 1 ? 3 : 4),
              i2 = d == 0 ? 2 : (d == 1 ? 4 : 5);
    const double cc = c * c;
#pragma unroll
    for (int q = 0; q < 4; ++q) sd.u[q] = u[q];
    sd.ft[0] = u[1 + d];
    sd.ft[1] = cc * P[i0];
    sd.ft[2] = cc * P[i1];
    sd.ft[3] = cc * P[i2];
    sd.sj = speed_jac(u, d, c);
    return sd;
}

// Transpose of the HLL face flux along axis d,
//   Phi = (a+ Ft(U_L) - a- Ft(U_R) + a+ a- (U_R - U_L)) / (a+ - a-),
// a- = min(0, lambda-_L, lambda-_R), a+ = max(0, lambda+_L, lambda+_R), for
// v = dL/dPhi, on one side (ME: the left state when ME_L):
//   (dPhi/dU_L)^T v = [a+ M_L^T v - a+ a- v + (v.(Ft_L + a- dU - Phi)) grad a+
//                      + (v.(a+ dU - Ft_R + Phi)) grad a-] / (a+ - a-),
//   (dPhi/dU_R)^T v = [-a- M_R^T v + a+ a- v + the same two terms] / (a+ - a-),
// dU = U_R - U_L, M = dFt_d/dU (J: that side's closure Jacobian); a speed's
// gradient term goes to the side whose speed the min/max selected (ties to
// the left state, none when the bound is 0).
template <bool ME_L>
__device__ inline void hll_face_adj_side(const SideData &me, const ClosureJac &J, const SideData &other, int d,
                                         double c, const double (&v)[4], double (&o)[4]) {
    const SideData &L = ME_L ? me : other;
    const SideData &R = ME_L ? other : me;
    const bool minR = R.sj.lmin < L.sj.lmin;
    const double m = minR ? R.sj.lmin : L.sj.lmin;
    const bool am0 = !(m < 0.0);
    const double am = am0 ? 0.0 : m;
    const bool maxR = L.sj.lmax < R.sj.lmax;
    const double M = maxR ? R.sj.lmax : L.sj.lmax;
    const bool ap0 = !(0.0 < M);
    const double ap = ap0 ? 0.0 : M;
    const double iD = recip_fp64(ap - am);
    double cp = 0.0, cm = 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double du = R.u[q] - L.u[q];
        const double phi = (ap * L.ft[q] - am * R.ft[q] + ap * am * du) * iD;
        cp += v[q] * (L.ft[q] + am * du - phi);
        cm += v[q] * (ap * du - R.ft[q] + phi);
    }
    double mm[4];
    flux_jac_t(J, d, c, v, mm);
    // the selected speeds' gradients count only when they are this side's
    const bool myp = !ap0 && (maxR != ME_L), mym = !am0 && (minR != ME_L);
    const double kp = myp ? cp * iD : 0.0, km = mym ? cm * iD : 0.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double lin = ME_L ? (ap * mm[q] - ap * am * v[q]) : (ap * am * v[q] - am * mm[q]);
        o[q] = lin * iD + kp * me.sj.gmax[q] + km * me.sj.gmin[q];
    }
}

// Transpose of the transport step with the HLL flux (gather form, one thread
// per cell and group, blockIdx.y = group), one launch per axis D: U*_i =
// U_i + lam sum_d (Phi_{i-1/2} - Phi_{i+1/2}), so with g = dL/dU*, dL/dU_i =
// g_i + the transposed face Jacobians of cell i's faces, its own side,
// applied to dL/dPhi = lam (g_right - g_left); at a non-periodic face only
// the cell inside is updated (-lam g_i across its plus face, lam g_i across
// its minus face), and the ghost's side maps back through ghost = U_i
// (transmissive), U_i with F_d reversed (reflective) or a constant (inflow).
// The x launch writes g_i plus its two faces' terms to (gN, gF), the y and z
// launches add theirs.  The cell's own face data along D is computed once.
template <typename S, int D>
__global__ __launch_bounds__(256) void k_transport_adj_hll(const S *__restrict__ N, const S *__restrict__ F,
                                                           const S *__restrict__ gU, S *__restrict__ gN,
                                                           S *__restrict__ gF, Grid gr, double c, double lam,
                                                           Bounds<S> bnd) {
    const int g = blockIdx.y;
    const int64_t V = gr.V;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= V) return;
    const int x = (int)(i % gr.nx), y = (int)((i / gr.nx) % gr.ny), z = (int)(i / ((int64_t)gr.nx * gr.ny));
    const S *__restrict__ Ng = N + (int64_t)g * V;
    const S *__restrict__ Fg = F + (int64_t)(3 * g) * V;
    const S *__restrict__ gUg = gU + (int64_t)(4 * g) * V;
    S *__restrict__ gNg = gN + (int64_t)g * V;
    S *__restrict__ gFg = gF + (int64_t)(3 * g) * V;
    const Nbrs nb = neighbours(gr, bnd, i, x, y, z);
    const double u[4] = {(double)Ng[i], (double)Fg[i], (double)Fg[V + i], (double)Fg[2 * V + i]};
    double gi[4], out[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) gi[q] = (double)gUg[(int64_t)q * V + i];
    if (D == 0) {
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] = gi[q];
    } else {
        out[0] = (double)gNg[i];
#pragma unroll
        for (int k = 0; k < 3; ++k) out[1 + k] = (double)gFg[(int64_t)k * V + i];
    }
    const SideData me = side_data(u, D, c);
    const ClosureJac Jme = closure_jac(u[0], u[1], u[2], u[3], c);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int face = nb.face[D][s];
        const int64_t j = nb.idx[D][s];
        double un[4], v[4];
        if (face < 0) {
            un[0] = (double)Ng[j];
#pragma unroll
            for (int k = 0; k < 3; ++k) un[1 + k] = (double)Fg[(int64_t)k * V + j];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const double gn = (double)gUg[(int64_t)q * V + j];
                v[q] = s ? lam * (gn - gi[q]) : lam * (gi[q] - gn);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                un[q] = u[q];
                v[q] = s ? -lam * gi[q] : lam * gi[q];
            }
            if (bnd.kind[face] == BC_REFLECTIVE) {
                un[1 + D] = -un[1 + D];
            } else if (bnd.kind[face] == BC_INFLOW) {
                const double phi = (double)bnd.phi[face][g];
                un[0] = phi / c;
                un[1] = un[2] = un[3] = 0.0;
                un[1 + D] = (face & 1) ? -phi : phi;
            }
        }
        const SideData nbr = side_data(un, D, c);
        double o[4];
        // the cell is the left state across its plus face (s = 1), the right
        // state across its minus face
        if (s) hll_face_adj_side<true>(me, Jme, nbr, D, c, v, o);
        else hll_face_adj_side<false>(me, Jme, nbr, D, c, v, o);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[q] += o[q];
        if (face >= 0 && bnd.kind[face] != BC_INFLOW) {
            // the ghost's side of the face, mapped back to the cell
            double og[4];
            const ClosureJac Jg = closure_jac(un[0], un[1], un[2], un[3], c);
            if (s) hll_face_adj_side<false>(nbr, Jg, me, D, c, v, og);
            else hll_face_adj_side<true>(nbr, Jg, me, D, c, v, og);
            if (bnd.kind[face] == BC_REFLECTIVE) og[1 + D] = -og[1 + D];
#pragma unroll
            for (int q = 0; q < 4; ++q) out[q] += og[q];
        }
    }
    gNg[i] = (S)out[0];
#pragma unroll
    for (int k = 0; k < 3; ++k) gFg[(int64_t)k * V + i] = (S)out[1 + k];
}

// dL/d(rate of source s) += sum_g frac_g / dx^3 dL/dS_g(host cell of s).
template <int G>
__global__ void k_src_grad(const int64_t *cell, int n, int64_t V, const int64_t *sorted_cell, const double *gS,
                           GroupConsts gc, double vol, double *g_rate) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t cs = cell[s];
    if (cs < 0 || cs >= V) return;
    const int r = lower_bound_cell(sorted_cell, n, cs);
    double acc = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) acc += gc.frac[g] / vol * gS[(int64_t)r * G + g];
    g_rate[s] += acc;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

}  // namespace emma
