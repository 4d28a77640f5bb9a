// kernels.hpp -- HIP kernels of the radiation step (gfx950, wave64).
//
//   k_src_*        source table: stable rank sort of the point sources by host
//                  cell, per-cell summed source density S_g = sum rate f_g / dx^3,
//                  and a one-bit-per-cell mask so the chemistry reads one bit per
//                  cell instead of a dense S field.
//   k_transport    M1 transport of all groups, one thread per cell, reference form
//                  (every face flux evaluated from both sides, like the paper's
//                  gather; kept as the simple second implementation that the
//                  fused kernel is tested against).
//   k_chem         per-cell FP64 thermochemistry subcycle.
//   k_fused        transport + chemistry in one pass (see fused.hpp).
//   k_diag_*       deterministic reductions for the diagnostics.
#pragma once

#include "physics.hpp"
#include "../../include/emma_rt.h"

namespace emma {

struct Grid {
    int nx, ny, nz;
    int64_t V;  // nx * ny * nz
};

// Counters accumulated when diagnostics are requested.
enum Counter {
    CNT_LIMITER = 0,
    CNT_NEG,
    CNT_XCLAMP,
    CNT_CAP,
    CNT_SUB,
    CNT_ATT,
    CNT_NONFINITE,
    CNT_BADSRC,
    CNT_BADREF,   // refined-cell list entries out of range or repeated, bad source children
    CNT_MAXSUB,   // max, via atomicMax
    CNT_HIST,     // EMMA_RT_SUBSTEP_BINS counters: substeps per cell-step histogram
    CNT_COUNT = CNT_HIST + EMMA_RT_SUBSTEP_BINS
};

// Kernel kinds for the per-kernel timing.
enum KernelKind {
    KID_SRC = 0,
    KID_TRANSPORT,
    KID_CHEM,
    KID_FUSED,
    KID_DIAG,
    KID_ADJ_CHEM,
    KID_ADJ_TRANSPORT,
    KID_ADJ_SRC,
    KID_ADJ_FWD,
    KID_CHEM_LIST,
    KID_CRTA,
    KID_ADJ_CHEM_LIST,
    KID_COUNT
};

__device__ inline int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline int wave_max(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Physical tile of block b when the hardware deals blocks to 8 XCDs
// round-robin: XCD k gets the logical range [k*q + min(k, r), ...).
__device__ inline int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int k = b & 7, i = b >> 3;
    return k * q + (k < r ? k : r) + i;
}

// Counters live in kCntSlots copies so that concurrent waves do not all hit
// one address; slot = block index mod kCntSlots, summed on the host.
constexpr int kCntSlots = 64;

__device__ inline unsigned long long *cnt_slot(unsigned long long *cnt) {
    return cnt + (blockIdx.x & (kCntSlots - 1)) * CNT_COUNT;
}

// Adds v into counter idx once per wave (all 64 lanes must call it).
__device__ inline void wave_count(unsigned long long *cnt, int idx, int64_t v) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && v != 0) atomicAdd(cnt_slot(cnt) + idx, (unsigned long long)v);
}

__device__ inline void wave_count_max(unsigned long long *cnt, int idx, int v) {
    v = wave_max(v);
    if ((threadIdx.x & 63) == 0 && v > 0) atomicMax(cnt_slot(cnt) + idx, (unsigned long long)v);
}

// Histogram bin of a cell-step with n accepted substeps: the bit length of n
// (0 for none), everything from 2^16 in the last bin.
__device__ inline int substep_bin(int n) {
    const int b = n <= 0 ? 0 : 32 - __clz(n);
    return b < EMMA_RT_SUBSTEP_BINS - 1 ? b : EMMA_RT_SUBSTEP_BINS - 1;
}

// Adds the lanes with `counted` set to the histogram bins of their substep
// counts n, one atomic per bin present in the wave (all 64 lanes must call it).
__device__ inline void wave_hist(unsigned long long *cnt, bool counted, int n) {
    const int b = substep_bin(n);
    unsigned long long todo = __ballot(counted);
    while (todo) {  // wave-uniform: one pass per distinct bin
        const int bl = __shfl(b, __ffsll((long long)todo) - 1, 64);
        const unsigned long long m = __ballot(counted && b == bl);
        if ((threadIdx.x & 63) == 0) atomicAdd(cnt_slot(cnt) + CNT_HIST + bl, (unsigned long long)__popcll(m));
        todo &= ~m;
    }
}

// ------------------------------------------------------------------ sources
__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int n, unsigned long long v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Sorting the source list by (cell, list position), cells outside the grid
// keyed INT64_MAX so that they sort last and are ignored: each block sorts a
// tile of kSrcTile sources in LDS (rank = number of smaller keys within the
// tile), then every source's rank in the whole list is the sum over tiles of
// the number of smaller keys there (a binary search in each sorted tile):
// O(n (n / kSrcTile) log kSrcTile) work instead of O(n^2).
constexpr int kSrcTile = 256;

__device__ inline int64_t src_key(const int64_t *cell, int s, int64_t V) {
    const int64_t k = cell[s];
    return (k < 0 || k >= V) ? INT64_MAX : k;
}

__global__ __launch_bounds__(kSrcTile) void k_src_tile_sort(const int64_t *cell, int n, int64_t V,
                                                            int64_t *tkey, int32_t *tidx,
                                                            unsigned long long *cnt) {
    __shared__ int64_t key[kSrcTile];
    const int t0 = blockIdx.x * kSrcTile, m = min(kSrcTile, n - t0);
    const int s = t0 + threadIdx.x;
    int64_t ks = INT64_MAX;
    if ((int)threadIdx.x < m) {
        ks = src_key(cell, s, V);
        if (ks == INT64_MAX) atomicAdd(cnt_slot(cnt) + CNT_BADSRC, 1ull);
    }
    key[threadIdx.x] = ks;
    __syncthreads();
    if ((int)threadIdx.x < m) {
        int rank = 0;
        for (int t = 0; t < m; ++t) rank += (key[t] < ks) || (key[t] == ks && t < (int)threadIdx.x);
        tkey[t0 + rank] = ks;
        tidx[t0 + rank] = s;
    }
}

// Rank of source s in the whole list from the sorted tiles; writes the
// sorted table (cell, list position).
__global__ void k_src_rank(const int64_t *cell, int n, int64_t V, const int64_t *tkey, const int32_t *tidx,
                           int64_t *sorted_cell, int32_t *sorted_idx) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    const int64_t ks = src_key(cell, s, V);
    int rank = 0;
    for (int t0 = 0; t0 < n; t0 += kSrcTile) {
        // keys (k, i) of the tile below (ks, s): k < ks, or k == ks and i < s
        int lo = 0, hi = min(kSrcTile, n - t0);
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            const int64_t k = tkey[t0 + mid];
            if (k < ks || (k == ks && tidx[t0 + mid] < s)) lo = mid + 1;
            else hi = mid;
        }
        rank += lo;
    }
    sorted_cell[rank] = ks;
    sorted_idx[rank] = s;
}

// At the head of every run of equal cells: S_g = sum over the run, in list
// order, of rate * frac_g / dx^3, and the cell's bit in the mask.
template <int G>
__global__ void k_src_heads(const int64_t *sorted_cell, const int32_t *sorted_idx,
                            const double *rate, int n, GroupConsts gc, double inv_vol_dx,
                            double vol, double *S, uint32_t *mask) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t c = sorted_cell[r];
    if (c == INT64_MAX) return;
    if (r > 0 && sorted_cell[r - 1] == c) return;
    double acc[G];
#pragma unroll
    for (int g = 0; g < G; ++g) acc[g] = 0.0;
    for (int q = r; q < n && sorted_cell[q] == c; ++q) {
        const double rt = rate[sorted_idx[q]];
#pragma unroll
        for (int g = 0; g < G; ++g) acc[g] += rt * gc.frac[g] / vol;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) S[(int64_t)r * G + g] = acc[g];
    atomicOr(mask + (c >> 5), 1u << (c & 31));
    (void)inv_vol_dx;
}

// First sorted position whose cell is >= c.
__device__ inline int lower_bound_cell(const int64_t *sorted_cell, int n, int64_t c) {
    int lo = 0, hi = n;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (sorted_cell[mid] < c) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int G>
__device__ inline void source_of(int64_t i, const uint32_t *mask, const int64_t *sorted_cell,
                                 const double *S, int n, double (&Sc)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) Sc[g] = 0.0;
    if ((mask[i >> 5] >> (i & 31)) & 1u) {
        const int r = lower_bound_cell(sorted_cell, n, i);
#pragma unroll
        for (int g = 0; g < G; ++g) Sc[g] = S[(int64_t)r * G + g];
    }
}

struct SrcTable {
    const uint32_t *mask;
    const int64_t *sorted_cell;
    const double *S;
    int n;
};

// --------------------------------------------------------------- boundaries
// Global boundaries (the gather step of Sec. 4 and the planar source of the
// Sec. 6 photo-evaporation test), faces x-, x+, y-, y+, z-, z+.  Across a
// non-periodic face the outside neighbour of a cell is a ghost made from the
// cell itself: transmissive = the cell; reflective = the cell with its normal
// flux component reversed; inflow = a beam entering along the face normal,
// F = phi_g n_in, N = phi_g / c, independent of the cell.
enum BcKind { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1, BC_REFLECTIVE = 2, BC_INFLOW = 3 };

template <typename R>
struct Bounds {
    int kind[6];
    R phi[6][EMMA_RT_MAX_GROUPS];  // inflow faces: photons cm^-2 s^-1 of each group
};

// Turn the state (n, f[3]) of the boundary cell into its ghost across face.
template <typename R>
__host__ __device__ __forceinline__ void ghost(const Bounds<R> &b, int face, int g, R c, R &n, R f[3]) {
    const int d = face >> 1;
    const int k = b.kind[face];
    if (k == BC_REFLECTIVE) {
        f[d] = -f[d];
    } else if (k == BC_INFLOW) {
        const R phi = b.phi[face][g];
        n = phi / c;
        f[0] = R(0); f[1] = R(0); f[2] = R(0);
        f[d] = (face & 1) ? -phi : phi;  // pointing into the domain
    }
}

// Neighbour cells of cell (x, y, z) across both faces of each axis: flat
// index (the cell itself across a non-periodic face) and the face whose
// ghost applies there (-1: an ordinary neighbour).
struct Nbrs {
    int64_t idx[3][2];
    int face[3][2];
};

template <typename R>
__host__ __device__ inline Nbrs neighbours(const Grid &gr, const Bounds<R> &b, int64_t i, int x, int y, int z) {
    Nbrs nb;
    const int c3[3] = {x, y, z};
    const int n3[3] = {gr.nx, gr.ny, gr.nz};
    const int64_t st[3] = {1, (int64_t)gr.nx, (int64_t)gr.nx * gr.ny};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            const int face = 2 * d + s;
            int q = c3[d] + (s ? 1 : -1);
            nb.face[d][s] = -1;
            if (q < 0 || q >= n3[d]) {
                if (b.kind[face] == BC_PERIODIC) {
                    q = s ? 0 : n3[d] - 1;
                } else {
                    q = c3[d];
                    nb.face[d][s] = face;
                }
            }
            nb.idx[d][s] = i + (int64_t)(q - c3[d]) * st[d];
        }
    }
    return nb;
}

// ---------------------------------------------------------------- transport
// Reference transport: one thread per cell, all groups.  The update of cell i
// is U* = U + (dt/dx) sum_d [flux(i-1/2) - flux(i+1/2)] with the flux of
// eq. (e:glf), then N* >= 0 and |F*| <= c N*.
template <typename R>
__device__ inline void glf(R NL, const R FL[3], const R PL[6], R NR, const R FR[3], const R PR[6],
                           int d, R c, R out[4]) {
    // column d of the symmetric tensor: rows x, y, z
    const int col[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    out[0] = R(0.5) * (FL[d] + FR[d]) - R(0.5) * c * (NR - NL);
#pragma unroll
    for (int k = 0; k < 3; ++k)
        out[1 + k] = R(0.5) * c * c * (PL[col[k][d]] + PR[col[k][d]]) - R(0.5) * c * (FR[k] - FL[k]);
}

// HLL flux across a face normal to axis d with the speeds of m1_speeds:
//   (a+ Ft(L) - a- Ft(R) + a+ a- (U_R - U_L)) / (a+ - a-),
// a- = min(0, speeds of both sides), a+ = max(0, speeds of both sides).
template <typename R>
__device__ inline void hll(R NL, const R FL[3], const R PL[6], R NR, const R FR[3], const R PR[6], int d, R c,
                           R out[4]) {
    const int col[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    R lmL, lpL, lmR, lpR;
    m1_speeds<R>(NL, FL[d], c, lmL, lpL);
    m1_speeds<R>(NR, FR[d], c, lmR, lpR);
    const R amr = lmL < lmR ? lmL : lmR;
    const R apr = lpL > lpR ? lpL : lpR;
    const R am = amr < R(0) ? amr : R(0);
    const R ap = apr > R(0) ? apr : R(0);
    const R inv = FastMath<R>::rcp(ap - am);
    const R cc = c * c, pm = ap * am;
    out[0] = (ap * FL[d] - am * FR[d] + pm * (NR - NL)) * inv;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        out[1 + k] = (ap * cc * PL[col[k][d]] - am * cc * PR[col[k][d]] + pm * (FR[k] - FL[k])) * inv;
}

// The transport update of one cell (all groups) from the state (N, F):
// U*_i = U_i + lam sum_d (flux(i - 1/2) - flux(i + 1/2)), the flux of eq.
// (e:glf) or, with HLLF, the HLL flux; then, unless NOLIMIT, the floor and
// the limiter (counted in nlim, nneg).
template <int G, typename R, bool NOLIMIT, bool HLLF>
__device__ inline void cell_transport(const R *__restrict__ N, const R *__restrict__ F, const Grid &gr, R c,
                                      R lam, const Bounds<R> &bnd, int64_t i, R (&us)[G][4], int64_t &nlim,
                                      int64_t &nneg) {
    const int x = (int)(i % gr.nx);
    const int y = (int)((i / gr.nx) % gr.ny);
    const int z = (int)(i / ((int64_t)gr.nx * gr.ny));
    const int64_t V = gr.V;
    const Nbrs nb = neighbours(gr, bnd, i, x, y, z);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const R *Ng = N + (int64_t)g * V;
        const R *Fg = F + (int64_t)g * 3 * V;
        const R Ni = Ng[i];
        const R Fi[3] = {Fg[i], Fg[V + i], Fg[2 * V + i]};
        R Pi[6];
        m1_pressure(Ni, Fi[0], Fi[1], Fi[2], c, Pi);
        R acc[4] = {R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t im = nb.idx[d][0], ip = nb.idx[d][1];
            R Nm = Ng[im], Np = Ng[ip];
            R Fm[3] = {Fg[im], Fg[V + im], Fg[2 * V + im]};
            R Fp[3] = {Fg[ip], Fg[V + ip], Fg[2 * V + ip]};
            if (nb.face[d][0] >= 0) ghost(bnd, nb.face[d][0], g, c, Nm, Fm);
            if (nb.face[d][1] >= 0) ghost(bnd, nb.face[d][1], g, c, Np, Fp);
            R Pm[6], Pp[6];
            m1_pressure(Nm, Fm[0], Fm[1], Fm[2], c, Pm);
            m1_pressure(Np, Fp[0], Fp[1], Fp[2], c, Pp);
            R lo[4], hi[4];
            if (HLLF) {
                hll(Nm, Fm, Pm, Ni, Fi, Pi, d, c, lo);
                hll(Ni, Fi, Pi, Np, Fp, Pp, d, c, hi);
            } else {
                glf(Nm, Fm, Pm, Ni, Fi, Pi, d, c, lo);
                glf(Ni, Fi, Pi, Np, Fp, Pp, d, c, hi);
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) acc[k] += lo[k] - hi[k];
        }
        R n = Ni + lam * acc[0];
        R f[3] = {Fi[0] + lam * acc[1], Fi[1] + lam * acc[2], Fi[2] + lam * acc[3]};
        if (!NOLIMIT) {
            const int taken = floor_limit_fwd(n, f[0], f[1], f[2], c);
            nneg += taken & 1;
            nlim += taken >> 1;
        }
        us[g][0] = n;
        us[g][1] = f[0];
        us[g][2] = f[1];
        us[g][3] = f[2];
    }
}

// NOLIMIT = true skips the floor and limiter (the adjoint needs the values
// before them).  HLLF selects the HLL flux instead of eq. (e:glf).
template <int G, typename R, bool DIAG, bool NOLIMIT = false, bool HLLF = false>
__global__ __launch_bounds__(256) void k_transport(const R *__restrict__ N, const R *__restrict__ F,
                                                   R *__restrict__ Ns, R *__restrict__ Fs, Grid gr,
                                                   R c, R lam, unsigned long long *cnt, Bounds<R> bnd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t nlim = 0, nneg = 0;
    if (i < gr.V) {
        const int64_t V = gr.V;
        R us[G][4];
        cell_transport<G, R, NOLIMIT, HLLF>(N, F, gr, c, lam, bnd, i, us, nlim, nneg);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            Ns[(int64_t)g * V + i] = us[g][0];
#pragma unroll
            for (int k = 0; k < 3; ++k) Fs[(int64_t)(3 * g + k) * V + i] = us[g][1 + k];
        }
    }
    if (DIAG) {
        wave_count(cnt, CNT_LIMITER, nlim);
        wave_count(cnt, CNT_NEG, nneg);
    }
}

// ---------------------------------------------------------------- chemistry
// Work list of cells whose subcycle did not finish within the first pass's
// substep budget.  Most cells need one or two substeps; the few heated cells
// near the sources need tens to hundreds, and in place they would hold their
// whole wave for that long.  They are finished by a second, persistent pass
// over the compacted list (same code, same inputs, same results).
#ifndef EMMA_CHEM_BUDGET
#define EMMA_CHEM_BUDGET 3
#endif
#ifndef EMMA_CHEM_BUDGET_FUSED
#define EMMA_CHEM_BUDGET_FUSED 2
#endif
constexpr int kChemBudget = EMMA_CHEM_BUDGET;
constexpr int kChemBudgetFused = EMMA_CHEM_BUDGET_FUSED;
// Total substeps after which the second pass hands a cell on to the
// cooperative pass (0: no cooperative pass).
#ifndef EMMA_CONT_BUDGET
#define EMMA_CONT_BUDGET 16
#endif
constexpr int kContBudget = EMMA_CONT_BUDGET;

struct WorkList {
    uint32_t *count;  // [1], reset before every first pass
    uint32_t *cells;  // [V]
};

// Appends cell i for every lane with defer set: one atomic per wave.
// Returns the lane's slot in the list (meaningless where defer is not set).
__device__ inline uint32_t defer_slot(const WorkList &wl, bool defer, uint32_t i) {
    const unsigned long long m = __ballot(defer);
    if (m == 0) return 0;
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (lane == __ffsll((long long)m) - 1) base = atomicAdd(wl.count, (uint32_t)__popcll(m));
    base = __shfl(base, __ffsll((long long)m) - 1, 64);
    const uint32_t k = base + __popcll(m & ((1ull << lane) - 1ull));
    if (defer) wl.cells[k] = i;
    return k;
}

__device__ inline void defer_push(const WorkList &wl, bool defer, uint32_t i) { (void)defer_slot(wl, defer, i); }

// Subcycle states of the cells the first pass stopped, by work-list slot
// (structure of arrays, so the second pass reads them coalesced).  Slots at
// or beyond cap have no state: the first pass finishes those cells itself.
struct ContBuf {
    double *N, *Pf;       // [G][cap]
    double *x, *e, *rem;  // [cap]
    int32_t *st;          // [4][cap]: substeps, attempts, cap, xclamp
    uint32_t *next;       // [cap]: slots the second pass hands on to the cooperative
                          // pass (their count at WorkList::count[1])
    uint32_t cap;
};

// Appends v for every lane with push set to list (count at *count): one
// atomic per wave.
__device__ inline void list_push(uint32_t *count, uint32_t *list, bool push, uint32_t v) {
    const unsigned long long m = __ballot(push);
    if (m == 0) return;
    const int lane = threadIdx.x & 63;
    const int first = __ffsll((long long)m) - 1;
    uint32_t base = 0;
    if (lane == first) base = atomicAdd(count, (uint32_t)__popcll(m));
    base = __shfl(base, first, 64);
    if (push) list[base + __popcll(m & ((1ull << lane) - 1ull))] = v;
}

template <int G>
__device__ __forceinline__ void cont_save(const ContBuf &cb, uint32_t k, const SubState<G> &s) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        cb.N[(size_t)g * cb.cap + k] = s.N[g];
        cb.Pf[(size_t)g * cb.cap + k] = s.Pf[g];
    }
    cb.x[k] = s.x;
    cb.e[k] = s.e;
    cb.rem[k] = s.rem;
    cb.st[k] = s.st.substeps;
    cb.st[(size_t)cb.cap + k] = s.st.attempts;
    cb.st[2 * (size_t)cb.cap + k] = s.st.cap;
    cb.st[3 * (size_t)cb.cap + k] = s.st.xclamp;
}

template <int G>
__device__ __forceinline__ void cont_load(const ContBuf &cb, uint32_t k, SubState<G> &s) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        s.N[g] = cb.N[(size_t)g * cb.cap + k];
        s.Pf[g] = cb.Pf[(size_t)g * cb.cap + k];
    }
    s.x = cb.x[k];
    s.e = cb.e[k];
    s.rem = cb.rem[k];
    s.st.substeps = cb.st[k];
    s.st.attempts = cb.st[(size_t)cb.cap + k];
    s.st.cap = cb.st[2 * (size_t)cb.cap + k];
    s.st.xclamp = cb.st[3 * (size_t)cb.cap + k];
}

// The first chemistry pass touches every element exactly once per step: its
// loads and stores are non-temporal (streamed past the caches).  F enters the
// subcycle only through the product of the substeps' factors, so it is read
// after the subcycle, which keeps it out of the registers the subcycle needs.
#ifndef EMMA_CHEM_MIN_BLOCKS
#define EMMA_CHEM_MIN_BLOCKS 1
#endif
// Threads per block of the first chemistry pass.  With FP32 storage, one
// wave: its waves run for different times (one substep or several); a
// one-wave block reuses the slot of a wave that finished early at once, where
// a four-wave block has to wait for room for all four (measured at 256^3:
// 0.507 ms against 0.574 ms with 256 threads, 0.514 ms with 128).  The FP64
// variant measured the other way (0.730 ms with 64 threads against 0.694 ms
// with 256) and keeps four-wave blocks.
#ifndef EMMA_CHEM_TB
#define EMMA_CHEM_TB 64
#endif
#ifndef EMMA_CHEM_TB_FP64
#define EMMA_CHEM_TB_FP64 256
#endif
template <typename S> constexpr int chem_tb() { return sizeof(S) == 4 ? EMMA_CHEM_TB : EMMA_CHEM_TB_FP64; }

template <typename T>
__device__ __forceinline__ T stream_ld(const T *p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void stream_st(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}

// One thread per cell: reads the post-transport N*, F* (storage type S), the
// gas state (x, T) and the cell's source density; writes the end-of-step N,
// F, x, T (in place, or into xo, To with TAPE).
// A cell still short of dt after kChemBudget substeps stops there: its
// subcycle state goes to the continuation buffer at its work-list slot and
// k_chem_cont finishes it (nothing written here); without a free slot it
// finishes here.  F_out = F* Pf with Pf the product of the substeps' factors.
// TAPE (the adjoint's segment forward): Ns, Fs hold the transport output
// before the floor and the limiter, which are applied here with the
// transport's own function (same bits as the step); x, T are only read and
// the results go to the distinct arrays xo, To; with multi, one bit per cell
// (one 64-bit word per wave of 64 consecutive cells), set unless the subcycle
// was a single accepted substep.
template <int G, typename S, bool DIAG, bool FAST, bool TAPE = false>
__global__ __launch_bounds__(chem_tb<S>(), EMMA_CHEM_MIN_BLOCKS) void k_chem(
    const S *__restrict__ Ns, const S *__restrict__ Fs, S *__restrict__ N, S *__restrict__ F,
    double *__restrict__ x, double *__restrict__ T, double *__restrict__ xo, double *__restrict__ To,
    const double *__restrict__ n0, int64_t V, SrcTable src, GroupConsts gc, ChemParams cp,
    unsigned long long *cnt, WorkList wl, ContBuf cb, const uint32_t *__restrict__ skip,
    uint64_t *__restrict__ multi) {
    double *__restrict__ xw = TAPE ? xo : x;
    double *__restrict__ Tw = TAPE ? To : T;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    SubState<G> s;
    s.st = ChemStats{0, 0, 0, 0};
    bool stopped = false, done = false;
    // skip: one bit per cell, set for the refined cells whose children run
    // the chemistry instead (null: every cell)
    const bool mine = i < V && !(skip && ((skip[i >> 5] >> (i & 31)) & 1u));
    double n0c = 0.0, Tc = 0.0, Sc[G];
    if (mine) {
        double Nc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            S n = stream_ld(Ns + (int64_t)g * V + i);
            if (TAPE && n < S(0)) n = S(0);  // the floor (the limiter leaves N alone)
            Nc[g] = (double)n;
        }
        // the gas state is loaded before the source lookup branches, so that
        // all of the cell's loads are in flight together
        const double xc = stream_ld(x + i);
        Tc = stream_ld(T + i);
        n0c = stream_ld(n0 + i);
        source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
        sub_start<G>(s, cp, Nc, xc, Tc, n0c);
        stopped = !sub_run<G, FAST>(s, gc, cp, n0c, Tc, Sc, kChemBudget);
    }
    const uint32_t k = defer_slot(wl, stopped, (uint32_t)i);
    if (stopped) {
        if (k < cb.cap) cont_save<G>(cb, k, s);
        else stopped = !sub_run<G, FAST>(s, gc, cp, n0c, Tc, Sc, 0x7fffffff);  // no slot: finish here
    }
    if (mine && !stopped) {
#pragma unroll
        for (int g = 0; g < G; ++g) {
            stream_st(N + (int64_t)g * V + i, (S)s.N[g]);
            S f[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) f[c] = stream_ld(Fs + ((int64_t)g * 3 + c) * V + i);
            if (TAPE) {
                S n = stream_ld(Ns + (int64_t)g * V + i);
                floor_limit_fwd<S>(n, f[0], f[1], f[2], (S)cp.c);
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) stream_st(F + ((int64_t)g * 3 + c) * V + i, (S)((double)f[c] * s.Pf[g]));
        }
        stream_st(xw + i, s.x);
        stream_st(Tw + i, sub_T<G, FAST>(s, cp, n0c, Tc));
        done = true;
    }
    if (TAPE && multi) {
        const unsigned long long m = __ballot(mine && !(done && s.st.substeps == 1));
        if ((threadIdx.x & 63) == 0) multi[i >> 6] = m;
    }
    if (stopped) s.st = ChemStats{0, 0, 0, 0};  // counted by the continuation pass
    if (DIAG) {
        wave_count(cnt, CNT_SUB, s.st.substeps);
        wave_count(cnt, CNT_ATT, s.st.attempts);
        wave_count(cnt, CNT_CAP, s.st.cap);
        wave_count(cnt, CNT_XCLAMP, s.st.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, s.st.substeps);
        wave_hist(cnt, done, s.st.substeps);
    }
}

// Second pass of the split path: continues the subcycles the first pass
// stopped, from their saved states (list slots below the buffer's capacity),
// grid-stride over the list.  T: the step's input temperature (used in the
// isothermal mode); writes N, F, xo, To of those cells.  TAPE: Ns, Fs are
// the transport output before the floor and the limiter, as in k_chem (Ns is
// read only then).
// The end of a continued cell's subcycle: N, F = F* Pf, x, T of cell i.
template <int G, typename S, bool FAST, bool TAPE>
__device__ __forceinline__ void cont_store(const S *Ns, const S *Fs, S *N, S *F, double *xo, double *To, int64_t V,
                                           int64_t i, const SubState<G> &s, const ChemParams &cp, double n0c,
                                           double Tc) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        N[(int64_t)g * V + i] = (S)s.N[g];
        S f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = Fs[((int64_t)g * 3 + c) * V + i];
        if (TAPE) {
            S n = Ns[(int64_t)g * V + i];
            floor_limit_fwd<S>(n, f[0], f[1], f[2], (S)cp.c);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) F[((int64_t)g * 3 + c) * V + i] = (S)((double)f[c] * s.Pf[g]);
    }
    xo[i] = s.x;
    To[i] = sub_T<G, FAST>(s, cp, n0c, Tc);
}

// budget: total accepted substeps after which a cell is handed on to the
// cooperative pass (its state back in its slot, the slot appended to cb.next).
template <int G, typename S, bool DIAG, bool FAST, bool TAPE = false>
__global__ __launch_bounds__(256) void k_chem_cont(const S *Ns, const S *Fs, S *N, S *F, const double *T, double *xo, double *To,
                                                   const double *__restrict__ n0, int64_t V, SrcTable src,
                                                   GroupConsts gc, ChemParams cp, unsigned long long *cnt,
                                                   WorkList wl, ContBuf cb, int budget) {
    const uint32_t n = min(*wl.count, cb.cap);
    const uint32_t stride = gridDim.x * blockDim.x;
    ChemStats tot{0, 0, 0, 0};
    int maxsub = 0;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int64_t i = wl.cells[k];
        SubState<G> s;
        cont_load<G>(cb, k, s);
        double Sc[G];
        source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
        const double n0c = n0[i], Tc = T[i];
        const bool handed = !sub_run<G, FAST>(s, gc, cp, n0c, Tc, Sc, budget);
        if (handed) cont_save<G>(cb, k, s);
        list_push(wl.count + 1, cb.next, handed, k);
        if (handed) continue;  // counted by the cooperative pass
        cont_store<G, S, FAST, TAPE>(Ns, Fs, N, F, xo, To, V, i, s, cp, n0c, Tc);
        if (DIAG) {
            tot.substeps += s.st.substeps;
            tot.attempts += s.st.attempts;
            tot.cap += s.st.cap;
            tot.xclamp += s.st.xclamp;
            maxsub = max(maxsub, s.st.substeps);
            atomicAdd(cnt_slot(cnt) + CNT_HIST + substep_bin(s.st.substeps), 1ull);
        }
    }
    if (DIAG) {
        wave_count(cnt, CNT_SUB, tot.substeps);
        wave_count(cnt, CNT_ATT, tot.attempts);
        wave_count(cnt, CNT_CAP, tot.cap);
        wave_count(cnt, CNT_XCLAMP, tot.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, maxsub);
    }
}

// ------------------------------------------------ cooperative long subcycles
// The cells still short of dt after the second pass's budget (the heated
// cells near the sources, up to ~100 substeps) are each one dependent chain:
// a wave holding them runs for the longest one, alone on its SIMD, so the
// chain's latency is the pass's time.  Here kCoopLanes lanes share a cell:
// the rate fits of a substep are evaluated side by side (lane q of each quad
// takes fit q, the four fits having one form, P exp(pre + a L - d ln(1 +
// exp(c (L - ln b))))) and the attempts of the 10 % rule are tried side by
// side (lane j with the first step halved j times, then 8 + j, ...), the
// first accepted one kept.  Every lane runs the arithmetic of the per-cell
// code on the same inputs, so the results (and the substep and attempt
// counts) are the ones the per-cell subcycle would give.  On-the-spot,
// energy-evolving mode only.
constexpr int kCoopLanes = 8;

// lane (q & 3) of a quad's value to every lane of the quad
template <int Q>
__device__ __forceinline__ double quad_bcast(double v) {
    constexpr int ctrl = Q * 0x55;  // quad_perm [Q, Q, Q, Q]
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), ctrl, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), ctrl, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

// rates_at<true>(T), each quad evaluating its four fits side by side
__device__ __forceinline__ RateSet rates_coop(double T) {
    const double invT = recip_fp64(T);
    const double lam = 2.0 * kTHI * invT;
    const double L = log_fp64(lam);
    const double lnT = 12.662275226919286 - L;  // ln(2 T_HI) - L
    const double sT = sqrt(T);
    const int q = threadIdx.x & 3;
    // 0: alpha_B, 1: recombination cooling, 2: collisional ionisation, 3:
    // collisional excitation (a = d = c = 0: the fit part is exactly zero)
    const double P = q == 0 ? 2.753e-14 : q == 1 ? 3.435e-30 * T : q == 2 ? 21.11 : 7.5e-19;
    const double pre = q <= 1 ? -0.0 : q == 2 ? beta_pre(lnT, lam) : -118348.0 * invT;
    const double a = q == 0 ? 1.500 : q == 1 ? 1.970 : q == 2 ? -1.089 : 0.0;
    const double lnb = q == 0 ? 1.007957920399979 : q == 1 ? 0.8109302162163288 : q == 2 ? -1.0384583658483626 : 0.0;
    const double c = q == 0 ? 0.407 : q == 1 ? 0.376 : q == 2 ? 0.874 : 0.0;
    const double d = q == 0 ? 2.242 : q == 1 ? 3.720 : q == 2 ? 1.101 : 0.0;
    const double R = recip_fp64(1.0 + sT * 0.003162277660168379);
    const double v = P * exp_fp64(pre + hg_fit(L, a, lnb, c, d)) * (q == 3 ? R : 1.0);
    RateSet r;
    r.alpha = quad_bcast<0>(v);
    r.dalpha = 0.0;
    r.crec = quad_bcast<1>(v);
    r.beta = quad_bcast<2>(v);
    r.cci = kKB * kTHI * r.beta;
    r.cce = quad_bcast<3>(v);
    r.cff = 1.42e-27 * 1.3 * sT;
    return r;
}

// substep<G, true> with the rates and the attempts shared by the lanes of a
// group (every lane of the group holds the same cell state and ends with the
// same new state)
template <int G>
__device__ __forceinline__ bool substep_coop(const GroupConsts &gc, const ChemParams &p, bool last, double n0,
                                             double eunit, const double (&S)[G], double (&N)[G], double &x,
                                             double &e, double &rem, double (&inv)[G], ChemStats &st) {
    const double c = p.c;
    if (!(e > 0.0 && e < HUGE_VAL)) return false;  // invalid input: leave the cell
    const double Tp = e * recip_fp64(eunit * (1.0 + x));
    const RateSet r = rates_coop(Tp);
    double D;
    int branch;
    const double dtau0 = first_dtau<G>(gc, c, false, last, n0, r, N, x, e, rem, D, branch);
    const int j = threadIdx.x & (kCoopLanes - 1);
    const int base = (threadIdx.x & 63) & ~(kCoopLanes - 1);
    double Nn[G], In[G], xn, en;
    int xcl, k = 0, src = 0, flags = 0;
    // ends by round kMaxHalvings / kCoopLanes at the latest: the attempt with
    // kMaxHalvings halvings is taken whether or not it passes (as substep())
    for (int round = 0;; ++round) {
        // the attempt with the first step halved k times (exact: a power of 2)
        k = kCoopLanes * round + j;
        attempt<G>(gc, c, false, n0, r, S, N, x, e, ldexp(dtau0, -k), Nn, In, xn, en, xcl);
        const bool pass = fabs(en - e) <= 0.1 * e;
        const bool take = k <= kMaxHalvings && (last ? k == 0 : (pass || k == kMaxHalvings));
        const unsigned m = (unsigned)(__ballot(take) >> base) & ((1u << kCoopLanes) - 1u);
        if (m) {
            src = base + __ffs(m) - 1;
            flags = (xcl != 0) | ((!last && !pass) ? 2 : 0);  // clamp; cap reached without passing
            break;
        }
    }
    k = __shfl(k, src, 64);
    flags = __shfl(flags, src, 64);
#pragma unroll
    for (int g = 0; g < G; ++g) {
        N[g] = __shfl(Nn[g], src, 64);
        inv[g] = __shfl(In[g], src, 64);
    }
    x = __shfl(xn, src, 64);
    e = __shfl(en, src, 64);
    st.attempts += k + 1;
    if (flags & 2) st.cap = 1;
    if (flags & 1) st.xclamp++;
    rem = rem - ldexp(dtau0, -k);
    st.substeps++;
    return true;
}

// Third pass: the slots the second pass handed on, kCoopLanes lanes per
// cell, grid-stride.
template <int G, typename S, bool DIAG, bool TAPE = false>
__global__ __launch_bounds__(256) void k_chem_coop(const S *Ns, const S *Fs, S *N, S *F, const double *T,
                                                   double *xo, double *To, const double *__restrict__ n0, int64_t V,
                                                   SrcTable src, GroupConsts gc, ChemParams cp,
                                                   unsigned long long *cnt, WorkList wl, ContBuf cb) {
    const uint32_t n = wl.count[1];
    const uint32_t stride = gridDim.x * blockDim.x / kCoopLanes;
    const bool lead = (threadIdx.x & (kCoopLanes - 1)) == 0;
    ChemStats tot{0, 0, 0, 0};
    int maxsub = 0;
    for (uint32_t q = (blockIdx.x * blockDim.x + threadIdx.x) / kCoopLanes; q < n; q += stride) {
        const uint32_t k = cb.next[q];
        const int64_t i = wl.cells[k];
        SubState<G> s;
        cont_load<G>(cb, k, s);
        double Sc[G];
        source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
        const double n0c = n0[i], Tc = T[i];
        const double eunit = 1.5 * n0c * kKB;
        while (s.rem > 0.0) {
            const bool last = s.st.substeps >= cp.max_substeps;
            double inv[G];
            if (!substep_coop<G>(gc, cp, last, n0c, eunit, Sc, s.N, s.x, s.e, s.rem, inv, s.st)) break;
#pragma unroll
            for (int g = 0; g < G; ++g) s.Pf[g] *= inv[g];
            if (last) { s.st.cap = 1; break; }
        }
        if (lead) {
            cont_store<G, S, true, TAPE>(Ns, Fs, N, F, xo, To, V, i, s, cp, n0c, Tc);
            if (DIAG) {
                tot.substeps += s.st.substeps;
                tot.attempts += s.st.attempts;
                tot.cap += s.st.cap;
                tot.xclamp += s.st.xclamp;
                maxsub = max(maxsub, s.st.substeps);
                atomicAdd(cnt_slot(cnt) + CNT_HIST + substep_bin(s.st.substeps), 1ull);
            }
        }
    }
    if (DIAG) {
        wave_count(cnt, CNT_SUB, tot.substeps);
        wave_count(cnt, CNT_ATT, tot.attempts);
        wave_count(cnt, CNT_CAP, tot.cap);
        wave_count(cnt, CNT_XCLAMP, tot.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, maxsub);
    }
}

// Second pass: the deferred cells, whole subcycle, grid-stride over the list.
// Ns, Fs hold the post-transport values (they may alias N, F: each cell is
// read before it is written by the same thread).
template <int G, typename S, bool DIAG, bool FAST>
__global__ __launch_bounds__(256) void k_chem_list(const S *Ns, const S *Fs, S *N, S *F, double *__restrict__ x,
                                                   double *__restrict__ T, const double *__restrict__ n0,
                                                   int64_t V, SrcTable src, GroupConsts gc, ChemParams cp,
                                                   unsigned long long *cnt, WorkList wl) {
    const uint32_t n = *wl.count;
    const uint32_t stride = gridDim.x * blockDim.x;
    ChemStats tot{0, 0, 0, 0};
    int maxsub = 0;
    for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) {
        const int64_t i = wl.cells[k];
        double Nc[G], Fc[G][3], Sc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            Nc[g] = (double)Ns[(int64_t)g * V + i];
#pragma unroll
            for (int q = 0; q < 3; ++q) Fc[g][q] = (double)Fs[((int64_t)g * 3 + q) * V + i];
        }
        source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
        double xc = x[i], Tc = T[i];
        const ChemStats st = chem_cell<G, FAST>(gc, cp, Nc, Fc, xc, Tc, n0[i], Sc);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            N[(int64_t)g * V + i] = (S)Nc[g];
#pragma unroll
            for (int q = 0; q < 3; ++q) F[((int64_t)g * 3 + q) * V + i] = (S)Fc[g][q];
        }
        x[i] = xc;
        T[i] = Tc;
        if (DIAG) {
            tot.substeps += st.substeps;
            tot.attempts += st.attempts;
            tot.cap += st.cap;
            tot.xclamp += st.xclamp;
            maxsub = max(maxsub, st.substeps);
            // few cells reach this pass: one atomic each
            atomicAdd(cnt_slot(cnt) + CNT_HIST + substep_bin(st.substeps), 1ull);
        }
    }
    if (DIAG) {
        wave_count(cnt, CNT_SUB, tot.substeps);
        wave_count(cnt, CNT_ATT, tot.attempts);
        wave_count(cnt, CNT_CAP, tot.cap);
        wave_count(cnt, CNT_XCLAMP, tot.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, maxsub);
    }
}

// One-pass step of the fused path with the HLL flux: one thread per cell
// reads its radius-1 neighbourhood of (N, F), updates its own U* (all
// groups, the floor and the limiter), and runs the chemistry on it in the
// same thread, writing (No, Fo) and x, T in place; a subcycle longer than
// kChemBudgetFused substeps writes U* instead and goes to the work list,
// which k_chem_list finishes in place.  (The tiled fused kernels split the
// GLF flux into per-cell parts shared through LDS; the HLL flux needs both
// sides' states and speeds at every face, which this form reads from memory.)
template <int G, typename R, bool DIAG, bool FAST>
__global__ __launch_bounds__(256) void k_step_cell(const R *__restrict__ N, const R *__restrict__ F,
                                                   R *__restrict__ No, R *__restrict__ Fo, double *__restrict__ x,
                                                   double *__restrict__ T, const double *__restrict__ n0, Grid gr,
                                                   R c, R lam, SrcTable src, GroupConsts gc, ChemParams cp,
                                                   unsigned long long *cnt, WorkList wl, Bounds<R> bnd) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t V = gr.V;
    int64_t nlim = 0, nneg = 0;
    bool deferred = false, done = false;
    ChemStats cs{0, 0, 0, 0};
    if (i < V) {
        R us[G][4];
        cell_transport<G, R, false, true>(N, F, gr, c, lam, bnd, i, us, nlim, nneg);
        double Nc[G], Pf[G], Sc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) Nc[g] = (double)us[g][0];
        source_of<G>(i, src.mask, src.sorted_cell, src.S, src.n, Sc);
        double xc = x[i], Tc = T[i];
        cs = chem_cell_nxt<G, FAST>(gc, cp, Nc, Pf, xc, Tc, n0[i], Sc, kChemBudgetFused, &deferred);
        if (!deferred) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                us[g][0] = (R)Nc[g];
#pragma unroll
                for (int k = 1; k < 4; ++k) us[g][k] = (R)((double)us[g][k] * Pf[g]);
            }
            x[i] = xc;
            T[i] = Tc;
            done = true;
        } else {
            cs = ChemStats{0, 0, 0, 0};  // counted by k_chem_list
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            No[(int64_t)g * V + i] = us[g][0];
#pragma unroll
            for (int k = 0; k < 3; ++k) Fo[(int64_t)(3 * g + k) * V + i] = us[g][1 + k];
        }
    }
    defer_push(wl, deferred, (uint32_t)i);
    if (DIAG) {
        wave_count(cnt, CNT_LIMITER, nlim);
        wave_count(cnt, CNT_NEG, nneg);
        wave_count(cnt, CNT_SUB, cs.substeps);
        wave_count(cnt, CNT_ATT, cs.attempts);
        wave_count(cnt, CNT_CAP, cs.cap);
        wave_count(cnt, CNT_XCLAMP, cs.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, cs.substeps);
        wave_hist(cnt, done, cs.substeps);
    }
}

// -------------------------------------------------------------- diagnostics
// Per-block partial sums of N (per group) and x n0, plus the non-finite count;
// the partials are summed in block order by k_diag_final (deterministic).
template <int G, typename S>
__global__ __launch_bounds__(256) void k_diag_partial(const S *N, const S *F, const double *x,
                                                      const double *T, const double *n0, int64_t V,
                                                      double *partial, unsigned long long *cnt) {
    __shared__ double sh[G + 1][256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[G + 1];
#pragma unroll
    for (int q = 0; q < G + 1; ++q) v[q] = 0.0;
    int64_t bad = 0;
    if (i < V) {
        bool fin = isfinite(x[i]) && isfinite(T[i]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double n = (double)N[(int64_t)g * V + i];
            v[g] = n;
            fin = fin && isfinite(n);
#pragma unroll
            for (int k = 0; k < 3; ++k) fin = fin && isfinite((double)F[((int64_t)g * 3 + k) * V + i]);
        }
        v[G] = x[i] * n0[i];
        bad = fin ? 0 : 1;
    }
    wave_count(cnt, CNT_NONFINITE, bad);
#pragma unroll
    for (int q = 0; q < G + 1; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < G + 1; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < G + 1; ++q) partial[(int64_t)blockIdx.x * (G + 1) + q] = sh[q][0];
    }
}

// ------------------------------------------------- refined cells (Sec. 5)
// The coarse radiative transport approximation with static refinement: the
// transport runs on the coarse grid only; a refined coarse cell carries
// NC = r^3 children with their own gas, whose chemistry runs with the
// parent's post-transport radiation injected (piecewise constant); the
// parent then holds the children's mean N, F, the n0-weighted mean x and the
// (1 + x) n0-weighted mean T (its photons, ionised atoms and internal energy
// are the children's).  Means are pairwise sums over the children in index
// order, ((c0 + c1) + (c2 + c3)) + ..., so equal children give the parent
// exactly.

// Marks the refined cells in a one-bit-per-cell mask (cleared beforehand);
// entries outside the grid or repeated are counted and ignored.
__global__ void k_mark_refined(const int64_t *__restrict__ cell, int n, int64_t V, uint32_t *mask,
                               unsigned long long *cnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    int64_t bad = 0;
    if (j < n) {
        const int64_t p = cell[j];
        if (p < 0 || p >= V) {
            bad = 1;
        } else {
            const uint32_t bit = 1u << (p & 31);
            if (atomicOr(mask + (p >> 5), bit) & bit) bad = 1;
        }
    }
    wave_count(cnt, CNT_BADREF, bad);
}

// Pairwise sum over the NC consecutive lanes of one parent (NC divides 64):
// after the step with mask m each lane holds the sum of its aligned block of
// 2m lanes, added as (lower half) + (upper half) up to commutation.
template <int NC>
__device__ __forceinline__ double child_sum(double v) {
#pragma unroll
    for (int m = 1; m < NC; m <<= 1) v += __shfl_xor(v, m);
    return v;
}

// One lane per child: chemistry on the injected radiation, then the
// restriction; lane 0 of each parent writes the parent.  Children's sources:
// the parent's sources (sorted table, list order) whose child index is this
// lane's, at rate * frac / volf, volf = (dx / r)^3.  The children's state is
// read from (xfi, Tfi) and written to (xf, Tf), which may be the same arrays.
// TAPE (the adjoint's segment forward): Ns, Fs are the transport output before
// the floor and the limiter, applied here to the parent's values with the
// transport's own function.
template <int G, typename S, bool DIAG, bool FAST, int NC, bool TAPE = false>
__global__ __launch_bounds__(256) void k_crta_fine(const S *__restrict__ Ns, const S *__restrict__ Fs,
                                                   S *__restrict__ N, S *__restrict__ F, double *__restrict__ x,
                                                   double *__restrict__ T, int64_t V,
                                                   const int64_t *__restrict__ ref_cell, int n_ref,
                                                   const double *xfi, const double *Tfi, double *xf, double *Tf,
                                                   const double *__restrict__ nf,
                                                   const int64_t *__restrict__ sorted_cell,
                                                   const int32_t *__restrict__ sorted_idx,
                                                   const double *__restrict__ rate,
                                                   const int32_t *__restrict__ src_child, int n_src,
                                                   GroupConsts gc, ChemParams cp, double volf,
                                                   unsigned long long *cnt) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t j = t / NC;
    const int ch = (int)(t % NC);
    ChemStats st{0, 0, 0, 0};
    int64_t bad = 0;
    const int64_t p = j < n_ref ? ref_cell[j] : -1;
    // every lane of a parent agrees on `live`, so the sums stay inside live lanes
    if (p >= 0 && p < V) {
        double Nc[G], Fc[G][3], Sc[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            S n = Ns[(int64_t)g * V + p];
            S fv[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) fv[k] = Fs[((int64_t)g * 3 + k) * V + p];
            if (TAPE) floor_limit_fwd<S>(n, fv[0], fv[1], fv[2], (S)cp.c);
            Nc[g] = (double)n;
#pragma unroll
            for (int k = 0; k < 3; ++k) Fc[g][k] = (double)fv[k];
            Sc[g] = 0.0;
        }
        if (n_src > 0) {
            for (int r = lower_bound_cell(sorted_cell, n_src, p); r < n_src && sorted_cell[r] == p; ++r) {
                const int s = sorted_idx[r];
                const int sc = src_child ? src_child[s] : 0;
                if (sc == ch) {
#pragma unroll
                    for (int g = 0; g < G; ++g) Sc[g] += rate[s] * gc.frac[g] / volf;
                }
                if (ch == 0 && (sc < 0 || sc >= NC)) bad++;
            }
        }
        const int64_t f = j * NC + ch;
        double xc = xfi[f], Tc = Tfi[f];
        const double nc = nf[f];
        st = chem_cell<G, FAST>(gc, cp, Nc, Fc, xc, Tc, nc, Sc);
        xf[f] = xc;
        Tf[f] = Tc;
        const double inv = 1.0 / NC;
        double No[G], Fo[G][3];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            No[g] = child_sum<NC>(Nc[g]) * inv;
#pragma unroll
            for (int k = 0; k < 3; ++k) Fo[g][k] = child_sum<NC>(Fc[g][k]) * inv;
        }
        const double nsum = child_sum<NC>(nc);
        const double xp = child_sum<NC>(xc * (nc / nsum));
        const double w = (1.0 + xc) * nc;
        const double msum = child_sum<NC>(w);
        const double Tp = child_sum<NC>(Tc * (w / msum));
        if (ch == 0) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                N[(int64_t)g * V + p] = (S)No[g];
#pragma unroll
                for (int k = 0; k < 3; ++k) F[((int64_t)g * 3 + k) * V + p] = (S)Fo[g][k];
            }
            x[p] = xp;
            T[p] = Tp;
        }
    }
    wave_count(cnt, CNT_BADREF, bad);
    if (DIAG) {
        wave_count(cnt, CNT_SUB, st.substeps);
        wave_count(cnt, CNT_ATT, st.attempts);
        wave_count(cnt, CNT_CAP, st.cap);
        wave_count(cnt, CNT_XCLAMP, st.xclamp);
        wave_count_max(cnt, CNT_MAXSUB, st.substeps);
        wave_hist(cnt, p >= 0 && p < V, st.substeps);
    }
}

template <int G>
__global__ __launch_bounds__(256) void k_diag_final(const double *partial, int nblk, double *out) {
    __shared__ double sh[G + 1][256];
    double v[G + 1];
#pragma unroll
    for (int q = 0; q < G + 1; ++q) v[q] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) {
#pragma unroll
        for (int q = 0; q < G + 1; ++q) v[q] += partial[(int64_t)b * (G + 1) + q];
    }
#pragma unroll
    for (int q = 0; q < G + 1; ++q) sh[q][threadIdx.x] = v[q];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
#pragma unroll
            for (int q = 0; q < G + 1; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
#pragma unroll
        for (int q = 0; q < G + 1; ++q) out[q] = sh[q][0];
    }
}

}  // namespace emma
