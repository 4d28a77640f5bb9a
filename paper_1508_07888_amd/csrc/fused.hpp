// fused.hpp -- z-marching, LDS-tiled M1 transport with an optional fused
// chemistry epilogue (one pass over HBM per step).
//
// The face flux of eq. (e:glf) splits into a part carried by each side:
//   flux(i+1/2) = A_d(U_i) - B_d(U_{i+1}),  A_d(U) = (Ft_d(U) + c U)/2,
//   B_d(U) = (c U - Ft_d(U))/2,  Ft_d(U) = (F_d, c^2 P_.d),
// so the conservative update of eq. (e:uprt), 3D unsplit, is
//   U* = U + (dt/dx) [ sum_d A_d(U_{i-e_d}) + B_d(U_{i+e_d}) - 3 c U_i ].
// Each cell's closure P(U) is computed once per step by the thread that owns
// its column (halo cells once more by the block that needs them); x/y
// neighbours are exchanged through LDS, z neighbours stay in registers while
// the block marches up its column chunk.
//
// Block: 64 x 4 threads own a 64 x 4 column tile and march over LZ planes.
// Blocks are numbered so that each XCD (blocks are dealt round-robin to the 8
// XCDs) receives a contiguous run of tiles: a tile's y neighbours are then
// processed on the same XCD at about the same time and their shared rows hit
// that XCD's L2.
//
// Global accesses use one uniform base pointer per (group, component) array
// and a 32-bit per-thread byte offset (< 4 GiB per array), so addresses are
// formed by the scalar unit.
#pragma once

#include "kernels.hpp"

namespace emma {

constexpr int kTX = 64;
constexpr int kTY = 4;
constexpr int kLX = kTX + 2;
constexpr int kLY = kTY + 2;

template <typename R> struct TileArgs {
    const R *N, *F;
    R *No, *Fo;
    double *x, *T;
    const double *n0;
    Grid gr;
    int ntx, nty, ntz, LZ;
    R c, lam;
    SrcTable src;
    GroupConsts gc;
    ChemParams cp;
    unsigned long long *cnt;
    WorkList wl;
};

// Physical tile of block b when the hardware deals blocks to 8 XCDs
// round-robin: XCD k gets the logical range [k*q + min(k, r), ...).
__device__ inline int xcd_tile(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int k = b & 7, i = b >> 3;
    return k * q + (k < r ? k : r) + i;
}

template <typename R> struct alignas(4 * sizeof(R) > 16 ? 16 : 4 * sizeof(R)) Vec4 {
    R n, fx, fy, fz;
};

template <typename T>
__device__ __forceinline__ T ld(const T *base, uint32_t byte_off) {
    return *(const T *)((const char *)base + byte_off);
}
template <typename T>
__device__ __forceinline__ void st(T *base, uint32_t byte_off, T v) {
    *(T *)((char *)base + byte_off) = v;
}

template <int G, typename R>
__device__ __forceinline__ void load_cell(const R *__restrict__ N, const R *__restrict__ F, int64_t V,
                                          uint32_t off, Vec4<R> (&u)[G]) {
#pragma unroll
    for (int g = 0; g < G; ++g) {
        u[g].n = ld(N + (int64_t)g * V, off);
        u[g].fx = ld(F + (int64_t)(3 * g + 0) * V, off);
        u[g].fy = ld(F + (int64_t)(3 * g + 1) * V, off);
        u[g].fz = ld(F + (int64_t)(3 * g + 2) * V, off);
    }
}

// A_z and B_z parts (times 2) of one state with its closure.
template <typename R>
__device__ __forceinline__ Vec4<R> az2(const Vec4<R> &u, const R P[6], R c) {
    return Vec4<R>{u.fz + c * u.n, c * c * P[2] + c * u.fx, c * c * P[4] + c * u.fy, c * c * P[5] + c * u.fz};
}
template <typename R>
__device__ __forceinline__ Vec4<R> bz2(const Vec4<R> &u, const R P[6], R c) {
    return Vec4<R>{c * u.n - u.fz, c * u.fx - c * c * P[2], c * u.fy - c * c * P[4], c * u.fz - c * c * P[5]};
}

template <int G, typename R, bool DIAG, bool FUSE, bool FAST>
__global__ __launch_bounds__(256) void k_tiled(TileArgs<R> a) {
    // plane z of the current group: state, (Pxx, Pxy, Pxz, Pyy) and Pyz, double-buffered
    __shared__ Vec4<R> ldsU[2][kLY][kLX];
    __shared__ Vec4<R> ldsP[2][kLY][kLX];
    __shared__ R ldsQ[2][kLY][kLX];
    const int tid = threadIdx.x;
    const int tx = tid & (kTX - 1), ty = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tile_x = t % a.ntx, tile_y = (t / a.ntx) % a.nty, tile_z = t / (a.ntx * a.nty);
    const int nx = a.gr.nx, ny = a.gr.ny, nz = a.gr.nz;
    const int64_t V = a.gr.V;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int x0 = tile_x * kTX, y0 = tile_y * kTY, z0 = tile_z * a.LZ;
    const int z1 = min(z0 + a.LZ, nz);
    const int w = min(kTX, nx - x0), h = min(kTY, ny - y0);
    const bool active = tx < w && ty < h;
    const uint32_t col = active ? (uint32_t)(y0 + ty) * nx + (x0 + tx) : 0u;  // cell within a plane
    constexpr uint32_t E = sizeof(R);

    // halo role: bottom row, top row, left column, right column of the tile
    int hrole = -1, hlx = 0, hly = 0;
    uint32_t hcol = 0;
    if (tid < kTX) {
        if (tid < w) { hrole = 0; hlx = tid + 1; hly = 0; hcol = (uint32_t)((y0 + ny - 1) % ny) * nx + x0 + tid; }
    } else if (tid < 2 * kTX) {
        const int cx = tid - kTX;
        if (cx < w) { hrole = 1; hlx = cx + 1; hly = h + 1; hcol = (uint32_t)((y0 + h) % ny) * nx + x0 + cx; }
    } else if (tid < 2 * kTX + kTY) {
        const int cy = tid - 2 * kTX;
        if (cy < h) { hrole = 2; hlx = 0; hly = cy + 1; hcol = (uint32_t)(y0 + cy) * nx + (x0 + nx - 1) % nx; }
    } else if (tid < 2 * kTX + 2 * kTY) {
        const int cy = tid - 2 * kTX - kTY;
        if (cy < h) { hrole = 3; hlx = w + 1; hly = cy + 1; hcol = (uint32_t)(y0 + cy) * nx + (x0 + w) % nx; }
    }

    const R c = a.c, half = R(0.5);
    // rolling column window: cur = plane z, nxt = plane z+1, Az2 = 2 A_z(plane z-1)
    Vec4<R> cur[G], nxt[G], nn[G], hal[G], hnext[G], Az2[G];
    R Pc[G][6], Pn[G][6];
    int64_t nlim = 0, nneg = 0;
    ChemStats tot{0, 0, 0, 0};
    int maxsub = 0;

    auto zwrap = [nz](int z) { return (uint32_t)((z % nz + nz) % nz); };
    {
        const Vec4<R> zero{R(0), R(0), R(0), R(0)};
#pragma unroll
        for (int g = 0; g < G; ++g) { cur[g] = zero; nxt[g] = zero; hal[g] = zero; }
        Vec4<R> um[G];
#pragma unroll
        for (int g = 0; g < G; ++g) um[g] = zero;
        if (active) {
            load_cell<G>(a.N, a.F, V, (zwrap(z0 - 1) * plane + col) * E, um);
            load_cell<G>(a.N, a.F, V, ((uint32_t)z0 * plane + col) * E, cur);
            load_cell<G>(a.N, a.F, V, (zwrap(z0 + 1) * plane + col) * E, nxt);
        }
        if (hrole >= 0) load_cell<G>(a.N, a.F, V, ((uint32_t)z0 * plane + hcol) * E, hal);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            R Pm[6];
            m1_pressure(um[g].n, um[g].fx, um[g].fy, um[g].fz, c, Pm);
            Az2[g] = az2(um[g], Pm, c);
            m1_pressure(cur[g].n, cur[g].fx, cur[g].fy, cur[g].fz, c, Pc[g]);
            m1_pressure(nxt[g].n, nxt[g].fx, nxt[g].fy, nxt[g].fz, c, Pn[g]);
        }
    }

    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        // prefetch: own column two planes up, halo one plane up, gas state of plane z
        const uint32_t zc = (uint32_t)z * plane + col;
        if (active) load_cell<G>(a.N, a.F, V, (zwrap(z + 2) * plane + col) * E, nn);
        if (hrole >= 0 && z + 1 < z1) load_cell<G>(a.N, a.F, V, ((uint32_t)(z + 1) * plane + hcol) * E, hnext);
        double xg = 0.0, Tg = 0.0, n0g = 0.0;
        if (FUSE && active) {
            xg = ld(a.x, zc * 8u);
            Tg = ld(a.T, zc * 8u);
            n0g = ld(a.n0, zc * 8u);
        }

        Vec4<R> us[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            // publish plane z of group g: own cell and halo cell
            if (active) {
                ldsU[buf][ty + 1][tx + 1] = cur[g];
                ldsP[buf][ty + 1][tx + 1] = Vec4<R>{Pc[g][0], Pc[g][1], Pc[g][2], Pc[g][3]};
                ldsQ[buf][ty + 1][tx + 1] = Pc[g][4];
            }
            if (hrole >= 0) {
                R Ph[6];
                m1_pressure(hal[g].n, hal[g].fx, hal[g].fy, hal[g].fz, c, Ph);
                ldsU[buf][hly][hlx] = hal[g];
                ldsP[buf][hly][hlx] = Vec4<R>{Ph[0], Ph[1], Ph[2], Ph[3]};
                ldsQ[buf][hly][hlx] = Ph[4];
            }
            __syncthreads();
            if (active) {
                const int lx = tx + 1, ly = ty + 1;
                const R cc = c * c;
                // 2 x (A_x of the left, B_x of the right, A_y below, B_y above)
                const Vec4<R> uL = ldsU[buf][ly][lx - 1], pL = ldsP[buf][ly][lx - 1];
                const Vec4<R> uR = ldsU[buf][ly][lx + 1], pR = ldsP[buf][ly][lx + 1];
                const Vec4<R> uD = ldsU[buf][ly - 1][lx], pD = ldsP[buf][ly - 1][lx];
                const Vec4<R> uT = ldsU[buf][ly + 1][lx], pT = ldsP[buf][ly + 1][lx];
                const R qD = ldsQ[buf][ly - 1][lx], qT = ldsQ[buf][ly + 1][lx];
                // ldsP holds (Pxx, Pxy, Pxz, Pyy) in (n, fx, fy, fz)
                R sN = (uL.fx + c * uL.n) + (c * uR.n - uR.fx) + (uD.fy + c * uD.n) + (c * uT.n - uT.fy);
                R sX = (cc * pL.n + c * uL.fx) + (c * uR.fx - cc * pR.n) + (cc * pD.fx + c * uD.fx) +
                       (c * uT.fx - cc * pT.fx);
                R sY = (cc * pL.fx + c * uL.fy) + (c * uR.fy - cc * pR.fx) + (cc * pD.fz + c * uD.fy) +
                       (c * uT.fy - cc * pT.fz);
                R sZ = (cc * pL.fy + c * uL.fz) + (c * uR.fz - cc * pR.fy) + (cc * qD + c * uD.fz) +
                       (c * uT.fz - cc * qT);
                // z: 2 A_z of plane z-1 (kept from the last iteration), 2 B_z of plane z+1
                const Vec4<R> bz = bz2(nxt[g], Pn[g], c);
                const R three_c = R(3) * c;
                R n = cur[g].n + a.lam * (half * (sN + Az2[g].n + bz.n) - three_c * cur[g].n);
                R fx = cur[g].fx + a.lam * (half * (sX + Az2[g].fx + bz.fx) - three_c * cur[g].fx);
                R fy = cur[g].fy + a.lam * (half * (sY + Az2[g].fy + bz.fy) - three_c * cur[g].fy);
                R fz = cur[g].fz + a.lam * (half * (sZ + Az2[g].fz + bz.fz) - three_c * cur[g].fz);
                if (n < R(0)) { n = R(0); nneg++; }
                const R F2 = fx * fx + fy * fy + fz * fz;
                const R cn = c * n;
                if (F2 > cn * cn) {
                    const R s = cn * FastMath<R>::rcp(FastMath<R>::sqrt(F2));
                    fx *= s; fy *= s; fz *= s;
                    nlim++;
                }
                us[g] = Vec4<R>{n, fx, fy, fz};
            }
            buf ^= 1;
        }

        // roll the z window up before the chemistry so that plane z's state and
        // closure are dead while it runs: 2 A_z(plane z) for the next plane
#pragma unroll
        for (int g = 0; g < G; ++g) {
            Az2[g] = az2(cur[g], Pc[g], c);
            cur[g] = nxt[g];
#pragma unroll
            for (int q = 0; q < 6; ++q) Pc[g][q] = Pn[g][q];
        }

        bool deferred = false;
        if (active) {
            if (FUSE) {
                double Nc[G], Fc[G][3], Sc[G];
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    Nc[g] = (double)us[g].n;
                    Fc[g][0] = (double)us[g].fx;
                    Fc[g][1] = (double)us[g].fy;
                    Fc[g][2] = (double)us[g].fz;
                }
                source_of<G>((int64_t)zc, a.src.mask, a.src.sorted_cell, a.src.S, a.src.n, Sc);
                const ChemStats cs =
                    chem_cell<G, FAST>(a.gc, a.cp, Nc, Fc, xg, Tg, n0g, Sc, kChemBudget, &deferred);
                if (!deferred) {
                    if (DIAG) {
                        tot.substeps += cs.substeps;
                        tot.attempts += cs.attempts;
                        tot.cap += cs.cap;
                        tot.xclamp += cs.xclamp;
                        maxsub = max(maxsub, cs.substeps);
                    }
#pragma unroll
                    for (int g = 0; g < G; ++g) {
                        us[g].n = (R)Nc[g];
                        us[g].fx = (R)Fc[g][0];
                        us[g].fy = (R)Fc[g][1];
                        us[g].fz = (R)Fc[g][2];
                    }
                    st(a.x, zc * 8u, xg);
                    st(a.T, zc * 8u, Tg);
                }
                // deferred: N*, F* go to the output below; x, T stay untouched
            }
#pragma unroll
            for (int g = 0; g < G; ++g) {
                st(a.No + (int64_t)g * V, zc * E, us[g].n);
                st(a.Fo + (int64_t)(3 * g + 0) * V, zc * E, us[g].fx);
                st(a.Fo + (int64_t)(3 * g + 1) * V, zc * E, us[g].fy);
                st(a.Fo + (int64_t)(3 * g + 2) * V, zc * E, us[g].fz);
            }
        }

        if (FUSE) defer_push(a.wl, deferred, zc);

        // the prefetched plane z+2 becomes plane z+1 of the next iteration
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (active) nxt[g] = nn[g];
            m1_pressure(nxt[g].n, nxt[g].fx, nxt[g].fy, nxt[g].fz, c, Pn[g]);
            if (hrole >= 0 && z + 1 < z1) hal[g] = hnext[g];
        }
    }
    if (DIAG) {
        wave_count(a.cnt, CNT_LIMITER, nlim);
        wave_count(a.cnt, CNT_NEG, nneg);
        if (FUSE) {
            wave_count(a.cnt, CNT_SUB, tot.substeps);
            wave_count(a.cnt, CNT_ATT, tot.attempts);
            wave_count(a.cnt, CNT_CAP, tot.cap);
            wave_count(a.cnt, CNT_XCLAMP, tot.xclamp);
            wave_count_max(a.cnt, CNT_MAXSUB, maxsub);
        }
    }
}

template <int G, typename S>
inline TileArgs<S> tile_args(const S *iN, const S *iF, S *oN, S *oF, double *x, double *T,
                             const double *n0, const Grid &gr, const SrcTable &src,
                             const GroupConsts &gc, const ChemParams &cp, double lam,
                             unsigned long long *cnt, int LZ, WorkList wl) {
    TileArgs<S> a;
    a.N = iN; a.F = iF; a.No = oN; a.Fo = oF;
    a.x = x; a.T = T; a.n0 = n0;
    a.gr = gr;
    a.ntx = (gr.nx + kTX - 1) / kTX;
    a.nty = (gr.ny + kTY - 1) / kTY;
    a.LZ = LZ;
    a.ntz = (gr.nz + LZ - 1) / LZ;
    a.c = (S)cp.c;
    a.lam = (S)lam;
    a.src = src;
    a.gc = gc;
    a.cp = cp;
    a.cnt = cnt;
    a.wl = wl;
    return a;
}

// Number of z planes per block: enough blocks to fill 256 CUs several times.
inline int pick_lz(const Grid &gr) {
    const int64_t cols = (int64_t)((gr.nx + kTX - 1) / kTX) * ((gr.ny + kTY - 1) / kTY);
    int lz = 32;
    while (lz > 4 && cols * ((gr.nz + lz - 1) / lz) < 2048) lz >>= 1;
    return lz;
}

// The 32-bit byte offsets address one (group, component) array and the
// double fields: V * 8 bytes must stay below 4 GiB.
inline bool tiled_supported(const Grid &gr) { return (uint64_t)gr.V * 8 < ((uint64_t)1 << 32); }

// Transport only (split path): one group per block, grid.y = group, which
// keeps one group's rolling window in registers instead of all G.
template <int G, typename S, bool DIAG>
inline int launch_transport_tiled(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, const Grid &gr,
                                  const ChemParams &cp, double lam, unsigned long long *cnt) {
    const int LZ = pick_lz(gr);
    for (int g = 0; g < G; ++g) {
        TileArgs<S> a = tile_args<1, S>(iN + (int64_t)g * gr.V, iF + (int64_t)3 * g * gr.V, oN + (int64_t)g * gr.V,
                                        oF + (int64_t)3 * g * gr.V, nullptr, nullptr, nullptr, gr, SrcTable{},
                                        GroupConsts{}, cp, lam, cnt, LZ, WorkList{});
        const int nb = a.ntx * a.nty * a.ntz;
        hipLaunchKernelGGL((k_tiled<1, S, DIAG, false, false>), dim3(nb), dim3(kTX * kTY), 0, st, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int G, typename S, bool DIAG>
inline int launch_fused(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, double *x, double *T,
                        const double *n0, const Grid &gr, const SrcTable &src, const GroupConsts &gc,
                        const ChemParams &cp, double lam, unsigned long long *cnt, WorkList wl) {
    const int LZ = pick_lz(gr);
    TileArgs<S> a = tile_args<G, S>(iN, iF, oN, oF, x, T, n0, gr, src, gc, cp, lam, cnt, LZ, wl);
    const int nb = a.ntx * a.nty * a.ntz;
    if (cp.otsa && !cp.isothermal)
        hipLaunchKernelGGL((k_tiled<G, S, DIAG, true, true>), dim3(nb), dim3(kTX * kTY), 0, st, a);
    else
        hipLaunchKernelGGL((k_tiled<G, S, DIAG, true, false>), dim3(nb), dim3(kTX * kTY), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace emma
