// fused.hpp -- z-marching, LDS-tiled M1 transport with an optional fused
// chemistry epilogue (one pass over HBM per step).
//
// The face flux of eq. (e:glf) splits into a part carried by each side:
//   flux(i+1/2) = A_d(U_i) - B_d(U_{i+1}),  A_d(U) = (Ft_d(U) + c U)/2,
//   B_d(U) = (c U - Ft_d(U))/2,  Ft_d(U) = (F_d, c^2 P_.d),
// so the conservative update of eq. (e:uprt), 3D unsplit, is
//   U* = U + (dt/dx) [ sum_d A_d(U_{i-e_d}) + B_d(U_{i+e_d}) - 3 c U_i ].
// Each cell's closure P(U) is computed once per step by the thread that owns
// its column (halo cells once more by the block that needs them), and the
// owner publishes the four x/y split vectors 2A_x, 2B_x, 2A_y, 2B_y in LDS:
// each neighbour then reads exactly the one 4-vector it needs.  z neighbours
// stay in registers while the block marches up its column chunk.
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
// Tile heights (rows of 64 cells per block) and the longest z chunk; tuning
// knobs, measured on the device.
#ifndef EMMA_TY_SPLIT
#define EMMA_TY_SPLIT 4
#endif
#ifndef EMMA_TY_FUSED
#define EMMA_TY_FUSED 4
#endif
#ifndef EMMA_LZ_MAX
#define EMMA_LZ_MAX 32
#endif
// prefetch depth of the z march (planes loaded ahead of use); FP32: one
// plane ahead and one LDS buffer (17.5 KB a block, 90 VGPRs: five waves per
// SIMD, where two buffers held it to four blocks per CU by their LDS)
#ifndef EMMA_PD_SPLIT
#define EMMA_PD_SPLIT 1
#endif
// FP64: one plane ahead and one LDS buffer (35 KB a block, 164 VGPRs: three
// waves per SIMD, where two buffers held it to two blocks per CU)
#ifndef EMMA_PD_SPLIT_FP64
#define EMMA_PD_SPLIT_FP64 1
#endif
// LDS buffers of the FP64 split transport's plane exchange (2 or 1)
#ifndef EMMA_NB_SPLIT_FP64
#define EMMA_NB_SPLIT_FP64 1
#endif
// LDS buffers of the FP32 split transport's plane exchange (2 or 1)
#ifndef EMMA_NB_SPLIT
#define EMMA_NB_SPLIT 1
#endif
#ifndef EMMA_PD_FUSED
#define EMMA_PD_FUSED 0
#endif

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
    ContBuf cb;   // continuation states of stopped cells (k_step_ws)
    Bounds<R> bnd;
    int nolimit;  // 1: write the values before the N >= 0 floor and the limiter (split transport)
};

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
// Stores of the split transport's output: read only by the chemistry pass
// after the whole grid, so they are streamed past the caches (non-temporal;
// 0.408 against 0.417 ms per step at 256^3).  Loads stay cached: a tile's
// rows are the halo rows of its neighbours.
template <typename T>
__device__ __forceinline__ void st_out(T *base, uint32_t byte_off, T v) {
    __builtin_nontemporal_store(v, (T *)((char *)base + byte_off));
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

// Ghost of a boundary cell's state across a non-periodic face.
template <typename R>
__device__ __forceinline__ Vec4<R> ghost4(const Bounds<R> &b, int face, int g, R c, Vec4<R> u) {
    R f[3] = {u.fx, u.fy, u.fz};
    ghost(b, face, g, c, u.n, f);
    return Vec4<R>{u.n, f[0], f[1], f[2]};
}

// The four x/y split vectors (times 2) of one state U = (N, F) with its
// flux-form closure cP = c^2 P: 2 A_d = Ft_d + c U, 2 B_d = c U - Ft_d with
// Ft_d = (F_d, c^2 P_xd, c^2 P_yd, c^2 P_zd).
template <typename R>
__device__ __forceinline__ void split_xy(const Vec4<R> &u, const R cP[6], R c, Vec4<R> &Ax, Vec4<R> &Bx,
                                         Vec4<R> &Ay, Vec4<R> &By) {
    Ax = Vec4<R>{c * u.n + u.fx, c * u.fx + cP[0], c * u.fy + cP[1], c * u.fz + cP[2]};
    Bx = Vec4<R>{c * u.n - u.fx, c * u.fx - cP[0], c * u.fy - cP[1], c * u.fz - cP[2]};
    Ay = Vec4<R>{c * u.n + u.fy, c * u.fx + cP[1], c * u.fy + cP[3], c * u.fz + cP[4]};
    By = Vec4<R>{c * u.n - u.fy, c * u.fx - cP[1], c * u.fy - cP[3], c * u.fz - cP[4]};
}

// A_z and B_z parts (times 2) of one state with its flux-form closure.
template <typename R>
__device__ __forceinline__ Vec4<R> az2(const Vec4<R> &u, const R cP[6], R c) {
    return Vec4<R>{c * u.n + u.fz, c * u.fx + cP[2], c * u.fy + cP[4], c * u.fz + cP[5]};
}
template <typename R>
__device__ __forceinline__ Vec4<R> bz2(const Vec4<R> &u, const R cP[6], R c) {
    return Vec4<R>{c * u.n - u.fz, c * u.fx - cP[2], c * u.fy - cP[4], c * u.fz - cP[5]};
}

// ------------------------------------------------------------ HLL, tiled
// The HLL flux with M1 wave speeds (reference path: kernels.hpp k_transport)
// does not split into per-cell parts: a face needs both sides' state U, flux
// Ft_d = (F_d, c^2 P_xd, c^2 P_yd, c^2 P_zd) and speeds.  Each cell computes
// its closure and its speeds along the three axes once, publishes (U, Ft_x, Ft_y, speeds) in LDS for its x/y
// neighbours, keeps the z side in registers, and evaluates its own faces.
template <typename R> struct Speeds2 {
    R lo, hi;  // min(0, lambda-), max(0, lambda+) along one axis
};

template <typename R>
__device__ __forceinline__ Speeds2<R> hll_speeds(const Vec4<R> &u, int d, R c) {
    const R fd = d == 0 ? u.fx : (d == 1 ? u.fy : u.fz);
    R lmn, lmx;
    m1_speeds<R>(u.n, fd, c, lmn, lmx);
    return Speeds2<R>{lmn < R(0) ? lmn : R(0), lmx > R(0) ? lmx : R(0)};
}

template <typename R>
__device__ __forceinline__ Vec4<R> hll_ft(const Vec4<R> &u, const R P[6], R c, int d) {
    const R cc = c * c;
    const int i0 = d == 0 ? 0 : (d == 1 ? 1 : 2), i1 = d == 0 ? 1 : (d == 1 ? 3 : 4),
              i2 = d == 0 ? 2 : (d == 1 ? 4 : 5);
    return Vec4<R>{d == 0 ? u.fx : (d == 1 ? u.fy : u.fz), cc * P[i0], cc * P[i1], cc * P[i2]};
}

// (a+ Ft(L) - a- Ft(R) + a+ a- (U_R - U_L)) / (a+ - a-)
template <typename R>
__device__ __forceinline__ Vec4<R> hll_face(const Vec4<R> &uL, const Vec4<R> &fL, Speeds2<R> sL, const Vec4<R> &uR,
                                            const Vec4<R> &fR, Speeds2<R> sR) {
    const R am = sL.lo < sR.lo ? sL.lo : sR.lo;
    const R ap = sL.hi > sR.hi ? sL.hi : sR.hi;
    const R inv = FastMath<R>::rcp(ap - am), pm = ap * am;
    return Vec4<R>{(ap * fL.n - am * fR.n + pm * (uR.n - uL.n)) * inv,
                   (ap * fL.fx - am * fR.fx + pm * (uR.fx - uL.fx)) * inv,
                   (ap * fL.fy - am * fR.fy + pm * (uR.fy - uL.fy)) * inv,
                   (ap * fL.fz - am * fR.fz + pm * (uR.fz - uL.fz)) * inv};
}

// Split-path transport with the HLL flux, the group in blockIdx.y, blocks of
// 64 x TY columns marching up LZ-plane z chunks.  Halo roles, ghosts and the
// z window follow k_tiled; LDS holds, per plane (NB = 2: double-buffered;
// NB = 1: one buffer and a second barrier per plane), U of the tile and its
// x/y halo, Ft_x and the x speeds of the tile and its x halo, Ft_y and the y
// speeds of the tile and its y halo.  One buffer (22 KB FP32, 44 KB FP64)
// measured faster than two: the FP64 double-buffered tiles (88 KB) fit once
// per CU (FP64 HLL step 2.69 -> 1.92 ms at 256^3; FP32 1.009 -> 1.002).
#ifndef EMMA_HLL_NB
#define EMMA_HLL_NB 1
#endif
template <typename R, bool DIAG, int TY, bool FULL, int NB = EMMA_HLL_NB>
__global__ __launch_bounds__(kTX * TY) void k_tiled_hll(TileArgs<R> a) {
    __shared__ Vec4<R> lU[NB][TY + 2][kTX + 2];
    __shared__ Vec4<R> lFx[NB][TY][kTX + 2];
    __shared__ Speeds2<R> lSx[NB][TY][kTX + 2];
    __shared__ Vec4<R> lFy[NB][TY + 2][kTX];
    __shared__ Speeds2<R> lSy[NB][TY + 2][kTX];
    const int tid = threadIdx.x;
    const int tx = tid & (kTX - 1), ty = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tile_x = t % a.ntx, tile_y = (t / a.ntx) % a.nty, tile_z = t / (a.ntx * a.nty);
    const int nx = a.gr.nx, ny = a.gr.ny, nz = a.gr.nz;
    const int64_t V = a.gr.V;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int x0 = tile_x * kTX, y0 = tile_y * TY, z0 = tile_z * a.LZ;
    const int z1 = min(z0 + a.LZ, nz);
    const int w = min(kTX, nx - x0), h = min(TY, ny - y0);
    const bool active = FULL || (tx < w && ty < h);
    const uint32_t col = active ? (uint32_t)(y0 + ty) * nx + (x0 + tx) : 0u;
    constexpr uint32_t E = sizeof(R);
    // one launch for all groups, blockIdx.y the group (as in k_tiled)
    const int gy = blockIdx.y;
    const R *__restrict__ Nin = a.N + (int64_t)gy * V;
    const R *__restrict__ Fin = a.F + (int64_t)3 * gy * V;
    R *__restrict__ Nout = a.No + (int64_t)gy * V;
    R *__restrict__ Fout = a.Fo + (int64_t)3 * gy * V;
    // read in place from the arguments (a local copy indexed by face would
    // live in scratch memory); the group's inflow fluxes are phi[face][gy + g]
    const Bounds<R> &bd = a.bnd;
    // halo role as in k_tiled: 0 row below, 1 row above, 2 column left, 3 column right
    int hrole = -1, hlx = 0, hly = 0, hface = -1;
    uint32_t hcol = 0;
    if (tid < kTX) {
        if (tid < w) {
            hrole = 0; hlx = tid + 1; hly = 0;
            int yy = y0 - 1;
            if (yy < 0) {
                if (bd.kind[2] == BC_PERIODIC) yy = ny - 1;
                else { yy = 0; hface = 2; }
            }
            hcol = (uint32_t)yy * nx + x0 + tid;
        }
    } else if (tid < 2 * kTX) {
        const int cx = tid - kTX;
        if (cx < w) {
            hrole = 1; hlx = cx + 1; hly = h + 1;
            int yy = y0 + h;
            if (yy >= ny) {
                if (bd.kind[3] == BC_PERIODIC) yy = 0;
                else { yy = ny - 1; hface = 3; }
            }
            hcol = (uint32_t)yy * nx + x0 + cx;
        }
    } else if (tid < 2 * kTX + TY) {
        const int cy = tid - 2 * kTX;
        if (cy < h) {
            hrole = 2; hlx = 0; hly = cy + 1;
            int xx = x0 - 1;
            if (xx < 0) {
                if (bd.kind[0] == BC_PERIODIC) xx = nx - 1;
                else { xx = 0; hface = 0; }
            }
            hcol = (uint32_t)(y0 + cy) * nx + xx;
        }
    } else if (tid < 2 * kTX + 2 * TY) {
        const int cy = tid - 2 * kTX - TY;
        if (cy < h) {
            hrole = 3; hlx = w + 1; hly = cy + 1;
            int xx = x0 + w;
            if (xx >= nx) {
                if (bd.kind[1] == BC_PERIODIC) xx = 0;
                else { xx = nx - 1; hface = 1; }
            }
            hcol = (uint32_t)(y0 + cy) * nx + xx;
        }
    }
    const bool zlo_ghost = bd.kind[4] != BC_PERIODIC, zhi_ghost = bd.kind[5] != BC_PERIODIC;
    int hkind = BC_PERIODIC, hd = 0;
    R hsgn = R(1), hphi = R(0);
    if (hface >= 0) {
        hkind = bd.kind[hface];
        hd = hface >> 1;
        hsgn = (hface & 1) ? R(-1) : R(1);
        hphi = bd.phi[hface][gy];
    }
    const uint32_t hsrc = hrole >= 0 ? hcol : col;
    const R c = a.c;
    auto zwrap = [nz](int z) { return (uint32_t)((z % nz + nz) % nz); };
    auto load1 = [&](uint32_t off) {
        Vec4<R> u[1];
        load_cell<1>(Nin, Fin, V, off * E, u);
        return u[0];
    };
    // z window: planes z (cur) and z + 1 (nxt) with their closures, the z
    // side (Ft_z, speeds) of both, and the flux through the face below z
    Vec4<R> cur = load1(zwrap(z0) * plane + col);
    Vec4<R> nxt = load1(zwrap(min(z0 + 1, z1)) * plane + col);
    Vec4<R> um = load1(zwrap(z0 - 1) * plane + col);
    if (z0 == 0 && zlo_ghost) um = ghost4(bd, 4, gy, c, cur);
    if (z0 + 1 == nz && zhi_ghost) nxt = ghost4(bd, 5, gy, c, cur);
    R Pc[6], Pn[6];
    Vec4<R> flo;
    {
        R Pm[6];
        m1_pressure(um.n, um.fx, um.fy, um.fz, c, Pm);
        m1_pressure(cur.n, cur.fx, cur.fy, cur.fz, c, Pc);
        flo = hll_face(um, hll_ft(um, Pm, c, 2), hll_speeds(um, 2, c), cur, hll_ft(cur, Pc, c, 2),
                       hll_speeds(cur, 2, c));
    }
    m1_pressure(nxt.n, nxt.fx, nxt.fy, nxt.fz, c, Pn);
    Vec4<R> hal = load1((uint32_t)z0 * plane + hsrc);
    int64_t nlim = 0, nneg = 0;
    int buf = 0;
    for (int z = z0; z < z1; ++z) {
        const uint32_t zc = (uint32_t)z * plane + col;
        // loads for the next plane fly during this one
        Vec4<R> nn = load1(zwrap(min(z + 2, z1)) * plane + col);
        const Vec4<R> hal_next = load1((uint32_t)min(z + 1, z1 - 1) * plane + hsrc);
        // publish plane z: own cell
        const Vec4<R> ftx = hll_ft(cur, Pc, c, 0), fty = hll_ft(cur, Pc, c, 1);
        const Speeds2<R> sx = hll_speeds(cur, 0, c), sy = hll_speeds(cur, 1, c);
        if (active) {
            lU[buf][ty + 1][tx + 1] = cur;
            lFx[buf][ty][tx + 1] = ftx;
            lSx[buf][ty][tx + 1] = sx;
            lFy[buf][ty + 1][tx] = fty;
            lSy[buf][ty + 1][tx] = sy;
        }
        // halo cell (the ghost across a non-periodic face)
        if (hrole >= 0) {
            Vec4<R> hv = hal;
            if (hkind == BC_REFLECTIVE) {
                if (hd == 0) hv.fx = -hv.fx;
                else hv.fy = -hv.fy;
            } else if (hkind == BC_INFLOW) {
                hv.n = hphi / c;
                hv.fx = hd == 0 ? hsgn * hphi : R(0);
                hv.fy = hd == 1 ? hsgn * hphi : R(0);
                hv.fz = R(0);
            }
            R Ph[6];
            m1_pressure(hv.n, hv.fx, hv.fy, hv.fz, c, Ph);
            lU[buf][hly][hlx] = hv;
            if (hrole <= 1) {  // row below / above: y side
                lFy[buf][hly][hlx - 1] = hll_ft(hv, Ph, c, 1);
                lSy[buf][hly][hlx - 1] = hll_speeds(hv, 1, c);
            } else {           // column left / right: x side
                lFx[buf][hly - 1][hlx] = hll_ft(hv, Ph, c, 0);
                lSx[buf][hly - 1][hlx] = hll_speeds(hv, 0, c);
            }
        }
        // z side of plane z + 1 and the face above z
        R Pnn[6];
        const Vec4<R> fup = hll_face(cur, hll_ft(cur, Pc, c, 2), hll_speeds(cur, 2, c), nxt, hll_ft(nxt, Pn, c, 2),
                                     hll_speeds(nxt, 2, c));
        __syncthreads();
        Vec4<R> us;
        {
            const Vec4<R> fxl = hll_face(lU[buf][ty + 1][tx], lFx[buf][ty][tx], lSx[buf][ty][tx], cur, ftx, sx);
            const Vec4<R> fxr =
                hll_face(cur, ftx, sx, lU[buf][ty + 1][tx + 2], lFx[buf][ty][tx + 2], lSx[buf][ty][tx + 2]);
            const Vec4<R> fyl = hll_face(lU[buf][ty][tx + 1], lFy[buf][ty][tx], lSy[buf][ty][tx], cur, fty, sy);
            const Vec4<R> fyr =
                hll_face(cur, fty, sy, lU[buf][ty + 2][tx + 1], lFy[buf][ty + 2][tx], lSy[buf][ty + 2][tx]);
            const R lam = a.lam;
            R n = cur.n + lam * ((fxl.n - fxr.n) + (fyl.n - fyr.n) + (flo.n - fup.n));
            R fx = cur.fx + lam * ((fxl.fx - fxr.fx) + (fyl.fx - fyr.fx) + (flo.fx - fup.fx));
            R fy = cur.fy + lam * ((fxl.fy - fxr.fy) + (fyl.fy - fyr.fy) + (flo.fy - fup.fy));
            R fz = cur.fz + lam * ((fxl.fz - fxr.fz) + (fyl.fz - fyr.fz) + (flo.fz - fup.fz));
            if (!a.nolimit) {
                const int taken = floor_limit_fwd(n, fx, fy, fz, c);
                if (active) {
                    nneg += taken & 1;
                    nlim += taken >> 1;
                }
            }
            us = Vec4<R>{n, fx, fy, fz};
        }
        if (active) {
            st(Nout, zc * E, us.n);
            st(Fout, zc * E, us.fx);
            st(Fout + V, zc * E, us.fy);
            st(Fout + 2 * V, zc * E, us.fz);
        }
        // roll the window
        if (z + 2 == nz && zhi_ghost) nn = ghost4(bd, 5, gy, c, nxt);
        m1_pressure(nn.n, nn.fx, nn.fy, nn.fz, c, Pnn);
        flo = fup;
        cur = nxt;
        nxt = nn;
#pragma unroll
        for (int q = 0; q < 6; ++q) {
            Pc[q] = Pn[q];
            Pn[q] = Pnn[q];
        }
        hal = hal_next;
        if (NB == 2) buf ^= 1;
        else __syncthreads();  // every read of this plane before the next writes
    }
    if (DIAG) {
        wave_count(a.cnt, CNT_LIMITER, nlim);
        wave_count(a.cnt, CNT_NEG, nneg);
    }
}

// FULL: every tile is a whole 64 x TY tile (nx % 64 == 0, ny % TY == 0), so
// every thread owns a cell and no store needs a predicate.
#ifndef EMMA_FUSED_MIN_BLOCKS
#define EMMA_FUSED_MIN_BLOCKS 2
#endif
template <int G, typename R, bool DIAG, bool FUSE, bool FAST, int TY, int PD, bool FULL, int NB = 2>
__global__ __launch_bounds__(kTX * TY, (FUSE && sizeof(R) == 4) ? EMMA_FUSED_MIN_BLOCKS : 1) void k_tiled(TileArgs<R> a) {
    // plane z of the current group, double-buffered (NB = 2; NB = 1: one
    // buffer and a second barrier per plane, half the LDS): only the split
    // vectors a neighbour reads.  Consumer (ty, tx) reads lAx[ty][tx] (left
    // cell's A_x), lBx[ty][tx + 1] (right cell's B_x), lAy[ty][tx] (A_y of the
    // cell below), lBy[ty][tx] (B_y of the cell above).
    __shared__ Vec4<R> lAx[NB][TY][kTX + 1];
    __shared__ Vec4<R> lBx[NB][TY][kTX + 1];
    __shared__ Vec4<R> lAy[NB][TY + 1][kTX];
    __shared__ Vec4<R> lBy[NB][TY][kTX];
    const int tid = threadIdx.x;
    const int tx = tid & (kTX - 1), ty = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tile_x = t % a.ntx, tile_y = (t / a.ntx) % a.nty, tile_z = t / (a.ntx * a.nty);
    const int nx = a.gr.nx, ny = a.gr.ny, nz = a.gr.nz;
    const int64_t V = a.gr.V;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int x0 = tile_x * kTX, y0 = tile_y * TY, z0 = tile_z * a.LZ;
    const int z1 = min(z0 + a.LZ, nz);
    const int w = min(kTX, nx - x0), h = min(TY, ny - y0);
    const bool active = FULL || (tx < w && ty < h);
    const uint32_t col = active ? (uint32_t)(y0 + ty) * nx + (x0 + tx) : 0u;  // cell within a plane
    constexpr uint32_t E = sizeof(R);

    // halo role: bottom row, top row, left column, right column of the tile;
    // across a non-periodic face the halo cell is the boundary cell itself and
    // hface names the face whose ghost it becomes
    // the split transport launches once for all groups: blockIdx.y is the
    // group (G = 1 then), whose arrays and inflow fluxes the block takes
    const int gy = blockIdx.y;
    const R *__restrict__ Nin = a.N + (int64_t)gy * V;
    const R *__restrict__ Fin = a.F + (int64_t)3 * gy * V;
    R *__restrict__ Nout = a.No + (int64_t)gy * V;
    R *__restrict__ Fout = a.Fo + (int64_t)3 * gy * V;
    // read in place from the arguments (a local copy indexed by face would
    // live in scratch memory); the group's inflow fluxes are phi[face][gy + g]
    const Bounds<R> &bd = a.bnd;
    int hrole = -1, hlx = 0, hly = 0, hface = -1;
    uint32_t hcol = 0;
    if (tid < kTX) {
        if (tid < w) {
            hrole = 0; hlx = tid + 1; hly = 0;
            int yy = y0 - 1;
            if (yy < 0) {
                if (bd.kind[2] == BC_PERIODIC) yy = ny - 1;
                else { yy = 0; hface = 2; }
            }
            hcol = (uint32_t)yy * nx + x0 + tid;
        }
    } else if (tid < 2 * kTX) {
        const int cx = tid - kTX;
        if (cx < w) {
            hrole = 1; hlx = cx + 1; hly = h + 1;
            int yy = y0 + h;
            if (yy >= ny) {
                if (bd.kind[3] == BC_PERIODIC) yy = 0;
                else { yy = ny - 1; hface = 3; }
            }
            hcol = (uint32_t)yy * nx + x0 + cx;
        }
    } else if (tid < 2 * kTX + TY) {
        const int cy = tid - 2 * kTX;
        if (cy < h) {
            hrole = 2; hlx = 0; hly = cy + 1;
            int xx = x0 - 1;
            if (xx < 0) {
                if (bd.kind[0] == BC_PERIODIC) xx = nx - 1;
                else { xx = 0; hface = 0; }
            }
            hcol = (uint32_t)(y0 + cy) * nx + xx;
        }
    } else if (tid < 2 * kTX + 2 * TY) {
        const int cy = tid - 2 * kTX - TY;
        if (cy < h) {
            hrole = 3; hlx = w + 1; hly = cy + 1;
            int xx = x0 + w;
            if (xx >= nx) {
                if (bd.kind[1] == BC_PERIODIC) xx = 0;
                else { xx = nx - 1; hface = 1; }
            }
            hcol = (uint32_t)(y0 + cy) * nx + xx;
        }
    }
    // z faces: ghosts of plane 0 below the grid and of plane nz-1 above it
    const bool zlo_ghost = bd.kind[4] != BC_PERIODIC, zhi_ghost = bd.kind[5] != BC_PERIODIC;

    const R c = a.c, cc = c * c, half = R(0.5);
    // The z march keeps a window of U = PD + 2 planes of the own column in
    // registers, W[(z - z0) mod U] = plane z, and of the halo column, H[...]:
    // the planes z and z+1 in use and PD planes in flight.  The loop is
    // unrolled by U so every slot is a fixed register set (no copies), and
    // every global load is issued unconditionally (planes past the chunk are
    // clamped to its last plane, threads without a halo cell load their own
    // column) so the compiler can wait for exactly the plane it needs instead
    // of draining all loads in flight.
    constexpr int U = PD + 2;
    Vec4<R> W[U][G], H[U][G], Az2[G], Bz2[G];
    R Pc[G][6], Pn[G][6];
    int64_t nlim = 0, nneg = 0;
    ChemStats tot{0, 0, 0, 0};
    int maxsub = 0;
    // the halo cell's ghost, read once (a face index into the argument block
    // would otherwise be a memory load inside the loop)
    int hkind = BC_PERIODIC, hd = 0;
    R hsgn = R(1), hphi[G];
#pragma unroll
    for (int g = 0; g < G; ++g) hphi[g] = R(0);
    if (hface >= 0) {
        hkind = bd.kind[hface];
        hd = hface >> 1;
        hsgn = (hface & 1) ? R(-1) : R(1);
#pragma unroll
        for (int g = 0; g < G; ++g) hphi[g] = bd.phi[hface][gy + g];
    }
    // threads without a halo cell reload their own column, except in the waves
    // that have no halo cell at all, which skip the halo loads (a wave-uniform
    // condition, so a scalar branch)
    const uint32_t hsrc = hrole >= 0 ? hcol : col;
    const bool hwave = __builtin_amdgcn_readfirstlane(tid >> 6) * kTX < 2 * kTX + 2 * TY;

    auto zwrap = [nz](int z) { return (uint32_t)((z % nz + nz) % nz); };
    {
        Vec4<R> um[G];
        load_cell<G>(Nin, Fin, V, (zwrap(z0 - 1) * plane + col) * E, um);
#pragma unroll
        for (int k = 0; k < U; ++k) load_cell<G>(Nin, Fin, V, (zwrap(min(z0 + k, z1)) * plane + col) * E, W[k]);
#pragma unroll
        for (int k = 0; k < U; ++k)
            if (hwave) load_cell<G>(Nin, Fin, V, ((uint32_t)min(z0 + k, z1 - 1) * plane + hsrc) * E, H[k]);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (z0 == 0 && zlo_ghost) um[g] = ghost4(bd, 4, gy + g, c, W[0][g]);
            if (z0 + 1 == nz && zhi_ghost) W[1][g] = ghost4(bd, 5, gy + g, c, W[0][g]);
            R Pm[6];
            m1_pressure(um[g].n, um[g].fx, um[g].fy, um[g].fz, c, Pm, cc);
            Az2[g] = az2(um[g], Pm, c);
            m1_pressure(W[0][g].n, W[0][g].fx, W[0][g].fy, W[0][g].fz, c, Pc[g], cc);
            m1_pressure(W[1][g].n, W[1][g].fx, W[1][g].fy, W[1][g].fz, c, Pn[g], cc);
            Bz2[g] = bz2(W[1][g], Pn[g], c);
        }
    }

    int buf = 0;
    // plane z: transport of every group, optional chemistry, store; then
    // refill the freed slots with plane z + U and prepare plane z + 2's closure
    auto plane_step = [&](const int z, Vec4<R>(&cur)[G], Vec4<R>(&nxt)[G], Vec4<R>(&nn)[G], Vec4<R>(&hal)[G]) {
        const uint32_t zc = (uint32_t)z * plane + col;
        double xg = 0.0, Tg = 0.0, n0g = 0.0;
        if (FUSE) {
            xg = ld(a.x, zc * 8u);
            Tg = ld(a.T, zc * 8u);
            n0g = ld(a.n0, zc * 8u);
            // the fused kernel recomputes plane z's closure rather than keeping
            // it live through the chemistry (registers, not ALU, limit it)
#pragma unroll
            for (int g = 0; g < G; ++g) m1_pressure(cur[g].n, cur[g].fx, cur[g].fy, cur[g].fz, c, Pc[g], cc);
        }

        Vec4<R> us[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            // publish plane z of group g: own cell and halo cell
            if (active) {
                Vec4<R> Ax, Bx, Ay, By;
                split_xy(cur[g], Pc[g], c, Ax, Bx, Ay, By);
                lAx[buf][ty][tx + 1] = Ax;
                lBx[buf][ty][tx] = Bx;
                lAy[buf][ty + 1][tx] = Ay;
                if (ty > 0) lBy[buf][ty - 1][tx] = By;
            }
            if (hrole >= 0) {
                Vec4<R> hv = hal[g];
                if (hkind == BC_REFLECTIVE) {
                    if (hd == 0) hv.fx = -hv.fx;
                    else if (hd == 1) hv.fy = -hv.fy;
                    else hv.fz = -hv.fz;
                } else if (hkind == BC_INFLOW) {  // beam into the domain across the face
                    hv.n = hphi[g] / c;
                    hv.fx = hd == 0 ? hsgn * hphi[g] : R(0);
                    hv.fy = hd == 1 ? hsgn * hphi[g] : R(0);
                    hv.fz = hd == 2 ? hsgn * hphi[g] : R(0);
                }
                R Ph[6];
                m1_pressure(hv.n, hv.fx, hv.fy, hv.fz, c, Ph, cc);
                Vec4<R> Ax, Bx, Ay, By;
                split_xy(hv, Ph, c, Ax, Bx, Ay, By);
                if (hrole == 0) lAy[buf][0][hlx - 1] = Ay;            // row below the tile
                else if (hrole == 1) lBy[buf][h - 1][hlx - 1] = By;   // row above
                else if (hrole == 2) lAx[buf][hly - 1][0] = Ax;       // column left
                else lBx[buf][hly - 1][w] = Bx;                       // column right
            }
            __syncthreads();
            {
                const Vec4<R> aL = lAx[buf][ty][tx], bR = lBx[buf][ty][tx + 1];
                const Vec4<R> aD = lAy[buf][ty][tx], bT = lBy[buf][ty][tx];
                // U + lam/2 (sum of the six split vectors (times 2) - 6 c U)
                // = (1 - 3 c lam) U + lam/2 (sum)
                const R hl = half * a.lam;
                const R k0 = R(1) - R(3) * c * a.lam;
                R n = k0 * cur[g].n + hl * ((aL.n + bR.n) + (aD.n + bT.n) + (Az2[g].n + Bz2[g].n));
                R fx = k0 * cur[g].fx + hl * ((aL.fx + bR.fx) + (aD.fx + bT.fx) + (Az2[g].fx + Bz2[g].fx));
                R fy = k0 * cur[g].fy + hl * ((aL.fy + bR.fy) + (aD.fy + bT.fy) + (Az2[g].fy + Bz2[g].fy));
                R fz = k0 * cur[g].fz + hl * ((aL.fz + bR.fz) + (aD.fz + bT.fz) + (Az2[g].fz + Bz2[g].fz));
                if (!a.nolimit) {
                    const int taken = floor_limit_fwd(n, fx, fy, fz, c);
                    if (active) {
                        nneg += taken & 1;
                        nlim += taken >> 1;
                    }
                }
                us[g] = Vec4<R>{n, fx, fy, fz};
            }
            if (NB == 2) buf ^= 1;
            else __syncthreads();  // every read of this plane before the next writes
        }

        // roll the z window before the chemistry so that plane z's state and
        // closure are dead while it runs: 2 A_z(plane z) for the next plane
#pragma unroll
        for (int g = 0; g < G; ++g) {
            Az2[g] = az2(cur[g], Pc[g], c);
            if (!FUSE) {
#pragma unroll
                for (int q = 0; q < 6; ++q) Pc[g][q] = Pn[g][q];
            }
        }
        // the slots of plane z are free: refill them with plane z + U (clamped
        // to the chunk's last plane, which is then loaded twice from L2); the
        // loads fly while the chemistry runs
        load_cell<G>(Nin, Fin, V, (zwrap(min(z + U, z1)) * plane + col) * E, cur);
        if (hwave) load_cell<G>(Nin, Fin, V, ((uint32_t)min(z + U, z1 - 1) * plane + hsrc) * E, hal);

        bool deferred = false, done = false;
        int nsub = 0;
        if (FUSE && active) {
            double Nc[G], Sc[G], Pf[G];
#pragma unroll
            for (int g = 0; g < G; ++g) Nc[g] = (double)us[g].n;
            source_of<G>((int64_t)zc, a.src.mask, a.src.sorted_cell, a.src.S, a.src.n, Sc);
            const ChemStats cs =
                chem_cell_nxt<G, FAST>(a.gc, a.cp, Nc, Pf, xg, Tg, n0g, Sc, kChemBudgetFused, &deferred);
            if (!deferred) {
                if (DIAG) {
                    tot.substeps += cs.substeps;
                    tot.attempts += cs.attempts;
                    tot.cap += cs.cap;
                    tot.xclamp += cs.xclamp;
                    maxsub = max(maxsub, cs.substeps);
                    done = true;
                    nsub = cs.substeps;
                }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    us[g].n = (R)Nc[g];
                    us[g].fx = (R)((double)us[g].fx * Pf[g]);
                    us[g].fy = (R)((double)us[g].fy * Pf[g]);
                    us[g].fz = (R)((double)us[g].fz * Pf[g]);
                }
                st(a.x, zc * 8u, xg);
                st(a.T, zc * 8u, Tg);
            }
            // deferred: N*, F* go to the output below; x, T stay untouched
        }
        if (DIAG && FUSE) wave_hist(a.cnt, done, nsub);
        if (active) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                st_out(Nout + (int64_t)g * V, zc * E, us[g].n);
                st_out(Fout + (int64_t)(3 * g + 0) * V, zc * E, us[g].fx);
                st_out(Fout + (int64_t)(3 * g + 1) * V, zc * E, us[g].fy);
                st_out(Fout + (int64_t)(3 * g + 2) * V, zc * E, us[g].fz);
            }
        }

        if (FUSE) defer_push(a.wl, deferred, zc);

        // plane z + 2 becomes the next step's upper neighbour
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (z + 2 == nz && zhi_ghost) nn[g] = ghost4(bd, 5, gy + g, c, nxt[g]);  // nxt = plane nz-1
            m1_pressure(nn[g].n, nn[g].fx, nn[g].fy, nn[g].fz, c, Pn[g], cc);
            Bz2[g] = bz2(nn[g], Pn[g], c);
        }
    };
    for (int zb = z0; zb < z1; zb += U) {
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (zb + j < z1) plane_step(zb + j, W[j], W[(j + 1) % U], W[(j + 2) % U], H[j]);
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
                             unsigned long long *cnt, int LZ, WorkList wl, int TY, const Bounds<S> &bnd) {
    TileArgs<S> a;
    a.N = iN; a.F = iF; a.No = oN; a.Fo = oF;
    a.x = x; a.T = T; a.n0 = n0;
    a.gr = gr;
    a.ntx = (gr.nx + kTX - 1) / kTX;
    a.nty = (gr.ny + TY - 1) / TY;
    a.LZ = LZ;
    a.ntz = (gr.nz + LZ - 1) / LZ;
    a.c = (S)cp.c;
    a.lam = (S)lam;
    a.src = src;
    a.gc = gc;
    a.cp = cp;
    a.cnt = cnt;
    a.wl = wl;
    a.cb = ContBuf{};
    a.bnd = bnd;
    a.nolimit = 0;
    return a;
}

// Number of z planes per block: enough blocks to fill 256 CUs several times.
inline int pick_lz(const Grid &gr, int TY) {
    const int64_t cols = (int64_t)((gr.nx + kTX - 1) / kTX) * ((gr.ny + TY - 1) / TY);
    int lz = EMMA_LZ_MAX;
    while (lz > 4 && cols * ((gr.nz + lz - 1) / lz) < 2048) lz >>= 1;
    return lz;
}

// The 32-bit byte offsets address one (group, component) array and the
// double fields: V * 8 bytes must stay below 4 GiB.
inline bool tiled_supported(const Grid &gr) { return (uint64_t)gr.V * 8 < ((uint64_t)1 << 32); }

// Transport only (split path): the kernel for one group (one group's
// rolling window in registers instead of all G), launched once for all
// groups with the group in blockIdx.y (no tail and launch gap between
// groups, as one launch per group had).
template <int G, typename S, bool DIAG>
inline int launch_transport_tiled(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, const Grid &gr,
                                  const ChemParams &cp, double lam, unsigned long long *cnt,
                                  const Bounds<S> &bnd, bool nolimit = false) {
    // double tiles need twice the LDS: at most 8 rows (136 KB)
    constexpr int TY = (sizeof(S) == 8 && EMMA_TY_SPLIT > 8) ? 8 : EMMA_TY_SPLIT;
    constexpr int PD = sizeof(S) == 8 ? EMMA_PD_SPLIT_FP64 : EMMA_PD_SPLIT;
    constexpr int NB = sizeof(S) == 8 ? EMMA_NB_SPLIT_FP64 : EMMA_NB_SPLIT;
    const int LZ = pick_lz(gr, TY);
    TileArgs<S> a = tile_args<1, S>(iN, iF, oN, oF, nullptr, nullptr, nullptr, gr, SrcTable{}, GroupConsts{}, cp,
                                    lam, cnt, LZ, WorkList{}, TY, bnd);
    a.nolimit = nolimit ? 1 : 0;
    const int nb = a.ntx * a.nty * a.ntz;
    if (gr.nx % kTX == 0 && gr.ny % TY == 0)
        hipLaunchKernelGGL((k_tiled<1, S, DIAG, false, false, TY, PD, true, NB>), dim3(nb, G), dim3(kTX * TY), 0, st, a);
    else
        hipLaunchKernelGGL((k_tiled<1, S, DIAG, false, false, TY, PD, false, NB>), dim3(nb, G), dim3(kTX * TY), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Split-path transport with the HLL flux: one launch for all groups.
template <int G, typename S, bool DIAG>
inline int launch_transport_tiled_hll(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, const Grid &gr,
                                      const ChemParams &cp, double lam, unsigned long long *cnt,
                                      const Bounds<S> &bnd, bool nolimit = false) {
    constexpr int TY = 4;
    const int LZ = pick_lz(gr, TY);
    // all groups in one launch (blockIdx.y = group)
    TileArgs<S> a = tile_args<1, S>(iN, iF, oN, oF, nullptr, nullptr, nullptr, gr, SrcTable{}, GroupConsts{}, cp, lam,
                                    cnt, LZ, WorkList{}, TY, bnd);
    a.nolimit = nolimit ? 1 : 0;
    const int nb = a.ntx * a.nty * a.ntz;
    if (gr.nx % kTX == 0 && gr.ny % TY == 0)
        hipLaunchKernelGGL((k_tiled_hll<S, DIAG, TY, true>), dim3(nb, G), dim3(kTX * TY), 0, st, a);
    else
        hipLaunchKernelGGL((k_tiled_hll<S, DIAG, TY, false>), dim3(nb, G), dim3(kTX * TY), 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int G, typename S, bool DIAG>
inline int launch_fused(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, double *x, double *T,
                        const double *n0, const Grid &gr, const SrcTable &src, const GroupConsts &gc,
                        const ChemParams &cp, double lam, unsigned long long *cnt, WorkList wl,
                        const Bounds<S> &bnd) {
    constexpr int TY = (sizeof(S) == 8 && EMMA_TY_FUSED > 8) ? 8 : EMMA_TY_FUSED;
    const int LZ = pick_lz(gr, TY);
    TileArgs<S> a = tile_args<G, S>(iN, iF, oN, oF, x, T, n0, gr, src, gc, cp, lam, cnt, LZ, wl, TY, bnd);
    const int nb = a.ntx * a.nty * a.ntz;
    const bool full = gr.nx % kTX == 0 && gr.ny % TY == 0;
    const bool fast = cp.otsa && !cp.isothermal;
    if (fast && full)
        hipLaunchKernelGGL((k_tiled<G, S, DIAG, true, true, TY, EMMA_PD_FUSED, true>), dim3(nb), dim3(kTX * TY), 0,
                           st, a);
    else if (fast)
        hipLaunchKernelGGL((k_tiled<G, S, DIAG, true, true, TY, EMMA_PD_FUSED, false>), dim3(nb), dim3(kTX * TY), 0,
                           st, a);
    else
        hipLaunchKernelGGL((k_tiled<G, S, DIAG, true, false, TY, EMMA_PD_FUSED, false>), dim3(nb), dim3(kTX * TY),
                           0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace emma
