// step_ws.hpp -- one pass over HBM per step with specialised waves.
//
// Each block owns a 64 x 4 column tile of the grid and marches up a z chunk,
// as k_tiled does, but its waves have two roles:
//   * 4 transport waves (one row of the tile each) run the M1 transport of
//     every group (Sec. 2.2.3, eqs. e:glf, e:uprt): closure, the split vectors
//     exchanged through LDS, the conservative update, the floor and limiter;
//     they hand N*, F* of each plane to the chemistry waves through LDS;
//   * 4 chemistry waves (one cell per lane) run the FP64 thermochemistry
//     subcycle (Sec. 2.2.4) on the plane the transport waves finished one
//     iteration earlier and write the end-of-step state.
// The two roles run in separate loops, so the transport's rolling z window
// and the chemistry's FP64 state are never live at the same time: the
// register budget of the kernel is the larger of the two, not their sum.
// Both loops execute the same two barriers per iteration:
//     [B_b(k-1) .. B_a(k)]  transport publishes plane k's split vectors;
//                           chemistry runs plane k-1 from the hand-off buffer
//     [B_a(k)   .. B_b(k)]  transport reads the vectors, updates plane k and
//                           writes N*, F* to hand-off buffer k & 1
// A cell that needs more than kChemBudget substeps stops there; its state
// goes to the continuation buffer and k_chem_cont finishes it.
#pragma once

#include "fused.hpp"

namespace emma {

constexpr int kWsTY = 4;  // rows of the tile = transport waves = chemistry waves

template <int G, typename R>
struct WsShared {
    // split vectors (times 2) of the plane being updated, every group
    Vec4<R> Ax[G][kWsTY][kTX + 1];
    Vec4<R> Bx[G][kWsTY][kTX + 1];
    Vec4<R> Ay[G][kWsTY + 1][kTX];
    Vec4<R> By[G][kWsTY][kTX];
    // N*, F* of a finished plane, [buffer][group][component][row][x]
    R hand[2][G][4][kWsTY][kTX];
};

template <int G, typename R, bool DIAG, bool FAST, bool FULL>
__global__ __launch_bounds__(2 * kTX * kWsTY, 2) void k_step_ws(TileArgs<R> a) {
    constexpr int TY = kWsTY;
    __shared__ WsShared<G, R> sh;
    const int wave = threadIdx.x >> 6;
    const int tid = threadIdx.x & (kTX * TY - 1);  // index within the role's 256 threads
    const int tx = tid & (kTX - 1), ty = tid >> 6;
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    const int tile_x = t % a.ntx, tile_y = (t / a.ntx) % a.nty, tile_z = t / (a.ntx * a.nty);
    const int nx = a.gr.nx, ny = a.gr.ny, nz = a.gr.nz;
    const int64_t V = a.gr.V;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    const int x0 = tile_x * kTX, y0 = tile_y * TY, z0 = tile_z * a.LZ;
    const int z1 = min(z0 + a.LZ, nz);
    const int np = z1 - z0;
    const int w = min(kTX, nx - x0), h = min(TY, ny - y0);
    const bool active = FULL || (tx < w && ty < h);
    const uint32_t col = active ? (uint32_t)(y0 + ty) * nx + (x0 + tx) : 0u;  // cell within a plane
    constexpr uint32_t E = sizeof(R);

    if (wave >= TY) {
        // ------------------------------------------------ chemistry waves
        ChemStats tot{0, 0, 0, 0};
        int maxsub = 0;
        // gas of the next plane, loaded one iteration ahead
        double xn = 0.0, Tn = 0.0, n0n = 0.0;
        if (active && np > 0) {
            const uint32_t zc = (uint32_t)z0 * plane + col;
            xn = ld(a.x, zc * 8u);
            Tn = ld(a.T, zc * 8u);
            n0n = ld(a.n0, zc * 8u);
        }
        for (int k = 0; k <= np; ++k) {
            bool stopped = false, done = false;
            SubState<G> s;
            s.st = ChemStats{0, 0, 0, 0};
            uint32_t zc = 0;
            if (k >= 1 && active) {
                const int buf = (k - 1) & 1;
                zc = (uint32_t)(z0 + k - 1) * plane + col;
                const double xg = xn, Tg = Tn, n0g = n0n;
                if (k < np) {  // prefetch the gas of the next plane
                    const uint32_t zn = zc + plane;
                    xn = ld(a.x, zn * 8u);
                    Tn = ld(a.T, zn * 8u);
                    n0n = ld(a.n0, zn * 8u);
                }
                double Nc[G], Sc[G];
#pragma unroll
                for (int g = 0; g < G; ++g) Nc[g] = (double)sh.hand[buf][g][0][ty][tx];
                source_of<G>((int64_t)zc, a.src.mask, a.src.sorted_cell, a.src.S, a.src.n, Sc);
                sub_start<G>(s, a.cp, Nc, xg, Tg, n0g);
                stopped = !sub_run<G, FAST>(s, a.gc, a.cp, n0g, Tg, Sc, kChemBudget);
                // the lanes that stopped take continuation slots (one atomic per wave)
                const uint32_t slot = defer_slot(a.wl, stopped, zc);
                if (stopped) {
                    if (slot < a.cb.cap) cont_save<G>(a.cb, slot, s);
                    else stopped = !sub_run<G, FAST>(s, a.gc, a.cp, n0g, Tg, Sc, 0x7fffffff);
                }
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    // F* goes to the output either way: a stopped cell's
                    // continuation scales it there by its factor product
                    const double pf = stopped ? 1.0 : s.Pf[g];
                    if (!stopped) st(a.No + (int64_t)g * V, zc * E, (R)s.N[g]);
#pragma unroll
                    for (int c = 1; c < 4; ++c)
                        st(a.Fo + (int64_t)(3 * g + c - 1) * V, zc * E,
                           (R)((double)sh.hand[buf][g][c][ty][tx] * pf));
                }
                if (!stopped) {
                    st(a.x, zc * 8u, s.x);
                    st(a.T, zc * 8u, sub_T<G, FAST>(s, a.cp, n0g, Tg));
                    done = true;
                }
            }
            if (DIAG && k >= 1) {
                const ChemStats c = done ? s.st : ChemStats{0, 0, 0, 0};
                tot.substeps += c.substeps;
                tot.attempts += c.attempts;
                tot.cap += c.cap;
                tot.xclamp += c.xclamp;
                maxsub = max(maxsub, c.substeps);
                wave_hist(a.cnt, done, c.substeps);
            }
            __syncthreads();  // B_a
            __syncthreads();  // B_b
        }
        if (DIAG) {
            wave_count(a.cnt, CNT_SUB, tot.substeps);
            wave_count(a.cnt, CNT_ATT, tot.attempts);
            wave_count(a.cnt, CNT_CAP, tot.cap);
            wave_count(a.cnt, CNT_XCLAMP, tot.xclamp);
            wave_count_max(a.cnt, CNT_MAXSUB, maxsub);
        }
        return;
    }

    // ---------------------------------------------------- transport waves
    // halo role: bottom row, top row, left column, right column of the tile;
    // across a non-periodic face the halo cell is the boundary cell itself and
    // hface names the face whose ghost it becomes
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
    const bool zlo_ghost = bd.kind[4] != BC_PERIODIC, zhi_ghost = bd.kind[5] != BC_PERIODIC;
    int hkind = BC_PERIODIC, hd = 0;
    R hsgn = R(1);
    if (hface >= 0) {
        hkind = bd.kind[hface];
        hd = hface >> 1;
        hsgn = (hface & 1) ? R(-1) : R(1);
    }
    const uint32_t hsrc = hrole >= 0 ? hcol : col;  // threads without a halo cell reload their own

    const R c = a.c, cc = c * c;
    const R hl = R(0.5) * a.lam, k0 = R(1) - R(3) * c * a.lam;
    auto zwrap = [nz](int z) { return (uint32_t)((z % nz + nz) % nz); };
    // rolling window of the own column: U of planes z (cur) and z + 1 (nxt),
    // 2 A_z of plane z - 1; plane z + 2 in flight (pre).  Closures are
    // recomputed where they are needed (plane z + 1's twice: for B_z of plane
    // z, then for its own split vectors) rather than kept across the barriers,
    // which keeps the transport role within the chemistry role's registers.
    // The halo cell's U is loaded within the phase that uses it.
    Vec4<R> cur[G], nxt[G], pre[G], Az2[G];
    int nlim = 0, nneg = 0;
    {
        Vec4<R> um[G];
        load_cell<G>(a.N, a.F, V, (zwrap(z0 - 1) * plane + col) * E, um);
        load_cell<G>(a.N, a.F, V, (zwrap(z0) * plane + col) * E, cur);
        load_cell<G>(a.N, a.F, V, (zwrap(min(z0 + 1, z1)) * plane + col) * E, nxt);
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (z0 == 0 && zlo_ghost) um[g] = ghost4(bd, 4, g, c, cur[g]);
            if (z0 + 1 == nz && zhi_ghost) nxt[g] = ghost4(bd, 5, g, c, cur[g]);
            R Pm[6];
            m1_pressure(um[g].n, um[g].fx, um[g].fy, um[g].fz, c, Pm, cc);
            Az2[g] = az2(um[g], Pm, c);
        }
    }

    for (int k = 0; k <= np; ++k) {
        const int z = z0 + k;
        Vec4<R> Azn[G];
        if (k < np) {
            Vec4<R> hal[G];
            load_cell<G>(a.N, a.F, V, ((uint32_t)z * plane + hsrc) * E, hal);
            // publish plane z: own cell and halo cell, every group
#pragma unroll
            for (int g = 0; g < G; ++g) {
                R Pc[6];
                m1_pressure(cur[g].n, cur[g].fx, cur[g].fy, cur[g].fz, c, Pc, cc);
                Azn[g] = az2(cur[g], Pc, c);
                if (active) {
                    Vec4<R> Ax, Bx, Ay, By;
                    split_xy(cur[g], Pc, c, Ax, Bx, Ay, By);
                    sh.Ax[g][ty][tx + 1] = Ax;
                    sh.Bx[g][ty][tx] = Bx;
                    sh.Ay[g][ty + 1][tx] = Ay;
                    if (ty > 0) sh.By[g][ty - 1][tx] = By;
                }
            }
            if (hrole >= 0) {
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    Vec4<R> hv = hal[g];
                    if (hkind == BC_REFLECTIVE) {
                        if (hd == 0) hv.fx = -hv.fx;
                        else if (hd == 1) hv.fy = -hv.fy;
                        else hv.fz = -hv.fz;
                    } else if (hkind == BC_INFLOW) {  // beam into the domain across the face
                        // the halo faces are x-, x+, y-, y+ (z faces are in the window)
                        const R phi = hface == 0 ? bd.phi[0][g]
                                    : hface == 1 ? bd.phi[1][g] : hface == 2 ? bd.phi[2][g] : bd.phi[3][g];
                        hv.n = phi / c;
                        hv.fx = hd == 0 ? hsgn * phi : R(0);
                        hv.fy = hd == 1 ? hsgn * phi : R(0);
                        hv.fz = hd == 2 ? hsgn * phi : R(0);
                    }
                    R Ph[6];
                    m1_pressure(hv.n, hv.fx, hv.fy, hv.fz, c, Ph, cc);
                    Vec4<R> Ax, Bx, Ay, By;
                    split_xy(hv, Ph, c, Ax, Bx, Ay, By);
                    if (hrole == 0) sh.Ay[g][0][hlx - 1] = Ay;            // row below the tile
                    else if (hrole == 1) sh.By[g][h - 1][hlx - 1] = By;   // row above
                    else if (hrole == 2) sh.Ax[g][hly - 1][0] = Ax;       // column left
                    else sh.Bx[g][hly - 1][w] = Bx;                       // column right
                }
            }
            // plane z + 2 (clamped to the first plane past the chunk: wrapped,
            // or replaced by a ghost across the top face) flies until the update
            load_cell<G>(a.N, a.F, V, (zwrap(min(z + 2, z1)) * plane + col) * E, pre);
        }
        __syncthreads();  // B_a
        if (k < np) {
            const int buf = k & 1;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const Vec4<R> aL = sh.Ax[g][ty][tx], bR = sh.Bx[g][ty][tx + 1];
                const Vec4<R> aD = sh.Ay[g][ty][tx], bT = sh.By[g][ty][tx];
                R Pn[6];
                m1_pressure(nxt[g].n, nxt[g].fx, nxt[g].fy, nxt[g].fz, c, Pn, cc);
                const Vec4<R> Bz = bz2(nxt[g], Pn, c);
                // (1 - 3 c lam) U + lam/2 (sum of the six split vectors, times 2)
                R n = k0 * cur[g].n + hl * ((aL.n + bR.n) + (aD.n + bT.n) + (Az2[g].n + Bz.n));
                R fx = k0 * cur[g].fx + hl * ((aL.fx + bR.fx) + (aD.fx + bT.fx) + (Az2[g].fx + Bz.fx));
                R fy = k0 * cur[g].fy + hl * ((aL.fy + bR.fy) + (aD.fy + bT.fy) + (Az2[g].fy + Bz.fy));
                R fz = k0 * cur[g].fz + hl * ((aL.fz + bR.fz) + (aD.fz + bT.fz) + (Az2[g].fz + Bz.fz));
                const int taken = floor_limit_fwd(n, fx, fy, fz, c);
                if (active) {
                    nneg += taken & 1;
                    nlim += taken >> 1;
                }
                sh.hand[buf][g][0][ty][tx] = n;
                sh.hand[buf][g][1][ty][tx] = fx;
                sh.hand[buf][g][2][ty][tx] = fy;
                sh.hand[buf][g][3][ty][tx] = fz;
                // roll the window up one plane
                Az2[g] = Azn[g];
                cur[g] = nxt[g];
                nxt[g] = pre[g];
                if (z + 2 == nz && zhi_ghost) nxt[g] = ghost4(bd, 5, g, c, cur[g]);  // cur = plane nz-1
            }
        }
        __syncthreads();  // B_b
    }
    if (DIAG) {
        wave_count(a.cnt, CNT_LIMITER, nlim);
        wave_count(a.cnt, CNT_NEG, nneg);
    }
}

template <int G, typename S, bool DIAG>
inline int launch_step_ws(hipStream_t st, const S *iN, const S *iF, S *oN, S *oF, double *x, double *T,
                          const double *n0, const Grid &gr, const SrcTable &src, const GroupConsts &gc,
                          const ChemParams &cp, double lam, unsigned long long *cnt, WorkList wl, ContBuf cb,
                          const Bounds<S> &bnd) {
    constexpr int TY = kWsTY;
    const int LZ = pick_lz(gr, TY);
    TileArgs<S> a = tile_args<G, S>(iN, iF, oN, oF, x, T, n0, gr, src, gc, cp, lam, cnt, LZ, wl, TY, bnd);
    a.cb = cb;
    const int nb = a.ntx * a.nty * a.ntz;
    const bool full = gr.nx % kTX == 0 && gr.ny % TY == 0;
    const bool fast = cp.otsa && !cp.isothermal;
    const dim3 blk(2 * kTX * TY);
    if (fast && full)
        hipLaunchKernelGGL((k_step_ws<G, S, DIAG, true, true>), dim3(nb), blk, 0, st, a);
    else if (fast)
        hipLaunchKernelGGL((k_step_ws<G, S, DIAG, true, false>), dim3(nb), blk, 0, st, a);
    else
        hipLaunchKernelGGL((k_step_ws<G, S, DIAG, false, false>), dim3(nb), blk, 0, st, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace emma
