// emma_rt.hip -- C ABI of the MI355X radiation step library (include/emma_rt.h).
//
// Host side: argument checks, scratch ownership, the per-call source table,
// the step loop and the diagnostics.  Every step of the path runs in the HIP
// kernels of kernels.hpp / fused.hpp / adjoint.hpp; nothing falls back to the
// host.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <new>
#include <vector>

#include "../../include/emma_rt.h"
#include "kernels.hpp"
#include "fused.hpp"
#include "step_ws.hpp"
#include "adjoint.hpp"

using namespace emma;

struct emma_rt_ctx {
    emma_rt_config cfg;
    hipStream_t stream;
    int device;
    Grid grid;
    size_t elem;           // bytes per N/F element (4 or 8)
    void *Ns, *Fs;         // transport output / fused ping-pong (storage precision)
    uint32_t *mask;        // one bit per cell: cell hosts a source
    uint32_t *refmask;     // one bit per cell: cell is refined (emma_rt_step_crta)
    int64_t mask_words;
    int64_t *sorted_cell;  // [EMMA_RT_MAX_SOURCES]
    int32_t *sorted_idx;
    int64_t *tile_key;     // [EMMA_RT_MAX_SOURCES]: sources sorted within tiles
    int32_t *tile_idx;
    double *S;             // [EMMA_RT_MAX_SOURCES][G]
    unsigned long long *cnt;     // [kCntSlots][CNT_COUNT]
    double *partial;             // [nblk][G+1]
    int diag_blocks;
    double *dsum;                // [G+1]
    uint32_t *work_count;        // [2]: cells deferred by the first chemistry pass; cells handed on
                                 // to the cooperative pass
    uint32_t *work_cells;        // [V]
    int list_blocks;             // grid of the second chemistry pass
    void *cont;                  // continuation states of the stopped cells (ContBuf)
    uint32_t cont_cap;
    AdjointScratch adj;
    Bounds<float> bnd_f;   // global boundaries in the storage precision
    Bounds<double> bnd_d;
    // kernel timing (emma_rt_profile_enable)
    int prof;
    std::vector<hipEvent_t> *ev;     // pool, pairs (start, stop)
    std::vector<int> *ev_kind;       // kernel kind of each pair in flight
    double prof_ms[KID_COUNT];
    int64_t prof_n[KID_COUNT];
    char err[512];
};

static char g_static_err[512] = "";

static int fail(emma_rt_ctx *c, int code, const char *fmt, ...) {
    char *buf = c ? c->err : g_static_err;
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, 512, fmt, ap);
    va_end(ap);
    return code;
}

#define HIP_TRY(ctx, call)                                                              \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail((ctx), EMMA_RT_EHIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

static int check_launch(emma_rt_ctx *c, const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(c, EMMA_RT_EHIP, "launch of %s failed: %s", what, hipGetErrorString(e));
    return EMMA_RT_OK;
}

// ---------------------------------------------------------- kernel timing
static const int kEventPairs = 512;

static int prof_flush(emma_rt_ctx *c) {
    const int n = (int)c->ev_kind->size();
    if (n == 0) return EMMA_RT_OK;
    HIP_TRY(c, hipEventSynchronize((*c->ev)[2 * n - 1]));
    for (int i = 0; i < n; ++i) {
        float ms = 0.f;
        HIP_TRY(c, hipEventElapsedTime(&ms, (*c->ev)[2 * i], (*c->ev)[2 * i + 1]));
        c->prof_ms[(*c->ev_kind)[i]] += ms;
        c->prof_n[(*c->ev_kind)[i]] += 1;
    }
    c->ev_kind->clear();
    return EMMA_RT_OK;
}

// Brackets one launch with events when timing is on.
struct Timed {
    emma_rt_ctx *c;
    int kind;
    bool on;
    Timed(emma_rt_ctx *c_, int kind_) : c(c_), kind(kind_), on(c_->prof != 0) {
        if (!on) return;
        if ((int)c->ev_kind->size() == kEventPairs) prof_flush(c);
        const int i = (int)c->ev_kind->size();
        (void)hipEventRecord((*c->ev)[2 * i], c->stream);
    }
    ~Timed() {
        if (!on) return;
        const int i = (int)c->ev_kind->size();
        (void)hipEventRecord((*c->ev)[2 * i + 1], c->stream);
        c->ev_kind->push_back(kind);
    }
};

static GroupConsts group_consts(const emma_rt_config &cfg) {
    GroupConsts gc;
    for (int g = 0; g < 4; ++g) {
        const bool on = g < cfg.n_groups;
        gc.sigN[g] = on ? cfg.sigma_N[g] : 0.0;
        gc.SigE[g] = on ? cfg.sigma_E[g] * cfg.mean_E[g] - cfg.sigma_N[g] * kE13 : 0.0;
        gc.frac[g] = on ? cfg.src_frac[g] : 0.0;
    }
    return gc;
}

template <typename S> static const Bounds<S> &bounds_of(const emma_rt_ctx *c);
template <> const Bounds<float> &bounds_of<float>(const emma_rt_ctx *c) { return c->bnd_f; }
template <> const Bounds<double> &bounds_of<double>(const emma_rt_ctx *c) { return c->bnd_d; }

template <typename S> static Bounds<S> make_bounds(const emma_rt_config &cfg) {
    Bounds<S> b;
    for (int f = 0; f < 6; ++f) {
        b.kind[f] = cfg.bc[f];
        for (int g = 0; g < EMMA_RT_MAX_GROUPS; ++g)
            b.phi[f][g] = (S)(cfg.bc[f] == BC_INFLOW && g < cfg.n_groups ? cfg.inflow[f] * cfg.src_frac[g] : 0.0);
    }
    return b;
}

static const char *config_error(const emma_rt_config *cfg) {
    if (!cfg) return "config is NULL";
    if (cfg->nx < 1 || cfg->ny < 1 || cfg->nz < 1) return "grid dimensions must be >= 1";
    // the chemistry work list holds 32-bit cell indices
    if ((int64_t)cfg->nx * cfg->ny * cfg->nz >= ((int64_t)1 << 32)) return "grid too large (at most 2^32 - 1 cells)";
    if (cfg->n_groups < 1 || cfg->n_groups > EMMA_RT_MAX_GROUPS) return "n_groups must be in 1..4";
    if (!(cfg->dx > 0) || !isfinite(cfg->dx)) return "dx must be > 0";
    if (!(cfg->c_red > 0) || cfg->c_red > kC * (1 + 1e-12)) return "c_red must be in (0, c]";
    if (cfg->precision != EMMA_RT_FP64 && cfg->precision != EMMA_RT_MIXED) return "bad precision";
    if (cfg->max_substeps < 1) return "max_substeps must be >= 1";
    if (cfg->adjoint_max_steps < 0) return "adjoint_max_steps must be >= 0";
    if (cfg->path < EMMA_RT_PATH_SPLIT || cfg->path > EMMA_RT_PATH_REFERENCE) return "bad path";
    for (int d = 0; d < 3; ++d) {
        const int a = cfg->bc[2 * d], b = cfg->bc[2 * d + 1];
        if (a < EMMA_RT_BC_PERIODIC || a > EMMA_RT_BC_INFLOW || b < EMMA_RT_BC_PERIODIC || b > EMMA_RT_BC_INFLOW)
            return "bc values must be emma_rt_bc kinds (0..3)";
        if ((a == EMMA_RT_BC_PERIODIC) != (b == EMMA_RT_BC_PERIODIC))
            return "both faces of an axis must be periodic or neither";
    }
    for (int f = 0; f < 6; ++f)
        if (!(cfg->inflow[f] >= 0) || !isfinite(cfg->inflow[f])) return "inflow must be finite and >= 0";
    if (cfg->flux != EMMA_RT_FLUX_GLF && cfg->flux != EMMA_RT_FLUX_HLL) return "bad flux";
    if (cfg->path != EMMA_RT_PATH_REFERENCE &&
        !tiled_supported(Grid{cfg->nx, cfg->ny, cfg->nz, (int64_t)cfg->nx * cfg->ny * cfg->nz}))
        return "grid too large for the tiled kernels (V * 8 bytes >= 4 GiB): use the reference path";
    for (int g = 0; g < cfg->n_groups; ++g) {
        if (!(cfg->sigma_N[g] >= 0) || !(cfg->sigma_E[g] >= 0) || !(cfg->mean_E[g] >= 0) ||
            !(cfg->src_frac[g] >= 0))
            return "group constants must be finite and >= 0";
    }
    return nullptr;
}

static int64_t field_bytes(const emma_rt_config *cfg) {
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    const int64_t e = cfg->precision == EMMA_RT_FP64 ? 8 : 4;
    return 4 * cfg->n_groups * V * e;  // N and F of all groups
}

// Slots of the continuation buffer: enough for every stopped cell in the
// workloads measured (well under 1 % of the cells per step) with a wide
// margin; cells stopped beyond it are finished by the first pass itself.
static uint32_t cont_capacity(int64_t V) {
    int64_t cap = V / 8 > 65536 ? V / 8 : 65536;
    return (uint32_t)(cap < V ? cap : V);
}

static int64_t cont_bytes(int G, uint32_t cap) { return (int64_t)cap * ((2 * G + 3) * 8 + 16 + 4); }

static ContBuf cont_view(void *base, int G, uint32_t cap) {
    ContBuf cb;
    double *d = (double *)base;
    cb.N = d;
    cb.Pf = d + (size_t)G * cap;
    cb.x = d + (size_t)2 * G * cap;
    cb.e = cb.x + cap;
    cb.rem = cb.e + cap;
    cb.st = (int32_t *)(cb.rem + cap);
    cb.next = (uint32_t *)(cb.st + (size_t)4 * cap);
    cb.cap = cap;
    return cb;
}

extern "C" int64_t emma_rt_scratch_bytes(const emma_rt_config *cfg) {
    if (config_error(cfg)) return -1;
    const int64_t V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    int64_t b = field_bytes(cfg);                          // Ns + Fs
    b += 2 * ((V + 31) / 32) * 4;                          // source and refinement masks
    b += V * 4 + 64;                                       // chemistry work list
    b += cont_bytes(cfg->n_groups, cont_capacity(V));      // continuation states
    b += (int64_t)EMMA_RT_MAX_SOURCES * (2 * (8 + 4) + 8 * cfg->n_groups);
    b += kCntSlots * CNT_COUNT * 8;
    b += ((V + 255) / 256) * (cfg->n_groups + 1) * 8 + (cfg->n_groups + 1) * 8;
    b += adjoint_scratch_bytes(*cfg);
    return b;
}

static void release(emma_rt_ctx *c) {
    if (!c) return;
    (void)hipFree(c->Ns);
    (void)hipFree(c->Fs);
    (void)hipFree(c->mask);
    (void)hipFree(c->refmask);
    (void)hipFree(c->sorted_cell);
    (void)hipFree(c->sorted_idx);
    (void)hipFree(c->tile_key);
    (void)hipFree(c->tile_idx);
    (void)hipFree(c->S);
    (void)hipFree(c->cnt);
    (void)hipFree(c->partial);
    (void)hipFree(c->dsum);
    (void)hipFree(c->work_count);
    (void)hipFree(c->work_cells);
    (void)hipFree(c->cont);
    adjoint_release(c->adj);
    if (c->ev) {
        for (hipEvent_t e : *c->ev) (void)hipEventDestroy(e);
        delete c->ev;
        delete c->ev_kind;
        c->ev = nullptr;
        c->ev_kind = nullptr;
    }
}

extern "C" int emma_rt_init(emma_rt_ctx **out, const emma_rt_config *cfg, void *stream) {
    if (!out) return fail(nullptr, EMMA_RT_EINVAL, "ctx out-pointer is NULL");
    *out = nullptr;
    if (const char *why = config_error(cfg)) return fail(nullptr, EMMA_RT_EINVAL, "%s", why);
    emma_rt_ctx *c = new (std::nothrow) emma_rt_ctx();
    if (!c) return fail(nullptr, EMMA_RT_ENOMEM, "host allocation failed");
    memset(c, 0, sizeof(*c));
    c->cfg = *cfg;
    c->stream = (hipStream_t)stream;
    c->grid.nx = cfg->nx;
    c->grid.ny = cfg->ny;
    c->grid.nz = cfg->nz;
    c->grid.V = (int64_t)cfg->nx * cfg->ny * cfg->nz;
    c->elem = cfg->precision == EMMA_RT_FP64 ? 8 : 4;
    c->bnd_f = make_bounds<float>(*cfg);
    c->bnd_d = make_bounds<double>(*cfg);
    (void)hipGetDevice(&c->device);
    const int64_t V = c->grid.V;
    const int G = cfg->n_groups;
    c->mask_words = (V + 31) / 32;
    c->cont_cap = cont_capacity(V);
    c->diag_blocks = (int)((V + 255) / 256);
    {
        // persistent second chemistry pass: a few waves per SIMD of the device
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess || cus < 1)
            cus = 256;
        const int64_t want = (int64_t)cus * 8;
        c->list_blocks = (int)(want < c->diag_blocks ? want : c->diag_blocks);
    }
    struct { void **p; size_t n; } allocs[] = {
        {&c->Ns, (size_t)(G * V) * c->elem},
        {&c->Fs, (size_t)(3 * G * V) * c->elem},
        {(void **)&c->mask, (size_t)c->mask_words * 4},
        {(void **)&c->refmask, (size_t)c->mask_words * 4},
        {(void **)&c->sorted_cell, (size_t)EMMA_RT_MAX_SOURCES * 8},
        {(void **)&c->sorted_idx, (size_t)EMMA_RT_MAX_SOURCES * 4},
        {(void **)&c->tile_key, (size_t)EMMA_RT_MAX_SOURCES * 8},
        {(void **)&c->tile_idx, (size_t)EMMA_RT_MAX_SOURCES * 4},
        {(void **)&c->S, (size_t)EMMA_RT_MAX_SOURCES * G * 8},
        {(void **)&c->cnt, (size_t)kCntSlots * CNT_COUNT * 8},
        {(void **)&c->partial, (size_t)c->diag_blocks * (G + 1) * 8},
        {(void **)&c->dsum, (size_t)(G + 1) * 8},
        {(void **)&c->work_count, (size_t)64},
        {(void **)&c->work_cells, (size_t)V * 4},
        {&c->cont, (size_t)cont_bytes(G, c->cont_cap)},
    };
    for (auto &a : allocs) {
        if (hipMalloc(a.p, a.n) != hipSuccess) {
            (void)hipGetLastError();
            release(c);
            delete c;
            return fail(nullptr, EMMA_RT_ENOMEM, "hipMalloc of %zu bytes failed", a.n);
        }
    }
    if (adjoint_alloc(c->adj, *cfg) != 0) {
        (void)hipGetLastError();
        release(c);
        delete c;
        return fail(nullptr, EMMA_RT_ENOMEM, "adjoint tape allocation failed");
    }
    c->err[0] = 0;
    *out = c;
    return EMMA_RT_OK;
}

extern "C" void emma_rt_free(emma_rt_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

extern "C" const char *emma_rt_last_error(const emma_rt_ctx *c) { return c ? c->err : g_static_err; }

// ------------------------------------------------------------ source table
template <int G>
static int build_sources(emma_rt_ctx *c, const int64_t *cell, const double *rate, int n) {
    const int tb = 256;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((c->mask_words + tb - 1) / tb)), dim3(tb), 0,
                       c->stream, c->mask, c->mask_words, 0u);
    if (int e = check_launch(c, "k_fill_u32")) return e;
    if (n == 0) return EMMA_RT_OK;
    Timed tr(c, KID_SRC);
    hipLaunchKernelGGL(k_src_tile_sort, dim3((n + kSrcTile - 1) / kSrcTile), dim3(kSrcTile), 0, c->stream, cell, n,
                       c->grid.V, c->tile_key, c->tile_idx, c->cnt);
    hipLaunchKernelGGL(k_src_rank, dim3((n + tb - 1) / tb), dim3(tb), 0, c->stream, cell, n, c->grid.V,
                       c->tile_key, c->tile_idx, c->sorted_cell, c->sorted_idx);
    if (int e = check_launch(c, "k_src_rank")) return e;
    const double vol = c->cfg.dx * c->cfg.dx * c->cfg.dx;
    hipLaunchKernelGGL(k_src_heads<G>, dim3((n + tb - 1) / tb), dim3(tb), 0, c->stream, c->sorted_cell,
                       c->sorted_idx, rate, n, group_consts(c->cfg), 0.0, vol, c->S, c->mask);
    return check_launch(c, "k_src_heads");
}

// --------------------------------------------------------------- step loop
// Second chemistry pass over the cells the first pass deferred (in = where
// their post-transport N*, F* are, out = where the step's result goes).
template <int G, typename S, bool DIAG>
static int launch_chem_list(emma_rt_ctx *c, const S *inN, const S *inF, S *oN, S *oF, double *x, double *T,
                            const double *n0, const SrcTable &src, const GroupConsts &gc, const ChemParams &cp) {
    const WorkList wl{c->work_count, c->work_cells};
    const unsigned nb = (unsigned)c->list_blocks;
    Timed t(c, KID_CHEM_LIST);
    if (cp.otsa && !cp.isothermal)
        hipLaunchKernelGGL((k_chem_list<G, S, DIAG, true>), dim3(nb), dim3(256), 0, c->stream, inN, inF, oN, oF, x,
                           T, n0, c->grid.V, src, gc, cp, c->cnt, wl);
    else
        hipLaunchKernelGGL((k_chem_list<G, S, DIAG, false>), dim3(nb), dim3(256), 0, c->stream, inN, inF, oN, oF,
                           x, T, n0, c->grid.V, src, gc, cp, c->cnt, wl);
    return check_launch(c, "k_chem_list");
}

// First chemistry pass over every cell (skip: refined cells, or null).
// xo, To null: x, T updated in place; else the tape form of k_chem: Ns, Fs
// before the floor and the limiter, x, T read only, the results in xo, To,
// and with multi the cells whose subcycle was not a single substep.
template <int G, typename S, bool DIAG, bool FAST>
static int launch_chem(emma_rt_ctx *c, const S *Ns, const S *Fs, S *N, S *F, double *x, double *T, double *xo,
                       double *To, const double *n0, const SrcTable &src, const GroupConsts &gc, const ChemParams &cp,
                       const uint32_t *skip, uint64_t *multi = nullptr) {
    const int64_t V = c->grid.V;
    const WorkList wl{c->work_count, c->work_cells};
    const int tb = chem_tb<S>();
    const ContBuf cb = cont_view(c->cont, G, c->cont_cap);
    const dim3 nb((unsigned)((V + tb - 1) / tb));
    if (xo)
        hipLaunchKernelGGL((k_chem<G, S, DIAG, FAST, true>), nb, dim3(tb), 0, c->stream, Ns, Fs, N, F, x, T, xo, To,
                           n0, V, src, gc, cp, c->cnt, wl, cb, skip, multi);
    else
        hipLaunchKernelGGL((k_chem<G, S, DIAG, FAST, false>), nb, dim3(tb), 0, c->stream, Ns, Fs, N, F, x, T,
                           nullptr, nullptr, n0, V, src, gc, cp, c->cnt, wl, cb, skip, nullptr);
    return check_launch(c, "chemistry");
}

// Second pass of the split path: the subcycles the first pass stopped,
// continued from their saved states.  Ns_pre non-null: the tape form (the
// transport output before the floor and the limiter, see k_chem).
template <int G, typename S, bool DIAG>
static int launch_chem_cont(emma_rt_ctx *c, const S *Fs, S *N, S *F, const double *T, double *xo, double *To,
                            const double *n0, const SrcTable &src, const GroupConsts &gc, const ChemParams &cp,
                            const S *Ns_pre = nullptr) {
    const WorkList wl{c->work_count, c->work_cells};
    const ContBuf cb = cont_view(c->cont, G, c->cont_cap);
    const unsigned nb = (unsigned)c->list_blocks;
    const bool fast = cp.otsa && !cp.isothermal;
    Timed t(c, KID_CHEM_LIST);
    const dim3 grid(nb), block(256);
    const int64_t V = c->grid.V;
    // on-the-spot, energy-evolving mode: cells still going after
    // kContBudget substeps finish in the cooperative pass
    const bool coop = fast && kContBudget > 0;
    const int budget = coop ? kContBudget : 0x7fffffff;
    if (Ns_pre) {
        if (fast)
            hipLaunchKernelGGL((k_chem_cont<G, S, DIAG, true, true>), grid, block, 0, c->stream, Ns_pre, Fs, N, F, T,
                               xo, To, n0, V, src, gc, cp, c->cnt, wl, cb, budget);
        else
            hipLaunchKernelGGL((k_chem_cont<G, S, DIAG, false, true>), grid, block, 0, c->stream, Ns_pre, Fs, N, F,
                               T, xo, To, n0, V, src, gc, cp, c->cnt, wl, cb, budget);
    } else if (fast) {
        hipLaunchKernelGGL((k_chem_cont<G, S, DIAG, true>), grid, block, 0, c->stream, nullptr, Fs, N, F, T, xo, To,
                           n0, V, src, gc, cp, c->cnt, wl, cb, budget);
    } else {
        hipLaunchKernelGGL((k_chem_cont<G, S, DIAG, false>), grid, block, 0, c->stream, nullptr, Fs, N, F, T, xo, To,
                           n0, V, src, gc, cp, c->cnt, wl, cb, budget);
    }
    if (int e = check_launch(c, "k_chem_cont")) return e;
    if (!coop) return EMMA_RT_OK;
    if (Ns_pre)
        hipLaunchKernelGGL((k_chem_coop<G, S, DIAG, true>), grid, block, 0, c->stream, Ns_pre, Fs, N, F, T, xo, To,
                           n0, V, src, gc, cp, c->cnt, wl, cb);
    else
        hipLaunchKernelGGL((k_chem_coop<G, S, DIAG>), grid, block, 0, c->stream, nullptr, Fs, N, F, T, xo, To, n0,
                           V, src, gc, cp, c->cnt, wl, cb);
    return check_launch(c, "k_chem_coop");
}

static int reset_worklist(emma_rt_ctx *c) {
    // [0]: the first pass's stopped cells, [1]: the ones handed on to the cooperative pass
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, c->work_count, (int64_t)2, 0u);
    return check_launch(c, "k_fill_u32 (work list)");
}

template <int G, typename S, bool DIAG>
static int run_steps(emma_rt_ctx *c, S *N, S *F, double *x, double *T, const double *n0, int n_src,
                     double dt, int n_steps) {
    const Grid gr = c->grid;
    const int64_t V = gr.V;
    const int tb = 256;
    const unsigned nblk = (unsigned)((V + tb - 1) / tb);
    const GroupConsts gc = group_consts(c->cfg);
    ChemParams cp;
    cp.c = c->cfg.c_red;
    cp.dt = dt;
    cp.otsa = c->cfg.otsa;
    cp.isothermal = c->cfg.isothermal;
    cp.max_substeps = c->cfg.max_substeps;
    SrcTable src{c->mask, c->sorted_cell, c->S, n_src};
    const WorkList wl{c->work_count, c->work_cells};
    S *Ns = (S *)c->Ns, *Fs = (S *)c->Fs;
    const S cr = (S)c->cfg.c_red;
    const S lam = (S)(dt / c->cfg.dx);
    if (c->cfg.path == EMMA_RT_PATH_FUSED) {
        // ping-pong: even steps read the caller's buffers, odd steps the scratch
        for (int s = 0; s < n_steps; ++s) {
            const bool even = (s & 1) == 0;
            S *iN = even ? N : Ns, *iF = even ? F : Fs;
            S *oN = even ? Ns : N, *oF = even ? Fs : F;
            if (int e = reset_worklist(c)) return e;
            if (c->cfg.flux == EMMA_RT_FLUX_HLL) {
                // the HLL flux: one thread per cell, transport then chemistry
                {
                    Timed t(c, KID_FUSED);
                    if (cp.otsa && !cp.isothermal)
                        hipLaunchKernelGGL((k_step_cell<G, S, DIAG, true>), dim3(nblk), dim3(tb), 0, c->stream, iN,
                                           iF, oN, oF, x, T, n0, gr, cr, lam, src, gc, cp, c->cnt, wl,
                                           bounds_of<S>(c));
                    else
                        hipLaunchKernelGGL((k_step_cell<G, S, DIAG, false>), dim3(nblk), dim3(tb), 0, c->stream, iN,
                                           iF, oN, oF, x, T, n0, gr, cr, lam, src, gc, cp, c->cnt, wl,
                                           bounds_of<S>(c));
                }
                if (int e = check_launch(c, "k_step_cell")) return e;
                if (int e = launch_chem_list<G, S, DIAG>(c, oN, oF, oN, oF, x, T, n0, src, gc, cp)) return e;
                continue;
            }
            int e;
            // single precision: the kernel with transport and chemistry waves
            // (step_ws.hpp); the FP64 state needs twice its LDS, so FP64 keeps
            // the kernel that runs both on the same waves (fused.hpp)
            constexpr bool ws = sizeof(S) == 4;
            {
                Timed t(c, KID_FUSED);
                if constexpr (ws)
                    e = launch_step_ws<G, S, DIAG>(c->stream, iN, iF, oN, oF, x, T, n0, gr, src, gc, cp,
                                                   dt / c->cfg.dx, c->cnt, wl, cont_view(c->cont, G, c->cont_cap),
                                                   bounds_of<S>(c));
                else
                    e = launch_fused<G, S, DIAG>(c->stream, iN, iF, oN, oF, x, T, n0, gr, src, gc, cp,
                                                 dt / c->cfg.dx, c->cnt, wl, bounds_of<S>(c));
            }
            if (e) return fail(c, EMMA_RT_EHIP, "fused kernel launch failed: %s",
                               hipGetErrorString(hipGetLastError()));
            if constexpr (ws) {
                // stopped cells: continue from their saved states; their F* is in the output
                if (int e2 = launch_chem_cont<G, S, DIAG>(c, oF, oN, oF, T, x, T, n0, src, gc, cp)) return e2;
            } else {
                // deferred cells: N*, F* were written to the output, finish them in place
                if (int e2 = launch_chem_list<G, S, DIAG>(c, oN, oF, oN, oF, x, T, n0, src, gc, cp)) return e2;
            }
        }
        if (n_steps & 1) {
            HIP_TRY(c, hipMemcpyAsync(N, Ns, (size_t)G * V * sizeof(S), hipMemcpyDeviceToDevice, c->stream));
            HIP_TRY(c, hipMemcpyAsync(F, Fs, (size_t)3 * G * V * sizeof(S), hipMemcpyDeviceToDevice, c->stream));
        }
        return EMMA_RT_OK;
    }
    for (int s = 0; s < n_steps; ++s) {
        if (c->cfg.path == EMMA_RT_PATH_SPLIT && c->cfg.flux == EMMA_RT_FLUX_HLL) {
            Timed t(c, KID_TRANSPORT);
            launch_transport_tiled_hll<G, S, DIAG>(c->stream, N, F, Ns, Fs, gr, cp, dt / c->cfg.dx, c->cnt,
                                                   bounds_of<S>(c));
        } else if (c->cfg.path == EMMA_RT_PATH_SPLIT) {
            Timed t(c, KID_TRANSPORT);
            launch_transport_tiled<G, S, DIAG>(c->stream, N, F, Ns, Fs, gr, cp, dt / c->cfg.dx, c->cnt,
                                               bounds_of<S>(c));
        } else if (c->cfg.flux == EMMA_RT_FLUX_HLL) {
            Timed t(c, KID_TRANSPORT);
            hipLaunchKernelGGL((k_transport<G, S, DIAG, false, true>), dim3(nblk), dim3(tb), 0, c->stream, N, F,
                               Ns, Fs, gr, cr, lam, c->cnt, bounds_of<S>(c));
        } else {
            Timed t(c, KID_TRANSPORT);
            hipLaunchKernelGGL((k_transport<G, S, DIAG>), dim3(nblk), dim3(tb), 0, c->stream, N, F, Ns,
                               Fs, gr, cr, lam, c->cnt, bounds_of<S>(c));
        }
        if (int e = check_launch(c, "k_transport")) return e;
        if (int e = reset_worklist(c)) return e;
        {
            Timed t(c, KID_CHEM);
            const int e = (cp.otsa && !cp.isothermal)
                              ? launch_chem<G, S, DIAG, true>(c, Ns, Fs, N, F, x, T, nullptr, nullptr, n0, src, gc, cp, nullptr)
                              : launch_chem<G, S, DIAG, false>(c, Ns, Fs, N, F, x, T, nullptr, nullptr, n0, src, gc,
                                                               cp, nullptr);
            if (e) return e;
        }
        if (int e = launch_chem_cont<G, S, DIAG>(c, Fs, N, F, T, x, T, n0, src, gc, cp)) return e;
    }
    return EMMA_RT_OK;
}

template <int G, typename S>
static int diag_finish(emma_rt_ctx *c, const S *N, const S *F, const double *x, const double *T,
                       const double *n0, emma_rt_diag *d) {
    hipLaunchKernelGGL((k_diag_partial<G, S>), dim3(c->diag_blocks), dim3(256), 0, c->stream, N, F, x, T,
                       n0, c->grid.V, c->partial, c->cnt);
    if (int e = check_launch(c, "k_diag_partial")) return e;
    hipLaunchKernelGGL((k_diag_final<G>), dim3(1), dim3(256), 0, c->stream, c->partial, c->diag_blocks,
                       c->dsum);
    if (int e = check_launch(c, "k_diag_final")) return e;
    unsigned long long slots[kCntSlots * CNT_COUNT], cnt[CNT_COUNT];
    double sums[EMMA_RT_MAX_GROUPS + 1];
    HIP_TRY(c, hipMemcpyAsync(slots, c->cnt, sizeof(slots), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipMemcpyAsync(sums, c->dsum, (G + 1) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < CNT_COUNT; ++k) {
        cnt[k] = 0;
        for (int j = 0; j < kCntSlots; ++j) {
            const unsigned long long v = slots[j * CNT_COUNT + k];
            cnt[k] = k == CNT_MAXSUB ? (v > cnt[k] ? v : cnt[k]) : cnt[k] + v;
        }
    }
    const double vol = c->cfg.dx * c->cfg.dx * c->cfg.dx;
    memset(d, 0, sizeof(*d));
    for (int g = 0; g < G; ++g) d->photons[g] = sums[g] * vol;
    d->ionised = sums[G] * vol;
    d->substeps = (int64_t)cnt[CNT_SUB];
    d->attempts = (int64_t)cnt[CNT_ATT];
    d->max_sub = (int32_t)cnt[CNT_MAXSUB];
    d->limiter_hits = (int64_t)cnt[CNT_LIMITER];
    d->neg_clamps = (int64_t)cnt[CNT_NEG];
    d->x_clamps = (int64_t)cnt[CNT_XCLAMP];
    d->cap_hits = (int64_t)cnt[CNT_CAP];
    d->nonfinite = (int64_t)cnt[CNT_NONFINITE];
    for (int b = 0; b < EMMA_RT_SUBSTEP_BINS; ++b) d->substep_hist[b] = (int64_t)cnt[CNT_HIST + b];
    if (cnt[CNT_BADSRC]) return fail(c, EMMA_RT_EINVAL, "%llu source cell indices outside the grid were ignored",
                                     cnt[CNT_BADSRC]);
    if (cnt[CNT_BADREF])
        return fail(c, EMMA_RT_EINVAL, "%llu refined-cell entries (outside the grid or repeated) or source children "
                    "outside 0..r^3-1 were ignored", cnt[CNT_BADREF]);
    if (d->nonfinite) return fail(c, EMMA_RT_ENONFINITE, "%lld cells hold NaN/Inf", (long long)d->nonfinite);
    if (d->cap_hits) return fail(c, EMMA_RT_ESUBSTEP, "substep guard fired in %lld cell-steps",
                                 (long long)d->cap_hits);
    return EMMA_RT_OK;
}

template <int G, typename S>
static int step_typed(emma_rt_ctx *c, S *N, S *F, double *x, double *T, const double *n0,
                      const int64_t *cell, const double *rate, int n_src, double dt, int n_steps,
                      emma_rt_diag *d) {
    if (d) {
        hipLaunchKernelGGL(k_fill_u64, dim3((kCntSlots * CNT_COUNT + 255) / 256), dim3(256), 0, c->stream,
                           c->cnt, (int)(kCntSlots * CNT_COUNT), 0ull);
        if (int e = check_launch(c, "k_fill_u64")) return e;
    }
    if (int e = build_sources<G>(c, cell, rate, n_src)) return e;
    int e = d ? run_steps<G, S, true>(c, N, F, x, T, n0, n_src, dt, n_steps)
              : run_steps<G, S, false>(c, N, F, x, T, n0, n_src, dt, n_steps);
    if (e) return e;
    if (d) return diag_finish<G, S>(c, N, F, x, T, n0, d);
    return EMMA_RT_OK;
}

// Checks shared by emma_rt_step and emma_rt_step_noalloc (c holds the config).
static int step_args(emma_rt_ctx *c, const void *N, const void *F, const double *x, const double *T,
                     const double *n0, const int64_t *cell, const double *rate, int32_t n_src, double dt,
                     int32_t n_steps) {
    if (!N || !F || !x || !T || !n0) return fail(c, EMMA_RT_EINVAL, "a field pointer is NULL");
    if (n_src < 0 || n_src > EMMA_RT_MAX_SOURCES)
        return fail(c, EMMA_RT_EINVAL, "n_src must be in 0..%d", EMMA_RT_MAX_SOURCES);
    if (n_src > 0 && (!cell || !rate)) return fail(c, EMMA_RT_EINVAL, "source arrays are NULL");
    if (n_steps < 0) return fail(c, EMMA_RT_EINVAL, "n_steps must be >= 0");
    if (!(dt > 0) || !isfinite(dt)) return fail(c, EMMA_RT_EINVAL, "dt must be > 0");
    if (dt > c->cfg.dx / (3.0 * c->cfg.c_red) * (1.0 + 1e-12))
        return fail(c, EMMA_RT_EINVAL, "dt = %g exceeds dx/(3 c_red) = %g", dt, c->cfg.dx / (3.0 * c->cfg.c_red));
    return EMMA_RT_OK;
}

static int step_dispatch(emma_rt_ctx *c, void *N, void *F, double *x, double *T, const double *n0,
                         const int64_t *cell, const double *rate, int32_t n_src, double dt, int32_t n_steps,
                         emma_rt_diag *d) {
    const int G = c->cfg.n_groups;
    const bool f64 = c->cfg.precision == EMMA_RT_FP64;
#define DISPATCH(GG)                                                                                      \
    case GG:                                                                                              \
        return f64 ? step_typed<GG, double>(c, (double *)N, (double *)F, x, T, n0, cell, rate, n_src, dt, \
                                            n_steps, d)                                                   \
                   : step_typed<GG, float>(c, (float *)N, (float *)F, x, T, n0, cell, rate, n_src, dt,    \
                                           n_steps, d);
    switch (G) {
        DISPATCH(1)
        DISPATCH(2)
        DISPATCH(3)
        DISPATCH(4)
    }
#undef DISPATCH
    return fail(c, EMMA_RT_EINVAL, "n_groups out of range");
}

extern "C" int emma_rt_step(emma_rt_ctx *c, void *N, void *F, double *x, double *T, const double *n0,
                            const int64_t *cell, const double *rate, int32_t n_src, double dt,
                            int32_t n_steps, emma_rt_diag *d) {
    if (!c) return fail(nullptr, EMMA_RT_EINVAL, "ctx is NULL");
    if (int e = step_args(c, N, F, x, T, n0, cell, rate, n_src, dt, n_steps)) return e;
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != c->device) return fail(c, EMMA_RT_EINVAL, "current device %d is not the context's %d", dev, c->device);
    c->err[0] = 0;
    return step_dispatch(c, N, F, x, T, n0, cell, rate, n_src, dt, n_steps, d);
}

// ------------------------------------------- allocation-free step variant
// emma_rt_step for callers that cannot allocate device memory: the scratch a
// context would own (transport output / ping-pong fields, source table,
// counters, chemistry work list) is carved out of this fixed array instead.
// In host code `scratch` only names the symbol; its device address comes from
// hipGetSymbolAddress, taken once per device on the first call there.
static __device__ __align__(256) unsigned char scratch[EMMA_RT_NOALLOC_SCRATCH_BYTES];

static const int kMaxDevices = 64;
static void *g_scratch_ptr[kMaxDevices];
static std::mutex g_scratch_mu;

// Device address of this device's copy of `scratch` (nullptr on failure,
// with the reason in g_static_err).
static void *scratch_on(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            fail(nullptr, EMMA_RT_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", dev,
                 hipGetErrorString(e));
            return nullptr;
        }
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}

// Places the step's scratch at 256-byte aligned offsets from base (which may
// be null to measure); returns the bytes used.
static int64_t noalloc_layout(emma_rt_ctx *c, unsigned char *base, int n_src) {
    const int64_t V = c->grid.V;
    const int G = c->cfg.n_groups;
    int64_t off = 0;
    auto take = [&](int64_t n) {
        unsigned char *p = base ? base + off : nullptr;
        off += (n + 255) / 256 * 256;
        return (void *)p;
    };
    c->Ns = take((int64_t)G * V * (int64_t)c->elem);
    c->Fs = take((int64_t)3 * G * V * (int64_t)c->elem);
    c->mask = (uint32_t *)take(c->mask_words * 4);
    c->sorted_cell = (int64_t *)take((int64_t)n_src * 8);
    c->sorted_idx = (int32_t *)take((int64_t)n_src * 4);
    c->tile_key = (int64_t *)take((int64_t)n_src * 8);
    c->tile_idx = (int32_t *)take((int64_t)n_src * 4);
    c->S = (double *)take((int64_t)n_src * G * 8);
    c->cnt = (unsigned long long *)take((int64_t)kCntSlots * CNT_COUNT * 8);
    c->work_count = (uint32_t *)take(64);
    c->work_cells = (uint32_t *)take(V * 4);
    c->cont = take(cont_bytes(G, c->cont_cap));
    return off;
}

extern "C" int emma_rt_step_noalloc(const emma_rt_config *cfg, void *stream, void *N, void *F, double *x,
                                    double *T, const double *n0, const int64_t *cell, const double *rate,
                                    int32_t n_src, double dt, int32_t n_steps) {
    if (const char *why = config_error(cfg)) return fail(nullptr, EMMA_RT_EINVAL, "%s", why);
    // a context on the stack: host memory only, its device pointers set below
    emma_rt_ctx c;
    memset(&c, 0, sizeof(c));
    c.cfg = *cfg;
    c.stream = (hipStream_t)stream;
    c.grid = Grid{cfg->nx, cfg->ny, cfg->nz, (int64_t)cfg->nx * cfg->ny * cfg->nz};
    c.elem = cfg->precision == EMMA_RT_FP64 ? 8 : 4;
    c.bnd_f = make_bounds<float>(*cfg);
    c.bnd_d = make_bounds<double>(*cfg);
    c.mask_words = (c.grid.V + 31) / 32;
    c.cont_cap = cont_capacity(c.grid.V);
    int rc = step_args(&c, N, F, x, T, n0, cell, rate, n_src, dt, n_steps);
    if (rc == EMMA_RT_OK) {
        const int64_t need = noalloc_layout(&c, nullptr, n_src);
        if (need > (int64_t)EMMA_RT_NOALLOC_SCRATCH_BYTES)
            rc = fail(&c, EMMA_RT_EINVAL,
                      "grid and sources need %lld bytes of scratch, above the fixed %lld of "
                      "emma_rt_step_noalloc: use emma_rt_init / emma_rt_step",
                      (long long)need, (long long)EMMA_RT_NOALLOC_SCRATCH_BYTES);
    }
    if (rc == EMMA_RT_OK) {
        int dev = -1;
        if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
            return fail(nullptr, EMMA_RT_EHIP, "no usable current HIP device");
        c.device = dev;
        void *base = scratch_on(dev);
        if (!base) return EMMA_RT_EHIP;
        noalloc_layout(&c, (unsigned char *)base, n_src);
        int cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
        const int64_t blocks = (c.grid.V + 255) / 256;
        c.list_blocks = (int)((int64_t)cus * 8 < blocks ? (int64_t)cus * 8 : blocks);
        // the counters take atomic adds (bad source cells) and must start at zero
        hipLaunchKernelGGL(k_fill_u64, dim3((kCntSlots * CNT_COUNT + 255) / 256), dim3(256), 0, c.stream, c.cnt,
                           (int)(kCntSlots * CNT_COUNT), 0ull);
        rc = check_launch(&c, "k_fill_u64");
        if (rc == EMMA_RT_OK) rc = step_dispatch(&c, N, F, x, T, n0, cell, rate, n_src, dt, n_steps, nullptr);
    }
    if (rc != EMMA_RT_OK) memcpy(g_static_err, c.err, sizeof(g_static_err));
    else g_static_err[0] = 0;
    return rc;
}

// ------------------------------------------------- refined cells (Sec. 5)
template <int G, typename S, bool DIAG, int NC>
static int crta_steps(emma_rt_ctx *c, S *N, S *F, double *x, double *T, const double *n0, const double *rate,
                      const int32_t *src_child, int n_src, double dt, int n_steps, const int64_t *ref_cell,
                      int n_ref, double *xf, double *Tf, const double *nf) {
    const Grid gr = c->grid;
    const int64_t V = gr.V;
    const int tb = 256;
    const unsigned nblk = (unsigned)((V + tb - 1) / tb);
    const GroupConsts gc = group_consts(c->cfg);
    ChemParams cp;
    cp.c = c->cfg.c_red;
    cp.dt = dt;
    cp.otsa = c->cfg.otsa;
    cp.isothermal = c->cfg.isothermal;
    cp.max_substeps = c->cfg.max_substeps;
    const bool fast = cp.otsa && !cp.isothermal;
    SrcTable src{c->mask, c->sorted_cell, c->S, n_src};
    S *Ns = (S *)c->Ns, *Fs = (S *)c->Fs;
    const S cr = (S)c->cfg.c_red;
    const S lam = (S)(dt / c->cfg.dx);
    const double hf = c->cfg.dx / (NC == 8 ? 2 : 4);
    const double volf = hf * hf * hf;
    const unsigned fblk = (unsigned)(((int64_t)n_ref * NC + tb - 1) / tb);
    for (int s = 0; s < n_steps; ++s) {
        {
            Timed t(c, KID_TRANSPORT);
            if (c->cfg.path != EMMA_RT_PATH_REFERENCE && c->cfg.flux == EMMA_RT_FLUX_HLL)
                launch_transport_tiled_hll<G, S, DIAG>(c->stream, N, F, Ns, Fs, gr, cp, dt / c->cfg.dx, c->cnt,
                                                       bounds_of<S>(c));
            else if (c->cfg.path != EMMA_RT_PATH_REFERENCE)
                launch_transport_tiled<G, S, DIAG>(c->stream, N, F, Ns, Fs, gr, cp, dt / c->cfg.dx, c->cnt,
                                                   bounds_of<S>(c));
            else if (c->cfg.flux == EMMA_RT_FLUX_HLL)
                hipLaunchKernelGGL((k_transport<G, S, DIAG, false, true>), dim3(nblk), dim3(tb), 0, c->stream, N,
                                   F, Ns, Fs, gr, cr, lam, c->cnt, bounds_of<S>(c));
            else
                hipLaunchKernelGGL((k_transport<G, S, DIAG>), dim3(nblk), dim3(tb), 0, c->stream, N, F, Ns, Fs, gr,
                                   cr, lam, c->cnt, bounds_of<S>(c));
        }
        if (int e = check_launch(c, "transport")) return e;
        if (int e = reset_worklist(c)) return e;
        {
            Timed t(c, KID_CHEM);
            const int e = fast ? launch_chem<G, S, DIAG, true>(c, Ns, Fs, N, F, x, T, nullptr, nullptr, n0, src, gc, cp,
                                                               c->refmask)
                               : launch_chem<G, S, DIAG, false>(c, Ns, Fs, N, F, x, T, nullptr, nullptr, n0, src, gc,
                                                                cp, c->refmask);
            if (e) return e;
        }
        if (int e = launch_chem_cont<G, S, DIAG>(c, Fs, N, F, T, x, T, n0, src, gc, cp)) return e;
        if (n_ref > 0) {
            Timed t(c, KID_CRTA);
            if (fast)
                hipLaunchKernelGGL((k_crta_fine<G, S, DIAG, true, NC>), dim3(fblk), dim3(tb), 0, c->stream, Ns, Fs,
                                   N, F, x, T, V, ref_cell, n_ref, xf, Tf, xf, Tf, nf, c->sorted_cell, c->sorted_idx,
                                   rate, src_child, n_src, gc, cp, volf, c->cnt);
            else
                hipLaunchKernelGGL((k_crta_fine<G, S, DIAG, false, NC>), dim3(fblk), dim3(tb), 0, c->stream, Ns,
                                   Fs, N, F, x, T, V, ref_cell, n_ref, xf, Tf, xf, Tf, nf, c->sorted_cell,
                                   c->sorted_idx, rate, src_child, n_src, gc, cp, volf, c->cnt);
            if (int e = check_launch(c, "k_crta_fine")) return e;
        }
    }
    return EMMA_RT_OK;
}

template <int G, typename S>
static int crta_typed(emma_rt_ctx *c, S *N, S *F, double *x, double *T, const double *n0, const int64_t *cell,
                      const double *rate, const int32_t *src_child, int n_src, double dt, int n_steps,
                      const int64_t *ref_cell, int n_ref, int ratio, double *xf, double *Tf, const double *nf,
                      emma_rt_diag *d) {
    const int tb = 256;
    if (d) {
        hipLaunchKernelGGL(k_fill_u64, dim3((kCntSlots * CNT_COUNT + 255) / 256), dim3(256), 0, c->stream,
                           c->cnt, (int)(kCntSlots * CNT_COUNT), 0ull);
        if (int e = check_launch(c, "k_fill_u64")) return e;
    }
    if (int e = build_sources<G>(c, cell, rate, n_src)) return e;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((c->mask_words + tb - 1) / tb)), dim3(tb), 0, c->stream,
                       c->refmask, c->mask_words, 0u);
    if (int e = check_launch(c, "k_fill_u32 (refined mask)")) return e;
    if (n_ref > 0) {
        hipLaunchKernelGGL(k_mark_refined, dim3((n_ref + tb - 1) / tb), dim3(tb), 0, c->stream, ref_cell, n_ref,
                           c->grid.V, c->refmask, c->cnt);
        if (int e = check_launch(c, "k_mark_refined")) return e;
    }
    int e;
    if (ratio == 2)
        e = d ? crta_steps<G, S, true, 8>(c, N, F, x, T, n0, rate, src_child, n_src, dt, n_steps, ref_cell, n_ref,
                                          xf, Tf, nf)
              : crta_steps<G, S, false, 8>(c, N, F, x, T, n0, rate, src_child, n_src, dt, n_steps, ref_cell, n_ref,
                                           xf, Tf, nf);
    else
        e = d ? crta_steps<G, S, true, 64>(c, N, F, x, T, n0, rate, src_child, n_src, dt, n_steps, ref_cell,
                                           n_ref, xf, Tf, nf)
              : crta_steps<G, S, false, 64>(c, N, F, x, T, n0, rate, src_child, n_src, dt, n_steps, ref_cell,
                                            n_ref, xf, Tf, nf);
    if (e) return e;
    if (d) return diag_finish<G, S>(c, N, F, x, T, n0, d);
    return EMMA_RT_OK;
}

extern "C" int emma_rt_step_crta(emma_rt_ctx *c, void *N, void *F, double *x, double *T, const double *n0,
                                 const int64_t *cell, const double *rate, const int32_t *src_child, int32_t n_src,
                                 double dt, int32_t n_steps, const int64_t *ref_cell, int32_t n_ref, int32_t ratio,
                                 double *x_fine, double *T_fine, const double *n_fine, emma_rt_diag *d) {
    if (!c) return fail(nullptr, EMMA_RT_EINVAL, "ctx is NULL");
    if (!N || !F || !x || !T || !n0) return fail(c, EMMA_RT_EINVAL, "a field pointer is NULL");
    if (n_src < 0 || n_src > EMMA_RT_MAX_SOURCES)
        return fail(c, EMMA_RT_EINVAL, "n_src must be in 0..%d", EMMA_RT_MAX_SOURCES);
    if (n_src > 0 && (!cell || !rate)) return fail(c, EMMA_RT_EINVAL, "source arrays are NULL");
    if (n_steps < 0) return fail(c, EMMA_RT_EINVAL, "n_steps must be >= 0");
    if (!(dt > 0) || !isfinite(dt)) return fail(c, EMMA_RT_EINVAL, "dt must be > 0");
    if (dt > c->cfg.dx / (3.0 * c->cfg.c_red) * (1.0 + 1e-12))
        return fail(c, EMMA_RT_EINVAL, "dt = %g exceeds dx/(3 c_red) = %g", dt, c->cfg.dx / (3.0 * c->cfg.c_red));
    if (ratio != 2 && ratio != 4) return fail(c, EMMA_RT_EINVAL, "ratio must be 2 or 4");
    if (n_ref < 0 || (int64_t)n_ref > c->grid.V) return fail(c, EMMA_RT_EINVAL, "n_ref must be in 0..cells");
    if ((int64_t)n_ref * ratio * ratio * ratio > ((int64_t)1 << 31) - 256)
        return fail(c, EMMA_RT_EINVAL, "too many children (n_ref * ratio^3)");
    if (n_ref > 0 && (!ref_cell || !x_fine || !T_fine || !n_fine))
        return fail(c, EMMA_RT_EINVAL, "refined-cell arrays are NULL");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != c->device) return fail(c, EMMA_RT_EINVAL, "current device %d is not the context's %d", dev, c->device);
    c->err[0] = 0;
    const int G = c->cfg.n_groups;
    const bool f64 = c->cfg.precision == EMMA_RT_FP64;
#define CDISPATCH(GG)                                                                                          \
    case GG:                                                                                                   \
        return f64 ? crta_typed<GG, double>(c, (double *)N, (double *)F, x, T, n0, cell, rate, src_child, n_src, \
                                            dt, n_steps, ref_cell, n_ref, ratio, x_fine, T_fine, n_fine, d)      \
                   : crta_typed<GG, float>(c, (float *)N, (float *)F, x, T, n0, cell, rate, src_child, n_src,    \
                                           dt, n_steps, ref_cell, n_ref, ratio, x_fine, T_fine, n_fine, d);
    switch (G) {
        CDISPATCH(1)
        CDISPATCH(2)
        CDISPATCH(3)
        CDISPATCH(4)
    }
#undef CDISPATCH
    return fail(c, EMMA_RT_EINVAL, "n_groups out of range");
}

// ----------------------------------------------------------------- adjoint
// The transport of one step before the floor and the limiter (the forward's
// own kernel arithmetic), state (iN, iF) into (uN, uF).
template <int G, typename S>
static int tape_transport(emma_rt_ctx *c, const S *iN, const S *iF, S *uN, S *uF, const ChemParams &cp) {
    const Grid gr = c->grid;
    const int tb = 256;
    const double lam = cp.dt / c->cfg.dx;
    Timed t(c, KID_ADJ_FWD);
    const bool hll = c->cfg.flux == EMMA_RT_FLUX_HLL;
    const dim3 grid((unsigned)((gr.V + tb - 1) / tb));
    if (c->cfg.path == EMMA_RT_PATH_REFERENCE && hll)
        hipLaunchKernelGGL((k_transport<G, S, false, true, true>), grid, dim3(tb), 0, c->stream, iN, iF, uN, uF, gr,
                           (S)c->cfg.c_red, (S)lam, c->cnt, bounds_of<S>(c));
    else if (c->cfg.path == EMMA_RT_PATH_REFERENCE)
        hipLaunchKernelGGL((k_transport<G, S, false, true>), grid, dim3(tb), 0, c->stream, iN, iF, uN, uF, gr,
                           (S)c->cfg.c_red, (S)lam, c->cnt, bounds_of<S>(c));
    else if (hll)
        launch_transport_tiled_hll<G, S, false>(c->stream, iN, iF, uN, uF, gr, cp, lam, c->cnt, bounds_of<S>(c),
                                                true);
    else
        launch_transport_tiled<G, S, false>(c->stream, iN, iF, uN, uF, gr, cp, lam, c->cnt, bounds_of<S>(c), true);
    return check_launch(c, "transport (tape)");
}

// The chemistry of one step from the transport output before the floor and
// the limiter (uN, uF) and the gas state (ix, iT) into the separate arrays
// (oN, oF, ox, oT), with the source table already built: the adjoint's
// forward, tape slot s into slot s + 1 without a copy.  Same bits as the
// step (the floor and the limiter are the transport's own function, applied
// at load).  multi: the cells whose subcycle was not a single substep.
template <int G, typename S>
static int tape_chem(emma_rt_ctx *c, const S *uN, const S *uF, const double *ix, const double *iT, S *oN, S *oF,
                     double *ox, double *oT, const double *n0, int n_src, const ChemParams &cp, uint64_t *multi,
                     const uint32_t *skip) {
    const GroupConsts gc = group_consts(c->cfg);
    const SrcTable src{c->mask, c->sorted_cell, c->S, n_src};
    if (int e = reset_worklist(c)) return e;
    {
        Timed t(c, KID_CHEM);
        const int e = (cp.otsa && !cp.isothermal)
                          ? launch_chem<G, S, false, true>(c, uN, uF, oN, oF, (double *)ix, (double *)iT, ox, oT,
                                                           n0, src, gc, cp, skip, multi)
                          : launch_chem<G, S, false, false>(c, uN, uF, oN, oF, (double *)ix, (double *)iT, ox, oT,
                                                            n0, src, gc, cp, skip, multi);
        if (e) return e;
    }
    return launch_chem_cont<G, S, false>(c, uF, oN, oF, iT, ox, oT, n0, src, gc, cp, uN);
}

// The refined cells of emma_rt_step_crta_adjoint (n_ref = 0: the plain step).
struct CrtaAdj {
    const int64_t *ref_cell;
    int n_ref, nc;                 // nc = ratio^3
    const int32_t *src_child;
    const double *xf0, *Tf0, *nf;  // children's start state, n_fine
    double *tape;                  // [K - 1][2][n_ref nc]: children's x, T after steps 1..K-1
    double *gxf, *gTf, *gnf;
};

template <int G, typename S, int NC>
static int crta_adj_launch(emma_rt_ctx *c, const S *Ut, const S *Ft, const double *xfi, const double *Tfi,
                           const double *rate, int n_src, const GroupConsts &gc, const ChemParams &cp,
                           const CrtaAdj &ca, const S *gN, const S *gF, double *gx, double *gT, double *g_rate,
                           S *gU) {
    const int tb = 256;
    const double hf = c->cfg.dx / (NC == 8 ? 2 : 4);
    const double volf = hf * hf * hf;
    const unsigned fblk = (unsigned)(((int64_t)ca.n_ref * NC + tb - 1) / tb);
    if (cp.otsa && !cp.isothermal)
        hipLaunchKernelGGL((k_crta_adj<G, S, true, NC>), dim3(fblk), dim3(tb), 0, c->stream, Ut, Ft, c->grid.V,
                           ca.ref_cell, ca.n_ref, xfi, Tfi, ca.nf, c->sorted_cell, c->sorted_idx, rate, ca.src_child,
                           n_src, gc, cp, volf, gN, gF, gx, gT, ca.gxf, ca.gTf, ca.gnf, g_rate, gU);
    else
        hipLaunchKernelGGL((k_crta_adj<G, S, false, NC>), dim3(fblk), dim3(tb), 0, c->stream, Ut, Ft, c->grid.V,
                           ca.ref_cell, ca.n_ref, xfi, Tfi, ca.nf, c->sorted_cell, c->sorted_idx, rate, ca.src_child,
                           n_src, gc, cp, volf, gN, gF, gx, gT, ca.gxf, ca.gTf, ca.gnf, g_rate, gU);
    return check_launch(c, "k_crta_adj");
}

// The refined cells' part of a tape step: the children's chemistry from the
// transport output before the floor and the limiter, children's state slot s
// into slot s + 1, the parents' restriction into the coarse tape slot s + 1.
template <int G, typename S, int NC>
static int crta_tape_launch(emma_rt_ctx *c, const S *uN, const S *uF, S *oN, S *oF, double *ox, double *oT,
                            const double *xfi, const double *Tfi, double *xfo, double *Tfo, const double *rate,
                            int n_src, const GroupConsts &gc, const ChemParams &cp, const CrtaAdj &ca) {
    const int tb = 256;
    const double hf = c->cfg.dx / (NC == 8 ? 2 : 4);
    const double volf = hf * hf * hf;
    const unsigned fblk = (unsigned)(((int64_t)ca.n_ref * NC + tb - 1) / tb);
    if (cp.otsa && !cp.isothermal)
        hipLaunchKernelGGL((k_crta_fine<G, S, false, true, NC, true>), dim3(fblk), dim3(tb), 0, c->stream, uN, uF,
                           oN, oF, ox, oT, c->grid.V, ca.ref_cell, ca.n_ref, xfi, Tfi, xfo, Tfo, ca.nf,
                           c->sorted_cell, c->sorted_idx, rate, ca.src_child, n_src, gc, cp, volf, c->cnt);
    else
        hipLaunchKernelGGL((k_crta_fine<G, S, false, false, NC, true>), dim3(fblk), dim3(tb), 0, c->stream, uN,
                           uF, oN, oF, ox, oT, c->grid.V, ca.ref_cell, ca.n_ref, xfi, Tfi, xfo, Tfo, ca.nf,
                           c->sorted_cell, c->sorted_idx, rate, ca.src_child, n_src, gc, cp, volf, c->cnt);
    return check_launch(c, "k_crta_fine (tape)");
}

template <int G, typename S>
static int adjoint_typed(emma_rt_ctx *c, const S *N0, const S *F0, const double *x0, const double *T0,
                         const double *n0, const int64_t *cell, const double *rate, int n_src, double dt,
                         int n_steps, S *gN, S *gF, double *gx, double *gT, double *g_n0, double *g_rate,
                         const CrtaAdj &ca = CrtaAdj{}) {
    const Grid gr = c->grid;
    const int64_t V = gr.V;
    const int tb = 256;
    const GroupConsts gc = group_consts(c->cfg);
    ChemParams cp;
    cp.c = c->cfg.c_red;
    cp.dt = dt;
    cp.otsa = c->cfg.otsa;
    cp.isothermal = c->cfg.isothermal;
    cp.max_substeps = c->cfg.max_substeps;
    const bool fast = cp.otsa && !cp.isothermal;
    const double lam = dt / c->cfg.dx;
    const double vol = c->cfg.dx * c->cfg.dx * c->cfg.dx;
    // tape: state at the start of every step of the segment; the first is
    // the caller's (read only), the others are written by the segment's
    // forward.  With the transport tape (ustar), the transport output of
    // every step before the floor and the limiter is kept too; without it
    // (it did not fit), the reverse sweep recomputes it into Ns, Fs.
    const int64_t step_bytes = c->adj.tape_bytes_per_step;
    auto slot = [&](int s) { return (char *)c->adj.tape + (s - 1) * step_bytes; };
    auto tN = [&](int s) { return s == 0 ? (S *)N0 : (S *)slot(s); };
    auto tF = [&](int s) { return s == 0 ? (S *)F0 : (S *)slot(s) + (int64_t)G * V; };
    auto tx = [&](int s) { return s == 0 ? (double *)x0 : (double *)((S *)slot(s) + (int64_t)4 * G * V); };
    auto tT = [&](int s) { return s == 0 ? (double *)T0 : tx(s) + V; };
    const bool keep_u = c->adj.ustar != nullptr;
    auto uN = [&](int s) { return keep_u ? (S *)c->adj.ustar + (int64_t)s * 4 * G * V : (S *)c->Ns; };
    auto uF = [&](int s) { return keep_u ? uN(s) + (int64_t)G * V : (S *)c->Fs; };
    if (int e = build_sources<G>(c, cell, rate, n_src)) return e;
    // refined cells: their mask (the coarse chemistry and its adjoint skip
    // them) and the children's tape, slot 0 the caller's
    const bool crta = ca.n_ref > 0;
    const uint32_t *skip = nullptr;
    const int64_t nfine = (int64_t)ca.n_ref * ca.nc;
    auto fx = [&](int s) { return s == 0 ? ca.xf0 : ca.tape + (int64_t)(s - 1) * 2 * nfine; };
    auto fT = [&](int s) { return s == 0 ? ca.Tf0 : ca.tape + (int64_t)(s - 1) * 2 * nfine + nfine; };
    if (crta) {
        hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((c->mask_words + tb - 1) / tb)), dim3(tb), 0, c->stream,
                           c->refmask, c->mask_words, 0u);
        hipLaunchKernelGGL(k_fill_u64, dim3((kCntSlots * CNT_COUNT + 255) / 256), dim3(256), 0, c->stream, c->cnt,
                           (int)(kCntSlots * CNT_COUNT), 0ull);
        hipLaunchKernelGGL(k_mark_refined, dim3((ca.n_ref + tb - 1) / tb), dim3(tb), 0, c->stream, ca.ref_cell,
                           ca.n_ref, V, c->refmask, c->cnt);
        if (int e = check_launch(c, "k_mark_refined")) return e;
        // a repeated parent would have two sets of children writing its
        // gradients: refuse the list instead (one small read-back)
        std::vector<unsigned long long> slots((size_t)kCntSlots * CNT_COUNT);
        HIP_TRY(c, hipMemcpyAsync(slots.data(), c->cnt, slots.size() * 8, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        unsigned long long bad = 0;
        for (int j = 0; j < kCntSlots; ++j) bad += slots[(size_t)j * CNT_COUNT + CNT_BADREF];
        if (bad) return fail(c, EMMA_RT_EINVAL, "ref_cell has %llu entries outside the grid or repeated", bad);
        skip = c->refmask;
    }
    // the segment forward, step s into tape slot s + 1, marking the cells whose
    // subcycle was not a single substep
    const int64_t mwords = c->adj.multi_words;
    auto multi = [&](int s) { return c->adj.multi + (int64_t)s * mwords; };
    for (int s = 0; s < n_steps; ++s) {
        if (s + 1 < n_steps || keep_u)
            if (int e = tape_transport<G, S>(c, tN(s), tF(s), uN(s), uF(s), cp)) return e;
        if (s + 1 < n_steps) {
            if (int e = tape_chem<G, S>(c, uN(s), uF(s), tx(s), tT(s), tN(s + 1), tF(s + 1), tx(s + 1), tT(s + 1),
                                        n0, n_src, cp, multi(s), skip))
                return e;
            if (crta) {
                double *xo = (double *)fx(s + 1), *To = (double *)fT(s + 1);
                const int e = ca.nc == 8
                                  ? crta_tape_launch<G, S, 8>(c, uN(s), uF(s), tN(s + 1), tF(s + 1), tx(s + 1),
                                                              tT(s + 1), fx(s), fT(s), xo, To, rate, n_src, gc, cp, ca)
                                  : crta_tape_launch<G, S, 64>(c, uN(s), uF(s), tN(s + 1), tF(s + 1), tx(s + 1),
                                                               tT(s + 1), fx(s), fT(s), xo, To, rate, n_src, gc, cp,
                                                               ca);
                if (e) return e;
            }
        }
    }
    SrcTable src{c->mask, c->sorted_cell, c->S, n_src};
    if (n_src > 0) {
        hipLaunchKernelGGL(k_fill_f64, dim3((n_src * G + tb - 1) / tb), dim3(tb), 0, c->stream, c->adj.gS,
                           (int64_t)n_src * G, 0.0);
        if (int e = check_launch(c, "k_fill_f64")) return e;
    }
    for (int s = n_steps - 1; s >= 0; --s) {
        if (!keep_u)
            if (int e = tape_transport<G, S>(c, tN(s), tF(s), uN(s), uF(s), cp)) return e;
        S *Ut = uN(s), *Ft = uF(s);
        if (int e = reset_worklist(c)) return e;
        // Cells whose subcycle was more than one substep (marked by the
        // segment's forward; the last step of the segment has no marks) take
        // the kept-state pass.  It runs on the side stream beside the
        // single-substep pass, so its long subcycles overlap the bulk instead
        // of trailing it (with kernel timing on, both run in turn on the
        // context's stream).  Cells outside the list that still need more than
        // one substep go through the work list to a kept-state pass after.
        const bool marked = s + 1 < n_steps;
        const bool side = marked && !c->prof;
        const hipStream_t ls = side ? c->adj.side : c->stream;
        if (marked) {
            const int64_t words = (V + 63) / 64;
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, c->stream, c->adj.list_count, (int64_t)1, 0u);
            hipLaunchKernelGGL(k_multi_list, dim3((unsigned)((words + tb - 1) / tb)), dim3(tb), 0, c->stream,
                               (const uint64_t *)multi(s), words, V, c->adj.list_count, c->adj.list);
            if (int e = check_launch(c, "k_multi_list")) return e;
            if (side) {
                HIP_TRY(c, hipEventRecord(c->adj.ev_in, c->stream));
                HIP_TRY(c, hipStreamWaitEvent(ls, c->adj.ev_in, 0));
            }
            Timed t(c, KID_ADJ_CHEM_LIST);
            const WorkList ml{c->adj.list_count, c->adj.list};
            if (fast)
                hipLaunchKernelGGL((k_chem_adj_list<G, S, true>), dim3(c->list_blocks), dim3(tb), 0, ls, Ut, Ft,
                                   tx(s), tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS, (S *)c->adj.gU, ml);
            else
                hipLaunchKernelGGL((k_chem_adj_list<G, S, false>), dim3(c->list_blocks), dim3(tb), 0, ls, Ut, Ft,
                                   tx(s), tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS, (S *)c->adj.gU, ml);
            if (int e = check_launch(c, "k_chem_adj_list (marked cells)")) return e;
            if (side) HIP_TRY(c, hipEventRecord(c->adj.ev_out, ls));
        }
        {
            Timed t(c, KID_ADJ_CHEM);
            const WorkList wl{c->work_count, c->work_cells};
            const uint64_t *ms = marked ? multi(s) : nullptr;
            const int atb = EMMA_ADJ_TB;
            const unsigned ablk = (unsigned)((V + atb - 1) / atb);
            if (fast)
                hipLaunchKernelGGL((k_chem_adj<G, S, true>), dim3(ablk), dim3(atb), 0, c->stream, Ut, Ft, tx(s),
                                   tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS, (S *)c->adj.gU, wl, ms,
                                   skip);
            else
                hipLaunchKernelGGL((k_chem_adj<G, S, false>), dim3(ablk), dim3(atb), 0, c->stream, Ut, Ft, tx(s),
                                   tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS, (S *)c->adj.gU, wl, ms,
                                   skip);
            if (int e = check_launch(c, "k_chem_adj")) return e;
        }
        if (side) HIP_TRY(c, hipStreamWaitEvent(c->stream, c->adj.ev_out, 0));
        {
            Timed t(c, KID_ADJ_CHEM_LIST);
            const WorkList wl{c->work_count, c->work_cells};
            if (fast)
                hipLaunchKernelGGL((k_chem_adj_list<G, S, true>), dim3(c->list_blocks), dim3(tb), 0, c->stream, Ut,
                                   Ft, tx(s), tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS,
                                   (S *)c->adj.gU, wl);
            else
                hipLaunchKernelGGL((k_chem_adj_list<G, S, false>), dim3(c->list_blocks), dim3(tb), 0, c->stream, Ut,
                                   Ft, tx(s), tT(s), n0, V, src, gc, cp, gN, gF, gx, gT, g_n0, c->adj.gS,
                                   (S *)c->adj.gU, wl);
        }
        if (int e = check_launch(c, "k_chem_adj_list")) return e;
        if (crta) {
            Timed t(c, KID_ADJ_CHEM);
            const int e = ca.nc == 8 ? crta_adj_launch<G, S, 8>(c, Ut, Ft, fx(s), fT(s), rate, n_src, gc, cp, ca, gN,
                                                                gF, gx, gT, g_rate, (S *)c->adj.gU)
                                     : crta_adj_launch<G, S, 64>(c, Ut, Ft, fx(s), fT(s), rate, n_src, gc, cp, ca,
                                                                 gN, gF, gx, gT, g_rate, (S *)c->adj.gU);
            if (e) return e;
        }
        {
            Timed t(c, KID_ADJ_TRANSPORT);
            if (c->cfg.flux == EMMA_RT_FLUX_HLL) {
                const dim3 grid((unsigned)((V + tb - 1) / tb), G);
                S *gUs = (S *)c->adj.gU;
                hipLaunchKernelGGL((k_transport_adj_hll<S, 0>), grid, dim3(tb), 0, c->stream, tN(s), tF(s), gUs, gN,
                                   gF, gr, c->cfg.c_red, lam, bounds_of<S>(c));
                hipLaunchKernelGGL((k_transport_adj_hll<S, 1>), grid, dim3(tb), 0, c->stream, tN(s), tF(s), gUs, gN,
                                   gF, gr, c->cfg.c_red, lam, bounds_of<S>(c));
                hipLaunchKernelGGL((k_transport_adj_hll<S, 2>), grid, dim3(tb), 0, c->stream, tN(s), tF(s), gUs, gN,
                                   gF, gr, c->cfg.c_red, lam, bounds_of<S>(c));
            } else {
                const unsigned tiles = (unsigned)(((gr.nx + 63) / 64) * ((gr.ny + 3) / 4) *
                                                  ((gr.nz + kAdjLZ - 1) / kAdjLZ));
                hipLaunchKernelGGL((k_transport_adj<S>), dim3(tiles, G), dim3(tb), 0, c->stream, tN(s), tF(s),
                                   (S *)c->adj.gU, gN, gF, gr, c->cfg.c_red, lam, bounds_of<S>(c));
            }
        }
        if (int e = check_launch(c, "k_transport_adj")) return e;
    }
    if (n_src > 0) {
        Timed t(c, KID_ADJ_SRC);
        hipLaunchKernelGGL(k_src_grad<G>, dim3((n_src + tb - 1) / tb), dim3(tb), 0, c->stream, cell, n_src, V,
                           c->sorted_cell, c->adj.gS, gc, vol, g_rate);
    }
    return check_launch(c, "k_src_grad");
}

extern "C" int emma_rt_step_adjoint(emma_rt_ctx *c, const void *N0, const void *F0, const double *x0,
                                    const double *T0, const double *n0, const int64_t *cell,
                                    const double *rate, int32_t n_src, double dt, int32_t n_steps, void *gN,
                                    void *gF, double *gx, double *gT, double *g_n0, double *g_rate) {
    if (!c) return fail(nullptr, EMMA_RT_EINVAL, "ctx is NULL");
    if (c->cfg.adjoint_max_steps < 1) return fail(c, EMMA_RT_EINVAL, "context was created without adjoint scratch");
    if (n_steps < 1 || n_steps > c->cfg.adjoint_max_steps)
        return fail(c, EMMA_RT_EINVAL, "n_steps must be in 1..%d", c->cfg.adjoint_max_steps);
    if (!N0 || !F0 || !x0 || !T0 || !n0 || !gN || !gF || !gx || !gT || !g_n0)
        return fail(c, EMMA_RT_EINVAL, "a field pointer is NULL");
    if (n_src < 0 || n_src > EMMA_RT_MAX_SOURCES)
        return fail(c, EMMA_RT_EINVAL, "n_src must be in 0..%d", EMMA_RT_MAX_SOURCES);
    if (n_src > 0 && (!cell || !rate || !g_rate)) return fail(c, EMMA_RT_EINVAL, "source arrays are NULL");
    if (!(dt > 0) || dt > c->cfg.dx / (3.0 * c->cfg.c_red) * (1.0 + 1e-12))
        return fail(c, EMMA_RT_EINVAL, "dt must be in (0, dx/(3 c_red)]");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != c->device) return fail(c, EMMA_RT_EINVAL, "current device %d is not the context's %d", dev, c->device);
    c->err[0] = 0;
    const int G = c->cfg.n_groups;
    const bool f64 = c->cfg.precision == EMMA_RT_FP64;
#define ADISPATCH(GG)                                                                                        \
    case GG:                                                                                                 \
        return f64 ? adjoint_typed<GG, double>(c, (const double *)N0, (const double *)F0, x0, T0, n0, cell,  \
                                               rate, n_src, dt, n_steps, (double *)gN, (double *)gF, gx, gT, \
                                               g_n0, g_rate)                                                 \
                   : adjoint_typed<GG, float>(c, (const float *)N0, (const float *)F0, x0, T0, n0, cell,     \
                                              rate, n_src, dt, n_steps, (float *)gN, (float *)gF, gx, gT,    \
                                              g_n0, g_rate);
    switch (G) {
        ADISPATCH(1)
        ADISPATCH(2)
        ADISPATCH(3)
        ADISPATCH(4)
    }
#undef ADISPATCH
    return fail(c, EMMA_RT_EINVAL, "n_groups out of range");
}

extern "C" int64_t emma_rt_crta_adjoint_work_bytes(int32_t n_steps, int32_t n_ref, int32_t ratio) {
    if (n_steps < 1 || n_ref < 0 || (ratio != 2 && ratio != 4)) return -1;
    return (int64_t)(n_steps - 1) * n_ref * ratio * ratio * ratio * 16;
}

extern "C" int emma_rt_step_crta_adjoint(emma_rt_ctx *c, const void *N0, const void *F0, const double *x0,
                                         const double *T0, const double *n0, const int64_t *cell,
                                         const double *rate, const int32_t *src_child, int32_t n_src, double dt,
                                         int32_t n_steps, const int64_t *ref_cell, int32_t n_ref, int32_t ratio,
                                         const double *x_fine0, const double *T_fine0, const double *n_fine,
                                         void *work, int64_t work_bytes, void *gN, void *gF, double *gx,
                                         double *gT, double *g_n0, double *g_rate, double *g_x_fine,
                                         double *g_T_fine, double *g_n_fine) {
    if (!c) return fail(nullptr, EMMA_RT_EINVAL, "ctx is NULL");
    if (c->cfg.adjoint_max_steps < 1) return fail(c, EMMA_RT_EINVAL, "context was created without adjoint scratch");
    if (n_steps < 1 || n_steps > c->cfg.adjoint_max_steps)
        return fail(c, EMMA_RT_EINVAL, "n_steps must be in 1..%d", c->cfg.adjoint_max_steps);
    if (!N0 || !F0 || !x0 || !T0 || !n0 || !gN || !gF || !gx || !gT || !g_n0)
        return fail(c, EMMA_RT_EINVAL, "a field pointer is NULL");
    if (n_src < 0 || n_src > EMMA_RT_MAX_SOURCES)
        return fail(c, EMMA_RT_EINVAL, "n_src must be in 0..%d", EMMA_RT_MAX_SOURCES);
    if (n_src > 0 && (!cell || !rate || !g_rate)) return fail(c, EMMA_RT_EINVAL, "source arrays are NULL");
    if (!(dt > 0) || dt > c->cfg.dx / (3.0 * c->cfg.c_red) * (1.0 + 1e-12))
        return fail(c, EMMA_RT_EINVAL, "dt must be in (0, dx/(3 c_red)]");
    if (ratio != 2 && ratio != 4) return fail(c, EMMA_RT_EINVAL, "ratio must be 2 or 4");
    if (n_ref < 0 || (int64_t)n_ref > c->grid.V) return fail(c, EMMA_RT_EINVAL, "n_ref must be in 0..cells");
    if ((int64_t)n_ref * ratio * ratio * ratio > ((int64_t)1 << 31) - 256)
        return fail(c, EMMA_RT_EINVAL, "too many children (n_ref * ratio^3)");
    if (n_ref > 0 && (!ref_cell || !x_fine0 || !T_fine0 || !n_fine || !g_x_fine || !g_T_fine || !g_n_fine))
        return fail(c, EMMA_RT_EINVAL, "refined-cell arrays are NULL");
    const int64_t need = emma_rt_crta_adjoint_work_bytes(n_steps, n_ref, ratio);
    if (need > 0 && (!work || work_bytes < need))
        return fail(c, EMMA_RT_EINVAL, "work must hold %lld bytes", (long long)need);
    if (need > 0 && ((uintptr_t)work & 7)) return fail(c, EMMA_RT_EINVAL, "work must be 8-byte aligned");
    int dev = -1;
    (void)hipGetDevice(&dev);
    if (dev != c->device) return fail(c, EMMA_RT_EINVAL, "current device %d is not the context's %d", dev, c->device);
    c->err[0] = 0;
    CrtaAdj ca{ref_cell, n_ref, ratio * ratio * ratio, src_child, x_fine0, T_fine0, n_fine, (double *)work,
               g_x_fine, g_T_fine, g_n_fine};
    const int G = c->cfg.n_groups;
    const bool f64 = c->cfg.precision == EMMA_RT_FP64;
#define RDISPATCH(GG)                                                                                        \
    case GG:                                                                                                 \
        return f64 ? adjoint_typed<GG, double>(c, (const double *)N0, (const double *)F0, x0, T0, n0, cell,  \
                                               rate, n_src, dt, n_steps, (double *)gN, (double *)gF, gx, gT, \
                                               g_n0, g_rate, ca)                                             \
                   : adjoint_typed<GG, float>(c, (const float *)N0, (const float *)F0, x0, T0, n0, cell,     \
                                              rate, n_src, dt, n_steps, (float *)gN, (float *)gF, gx, gT,    \
                                              g_n0, g_rate, ca);
    switch (G) {
        RDISPATCH(1)
        RDISPATCH(2)
        RDISPATCH(3)
        RDISPATCH(4)
    }
#undef RDISPATCH
    return fail(c, EMMA_RT_EINVAL, "n_groups out of range");
}

// ------------------------------------------------------------ profiling
static const char *kKindNames[KID_COUNT] = {"src_table", "transport", "chemistry", "fused_step",
                                            "diagnostics", "adj_chemistry", "adj_transport",
                                            "adj_sources", "adj_forward", "chemistry_deferred",
                                            "chemistry_refined", "adj_chemistry_deferred"};

extern "C" int emma_rt_profile_enable(emma_rt_ctx *c, int32_t enable) {
    if (!c) return fail(nullptr, EMMA_RT_EINVAL, "ctx is NULL");
    if (enable && !c->ev) {
        c->ev = new std::vector<hipEvent_t>(2 * kEventPairs);
        c->ev_kind = new std::vector<int>();
        c->ev_kind->reserve(kEventPairs);
        for (auto &e : *c->ev) HIP_TRY(c, hipEventCreate(&e));
    }
    if (!enable && c->ev) {
        if (int e = prof_flush(c)) return e;
    }
    c->prof = enable ? 1 : 0;
    return EMMA_RT_OK;
}

extern "C" int emma_rt_profile_read(emma_rt_ctx *c, emma_rt_kernel_time *out, int32_t max_out,
                                    int32_t *n_out) {
    if (!c || !n_out || (max_out > 0 && !out)) return fail(c, EMMA_RT_EINVAL, "bad arguments");
    *n_out = 0;
    if (c->ev) {
        if (int e = prof_flush(c)) return e;
    }
    for (int k = 0; k < KID_COUNT; ++k) {
        if (c->prof_n[k] == 0) continue;
        if (*n_out < max_out) {
            emma_rt_kernel_time &r = out[*n_out];
            memset(&r, 0, sizeof(r));
            strncpy(r.name, kKindNames[k], sizeof(r.name) - 1);
            r.launches = c->prof_n[k];
            r.total_ms = c->prof_ms[k];
            (*n_out)++;
        }
        c->prof_n[k] = 0;
        c->prof_ms[k] = 0.0;
    }
    return EMMA_RT_OK;
}

// ------------------------------------------------------- group constants
// Hydrogen photo-ionisation cross-section, exact hydrogenic form
// (Osterbrock & Ferland): s(E) = 6.30e-18 (E0/E)^4 exp(4 - 4 atan(q)/q) /
// (1 - exp(-2 pi / q)), q = sqrt(E/E0 - 1), zero below E0 = 13.6 eV.
static double h_cross_section(double E) {
    const double E0 = 13.6;
    if (E < E0) return 0.0;
    const double r = E / E0;
    const double q2 = r - 1.0;
    if (q2 < 1e-12) return 6.30e-18;
    const double q = sqrt(q2);
    const double at = atan(q) / q;
    return 6.30e-18 / (r * r * r * r) * exp(4.0 - 4.0 * at) / (-expm1(-2.0 * M_PI / q));
}

// Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on P_n.
static void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w) {
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            const double dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        const double dp = n * (z * p1 - p0) / (z * z - 1.0);
        t[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

extern "C" int emma_rt_group_constants(double T_bb, const double *edges, int32_t G, double *sigN,
                                       double *sigE, double *meanE, double *frac) {
    if (G < 1 || G > EMMA_RT_MAX_GROUPS || !edges || !sigN || !sigE || !meanE || !frac || !(T_bb > 0))
        return EMMA_RT_EINVAL;
    for (int g = 0; g < G; ++g)
        if (!(edges[g] >= 13.6) || !(edges[g + 1] > edges[g])) return EMMA_RT_EINVAL;
    const double kT = kKB * T_bb / kEV;  // eV
    std::vector<double> t, w;
    const int order = 48, panels = 96;
    gauss_legendre(order, t, w);
    double tot = 0.0;
    std::vector<double> num(G);
    for (int g = 0; g < G; ++g) {
        // photon spectrum per unit energy E^2 / (exp(E/kT) - 1), integrated in
        // u = ln E (dE = E du) over equal panels
        const double a = log(edges[g]), b = log(edges[g + 1]);
        const double h = (b - a) / panels;
        double In = 0, Is = 0, Ie = 0, Ise = 0;
        for (int p = 0; p < panels; ++p) {
            const double mid = a + (p + 0.5) * h;
            for (int k = 0; k < order; ++k) {
                const double E = exp(mid + 0.5 * h * t[k]);
                const double wt = 0.5 * h * w[k] * E * E * E / expm1(E / kT);
                const double s = h_cross_section(E);
                In += wt;
                Is += wt * s;
                Ie += wt * E;
                Ise += wt * s * E;
            }
        }
        const double mE = Ie / In;
        sigN[g] = Is / In;
        sigE[g] = Ise / Ie;
        meanE[g] = mE * kEV;
        num[g] = In;
        tot += In;
    }
    for (int g = 0; g < G; ++g) frac[g] = num[g] / tot;
    return EMMA_RT_OK;
}
