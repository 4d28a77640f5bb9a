/*
 * emma_rt.h -- C ABI of the MI355X radiation step library (libemma_rt.so).
 *
 * One call advances the coarse-grid radiation of the EMMA code (Aubert,
 * Deparis & Ocvirk 2015) by n_steps explicit steps on a uniform grid (periodic,
 * or with the transmissive / reflective / inflow faces of Sec. 4 and Sec. 6)
 * with the gas frozen, as the coarse radiative transport approximation (Sec. 5)
 * does between two dynamical steps.  Each step is
 *   1. the M1 transport of every frequency group (Sec. 2.2.3): Eddington
 *      tensor closure, Lax-Friedrichs / HLL(+-c_red) face fluxes (eq. e:glf)
 *      or HLL with M1 wave speeds, and the unsplit conservative update
 *      (eq. e:uprt), then
 *   2. the per-cell sub-cycled hydrogen thermochemistry (Sec. 2.2.4):
 *      source injection, photo-ionisation, recombination, collisional
 *      ionisation, heating and cooling, coupled back into N and F.
 *
 * Conventions for every entry point
 *   - Field pointers are HIP device memory owned by the caller.  Layout is C
 *     order with x fastest: N[G][nz][ny][nx], F[G][3][nz][ny][nx] (component
 *     major), x_HII, T, n_H [nz][ny][nx].  Cell index = (z*ny + y)*nx + x.
 *   - Units CGS: N photons cm^-3, F photons cm^-2 s^-1, T K, n_H cm^-3 (the
 *     TOTAL hydrogen density n0; the neutral density is (1-x_HII) n0), dx cm,
 *     dt s, c_red cm s^-1, source rates photons s^-1.
 *   - Storage: EMMA_RT_FP64 keeps N, F in double; EMMA_RT_MIXED keeps N, F in
 *     float (transport computed in float, chemistry in double).  x_HII, T and
 *     n_H are always double.
 *   - Calls are asynchronous on the context's stream; only a call given a
 *     non-NULL diag waits for its own work.  Calls on one context must not
 *     overlap (the context owns scratch that every call reuses).
 *   - Errors are returned as emma_rt_status codes; nothing aborts or throws
 *     across the ABI.  emma_rt_last_error() gives the context's last message.
 */
#ifndef EMMA_RT_H
#define EMMA_RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct emma_rt_ctx emma_rt_ctx;

typedef enum {
    EMMA_RT_OK = 0,
    EMMA_RT_EINVAL = -1,     /* bad argument; nothing was launched */
    EMMA_RT_ENOMEM = -2,     /* device allocation failed (init only) */
    EMMA_RT_EHIP = -3,       /* a HIP runtime call failed */
    EMMA_RT_ESUBSTEP = -4,   /* chemistry guard fired in some cell (diag only);
                                outputs are written, count in diag->cap_hits */
    EMMA_RT_ENONFINITE = -5  /* NaN/Inf found in the end state (diag only) */
} emma_rt_status;

typedef enum { EMMA_RT_FP64 = 0, EMMA_RT_MIXED = 1 } emma_rt_precision;
typedef enum { EMMA_RT_PATH_SPLIT = 0, EMMA_RT_PATH_FUSED = 1, EMMA_RT_PATH_REFERENCE = 2 } emma_rt_path;
/* Global boundary of one face (Sec. 4, gather step; Sec. 6 test set-ups).
 * Across a non-periodic face the outside neighbour of a boundary cell is:
 *   TRANSMISSIVE  the cell itself;
 *   REFLECTIVE    the cell with its face-normal flux component reversed;
 *   INFLOW        a planar source: a beam entering along the face normal with
 *                 photon flux density inflow[face] (photons cm^-2 s^-1) split
 *                 over the groups by src_frac, N = flux / c_red (f = 1). */
typedef enum {
    EMMA_RT_BC_PERIODIC = 0,
    EMMA_RT_BC_TRANSMISSIVE = 1,
    EMMA_RT_BC_REFLECTIVE = 2,
    EMMA_RT_BC_INFLOW = 3
} emma_rt_bc;
/* Face flux: GLF = eq. (e:glf), HLL with signal speeds +-c_red;
 * HLL = HLL with, along axis d, the eigenvalues of the one-dimensional M1
 * system at the normal reduced flux F_d/(c_red N) as signal speeds. */
typedef enum { EMMA_RT_FLUX_GLF = 0, EMMA_RT_FLUX_HLL = 1 } emma_rt_flux;

#define EMMA_RT_MAX_GROUPS 4
#define EMMA_RT_SUBSTEP_BINS 18
#define EMMA_RT_MAX_SOURCES 65536

typedef struct {
    int32_t nx, ny, nz;         /* grid, each >= 1, at most 2^32 - 1 cells in all */
    int32_t n_groups;           /* 1 .. EMMA_RT_MAX_GROUPS frequency groups */
    double dx;                  /* cell size, cm */
    double c_red;               /* reduced speed of light (Sec. 2.2.3), 0 < c_red <= c */
    int32_t precision;          /* emma_rt_precision */
    int32_t otsa;               /* 1: on-the-spot (alpha_A := alpha_B, no recombination
                                   photons); 0: case A with recombination photons
                                   into group 1 (eq. e:therm1g) */
    int32_t isothermal;         /* 1: validation mode, one substep of dt, T frozen */
    int32_t max_substeps;       /* accepted substeps per cell per step before the
                                   guard takes one last substep of the remainder */
    int32_t adjoint_max_steps;  /* K: longest segment emma_rt_step_adjoint accepts;
                                   0 = no adjoint scratch */
    int32_t path;               /* kernels of the step: EMMA_RT_PATH_SPLIT (default:
                                   tiled transport, then chemistry), _FUSED (one
                                   kernel, chemistry on the transport's registers:
                                   one pass over HBM but fewer waves per SIMD) or
                                   _REFERENCE (one-cell-per-thread transport, then
                                   chemistry); all compute the same step */
    /* Per-group constants (Sec. 2.2.3-2.2.4, eq. e:siggroup and the sigma_E and
       <E> definitions): number- and energy-weighted cross-sections (cm^2), mean
       photon energy (erg) and fraction of a source's photons in the group. */
    double sigma_N[EMMA_RT_MAX_GROUPS];
    double sigma_E[EMMA_RT_MAX_GROUPS];
    double mean_E[EMMA_RT_MAX_GROUPS];
    double src_frac[EMMA_RT_MAX_GROUPS];
    /* Faces in the order x-, x+, y-, y+, z-, z+; emma_rt_bc values, 0 (periodic)
       by default.  Both faces of an axis are periodic or neither. */
    int32_t bc[6];
    int32_t flux;               /* emma_rt_flux; EMMA_RT_FLUX_HLL runs on every path
                                   (fused: one thread per cell, transport then
                                   chemistry), adjoint included */
    int32_t reserved;           /* 0 */
    double inflow[6];           /* photons cm^-2 s^-1 through each INFLOW face, >= 0 */
} emma_rt_config;

typedef struct {
    double photons[EMMA_RT_MAX_GROUPS]; /* sum over cells of N dx^3, end state */
    double ionised;                     /* sum over cells of x_HII n_H dx^3 */
    int64_t substeps;                   /* accepted chemistry substeps, all cells and steps */
    int64_t attempts;                   /* substep attempts including 10 % halvings */
    int32_t max_sub;                    /* most accepted substeps of one cell in one step */
    int32_t reserved;
    int64_t limiter_hits;               /* transport: |F*| > c N* rescaled */
    int64_t neg_clamps;                 /* transport: N* < 0 set to 0 */
    int64_t x_clamps;                   /* chemistry: x_HII clamped to [0, 1] */
    int64_t cap_hits;                   /* chemistry: cells where the substep guard fired */
    int64_t nonfinite;                  /* cells with a NaN/Inf in the end state */
    /* Histogram of accepted substeps per cell and step (refined cells: per
       child), all steps of the call: bin 0 counts cell-steps with none (an
       invalid energy leaves the cell untouched), bin k (1..16) those with
       2^(k-1) <= n < 2^k, the last bin those with n >= 2^16. */
    int64_t substep_hist[EMMA_RT_SUBSTEP_BINS];
} emma_rt_diag;

/* Create a context on the current HIP device.  cfg is copied.  hip_stream is a
 * hipStream_t (NULL = the default stream).  Allocates every piece of scratch
 * the later calls use (transport ping-pong fields, source tables, counters,
 * adjoint tape of adjoint_max_steps - 1 states; its transport part,
 * adjoint_max_steps steps of N*, F*, only if the device then still has the
 * room of four more states free: without it the adjoint recomputes them).  Returns EINVAL for a bad config,
 * ENOMEM when the scratch does not fit; *ctx is NULL on any error. */
int emma_rt_init(emma_rt_ctx **ctx, const emma_rt_config *cfg, void *hip_stream);

/* Advance (N, F, x_HII, T) in place by n_steps steps of dt (Sec. 2.2.3-2.2.4,
 * Sec. 5), with the gas density n_H and the source list held fixed.
 *   N, F            device, float or double per precision, read and written
 *   x_HII, T        device double, read and written
 *   n_H             device double, read only
 *   src_cell        device int64 [n_src], flat cell index of each point source;
 *                   entries outside the grid are ignored, and reported (EINVAL)
 *                   only when diag is given (without diag nothing is read back)
 *   src_rate        device double [n_src], photons s^-1; sources sharing a cell add
 *   dt              must satisfy 0 < dt <= dx / (3 c_red) (positivity of the
 *                   unsplit 3D update); larger dt returns EINVAL
 *   diag            NULL: no reductions, no wait.  Else filled after the call waits.
 * Returns OK, EINVAL, EHIP, or (diag only) ESUBSTEP / ENONFINITE. */
int emma_rt_step(emma_rt_ctx *ctx, void *N, void *F, double *x_HII, double *T,
                 const double *n_H, const int64_t *src_cell, const double *src_rate,
                 int32_t n_src, double dt, int32_t n_steps, emma_rt_diag *diag);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): emma_rt_step
 * without a context.  The scratch a context would own (transport output or
 * ping-pong fields, source table, counters, chemistry work list) lives in one
 * fixed device array of EMMA_RT_NOALLOC_SCRATCH_BYTES compiled into the
 * library; every GPU the library runs on holds its own copy until the process
 * ends.  Nothing is allocated: no hipMalloc, hipFree or allocating library call.
 *   cfg             as for emma_rt_init (read here, not kept); adjoint_max_steps
 *                   is ignored
 *   hip_stream      hipStream_t of the call (NULL = the default stream)
 *   N ... n_steps   as emma_rt_step (no diagnostics: src_cell entries outside
 *                   the grid are ignored without a report)
 * Scratch needed, each piece rounded up to 256 bytes: 4 G V e (N and F; e = 4
 * mixed, 8 FP64) + 4 V (work list) + V/8 (source mask) + 24 n_src + 8 G n_src
 * (source table) + 14336 (counters) + 64 + (16 G + 44) C (continuation states
 * of the chemistry, C = min(V, max(65536, V/8)) slots).  A grid and source list needing more
 * than EMMA_RT_NOALLOC_SCRATCH_BYTES return EINVAL before anything runs (a
 * 128^3 grid with 3 groups in mixed precision fits; in FP64 it does not).
 * All calls on one GPU share that GPU's array and the next call overwrites it:
 * calls that overlap on one GPU (two streams, two host threads) race and must
 * be serialised by the caller.  Errors are reported through
 * emma_rt_last_error(NULL) (one message per process, not per thread).
 * Returns OK, EINVAL or EHIP. */
#define EMMA_RT_NOALLOC_SCRATCH_BYTES (128ll << 20)
int emma_rt_step_noalloc(const emma_rt_config *cfg, void *hip_stream, void *N, void *F,
                         double *x_HII, double *T, const double *n_H, const int64_t *src_cell,
                         const double *src_rate, int32_t n_src, double dt, int32_t n_steps);

/* emma_rt_step with static refinement: the coarse radiative transport
 * approximation of Sec. 5.  The transport runs on the coarse grid only; each
 * refined coarse cell has r^3 children (r = ratio, 2 or 4) with their own gas,
 * whose chemistry runs with the parent's post-transport N, F injected
 * (piecewise constant) and with their own sources; the parent then holds the
 * children's mean N and F, the n_H-weighted mean x_HII and the (1 + x) n_H-
 * weighted mean T (its photons, ionised atoms and internal energy are the
 * children's; means are pairwise sums in child order, so children equal to
 * the parent reproduce emma_rt_step on the split path exactly).
 *   N, F, x_HII, T, n_H, src_cell, src_rate, dt, n_steps, diag: as emma_rt_step
 *                   (x_HII, T of refined cells are overwritten by the means)
 *   src_child       device int32 [n_src], child index of each source whose
 *                   host cell is refined (ignored for other sources); NULL = 0
 *   ref_cell        device int64 [n_ref], distinct refined coarse cells
 *   x_fine, T_fine  device double [n_ref][ratio^3], read and written; child
 *                   index (cz ratio + cy) ratio + cx within the parent
 *   n_fine          device double [n_ref][ratio^3], read only
 * Child sources have density rate * src_frac / (dx / ratio)^3.  The transport
 * uses the split path's tiled kernel (fused and split paths; the tiled HLL
 * kernel with EMMA_RT_FLUX_HLL) or the reference kernel (reference path).
 * Entries of ref_cell outside the grid or repeated, and source children
 * outside 0..ratio^3-1, are ignored and reported as EINVAL when diag is
 * given.  Its adjoint is emma_rt_step_crta_adjoint.  Returns as emma_rt_step,
 * and EINVAL for ratio not 2 or 4 or NULL arrays with n_ref > 0. */
int emma_rt_step_crta(emma_rt_ctx *ctx, void *N, void *F, double *x_HII, double *T,
                      const double *n_H, const int64_t *src_cell, const double *src_rate,
                      const int32_t *src_child, int32_t n_src, double dt, int32_t n_steps,
                      const int64_t *ref_cell, int32_t n_ref, int32_t ratio,
                      double *x_fine, double *T_fine, const double *n_fine, emma_rt_diag *diag);

/* Vector-Jacobian product of n_steps steps (1 <= n_steps <= adjoint_max_steps),
 * the exact derivative of the discrete map computed by emma_rt_step along the
 * branches (substep lengths, halvings, clamps) that the forward run takes.
 *   N0, F0, x0, T0  device, the state at the start of the segment (not modified)
 *   gN, gF, gx, gT  device, same layouts as the state (gN, gF in the state's
 *                   precision): on entry dL/d(state at segment end), on exit
 *                   dL/d(state at segment start)
 *   g_nH            device double [cells], dL/dn_H is ADDED to it
 *   g_src_rate      device double [n_src], dL/d(src_rate) is ADDED to it (nothing
 *                   for a source whose cell is outside the grid: such sources are
 *                   ignored by the forward step, and this call does not report them)
 * The floor N >= 0 and the limiter |F| <= c_red N are reversed along the
 * decisions the forward took, with the forward's own arithmetic.
 * The segment is recomputed forward from (N0, F0, x0, T0) into the context's
 * tape (the states of its steps, the transport output of each step before the
 * floor and the limiter when that part of the tape was allocated, and which
 * cells took more than one chemistry substep); then the steps are reversed
 * from the last.  The call uses a second stream of its own beside the
 * context's stream and joins it before returning (all its work is ordered
 * after earlier work on the context's stream).  Every boundary kind is
 * differentiated (an inflow face's beam is a constant); so is the HLL flux
 * (its signal speeds included).  Returns OK, EINVAL or EHIP. */
int emma_rt_step_adjoint(emma_rt_ctx *ctx, const void *N0, const void *F0,
                         const double *x0, const double *T0, const double *n_H,
                         const int64_t *src_cell, const double *src_rate, int32_t n_src,
                         double dt, int32_t n_steps,
                         void *gN, void *gF, double *gx, double *gT,
                         double *g_nH, double *g_src_rate);

/* Bytes of the device workspace emma_rt_step_crta_adjoint needs for a segment
 * of n_steps steps: the children's x_HII and T after each step but the last,
 * (n_steps - 1) n_ref ratio^3 16.  -1 for n_steps < 1, n_ref < 0 or ratio
 * not 2 or 4. */
int64_t emma_rt_crta_adjoint_work_bytes(int32_t n_steps, int32_t n_ref, int32_t ratio);

/* Vector-Jacobian product of n_steps steps of emma_rt_step_crta (the coarse
 * radiative transport approximation of Sec. 5), with the same conventions as
 * emma_rt_step_adjoint: the derivative of the discrete map along the branches
 * the forward run takes.
 *   N0 ... n_steps  as emma_rt_step_adjoint, plus src_child as emma_rt_step_crta
 *   ref_cell, n_ref, ratio, n_fine   as emma_rt_step_crta; ref_cell entries
 *                   must lie in the grid and be distinct (else EINVAL, after
 *                   one small device-to-host read, before the segment runs)
 *   x_fine0, T_fine0 device double [n_ref][ratio^3], the children's state at
 *                   the start of the segment (not modified)
 *   work, work_bytes device workspace of at least
 *                   emma_rt_crta_adjoint_work_bytes(n_steps, n_ref, ratio)
 *                   bytes, 8-byte aligned, owned by the caller; NULL when
 *                   that is 0; its contents on return are unspecified
 *   gN ... g_src_rate as emma_rt_step_adjoint (on exit, gx and gT of refined
 *                   cells are 0: the forward overwrites those cells' x_HII and
 *                   T with the children's means; a source whose src_child is
 *                   outside 0..ratio^3-1 in a refined cell gets nothing, as
 *                   the forward ignores it)
 *   g_x_fine, g_T_fine device double [n_ref][ratio^3]: on entry dL/d(children's
 *                   x_HII, T at segment end), on exit dL/d(at segment start)
 *   g_n_fine        device double [n_ref][ratio^3], dL/dn_fine is ADDED to it
 * Needs the context's adjoint scratch (adjoint_max_steps >= n_steps); the
 * children's part of the tape lives in work.  Returns OK, EINVAL or EHIP. */
int emma_rt_step_crta_adjoint(emma_rt_ctx *ctx, const void *N0, const void *F0,
                              const double *x0, const double *T0, const double *n_H,
                              const int64_t *src_cell, const double *src_rate,
                              const int32_t *src_child, int32_t n_src, double dt,
                              int32_t n_steps, const int64_t *ref_cell, int32_t n_ref,
                              int32_t ratio, const double *x_fine0, const double *T_fine0,
                              const double *n_fine, void *work, int64_t work_bytes,
                              void *gN, void *gF, double *gx, double *gT, double *g_nH,
                              double *g_src_rate, double *g_x_fine, double *g_T_fine,
                              double *g_n_fine);

/* Release the context and all its device scratch.  NULL is a no-op. */
void emma_rt_free(emma_rt_ctx *ctx);

/* Message of the context's most recent error ("" if none); a static message
 * when ctx is NULL (e.g. after a failed init). */
const char *emma_rt_last_error(const emma_rt_ctx *ctx);

/* Group constants of a black-body source spectrum of temperature T_bb (K) over
 * the group edges edges_eV[0..G] (Sec. 2.2.3-2.2.4): sigma_N, sigma_E (cm^2),
 * mean_E (erg) and the photon fraction of each group, by Gauss-Legendre
 * quadrature of the hydrogen photo-ionisation cross-section.  Host memory.
 * Returns EINVAL for G outside 1..EMMA_RT_MAX_GROUPS or unsorted edges. */
int emma_rt_group_constants(double T_bb, const double *edges_eV, int32_t G,
                            double *sigma_N, double *sigma_E, double *mean_E,
                            double *src_frac);

/* Per-kernel timing.  While enabled, every kernel that emma_rt_step and
 * emma_rt_step_adjoint launch is bracketed by HIP events recorded on the
 * context's stream (a few microseconds of overhead per launch; the events
 * are created here, not in the step).  emma_rt_profile_read waits for the
 * stream, returns one record per kernel kind that ran since the last read
 * (name, launches, summed duration in ms) and resets the sums.  Host memory;
 * *n_out is the number of records written (at most max_out).  Returns EINVAL
 * for a NULL context, EHIP on a runtime failure. */
typedef struct {
    char name[32];
    int64_t launches;
    double total_ms;
} emma_rt_kernel_time;

int emma_rt_profile_enable(emma_rt_ctx *ctx, int32_t enable);
int emma_rt_profile_read(emma_rt_ctx *ctx, emma_rt_kernel_time *out, int32_t max_out,
                         int32_t *n_out);

/* Size in bytes of the device scratch a context with this config allocates
 * (at most: the adjoint's transport tape is left out when memory is short). */
int64_t emma_rt_scratch_bytes(const emma_rt_config *cfg);

#ifdef __cplusplus
}
#endif

#endif /* EMMA_RT_H */
