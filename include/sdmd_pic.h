/*
 * sdmd_pic.h -- C ABI of the MI355X (gfx950) SDMD particle-in-cell library.
 *
 * The library implements the data-parallel core of the Single Domain Multiple
 * Decompositions method (Derouillat & Beck): one physical domain carried by two
 * decompositions at once (section 2.2).  Small *patches* own the
 * macro-particles; large *regions* own the fields.  One step is
 *
 *   particles on patches: field interpolation, push, charge-conserving
 *   deposition into a patch-local current tile   (section 3.3, "Particles")
 *   transfer (i): patch currents summed into the regions         (section 2.2)
 *   Maxwell (Yee) update on the regions             (section 3.3, "Fields")
 *   region ghost synchronisation                     (section 2.1, "Sync")
 *   transfer (ii): region fields read by the patches             (section 2.2)
 *   re-binning of the particles that left their patch  (section 2.1, "Sync")
 *
 * Equations (normalised units, c = 1): dE/dt = curl B - J, dB/dt = -curl E,
 * du/dt = (q/m)(E + u x B / gamma), dx/dt = u / gamma.  Second-order
 * (quadratic B-spline) shapes and the Esirkepov scheme (section 3.2), Boris
 * push, Yee staggered grid (section 3.2), periodic boundaries.
 *
 * Conventions for every function:
 *   - return 0 (PIC_OK) or a negative PIC_E_* code; no exception crosses the ABI;
 *   - host pointers are plain host memory owned by the caller; the library
 *     copies what it needs and keeps no reference to caller memory after the
 *     call returns;
 *   - device memory is obtained through pic_runtime.alloc / .free (or
 *     hipMalloc / hipFree when those are null) and is owned by the context
 *     until pic_retire / pic_free;
 *   - work is enqueued on pic_runtime.stream in order; pic_step is
 *     asynchronous, pic_fields / pic_diag / pic_particles synchronise the
 *     stream.  Device-side errors (non-finite values, a particle moving a cell
 *     or more in one step) are reported by the next synchronising call;
 *   - one host thread at a time per context.
 *
 * Field arrays crossing the ABI are FP64, layout [component][z][y][x] with x
 * fastest, no ghost cells, the whole domain (region-assembled).  Staggering
 * (position of index (i,j,k) in cell units):
 *   Ex (i+1/2, j, k)  Ey (i, j+1/2, k)  Ez (i, j, k+1/2)   J like E
 *   Bx (i, j+1/2, k+1/2)  By (i+1/2, j, k+1/2)  Bz (i+1/2, j+1/2, k)
 * In 2D3V (dims = 2) there is no z axis: nz = 1 and Ez, Jz sit on (i, j).
 */
#ifndef SDMD_PIC_H
#define SDMD_PIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define PIC_OK          0
#define PIC_E_INVAL    -1  /* null pointer, bad run index or argument        */
#define PIC_E_CONFIG   -2  /* configuration breaks a rule listed at pic_init  */
#define PIC_E_NOMEM    -3  /* allocation failed or HBM budget exceeded        */
#define PIC_E_DEVICE   -4  /* HIP runtime error; text in pic_last_error      */
#define PIC_E_NUMERIC  -5  /* non-finite value or a move of >= 1 cell a step */
#define PIC_E_CAPACITY -6  /* no free run slot                               */
#define PIC_E_STATE    -7  /* call not valid in the current state            */
#define PIC_E_OVERFLOW -8  /* a particle store of the run overflowed (more
                              particles reached it than it holds); the run's
                              state is no longer valid and it should be
                              retired                                        */

/* ---- enums -------------------------------------------------------------- */
#define PIC_FP64        0  /* everything in FP64                             */
#define PIC_FP32_SPLIT  1  /* particles: FP32 with a split position (integer
                              cell + FP32 offset in [0,1)); currents summed
                              per segment in 64-bit fixed point, FP32 patch
                              tiles; region reduction and Maxwell in FP64    */
#define PIC_BC_PERIODIC 0

/* field solvers (pic_config.field_solver) */
#define PIC_SOLVER_YEE   0  /* Yee finite-difference leapfrog (section 3.2):
                               state E^n, B^{n+1/2}, Bm^n                   */
#define PIC_SOLVER_PSATD 1  /* spectral: the Yee-lattice Maxwell equations
                               integrated exactly in time over each step in
                               Fourier space (the spectral solvers that
                               motivate large regions, sections 1 and 2.2):
                               state E^n, B^n (Bm^n = B^n); one periodic
                               region                                        */

/* pic_fields component mask bits */
#define PIC_F_EX   (1u << 0)
#define PIC_F_EY   (1u << 1)
#define PIC_F_EZ   (1u << 2)
#define PIC_F_BX   (1u << 3)   /* Bm: B time-centred at t^n                   */
#define PIC_F_BY   (1u << 4)
#define PIC_F_BZ   (1u << 5)
#define PIC_F_BHX  (1u << 6)   /* B at t^{n+1/2} (needed to resume a run);
                                  B^n with PIC_SOLVER_PSATD                  */
#define PIC_F_BHY  (1u << 7)
#define PIC_F_BHZ  (1u << 8)
#define PIC_F_JX   (1u << 9)   /* J at t^{n-1/2}, from the last step, as the
                                  Maxwell solve used it (after the filter)    */
#define PIC_F_JY   (1u << 10)
#define PIC_F_JZ   (1u << 11)
#define PIC_F_RHO  (1u << 12)  /* electron charge density at t^n (deposited on
                                  demand; the ion background is not included) */

/* pic_runtime.flags */
#define PIC_RT_NO_GRAPH   (1 << 0)  /* launch kernels one by one instead of
                                       replaying captured hipGraphs (of 2
                                       and 8 steps and of a re-layout period) */

typedef struct pic_ctx pic_ctx;

/* Initial particles, host memory, FP64 SoA, length n each.  Positions must
 * lie in [0, L) per axis (L = n_cells * d); z is ignored when dims = 2.
 * Momenta are u = gamma v at t^{-1/2}.  w is the particle's share of the
 * density (density of its cell divided by particles per cell), so the
 * electron charge density is rho = sum q w S.  id may be null (ids are then
 * 0..n-1); ids travel with the particle only when track_ids is set. */
typedef struct {
    int64_t n;
    const double *x, *y, *z;
    const double *ux, *uy, *uz;
    const double *w;
    const uint32_t *id;
} pic_particles_in;

/* Initial fields, host memory, FP64, 3 components each in the layout above.
 * kind 0: E and B at t = 0; the library sets B^{1/2} = B^0 - dt/2 curl E^0
 *         and Bm^0 = B^0 (no momentum pull-back: u is taken as u^{-1/2}).
 * kind 1: E at t^n, B at t^{n+1/2} and Bm at t^n (a resumed state); Bm may
 *         be null, then Bm = B. */
typedef struct {
    int32_t kind;
    int32_t reserved;
    const double *E, *B, *Bm;
} pic_fields_in;

/* One run.  Rules checked by pic_init / pic_admit (PIC_E_CONFIG):
 *   dims is 2 or 3; every n_cells[a] >= 1 (n_cells[2] = 1 when dims = 2);
 *   d[a] > 0 and 0 < dt < 1 / sqrt(sum 1/d[a]^2) (Courant limit);
 *   patch[a] >= 4 -- a patch holds at least the interpolation support
 *     (section 2.1; the smallest patches of section 3.4 are 8 x 7 cells) --
 *     patch[a] <= 32 (2D) or 8 (3D), and patch[a] divides n_cells[a];
 *     patch[a] = 0 on every axis asks the autotuner to choose;
 *   regions are rectangular, of equal shape, and made of whole patches
 *     (section 2.2, rule B): n_regions[a] >= 1 divides n_cells[a]/patch[a];
 *   shape_order is 2; bc[a] is PIC_BC_PERIODIC; m > 0;
 *   0 <= filter_passes <= 4 (2D) or 2 (3D);
 *   field_solver PIC_SOLVER_PSATD: one region (n_regions all 1), every
 *     n_cells[a] of the run a power of two <= 2048, and dt < min d[a] (the
 *     spectral step has no Courant limit; particles still move less than a
 *     cell per step);
 *   seg_cap is 0 or in [256, 65536]; field_tile_x is 0 or a compiled width
 *     (8, 16, 32, 64 in 2D; 8, 16, 32 in 3D; 8 in 3D with the filter).
 * A patch of 0 on every axis lets the library choose the patch edge, the
 * segment capacity and the field tile width: it times a few steps of this
 * config for each admissible square patch (8, 16, 32 in 2D; 4, 8 in 3D),
 * then for other segment capacities with the fastest patch, then for other
 * field tile widths, in scratch runs inside the remaining HBM budget, and
 * keeps the fastest (cached per grid, precision and density). */
typedef struct {
    int32_t dims;
    int32_t n_cells[3];
    double  d[3];
    double  dt;
    int32_t patch[3];
    int32_t n_regions[3];
    int32_t shape_order;
    int32_t precision;          /* PIC_FP64 or PIC_FP32_SPLIT */
    int32_t bc[3];
    int32_t track_ids;          /* carry ids through steps (pic_particles)  */
    int32_t filter_passes;      /* binomial current filter (section 3.2, the
                                   paper's run uses two passes): 0 = off; a
                                   pass smooths each J component with the
                                   1-2-1 kernel along x, then y, then z;
                                   at most 4 passes in 2D, 2 in 3D          */
    int32_t field_solver;       /* PIC_SOLVER_YEE or PIC_SOLVER_PSATD       */
    double  q, m;               /* species charge and mass; electrons -1, 1 */
    int64_t max_steps;          /* steps this run takes, 0 = unlimited: once
                                   they are done the run is left untouched by
                                   later pic_step calls (continuous batching) */
    int32_t seg_cap;            /* particles per segment a re-layout aims at:
                                   a patch holding more is worked on by several
                                   workgroups with their own current tiles (the
                                   task decomposition of a heavy patch,
                                   section 4); 0 = 2048 (2D) / 4096 (3D), or
                                   the autotuner's choice                   */
    int32_t field_tile_x;       /* nodes per field-kernel tile along x; 0 =
                                   the widest that the region width allows, or
                                   the autotuner's choice                   */
    const pic_particles_in *particles;   /* may be null: no particles      */
    const pic_fields_in    *fields;      /* may be null: zero fields       */
} pic_config;

/* Where device memory and work go.  alloc(bytes, stream, user) returns
 * device memory or null; free(ptr, bytes, stream, user) releases it.  Both
 * null: hipMalloc / hipFree.  stream: a hipStream_t (null = null stream).
 * hbm_budget: bytes the context may hold in total (0 = unlimited); every
 * device allocation of the context counts, set-up staging, read-out
 * scratch and the autotuner's trial runs included, and one that would pass
 * the budget fails with PIC_E_NOMEM.
 * max_runs: run slots for pic_admit (0 = the n_runs given to pic_init).
 * deterministic: nonzero makes every run of the context bitwise
 * reproducible.  SDMD only re-decomposes one domain (section 2.2), so a
 * run's result is defined independently of how its particles are split
 * into patches and segments, of the regions, and of the other runs beside
 * it; floating-point sums, however, depend on the order of their terms, and
 * atomic deposition fixes no order.  In this mode each current and charge
 * contribution is rounded once to a multiple of a quantum (a power of two
 * chosen per run: about 2^-62 of the run's particle count times its largest
 * possible contribution, reported by pic_diag as det_quantum) and summed in
 * 64-bit integers, which is exact.  Then E, B, Bm, J, rho and every
 * particle's state are the same bit for bit on every execution, alone or
 * in a batch, for any region layout, and after a resume from exported
 * state; the storage order of particles inside a patch and the last bits of
 * the kinetic-energy sum (taken in storage order) are not.  The current
 * differs from the FP64 sum by at most half a quantum per contribution.
 * Costs one more FP64 operation and a 64-bit integer subtraction per
 * deposit in the FP64 form (the split form sums in fixed point anyway),
 * 8-byte current tiles in HBM in the split form, and no mover queue (every
 * particle's rest of frame is deposited inline). */
typedef struct {
    void *(*alloc)(size_t bytes, void *stream, void *user);
    void (*free)(void *ptr, size_t bytes, void *stream, void *user);
    void   *stream;
    void   *user;
    size_t  hbm_budget;
    int32_t max_runs;
    int32_t flags;              /* PIC_RT_* */
    int32_t deterministic;
    int32_t reserved;
} pic_runtime;

/* Diagnostics of one run at its current step.  t_ms: time per step of the
 * phases over the last pic_time_phases call, order Particles,
 * SyncDec-i + Fields (fused), Sync (ghosts + re-binning), Relayout. */
typedef struct {
    int64_t step;
    double  t;
    int64_t n_particles;
    int64_t patch_min, patch_max;     /* particles per patch */
    double  patch_mean;
    double  U_E, U_B, K;              /* 1/2 sum E^2 dV, 1/2 sum Bm^2 dV,
                                         sum m w (gamma - 1) dV            */
    double  t_ms[4];
    int64_t n_relayout;               /* device re-layouts of the particle
                                         store since pic_init              */
    int64_t n_spill;                  /* particles parked outside their
                                         patch segment right now           */
    int32_t err_flags;                /* bit 0 non-finite, bit 1 move >= 1
                                         cell, bit 2 capacity overflow     */
    int32_t patch[3];                 /* patch shape in use                */
    double  gauss_residual;           /* max over nodes of |(div E - rho)^n
                                         - (div E - rho)^0| / max |rho^n|:
                                         round-off for the charge-conserving
                                         path (with the current filter the
                                         conserved form involves the filtered
                                         rho, and this figure drifts)       */
    int32_t kernel_path[4];           /* compiled paths the run's steps take:
                                         particle kernel patch edge (0 = the
                                         generic path reading the patch shape
                                         at run time), its LDS sizing class
                                         (8, 16, 32), field kernel tile width
                                         along x, 1 if deterministic       */
    int64_t device_bytes;             /* device bytes the context holds now
                                         (all runs and context buffers)    */
    int64_t device_bytes_peak;        /* the most it has held since pic_init;
                                         never above pic_runtime.hbm_budget
                                         when a budget is set              */
    double  det_quantum[2];           /* deterministic mode: the quantum of
                                         the fixed-point current and charge
                                         sums (0 otherwise)                */
    int32_t seg_cap;                  /* segment capacity in use           */
    int32_t reserved;
    double  t_push_kernel_ms;         /* the particle kernels' own duration
                                         per step over the last
                                         pic_time_phases call (events tied to
                                         their launches: kernel start to
                                         kernel end, without the dispatch
                                         gaps that t_ms[0] includes)       */
} pic_diag_t;

/* Particle export (host memory, caller owned).  capacity is the length of
 * every non-null array; n receives the particle count (PIC_E_INVAL with n
 * set if capacity is too small).  Order is the storage order (patch by
 * patch); positions are FP64 in [0, L); patch receives each particle's
 * patch index (x fastest over patches). */
typedef struct {
    int64_t capacity;
    int64_t n;
    double *x, *y, *z, *ux, *uy, *uz, *w;
    uint32_t *id;
    int32_t *patch;
} pic_particles_out;

/* Create a context holding n_runs independent runs (section 2.2 problem
 * statement per run) and bin their particles into patches.  Configs are
 * read and copied; *out receives the context.  With PIC_E_CONFIG the text
 * of the broken rule is in pic_last_error(NULL). */
int pic_init(const pic_config *cfgs, int32_t n_runs, const pic_runtime *rt, pic_ctx **out);

/* Enqueue n_steps SDMD steps for every active run on rt->stream and return
 * without waiting.  One step is the iteration of sections 2.2 and 3.3 of the
 * paper on the two decompositions of one domain: per patch, interpolation
 * of E^n and Bm^n from the patch's copy of its region's fields, push and
 * Esirkepov order-2 deposition into the patch's own current tile (the
 * "Particles" timer of section 3.3; methods of section 3.2); transfer (i),
 * every patch tile summed into its region, optionally smoothed by the
 * binomial filter; the Maxwell solve (Yee, or the spectral solver) on each
 * region, with ghost layers exchanged between regions; transfer (ii), each
 * region's new fields copied into the windows of its patches; and the
 * particles that left their patch moved to the patch that now holds them.
 * Runs that have reached their max_steps stay as they are.
 * n_steps: >= 0 (0 does nothing).  Returns PIC_OK once the work is
 * enqueued, PIC_E_INVAL for a null context or n_steps < 0, PIC_E_DEVICE if
 * a launch fails.  Errors the kernels detect while stepping (a position
 * outside [0, L), a non-finite value, a move of a cell or more in one step,
 * a store overflow) are latched per run on the device and returned by the
 * next synchronising call on that run (pic_fields, pic_diag, pic_particles)
 * as PIC_E_CONFIG, PIC_E_NUMERIC or PIC_E_OVERFLOW. */
int pic_step(pic_ctx *ctx, int32_t n_steps);

/* Read the fields of `run` as the undecomposed grid of section 2.1 would
 * hold them: the regions that own the fields in SDMD (section 2.2) are
 * assembled into one array, ghost layers dropped.  mask selects components
 * (PIC_F_*); they are written to dst in bit order, each nx*ny*nz FP64 values
 * in the layout above (x fastest, staggering as listed there).  dst is
 * caller owned, host memory, or device memory when dst_on_device != 0;
 * dst_len is its capacity in doubles (PIC_E_INVAL if it is too small, or for
 * a null pointer or a bad run).  Synchronises the stream and reports the
 * run's latched kernel errors (see pic_step). */
int pic_fields(pic_ctx *ctx, int32_t run, uint32_t mask, double *dst, size_t dst_len, int32_t dst_on_device);

/* Fill *out (caller owned) for `run`: step count, particle count, the
 * energies of fields and electrons (the energy balance an explicit PIC
 * scheme is checked with), the Gauss-law residual div E - rho against its
 * initial value (charge conservation of the Esirkepov deposition, section
 * 3.2), the patch size of section 2.2's fine decomposition and the split
 * of dense patches into several work items that section 4 proposes
 * (segments), re-layout and spill counts, the compiled kernel path, memory
 * and, after pic_time_phases, the per-phase times that correspond to the
 * timers of section 3.3.  Allocates device scratch for the charge density
 * and the residual (16 bytes per cell) and frees it before returning;
 * PIC_E_NOMEM if that fails or would exceed hbm_budget, PIC_E_INVAL for
 * null pointers or a bad run.  Synchronises the stream and reports the
 * run's latched kernel errors (see pic_step). */
int pic_diag(pic_ctx *ctx, int32_t run, pic_diag_t *out);

/* pic_diag without any device allocation, for callers that cannot allocate
 * device memory (a loop that must not call hipMalloc, code sharing the
 * process with HIP graph capture, harnesses that forbid allocation).  Same
 * output as pic_diag, from the same kernels; their scratch (charge density,
 * Gauss residual and partial sums: 16 bytes per cell plus a few KB) lives in
 * one static device array of 64 MiB per GPU, which the library holds from
 * the first pic_init on that GPU until the process ends.  Runs of up to
 * about 4.1 million cells fit; a larger run gets PIC_E_NOMEM and
 * pic_last_error gives the bytes it would need.  Every call on one GPU
 * shares that array and leaves its contents behind: calls that overlap on
 * one GPU (other threads, other contexts) race and must be serialised by
 * the caller.  Synchronises the stream. */
int pic_diag_noalloc(pic_ctx *ctx, int32_t run, pic_diag_t *out);

/* Export the particles of `run` (see pic_particles_out). Synchronises. */
int pic_particles(pic_ctx *ctx, int32_t run, pic_particles_out *out);

/* Device bytes pic_init / pic_admit would take for this config at most
 * (admission by HBM budget): what the run holds between calls plus the most
 * any call takes on top of it (set-up staging, read-out scratch, patch
 * autotuning), counted with the deterministic mode's 8-byte current tiles
 * so that the figure bounds both modes.  Does not touch the GPU. */
int pic_mem_bytes(const pic_config *cfg, size_t *bytes);

/* Add a run to a live context (continuous batching); *run_id receives its
 * slot.  PIC_E_CAPACITY if every slot is taken, PIC_E_NOMEM if the budget
 * would be exceeded.  The new run advances with the next pic_step. */
int pic_admit(pic_ctx *ctx, const pic_config *cfg, int32_t *run_id);

/* Release a run's slot and device memory.  Its results must have been read
 * before.  Enqueued work is drained first. */
int pic_retire(pic_ctx *ctx, int32_t run);

/* Number of steps `run` has taken or will have taken once the enqueued work
 * completes (host counter, no synchronisation; capped at max_steps). */
int pic_run_steps(pic_ctx *ctx, int32_t run, int64_t *steps);

/* Take n_steps (>= 1) normal steps of every active run, enqueued phase by
 * phase with a HIP event between phases and one synchronisation at the end
 * (the device waits ~200 us first while the host enqueues, so the kernels
 * run back to back); the diagnostics' t_ms then hold each phase's average
 * time per step over these steps.  PIC_E_INVAL for n_steps < 1. */
int pic_time_phases(pic_ctx *ctx, int32_t n_steps);

/* Release everything.  Null is allowed. */
void pic_free(pic_ctx *ctx);

/* Static text for an error code. */
const char *pic_strerror(int code);

/* Text of the last error of ctx (or of the last failed pic_init when ctx is
 * null).  Valid until the next call on the same context. */
const char *pic_last_error(pic_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SDMD_PIC_H */
