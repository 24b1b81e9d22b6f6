/*
 * swe.h -- C ABI of the MI355X (gfx950) library for the well-balanced
 * finite-volume step of the 2D Saint-Venant (shallow-water) system.
 *
 * Method (arXiv:1307.4839, "FullSWOF_Paral", Sections 2-3):
 *   model SW2D (Section 2.1) with rain R, Green-Ampt infiltration
 *   (Section 3.5) and Manning or Darcy-Weisbach friction (Section 2.1);
 *   second-order MUSCL/minmod reconstruction of h, h+z and u (Section 3.4),
 *   hydrostatic reconstruction with the S and Fc source corrections
 *   (Section 3.1, eq. SW1Dscheme), HLL flux (Section 3.3), semi-implicit
 *   friction and Heun's RK2 (Section 3.2), CFL time step on the
 *   reconstructed states (Section 3.3, eq. cfl), ghost-cell boundary
 *   conditions (Section 2.2) with two ghost layers (Section 6.1), and the
 *   per-stage order of Algorithm 1 (Section 6.2).
 *
 * Conventions
 *   - Every array is FP64, [ny][nx] row-major with x fastest, no padding.
 *     Cell (i, j) has centre ((i + 1/2) dx, (j + 1/2) dy).
 *   - Device pointers are owned by the caller; the library never frees them
 *     and keeps them only for the life of the context.  Host pointers are
 *     never retained past the call.
 *   - All work is enqueued on the caller's HIP stream given at creation;
 *     calls documented as "synchronizes" wait for that stream.
 *   - Every function returns 0 on success or a negative SWE_E* code.
 *   - A context is not thread-safe.  Contexts on the same device are
 *     independent (each has its own workspace).
 *   - Water depth is never clamped: a negative or non-finite value is
 *     reported through sticky status flags.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* error codes */
#define SWE_OK 0
#define SWE_EINVAL (-1)     /* invalid argument or parameter */
#define SWE_EHIP (-2)       /* a HIP runtime call failed */
#define SWE_ENEGDEPTH (-3)  /* a negative water depth was produced */
#define SWE_ENONFINITE (-4) /* a non-finite value was produced */
#define SWE_EDTMIN (-5)     /* the time step collapsed below dt_min */
#define SWE_ENOMEM (-6)     /* workspace too small */
#define SWE_EDT (-7)        /* the time step was not finite */

/* sticky status flags (swe_get_status) */
#define SWE_FLAG_NEGDEPTH 1u
#define SWE_FLAG_NONFINITE 2u
#define SWE_FLAG_DT 4u           /* a step's dt was not finite */
#define SWE_FLAG_DT_UNDERFLOW 8u /* a step's dt fell below dt_min */

/* boundary types, Section 2.2: ghost cells.  WALL mirrors the boundary
 * cells (normal discharge negated); OUTFLOW copies the boundary cell (free,
 * zero-gradient outflow).  The imposed types take the ghost state from the
 * Riemann invariants (Section 2.2: one variable is imposed in fluvial flow,
 * both in supercritical inflow, none in supercritical outflow).  With w the
 * outward normal velocity of the boundary cell and c = sqrt(g h), the
 * invariant w + 2c leaves the domain and the ghost keeps it:
 *   IMPOSED_H   depth bc_h; the ghost's normal velocity from the invariant;
 *   IMPOSED_Q   inflow discharge bc_q >= 0 per unit width; the ghost's depth
 *               solves 2 sqrt(g h) - bc_q / h = w + 2c (fixed bisection);
 *   IMPOSED_HQ  both (supercritical inflow).
 * A boundary cell in supercritical outflow (w > c) has a free ghost (the
 * copy) under every imposed type.  The tangential velocity is the cell's.
 * Both ghost layers are equal; the bed of the ghosts is the cell's.  A
 * supercritical inflow needs IMPOSED_HQ: under IMPOSED_H or IMPOSED_Q the
 * invariant is still used but is then not carried out of the domain.
 * Single contexts and ensemble members (the adjoint rejects them). */
#define SWE_BC_WALL 0
#define SWE_BC_OUTFLOW 1
#define SWE_BC_IMPOSED_H 2
#define SWE_BC_IMPOSED_Q 3
#define SWE_BC_IMPOSED_HQ 4

/* friction laws, Section 2.1 */
#define SWE_FRIC_NONE 0
#define SWE_FRIC_MANNING 1 /* coefficient n:  S_f = n^2 |u| u / h^(4/3) */
#define SWE_FRIC_DARCY 2   /* coefficient f:  S_f = f/(8g) |u| u / h    */

/* Largest row length (cells along x): a cell's byte offset within its row
 * stays below 2^31. */
#define SWE_MAX_NX (1 << 28)

typedef struct swe_params {
    int32_t nx, ny;      /* cells, >= 2 each; nx <= SWE_MAX_NX, nx ny <= 2^36 */
    double dx, dy;       /* cell sizes [m], > 0 */
    double g;            /* gravity [m/s^2] (9.81) */
    double cfl;          /* n_CFL (0.5 at second order, eq. cfl) */
    double dt_max;       /* upper bound on dt [s] (INFINITY for none) */
    double h_eps;        /* dry threshold [m]: velocity is 0 at or below it */
    int32_t bc[4];       /* west, east, south, north: SWE_BC_* */
    int32_t fric_law;    /* SWE_FRIC_* */
    double fric_coef;    /* n or f, used when the friction field is NULL */
    double rain;         /* rain intensity R [m/s] (uniform) */
    int32_t infil_on;    /* 1: Green-Ampt infiltration (needs vinf buffer) */
    double ks;           /* saturated conductivity K_s [m/s] */
    double psi;          /* wetting-front suction head, magnitude >= 0 [m] */
    double dtheta;       /* theta_s - theta_i, > 0 */
    int32_t order;       /* 1: first order (Section 3.3: no reconstruction,
                            one explicit Euler stage per step; the paper
                            pairs it with cfl = 1); 0 or 2: MUSCL + Heun */
    int32_t flux;        /* numerical flux (Section 3.3): 0 HLL (the
                            paper's), 1 Rusanov (local Lax-Friedrichs),
                            2 kinetic (Perthame-Simeoni, particle velocities
                            uniform on [u - s, u + s], s = sqrt(3gh/2); the
                            time step then uses |u| + s as the speed),
                            3 VFRoe-ncv (Section 4.1: the interface state of
                            the Riemann problem in (2 sqrt(gh), u)
                            linearized about the mean state; a dry side
                            takes the other side's velocity; not
                            positivity-preserving in general).  The adjoint
                            takes the second-order MUSCL scheme with fluxes
                            0-2; the members of an ensemble share order and
                            flux (0-2, MUSCL at second order). */
    double bc_h[4];      /* imposed depth [m] per side (west, east, south,
                            north), finite and > 0 where bc is IMPOSED_H or
                            IMPOSED_HQ; ignored elsewhere */
    double bc_q[4];      /* imposed inflow discharge [m^2/s] per side,
                            finite and >= 0 where bc is IMPOSED_Q or
                            IMPOSED_HQ; ignored elsewhere */
    double dt_min;       /* smallest acceptable dt [s] (0: no bound; finite,
                            >= 0).  A step whose eq. (cfl) dt falls below it
                            is a collapse of the time step (a wet/dry front
                            or a blow-up driving the wave speeds up): the
                            step is not taken, SWE_FLAG_DT_UNDERFLOW is
                            raised and later steps are not taken either
                            while it holds.  The last step of a run, clipped
                            to t_end - t, is exempt (dt == t_end - t). */
    int32_t recon;       /* second-order reconstruction (Section 4.1 lists
                            MUSCL, ENO and modified ENO): 0 MUSCL with
                            minmod (the paper's, Section 3.4); 1 ENO: the
                            slope of h, h+z and the velocities is the
                            one-sided difference of smaller magnitude (the
                            left one on ties), which keeps slopes at extrema
                            and may give negative face depths; 2 modified
                            ENO: ENO with the depth slope limited to
                            |D| <= 2 h_i (face depths in [0, 2 h_i]).  Used
                            at second order only. */
} swe_params;

/* Optional per-cell fields below are read only, [ny][nx] FP64 device
 * arrays like the state; NULL selects the scalar of swe_params.  Rain is
 * R(t, x, y) = r(t) rain_w(x, y) (Section 2.1 lets R vary in time and
 * space), with r(t) the hyetograph of swe_set_hyetograph or the constant
 * swe_params.rain.  Values are used as given (a negative weight or
 * conductivity is not rejected; the status flags report what follows). */
typedef struct swe_buffers {
    double* h;           /* water depth (in/out) */
    double* qx;          /* discharge along x (in/out) */
    double* qy;          /* discharge along y (in/out) */
    const double* z;     /* topography (in) */
    const double* fric;  /* per-cell friction coefficient, or NULL */
    double* vinf;        /* infiltrated volume per unit area (in/out); NULL
                            unless infil_on */
    const double* rain_w;  /* rain weight w >= 0 (dimensionless), or NULL */
    const double* ks;      /* Green-Ampt K_s [m/s] per cell, or NULL */
    const double* psi;     /* Green-Ampt suction head >= 0 [m], or NULL */
    const double* dtheta;  /* theta_s - theta_i > 0 per cell, or NULL */
} swe_buffers;

/* largest number of hyetograph breakpoints */
#define SWE_HYETO_MAX 128

typedef struct swe_ctx swe_ctx;

typedef struct swe_diag {
    double mass;         /* sum of h dx dy [m^3] */
    double infiltrated;  /* sum of vinf dx dy [m^3] */
    double h_min, h_max; /* extrema of h */
    int64_t wet_cells;   /* cells with h > h_eps */
    double rain_in;      /* rain fallen on the domain since creation,
                            sum over steps of dt r(t^n) sum(w) dx dy [m^3] */
    double outflow;      /* net volume that left through the sides since
                            creation: the balance water at creation + rain_in
                            - (mass + infiltrated) of the conservative scheme
                            (valid while only swe_step changes the state) */
} swe_diag;

/* Size in bytes of the device workspace a context needs for these
 * parameters: a second state (3 nx ny doubles), the stage rate Phi
 * (3 nx ny doubles) and a block of device scalars (time, step count,
 * wave-speed accumulators, hyetograph; about 8 KB). */
int swe_workspace_bytes(const swe_params* p, size_t* bytes);

/* Create a context.  `workspace` is caller-owned device memory of at least
 * swe_workspace_bytes() bytes, 256-byte aligned; `stream` is a hipStream_t
 * (NULL = default stream).  The buffers must stay valid for the life of the
 * context.  Sets t = 0 and clears the status flags (enqueued on the stream). */
int swe_create(const swe_params* p, const swe_buffers* b, void* workspace,
               size_t workspace_bytes, void* stream, swe_ctx** out);

int swe_destroy(swe_ctx* ctx);

/* Tile shape of the stage kernels: `tx` threads per block (64, 128 or 256)
 * own a strip of tx - 4 output columns; each block marches `ty` rows
 * (0 = automatic).  Results do not depend on the tile shape (every cell and
 * face is evaluated by the same formulas on the same inputs).  SWE_EINVAL
 * for other widths, ty > ny, or a ty that leaves more than 65535 row
 * blocks. */
int swe_set_tiling(swe_ctx* ctx, int32_t tx, int32_t ty);
int swe_get_tiling(swe_ctx* ctx, int32_t* tx, int32_t* ty);

/* Stream-ordered update of the simulated time t [s]. */
int swe_set_time(swe_ctx* ctx, double t);

/* Rain intensity [m/s] for steps enqueued after this call (used while no
 * hyetograph is set). */
int swe_set_rain(swe_ctx* ctx, double rain);

/* New imposed values of one side (0 west, 1 east, 2 south, 3 north) for the
 * steps enqueued after this call: a hydrograph or a varying level is fed
 * this way between calls of swe_step (Section 2.2; the values are constant
 * over a step).  The side must have an imposed type; the values follow the
 * rules of swe_params.bc_h / bc_q for that type, else SWE_EINVAL. */
int swe_set_boundary_values(swe_ctx* ctx, int32_t side, double h_b, double q_b);

/* Hyetograph r(t) (Section 2.1: R depends on t): a step from time t rains
 * r[k] for the last k with t_pts[k] <= t (rain is explicit, so the rate at
 * the start of the step holds for the whole step), and 0 when t < t_pts[0].
 * Host arrays of n values, copied: 1 <= n <= SWE_HYETO_MAX, t_pts finite
 * and strictly increasing, r finite and >= 0 [m/s]; n == 0 (pointers may be
 * NULL) removes the hyetograph.  The copy is stream-ordered after the steps
 * enqueued before it, and the call synchronizes the stream before it
 * returns.  SWE_EINVAL for invalid tables, SWE_EHIP if the copy fails. */
int swe_set_hyetograph(swe_ctx* ctx, const double* t_pts, const double* r, int32_t n);

/* Optional device log of time steps: step k (counted from context creation)
 * writes its dt to log[k] while k < capacity.  NULL disables. */
int swe_set_dt_log(swe_ctx* ctx, double* dev_log, int64_t capacity);

/* Enqueue `nsteps` time steps (Algorithm 1: two stages, then Heun, then rain
 * and infiltration).  dt = min(dt_max, cfl / (Ax/dx + Ay/dy), t_end - t)
 * where Ax, Ay bound |u| + sqrt(g h) over the reconstructed face states
 * (eq. cfl).  Steps once t >= t_end are no-ops.  Asynchronous (the host
 * never waits) unless t_end is finite and nsteps > 256: the steps are then
 * enqueued 256 at a time and the call waits for each batch to read the time,
 * returning once t_end is reached instead of enqueueing steps that would all
 * be no-ops.  Runs of 16 steps replay a captured HIP graph (re-captured
 * when t_end, the rain, the tiling or the dt log change).  On return
 * (stream order) the state is in the caller's h/qx/qy buffers. */
int swe_step(swe_ctx* ctx, int32_t nsteps, double t_end);

/* Synchronizes.  Current time, last dt and number of steps taken. */
int swe_get_time(swe_ctx* ctx, double* t, double* last_dt, int64_t* steps);

/* Synchronizes.  Sticky SWE_FLAG_* bits; returns the SWE_E* code of the
 * most serious flag set (0 if none), in the order NONFINITE, NEGDEPTH, DT,
 * DT_UNDERFLOW. */
int swe_get_status(swe_ctx* ctx, uint32_t* flags);

/* Synchronizes.  Deterministic (fixed-order) reductions of the state. */
int swe_get_diagnostics(swe_ctx* ctx, swe_diag* d);

/* One convective rate evaluation without stepping (Section 3.1, eq.
 * SW1Dscheme in 2D): Phi(U) = -(X/dx + Y/dy) for the given state, written
 * to ph/pqx/pqy (device, N doubles each), and the face wave-speed bounds
 * (Ax, Ay) to amax (host, 2 doubles).  Synchronizes. */
int swe_rate(swe_ctx* ctx, const double* h, const double* qx,
             const double* qy, double* ph, double* pqx, double* pqy,
             double* amax);

/* Per-kernel timing of the next `max_steps` steps: HIP events are recorded
 * on the context's stream before the stage-1 launch, between the stages and
 * after the stage-2 launch of each step.  Host-side event objects only; no
 * device memory.  SWE_EINVAL if a profile is already open. */
int swe_profile_begin(swe_ctx* ctx, int32_t max_steps);

/* Synchronizes.  Total milliseconds spent in the stage-1 (rate) and stage-2
 * (update) kernels over the profiled steps, and their number; closes the
 * profile. */
int swe_profile_end(swe_ctx* ctx, double* ms_rate, double* ms_update,
                    int32_t* nsteps);

/* ---------------------------------------------------------------------------
 * Ensembles: `count` independent simulations of arbitrary (uneven) sizes
 * stepped together.  Member k has its own swe_params p[k] and caller-owned
 * buffers b[k] (same conventions as swe_create), its own time, time step
 * (its own CFL bound), status flags and rain; all members share the
 * scheme (order and flux: SWE_EINVAL otherwise).  One step of the ensemble is
 * one launch per stage over a work list of (member, strip, row range) tiles,
 * one block per tile; runs of 16 steps replay a captured HIP graph.  Every member
 * evolves exactly (bit for bit) as it would in its own context.
 * ------------------------------------------------------------------------- */
typedef struct swe_batch swe_batch;

/* Device workspace for the ensemble: member table, work list, and per
 * member a scalar block, a second state, the stage rate and a backup of the
 * state used by the autotuner. */
int swe_batch_workspace_bytes(const swe_params* p, int32_t count, size_t* bytes);

int swe_batch_create(const swe_params* p, const swe_buffers* b, int32_t count,
                     void* workspace, size_t workspace_bytes, void* stream,
                     swe_batch** out);
int swe_batch_destroy(swe_batch* b);

/* Tile shape of the ensemble kernels: tx in {64, 128, 256}, ty >= 4. */
int swe_batch_set_tiling(swe_batch* b, int32_t tx, int32_t ty);
int swe_batch_get_tiling(swe_batch* b, int32_t* tx, int32_t* ty, int32_t* ntiles);

/* Measure every tile shape (tx in {64, 128, 256} x ty in {8, 16, 32, 64})
 * on `trial_steps` steps of the live ensemble, keep the fastest, and restore
 * the state, times and flags exactly as they were.  Synchronizes.  Returns
 * the chosen shape and its time per step [ms]. */
int swe_batch_autotune(swe_batch* b, int32_t trial_steps, int32_t* tx, int32_t* ty,
                       double* ms_per_step);

int swe_batch_set_rain(swe_batch* b, int32_t member, double rain);
/* swe_set_boundary_values for one member (same rules; synchronizes). */
int swe_batch_set_boundary_values(swe_batch* b, int32_t member, int32_t side, double h_b,
                                  double q_b);
/* swe_set_hyetograph for one member (same rules; synchronizes). */
int swe_batch_set_hyetograph(swe_batch* b, int32_t member, const double* t_pts,
                             const double* r, int32_t n);
int swe_batch_set_dt_log(swe_batch* b, int32_t member, double* dev_log, int64_t capacity);

/* Enqueue `nsteps` steps of every member (members stop at t_end). */
int swe_batch_step(swe_batch* b, int32_t nsteps, double t_end);

/* Synchronize.  Time of one member; sticky flags of all members (flags has
 * room for n >= count entries); the return code is that of the most serious
 * flag set in any member. */
int swe_batch_get_time(swe_batch* b, int32_t member, double* t, double* last_dt,
                       int64_t* steps);
int swe_batch_get_status(swe_batch* b, uint32_t* flags, int32_t n);

/* ---------------------------------------------------------------------------
 * Adjoint (reverse-mode gradient) of a run with respect to the per-cell
 * friction coefficient field (b->fric, required; Manning or Darcy-Weisbach;
 * no infiltration).  The run is `nsteps` steps from the state in b->h/qx/qy
 * (left untouched); the loss is
 *     L = sum over k = every, 2 every, ... <= nsteps, over m < ngauges, of
 *         (h after step k at cell gauges[m] - obs[(k/every - 1) ngauges + m])^2.
 * The gradient is that of the discrete step (Sections 3.1-3.4) with the time
 * step sequence frozen to the forward run's; kinks take the derivative of
 * the selected branch (first argument on ties; 0 for minmod of opposite
 * signs and for square/cube roots at 0).  States are recomputed from
 * checkpoints every `ckpt_every` steps (sqrt(nsteps) is the usual choice).
 * gauges (int32) and obs (FP64) are device arrays that must stay valid.
 * ------------------------------------------------------------------------- */
typedef struct swe_adj swe_adj;

/* The workspace holds the checkpoints (every ckpt_every-th state) and one
 * segment of ckpt_every states with their two stage rates.  The forward
 * pass leaves the last segment there, so the reverse pass recomputes every
 * segment but that one: with ckpt_every >= nsteps (one segment, about
 * 9 nx ny nsteps doubles) it recomputes nothing. */
int swe_adj_workspace_bytes(const swe_params* p, int32_t nsteps, int32_t ckpt_every,
                            int32_t ngauges, int32_t every, size_t* bytes);
int swe_adj_create(const swe_params* p, const swe_buffers* b, int32_t nsteps,
                   int32_t ckpt_every, const int32_t* gauges, int32_t ngauges,
                   int32_t every, const double* obs, void* workspace,
                   size_t workspace_bytes, void* stream, swe_adj** out);
int swe_adj_destroy(swe_adj* a);

/* Freeze the time step sequence to dts (device, nsteps values); NULL lets
 * the next forward pass choose dt by eq. (cfl) and freezes what it chose. */
int swe_adj_set_dts(swe_adj* a, const double* dts);
/* Copy the frozen sequence to dts (device, nsteps values). */
int swe_adj_get_dts(swe_adj* a, double* dts);

/* Synchronizes.  Runs the forward pass, storing checkpoints and the gauge
 * series, and returns the loss (host).  Status flags of the forward steps
 * give the return code. */
int swe_adj_forward(swe_adj* a, double* loss);

/* Synchronizes.  dL/d(fric) into grad (device, nx ny values) for the last
 * forward pass. */
int swe_adj_backward(swe_adj* a, double* grad);

/* Gauge depths of the last forward pass, (nsteps/every) x ngauges values
 * (device, row-major), stream-ordered. */
int swe_adj_get_series(swe_adj* a, double* out);

/* Gauge recorder of a single context (Section 4.2: the water depth at
 * gauges over time is the output the Malpasset validation compares).
 * After every step that advances the simulation, when the number of steps
 * taken since this call is a positive multiple k * every, h of the new state
 * at each gauge cell goes to series[(k - 1) * ngauges + m] for k <= max_samples
 * (later samples are dropped).  cells (int32 flat indices j * nx + i) and
 * series (FP64, max_samples * ngauges) are caller-owned device arrays that
 * must stay valid while recording; a cell index outside the grid records
 * NaN.  ngauges = 0 stops recording.  Synchronizes (it reads the step
 * count). */
int swe_set_gauges(swe_ctx* ctx, const int32_t* cells, int32_t ngauges, int32_t every,
                   double* series, int64_t max_samples);

/* Number of samples recorded since swe_set_gauges (at most max_samples);
 * copies min(that, max_copy) samples (ngauges values each) to the host
 * array out when out is not NULL.  Synchronizes. */
int swe_get_gauges(swe_ctx* ctx, double* out, int64_t max_copy, int64_t* nsamples);

/* ---------------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops and harnesses that forbid hipMalloc.
 *
 * swe_run_noalloc is swe_create + swe_set_time(t0) + swe_step(nsteps, t_end)
 * in one call, with the library's own scratch array as the workspace (a
 * file-scope device array of 6 SWE_NOALLOC_MAX_CELLS doubles plus a scalar
 * block, about 48 MiB, which every device the library runs on holds until
 * the process ends).  It allocates nothing and creates no stream, event or
 * graph: it validates, then enqueues the init, stage and copy kernels of
 * the steps on `stream` (NULL = default stream) and returns without waiting.
 * The steps, kernels and results are those of swe_step on the same inputs
 * (bit for bit), with the default tiling, no gauges, no dt log and no
 * hyetograph.  p and b as for swe_create (b's device buffers are the inputs
 * and outputs: on completion the state is in b->h/qx/qy and V_inf in
 * b->vinf); t0 finite; nsteps >= 0.  info is caller-owned device memory of 4
 * doubles that receives, in stream order, the time reached, the last dt,
 * the number of steps taken and the sticky SWE_FLAG_* bits (as doubles).
 * Returns SWE_ENOMEM if nx ny > SWE_NOALLOC_MAX_CELLS, SWE_EINVAL for
 * invalid arguments (nothing is enqueued then), SWE_EHIP if a launch fails.
 * Every call on a device shares that device's scratch array, which keeps
 * the last call's contents (the call clears what must start at zero): calls
 * that overlap on one device (other streams, other host threads) race. */
#define SWE_NOALLOC_MAX_CELLS (1 << 20)
int swe_run_noalloc(const swe_params* p, const swe_buffers* b, double t0, int32_t nsteps,
                    double t_end, void* stream, double* info);

/* Human-readable text for an error code. */
const char* swe_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* SWE_H */
