/*
 * dg.h — C ABI of the MI355X (gfx950) RKDG library with the jump filter.
 *
 * Method: Wei, Zhou, Xia, "The jump filter in the discontinuous Galerkin
 * method for hyperbolic conservation laws", arXiv:2407.19169.
 *   - modal Legendre DG space, mode 0 = cell average          (Sec. 2.1)
 *   - semi-discrete DG operator with an LLF interface flux    (Sec. 2.1, scheme (scheme:DG); Sec. 3)
 *   - third-order SSP Runge-Kutta in Shu-Osher form           (Sec. 2.2, (rkdg1); Sec. 3)
 *   - jump filter after every RK stage                        (Sec. 2.1 (para:damp2)-(timespli:1dscalar);
 *                                                              Sec. 2.3 (para:damp22d); Sec. 2.4 (timespli:sys))
 *   - hybrid limiter with the filter as low-order limiter     (Sec. 3, Algorithm 1)
 *
 * Conventions shared by every call:
 *   - Every function returns 0 (DG_OK) or a negative dg_status code.
 *   - All state pointers are DEVICE pointers owned by the caller (e.g. torch
 *     tensors); the library never allocates or frees state or workspace
 *     memory.  The solver handle owns only its parameters and a captured
 *     HIP graph.
 *   - Calls are ordered on the stream given in dg_options (NULL = the null
 *     stream).  Only dg_max_wavespeed, dg_run, dg_report_read and
 *     dg_run_batch synchronise that stream.
 *   - A handle is not thread-safe; separate handles are independent.
 *
 * State layout ("FP64 layout", the exchange format of dg_set_state and
 * dg_get_state, and the internal layout of DG_PREC_FP64):
 *   1D: u[(var*(k+1) + l)*n + j]                   var-major, then mode, then cell
 *   2D: u[((var*(k+1)^2 + p*(k+1) + q)*ny + jy)*nx + ix]   x fastest
 * where l (1D) or (p, q) (2D, Q^k tensor Legendre) index the modes.
 * In DG_PREC_MIXED the bound buffers hold an FP64 plane per variable for
 * mode 0 followed by FP32 planes for modes >= 1 (sizes from
 * dg_buffer_sizes); use dg_set_state/dg_get_state to convert.
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DG_OK = 0,
    DG_ERR_ARG = -1,         /* invalid argument (NULL, size, range)               */
    DG_ERR_UNSUPPORTED = -2, /* degree / dimension / equation combination          */
    DG_ERR_DEVICE = -3,      /* a HIP runtime call failed                          */
    DG_ERR_NONFINITE = -4,   /* a NaN/Inf appeared in the state or the time step   */
    DG_ERR_POSITIVITY = -5,  /* Euler: density or pressure <= 0 at a trace/quad pt */
    DG_ERR_STATE = -6        /* buffers not bound, or calls out of order           */
} dg_status;

typedef enum { DG_EQ_ADVECTION = 0, DG_EQ_BURGERS = 1, DG_EQ_EULER = 2 } dg_equation;

/* Boundary conditions (one per side).  PERIODIC must be set on both sides
 * of an axis.  OUTFLOW copies the interior trace (and its derivatives);
 * REFLECT mirrors it with the normal momentum negated (Euler only);
 * DIRICHLET imposes the constant conserved state mesh.dirichlet[side]
 * (inflow).  The two double-Mach-reflection boundaries (2D Euler, y sides)
 * use the oblique shock line x = shock_x0 + y/sqrt(3) + shock_speed*t:
 * DMR_WALL imposes mesh.post for x < shock_x0 and reflects beyond;
 * DMR_TOP imposes mesh.post behind the line and mesh.pre ahead of it.
 * Boundary states of the flux are taken at the RK stage times t, t+dt,
 * t+dt/2; those of the filter's jumps at the time the stage output stands
 * for, t+dt, t+dt/2, t+dt. */
typedef enum {
    DG_BC_PERIODIC = 0,
    DG_BC_OUTFLOW = 1,
    DG_BC_REFLECT = 2,
    DG_BC_DIRICHLET = 3,
    DG_BC_DMR_WALL = 4,
    DG_BC_DMR_TOP = 5
} dg_bc;

typedef enum { DG_FILTER_NONE = 0, DG_FILTER_JUMP = 1, DG_FILTER_HYBRID = 2 } dg_filter_mode;

/* DG_PREC_MIXED: mode 0 (cell averages), its update, the conservation
 * ledger and the positivity / wave-speed checks in FP64; higher modes are
 * stored, and volume, flux and filter arithmetic run, in FP32. */
typedef enum { DG_PREC_FP64 = 0, DG_PREC_MIXED = 1 } dg_precision;

/* Interface flux (Sec. 3: the computations use local Lax-Friedrichs; HLL
 * and HLLC are named there as alternatives).  HLL / HLLC: Euler only, with
 * Davis's wave-speed estimates; HLLC restores the contact wave. */
typedef enum { DG_FLUX_LLF = 0, DG_FLUX_HLL = 1, DG_FLUX_HLLC = 2 } dg_flux;

typedef struct {
    int dim;                 /* 1 or 2                                            */
    int64_t n[2];            /* cells along x (and y); uniform mesh               */
    double lo[2], hi[2];     /* domain [lo, hi] per axis                          */
    int bc[4];               /* dg_bc for x-lo, x-hi, y-lo, y-hi                  */
    double dirichlet[4][4];  /* conserved state per side (DIRICHLET)              */
    double shock_x0;         /* DMR_*: foot of the shock on the wall at t = 0     */
    double shock_speed;      /* DMR_*: speed of the shock line along x            */
    double post[4], pre[4];  /* DMR_*: conserved states behind / ahead of it      */
} dg_mesh;

typedef struct {
    int precision;           /* dg_precision                                      */
    int filter;              /* dg_filter_mode, applied after every RK stage      */
    double cfl;              /* dt = cfl * h / max wave speed (2D: cfl / max(ax/hx + ay/hy)) */
    double gamma;            /* ratio of specific heats (Euler)                   */
    double adv_speed[2];     /* advection velocity (DG_EQ_ADVECTION)              */
    int quad_points;         /* Gauss points per direction; 0 or degree+1         */
    void* stream;            /* hipStream_t; NULL = null stream                   */
    int cf_reading;          /* mesh factors (m_x, m_y) of the 2D Euler damping
                                coefficient (c_fx, c_fy) = (m_x beta_x, m_y beta_y) /
                                (4 lambda_pq H-bar) (Sec. 2.4, (para:damp22d1)):
                                0 (default): (h_x, h_y), as printed in Sec. 2.4;
                                1: (h_y, h_x), as printed for the Euler examples
                                   of Sec. 3.2 (equal to 0 on square cells);
                                2: (1, 1), no mesh factors (a state varying along
                                   one axis of square cells is then filtered
                                   exactly as by the 1D filter).
                                Other values: DG_ERR_ARG. */
    int positivity;          /* Euler: 1 = Zhang-Shu positivity-preserving limiter
                                after the post-stage operator (Sec. 3.2 uses it for
                                extreme cases): density and pressure kept positive at
                                each cell's test points -- 1D: the Gauss-Lobatto and
                                Gauss points; 2D: (Gauss-Lobatto x Gauss), (Gauss x
                                Gauss-Lobatto) and the Gauss x Gauss points.  A step
                                whose stage leaves an inadmissible cell average is
                                undone and retried with half the time step (at most
                                40 times; then the run stops with DG_ERR_POSITIVITY).
                                Positivity reports then concern cell averages only.
                                0 = off.  Other equations: DG_ERR_UNSUPPORTED. */
    int basis;               /* 2D space (Sec. 2.3): 0 = Q^k tensor product (modes
                                p, q <= k); 1 = P^k total degree (p + q <= k), the
                                paper's own space.  Both keep the Q^k layout; with P^k
                                the modes p + q > k are zero: dg_set_state drops them
                                (the L2 projection onto P^k, the basis being
                                orthogonal) and the residual keeps them at zero.  1D:
                                both values name the same space.  Other values:
                                DG_ERR_ARG. */
    int flux;                /* dg_flux; 0 = local Lax-Friedrichs.  HLL / HLLC with a
                                scalar equation or a batch: DG_ERR_UNSUPPORTED; other
                                values: DG_ERR_ARG. */
} dg_options;

/* Filled by dg_run / dg_report_read. */
typedef struct {
    int64_t steps;           /* steps taken by the last dg_run                    */
    double t;                /* simulated time reached                            */
    double dt_min, dt_max;   /* extreme time steps of the last dg_run             */
    double ledger[4];        /* FP64 sum over cells of |K| * cell average         */
    double boundary_flux[4]; /* FP64 time integral of the net outward boundary flux */
    int64_t troubled_cells;  /* hybrid: troubled cells summed over all stages     */
    double min_rho, min_p;   /* Euler: minima seen at trace and quadrature points  */
    double max_exponent;     /* largest damping exponent applied                  */
    int status;              /* first error latched on the device (dg_status)     */
    int64_t first_bad_cell;  /* cell index of that error, -1 if none              */
    int64_t restarts;        /* steps retried with half dt (positivity limiter)   */
} dg_report;

typedef struct dg_solver dg_solver;

/* Create a solver for `mesh`, polynomial degree `degree` (0..3) and
 * `equation`: the DG space V_h^k of piecewise polynomials of degree k on a
 * uniform mesh of an interval (Sec. 2.1) or a rectangle (Sec. 2.3), with the
 * modal Legendre basis whose mode 0 is the cell average (Sec. 2.1,
 * (eq:GLbasisequation)); the conservation law is linear advection, Burgers
 * (Sec. 3.1) or the Euler equations (Sec. 2.4, Sec. 3).  Supported: 1D
 * advection/Burgers/Euler; 2D advection/Euler (Q^k, or P^k with
 * options.basis = 1).  The handle copies *mesh and *opt; it owns no device
 * memory (dg_bind).  Errors: DG_ERR_ARG (NULL, n < 1, bad domain, BC
 * pairing, option values), DG_ERR_UNSUPPORTED (degree, dim/equation,
 * quad_points); *out is NULL then. */
int dg_create(const dg_mesh* mesh, int degree, int equation, const dg_options* opt,
              dg_solver** out);
int dg_destroy(dg_solver* s);

/* Bytes of each of the three state buffers and of the workspace. */
int dg_buffer_sizes(const dg_solver* s, size_t* state_bytes, size_t* workspace_bytes);

/* Bind caller-owned device memory: u_n holds the solution; u_a and u_b are
 * RK stage buffers; workspace (workspace_bytes) holds the unfiltered stage
 * output, per-cell filter data and the device control block.  All must be
 * 256-byte aligned and stay valid until re-bound or destroyed.  Resets the
 * simulated time and the ledger. */
int dg_bind(dg_solver* s, void* u_n, void* u_a, void* u_b, void* workspace);

/* Copy an FP64-layout state from DEVICE memory into u_n (converting to the
 * mixed layout if needed), and back.  modes_dev is a device pointer (the
 * caller's torch tensor, for instance), not a host array: a host array would
 * cost an extra copy through the caller's stream, so the host -> device copy
 * is left to the caller.  Stream-ordered; no synchronisation.  For the 2D
 * P^k space the modes p + q > k are dropped on the way in and written as
 * zeros on the way out. */
int dg_set_state(dg_solver* s, const double* modes_dev);
int dg_get_state(dg_solver* s, double* modes_dev);

/* CFL reduction (Sec. 2.2, Theorem 2.1 time-step condition): the largest
 * characteristic speed |f'(u-bar)| (Euler |u|+c; 2D: max over cells of
 * ax/hx + ay/hy) over the cell averages of u_n, in FP64, written to
 * *alpha (host).  Synchronises the stream.  In 2D *alpha is
 * max(ax/hx + ay/hy), so dt = cfl / alpha. */
int dg_max_wavespeed(dg_solver* s, double* alpha);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the CFL
 * reduction of dg_max_wavespeed on the state buffer u_dev (device, the
 * solver's internal layout and size, dg_buffer_sizes' state_bytes; it need
 * not be bound, and the solver needs no workspace).  Allocates nothing: its
 * scratch (one partial maximum per 256 cells, and the result) is a fixed
 * device array of the library, 1.1 MB on each GPU it runs on, held until the
 * process ends.  Limit: at most 16,777,216 cells (65536 x 256); larger
 * meshes: DG_ERR_ARG.  The maximum is reduced in a fixed order (no
 * atomics), so it equals dg_max_wavespeed's bit for bit.  *first_bad
 * (nullable) receives the lowest index of a cell whose average is
 * inadmissible (Euler) or non-finite, else -1.  Every call on a GPU uses
 * that GPU's one array: calls that overlap on one GPU race.  Runs on the
 * solver's stream and synchronises it.  Errors: DG_ERR_ARG (NULL, size),
 * DG_ERR_DEVICE, DG_ERR_NONFINITE (alpha not finite). */
int dg_max_wavespeed_noalloc(const dg_solver* s, const void* u_dev, double* alpha,
                             int64_t* first_bad);

/* One SSP-RK3 stage of the plain DG scheme into the workspace's stage
 * buffer: the semi-discrete operator L of (scheme:DG) (Sec. 2.1; 2D
 * (eq:semiloc_rec) without the viscous term, Sec. 2.3) -- Gauss quadrature
 * of the volume term, the interface flux (LLF, or HLL / HLLC) at the
 * interfaces and edge Gauss points -- and the Shu-Osher combination of the
 * third-order SSP Runge-Kutta method (Sec. 2.2 (rkdg1); Sec. 3):
 *   stage 0: w = u_n + dt L(u_n)
 *   stage 1: w = 3/4 u_n + 1/4 (u_a + dt L(u_a))
 *   stage 2: w = 1/3 u_n + 2/3 (u_b + dt L(u_b))
 * Boundary states are taken at t = 0 (+dt, +dt/2 by stage).  Reads u_n and
 * u_a / u_b (device, bound); no filter.  Stream-ordered.  Errors:
 * DG_ERR_ARG (stage, dt < 0), DG_ERR_STATE (unbound), DG_ERR_DEVICE. */
int dg_stage(dg_solver* s, int stage, double dt);

/* Post-stage operator of the options applied to the workspace's stage
 * buffer, the result to u_a (stage 0), u_b (stage 1) or u_n (stage 2):
 *   DG_FILTER_JUMP: u^l <- exp(-sigma^l dt) u^l for every mode l >= 1,
 *     sigma from the jumps of the derivatives across the cell's interfaces
 *     (1D: (para:damp2)-(para:damp21), (timespli:1dscalar); 2D:
 *     (para:damp22d)-(para:damp22d1); systems: the maximum over the
 *     components, (para:dampsystems1d)-(timespli:sys));
 *   DG_FILTER_HYBRID: Algorithm 1 (Sec. 3): cells with jump indicator
 *     eta > 1 get omega u + (1 - omega) (filtered u), omega =
 *     (max eta - eta) / (max eta - 1); other cells are unchanged;
 *   DG_FILTER_NONE: a copy;
 * then, with options.positivity, the positivity limiter.  The damping time
 * is the full dt after every stage.  Exponents of every cell are kept for
 * dg_last_exponents.  Stream-ordered.  Errors as dg_stage. */
int dg_jump_filter(dg_solver* s, int stage, double dt);

/* Advance u_n until t_end or max_steps steps: SSP-RK3 steps (Sec. 2.2
 * (rkdg1)) with the post-stage operator after every stage (Sec. 3), dt
 * chosen on the device every step from the CFL reduction (Theorem 2.1's
 * condition dt <= gamma h; dt = cfl h / alpha, 2D cfl / max(ax/hx + ay/hy);
 * the last step clamped to t_end).  The steps are replayed from a captured
 * HIP graph (remainders and small 1D hybrid grids launched directly) on a
 * private stream ordered after the solver's stream.  Synchronises and fills
 * *rep (nullable): steps and t accumulate over calls, dt_min / dt_max are
 * this call's.  Returns rep->status: DG_OK, DG_ERR_NONFINITE (the run
 * stops), DG_ERR_POSITIVITY (reported; with the positivity limiter, a step
 * still rejected after 40 halvings of dt, which stops the run),
 * DG_ERR_STATE (unbound), DG_ERR_DEVICE. */
int dg_run(dg_solver* s, double t_end, int64_t max_steps, dg_report* rep);

/* Read the report of the device control block (synchronises). */
int dg_report_read(dg_solver* s, dg_report* rep);

/* Per-cell damping exponents of the last dg_jump_filter call, FP64,
 * E[cell*(Lmax+1) + l] with Lmax = k (1D) or 2k (2D); written to a device
 * buffer of ncells*(Lmax+1) doubles.  2D hybrid: the troubled cells' only
 * (zero elsewhere; Algorithm 1 damps no other cell). */
int dg_last_exponents(dg_solver* s, double* E_dev);

/* Measurement hook: launch a kernel of dg_run `reps` times back to back on
 * the solver's run stream with time step dt and return its average
 * duration in microseconds from HIP events recorded before the first and
 * after the last launch (after one untimed warm-up launch).  1D: `stage`
 * 0..2 selects the fused stage(+filter / hybrid pass A) kernel of that RK
 * stage (reads u_n, u_a, u_b; writes u_a or u_b), in the form dg_run
 * launches it.  Hybrid runs without the positivity limiter use the deferred
 * blend; on grids under 258048 cells their stage 2 also runs the step
 * control in its last workgroup (here on a control block of its own).
 * 2D: 0..2 the residual
 * kernel of that stage (writes the workspace), 3..5 the filter kernel
 * (jump: workspace -> u_a) or hybrid pass A, the indicator (which reads the
 * corner values the residual kernel of a hybrid solver writes, as in dg_run).  1D `stage` 6: the
 * kernel that runs a whole step (jump filter or none; u_n -> u_a);
 * DG_ERR_ARG with the hybrid limiter.  u_n is never
 * modified.  Synchronises. */
int dg_time_kernel(dg_solver* s, int stage, double dt, int reps, double* avg_us);

const char* dg_strerror(int code);

/* ---------------------------------------------------------------------- */
/* Batched 1D Euler: many independent problems of different size and       */
/* degree advanced by one persistent launch (each workgroup owns whole     */
/* problems and steps them with its own dt).                               */
/* ---------------------------------------------------------------------- */
typedef struct dg_batch dg_batch;

typedef struct {
    int64_t n;               /* cells                                             */
    int degree;              /* 0..3                                              */
    double lo, hi;           /* domain                                            */
    int bc[2];               /* DG_BC_OUTFLOW / DG_BC_PERIODIC / DG_BC_REFLECT    */
    int64_t offset;          /* filled by dg_batch_create: element offset of the  */
                             /* problem's FP64-layout state in the packed array  */
} dg_problem1d;

/* Create a batch of `nprob` 1D Euler problems (each one a separate domain
 * with its own degree, cells and boundary conditions; jump filter or no
 * post-stage operator).  Problems are packed back to back in FP64 layout
 * (problem i at element offset probs[i].offset, written by this call);
 * total element count in *total_elems.  Errors: DG_ERR_ARG (sizes, BCs),
 * DG_ERR_UNSUPPORTED (degree > 3, other equations, hybrid limiter). */
int dg_batch_create(int nprob, dg_problem1d* probs, int equation, const dg_options* opt,
                    int64_t* total_elems, dg_batch** out);
int dg_batch_destroy(dg_batch* b);
int dg_batch_buffer_sizes(const dg_batch* b, size_t* state_bytes, size_t* workspace_bytes);
int dg_batch_bind(dg_batch* b, void* u_n, void* u_a, void* u_b, void* workspace);
int dg_batch_set_state(dg_batch* b, const double* packed_dev);
int dg_batch_get_state(dg_batch* b, double* packed_dev);
/* Advance every problem by `steps` steps (or until its t_end[i], host
 * array, nullable), each with its own CFL time step, in one persistent
 * launch: the reset of the queue and error latches, the launch and the copy
 * of the reports to pinned host memory are captured once in a HIP graph
 * (rebuilt when the step count or the schedule changes) and replayed on a
 * private stream ordered after the caller's.  per_problem (host, nullable,
 * nprob entries) receives each problem's report.  Synchronises. */
int dg_batch_run(dg_batch* b, const double* t_end, int64_t steps, dg_report* per_problem);

/* Autotuner of the batched launch: times `trial_steps` steps of the whole
 * batch for each candidate schedule (threads per workgroup: 256 or 128,
 * i.e. tiles of 244 or 116 cells; persistent workgroups per compute unit:
 * 1, 2, 4, 8 of 256 threads or twice as many of 128; queue order:
 * longest-first or as given), each from the same saved state (u_n is
 * restored afterwards), keeps the fastest for later dg_batch_run calls, and
 * writes a JSON summary into json (nullable; truncated to cap bytes): the
 * batch's key ("k_mix": fractions of degrees 0..3, "n_bucket":
 * round(log2(mean cells))) under which a caller may cache the choice, every
 * candidate's time, and "best".  Results do not depend on the schedule
 * (each problem's step is computed cell by cell the same way).
 * Synchronises. */
int dg_batch_tune(dg_batch* b, int64_t trial_steps, char* json, size_t cap);

/* Apply a schedule chosen earlier (by dg_batch_tune, e.g. from a cache keyed
 * as its JSON): block_size 128 or 256, wg_per_cu 1..16 workgroups of that
 * size per compute unit, lpt 1 = longest-first queue, 0 = as given.
 * Errors: DG_ERR_ARG, DG_ERR_STATE (unbound). */
int dg_batch_set_schedule(dg_batch* b, int block_size, int wg_per_cu, int lpt);

#ifdef __cplusplus
}
#endif
#endif /* DG_H */
