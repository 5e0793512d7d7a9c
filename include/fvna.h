/*
 * fvna.h -- C ABI of libfvna, the gfx950 (MI355X) implementation of the
 * dimensionally split high-resolution finite-volume step for the nonlinear
 * thermoviscous acoustic balance laws of Velasco-Segura & Rendon,
 * "A Finite Volume Approach for the Simulation of Nonlinear Dissipative
 * Acoustic Wave Propagation" (arXiv:1311.3004).
 *
 * What one step computes (paper Sec. 3 and the opening of Sec. 4):
 *   - the balance laws of eq. OurSystem in the conservation form of eq.
 *     OurSysAdim / adim:q, split as eqs. fs:cl1, fs:cl2, fs:source;
 *   - each split direction: Roe linearisation (Sec. 3.2, eqs. RoeCond,
 *     lambda1-3), waves and fluctuations (eqs. fluc:m, fluc:p), the MC-limited
 *     high-resolution correction (eq. limiter) and the update of eq. fv-hr;
 *   - the source step with central differences (end of Sec. 3 intro), plus,
 *     in axisymmetric geometry, the cylindrical terms of eq. OurSystem;
 *   - the CFL number nu = (dt/dx) max|s^p| over the mesh, both directions and
 *     all p, and the time-step control that keeps nu near the wished nu_W.
 *
 * Conventions shared by every call:
 *   - All physical inputs and outputs are SI.  Inside, lengths are in cells
 *     (dx = 1) and time in dx/c0; the state is held as perturbations
 *     R = rho'/rho0, M = rho u/(rho0 c0), N = rho v/(rho0 c0).
 *   - Fields at the boundary of the library are host arrays of doubles,
 *     row-major [ny][nx] with x1 (i) contiguous; cell (i, j) is centred at
 *     ((i + 1/2) dx, (j + 1/2) dx).  In axisymmetric geometry x1 = z and
 *     x2 = r, and the side y- (j = -1/2) is the symmetry axis r = 0.
 *   - Device memory is owned by the caller (e.g. PyTorch tensors): the
 *     library records the pointers it is given and never frees them.  Sizes
 *     come from fvna_workspace_size().  The HIP stream is borrowed.
 *   - Every call returns an fvna_status; no C++ exception crosses the ABI.
 *     On failure fvna_last_error() returns a thread-local message.
 *   - Errors found on the device while stepping (non-real Roe speeds,
 *     non-finite speeds, too many rejected steps) are latched in a device
 *     status word and reported by the next synchronising call (fvna_sync,
 *     fvna_get_state, fvna_get_stats).  The state then holds the last
 *     accepted step and further fvna_step calls are no-ops until
 *     fvna_set_state or fvna_set_clock.
 *   - Calls on one context are not thread-safe; distinct contexts are
 *     independent.
 */
#ifndef FVNA_H
#define FVNA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    FVNA_OK = 0,
    FVNA_E_INVALID = 1,        /* bad argument; nothing changed */
    FVNA_E_NOMEM = 2,          /* host allocation failed */
    FVNA_E_HIP = 3,            /* a HIP runtime call failed (message has the HIP error) */
    FVNA_E_NONHYPERBOLIC = 4,  /* Roe discriminant <= 0 or NaN (eigenvalues not real, Sec. 3.2) */
    FVNA_E_NONFINITE = 5,      /* otherwise: a discriminant or the largest wave speed is +Inf or NaN */
    FVNA_E_RETRIES = 6,        /* more than max_retries rejected attempts in a row */
    FVNA_E_STATE = 7           /* call not valid in the current state */
} fvna_status;

typedef enum { FVNA_CARTESIAN = 0, FVNA_AXISYMMETRIC = 1 } fvna_geometry;

/* Arithmetic and storage precision of the step.  FP32 and the FP16/BF16
 * storage variants compute in FP32; the half-width variants store each field
 * as field/scale rounded to nearest-even (store_scale below): with v the field
 * in FP32 and inv = 1/scale rounded to FP32, FP16 rounds the exact product
 * v * inv once (a fused multiply-convert; a zero is stored as +0), BF16 rounds
 * v * inv to FP32 and then to BF16.  Loads return the stored value times scale
 * in FP32. */
typedef enum { FVNA_F64 = 0, FVNA_F32 = 1, FVNA_F32_F16STORE = 2, FVNA_F32_BF16STORE = 3 } fvna_precision;

/* Boundary kinds (ghost cells), per side: 0 = x-, 1 = x+, 2 = y-, 3 = y+.
 *   PERIODIC: wrap (both sides of an axis must be periodic together).
 *   EXTRAP0:  zero-order extrapolation, the paper's simple absorbing side (Sec. 4.2).
 *   REFLECT:  mirror with the momentum normal to the side negated (Sec. 4.2);
 *             the r = 0 axis of the axisymmetric geometry.
 *   TAYLOR:   the analytic Taylor shock-like profile of eq. OurTaylorS,
 *             set by fvna_set_taylor, evaluated at the ghost-cell centre at
 *             t_n.  On a y side the ghost rows that the x2 sweep reads hold
 *             the x1 sweep of that analytic data (the same first fractional
 *             step as the interior) rather than the data themselves.
 * Side data enter at t_n, the start of the step (all kinds).
 *   SOURCE:   the focused boundary source of eq. hifuBC on side x- only,
 *             set by fvna_set_source; zero-order extrapolation outside the
 *             aperture. */
typedef enum {
    FVNA_BC_PERIODIC = 0, FVNA_BC_EXTRAP0 = 1, FVNA_BC_REFLECT = 2,
    FVNA_BC_TAYLOR = 3, FVNA_BC_SOURCE = 4
} fvna_bc;

typedef struct {
    int32_t nx, ny;            /* cells along x1 and x2, each >= 4 */
    double dx;                 /* mesh spacing [m], > 0 (Sec. 4: dx1 = dx2) */
    double c0, rho0;           /* ambient sound speed [m/s] and density [kg/m^3], > 0 */
    double beta;               /* coefficient of nonlinearity 1 + B/2A, >= 1 */
    double delta;              /* sound diffusivity [m^2/s] (eq. def-delta), >= 0 */
    int32_t geometry;          /* fvna_geometry */
    int32_t precision;         /* fvna_precision */
    int32_t bc[4];             /* initial fvna_bc per side (x-, x+, y-, y+) */
    double cfl_target;         /* wished CFL number nu_W, in (0, cfl_max) */
    double cfl_max;            /* attempts with nu > cfl_max are rejected and redone */
    int32_t max_retries;       /* rejected attempts allowed in a row (>= 0) */
    double dt0;                /* first time step [s]; <= 0: nu_W dx / (c0 max|s|) of the
                                  initial state (a dry pass of the Roe speeds) */
    int32_t fixed_dt;          /* 1: never change dt and never reject (nu still recorded) */
    double store_scale[3];     /* FP16/BF16 storage: per-field scale of (R, M, N), in the
                                  dimensionless units above; 0 = 1.0 */
    int32_t tile_rows;         /* rows per wavefront segment; 0 = library default */
} fvna_params;

/* Focused boundary source of eq. hifuBC on side x-: for the ghost rows whose
 * centre r (distance from side y-) is <= aperture (all other rows of the side
 * are zero-order extrapolation),
 *   R = g, M = F g / sqrt(r^2 + F^2), N = -r g / sqrt(r^2 + F^2),
 *   g = (p_surface / (rho0 c0^2)) w sin(2 pi freq tau),  tau = t + r^2 / (2 F c0),
 * with the envelope w chosen by `envelope`:
 *   FVNA_ENV_RAMP:   w(t) = sin^2(pi freq t / (2 ramp_cycles)) for
 *                    0 < t < ramp_cycles/freq, 0 for t <= 0, 1 afterwards
 *                    (a continuous focused field; not in the paper);
 *   FVNA_ENV_PACKET: w = exp(-(freq tau / packet_cycles)^10), the packet of
 *                    eq. hifuBC:g (exponent read as +10: a flat-top packet of
 *                    half-width packet_cycles periods centred on tau = 0; the
 *                    paper uses 4 and starts the run at a negative time, see
 *                    fvna_set_clock). */
/* With second_stage = 1 the run has the two stages of Sec. 4.2: from the
 * first step whose start time t_n is >= stage2_time on, the whole side x- is
 * zero-order extrapolation (the source rows included). */
typedef enum { FVNA_ENV_RAMP = 0, FVNA_ENV_PACKET = 1 } fvna_envelope;
typedef struct {
    double freq;               /* [Hz] > 0 */
    double p_surface;          /* [Pa] */
    double focal_length;       /* F [m] > 0 */
    double aperture;           /* [m] >= 0 */
    double ramp_cycles;        /* > 0 (FVNA_ENV_RAMP) */
    int32_t envelope;          /* fvna_envelope */
    double packet_cycles;      /* > 0 (FVNA_ENV_PACKET) */
    int32_t second_stage;      /* 0: the source stays on; 1: switch at stage2_time */
    double stage2_time;        /* [s], finite (second_stage = 1) */
} fvna_source;

typedef struct {
    double t;                  /* time of the current state [s] */
    double dt_next;            /* step the next attempt will use [s] */
    double nu_last;            /* CFL number of the last attempt */
    double nu_mean, nu_std;    /* over accepted steps since the last set_state/set_clock */
    int64_t steps;             /* accepted steps since the last set_state/set_clock */
    int64_t rejected;          /* rejected attempts since then */
    int32_t status;            /* latched fvna_status of the device (FVNA_OK if none) */
    int64_t status_step;       /* accepted steps when the error was latched */
} fvna_stats;

typedef struct fvna_ctx fvna_ctx;
typedef struct fvna_batch fvna_batch;

/* Bytes of ONE state buffer (two are needed, A and B) and of the scratch
 * buffer for these parameters.  Validates the parameters. */
fvna_status fvna_workspace_size(const fvna_params* p, size_t* state_bytes, size_t* scratch_bytes);

/* Create a simulation on the current HIP device.  state_a, state_b, scratch:
 * caller-owned device buffers of the sizes above (alignment >= 256 bytes).
 * hip_stream: a hipStream_t (NULL = default stream).  The state starts at
 * rest (all zero), t = 0. */
fvna_status fvna_create(const fvna_params* p, void* state_a, void* state_b, void* scratch,
                        void* hip_stream, fvna_ctx** out);

/* Change the boundary kind of one side (0 x-, 1 x+, 2 y-, 3 y+).  Periodic
 * must be set on both sides of an axis; SOURCE only on side 0; the
 * axisymmetric geometry needs REFLECT on side 2.  Waits for the context's
 * stream first when steps were enqueued (the captured step graph is rebuilt). */
fvna_status fvna_set_bc(fvna_ctx* c, int32_t side, int32_t bc);

/* Parameters of the focused source (side must be 0).  Fills the per-row
 * table of the source (focusing delay and direction cosines, in the scratch
 * buffer) with a synchronous copy: waits for the context's stream first.
 * Until it is called, a SOURCE side holds zero ghost cells. */
fvna_status fvna_set_source(fvna_ctx* c, int32_t side, const fvna_source* s);

/* Parameters of the Taylor profile used by TAYLOR sides (eq. OurTaylorS with
 * the rotation of Sec. 4.1): p' = -A tanh((xi - c0 t)/w), xi = (x - x0) cos(angle)
 * + y sin(angle), rho u = (p'/c0) (cos, sin), w = delta rho0 c0 / (beta A).
 * Waits for the context's stream first when steps were enqueued. */
fvna_status fvna_set_taylor(fvna_ctx* c, double amplitude_pa, double x0_m, double angle);

/* Copy a host state in: rho' [kg/m^3], rho u, rho v [kg m^-2 s^-1], each [ny][nx]
 * doubles.  Resets t to 0, the step counters and the latched status, and
 * recomputes the first time step (dt0 rule above).  Synchronises the stream. */
fvna_status fvna_set_state(fvna_ctx* c, const double* rho_p, const double* mom_x, const double* mom_y);

/* Set the time of the current state and the next time step (resume).  dt_next <= 0
 * recomputes it from the state.  Clears the latched status and counters. */
fvna_status fvna_set_clock(fvna_ctx* c, double t, double dt_next);

/* Enqueue nsteps accepted steps on the stream (asynchronous).  Rejected attempts
 * are redone on the device; fvna_sync finishes any that remain. */
fvna_status fvna_step(fvna_ctx* c, int64_t nsteps);

/* Wait for the stream, complete steps still owed after rejections, and return
 * the latched device status. */
fvna_status fvna_sync(fvna_ctx* c);

/* Move the domain ncols cells along +x1 (the moving domain of Sec. 4):
 * afterwards column i holds what column i + ncols held, and the ncols columns
 * that enter on the right hold undisturbed medium (zero perturbation) or, when
 * side x+ is TAYLOR, the Taylor profile at their path columns at the current
 * time (the medium ahead of the front).  The kept values are copied as they
 * are (exact in every precision).  Time, time step and statistics are
 * unchanged.  The focused source stays at the domain's left edge; Taylor data
 * (side and ghost values) stay anchored on the path: column i of a domain that
 * has moved x_off cells lies at path column x_off + i, where the profile of
 * fvna_set_taylor is evaluated.  The x axis must not be periodic.
 * 0 <= ncols <= nx; 0 does nothing.  Asynchronous on the stream;
 * FVNA_E_INVALID for a bad argument. */
fvna_status fvna_shift(fvna_ctx* c, int32_t ncols);

/* The two stages of Sec. 4 on a moving domain: the domain stays still until
 * the wave reaches its middle at t1; from then on it follows the wave.  The
 * paper gives no rule for the moves; here the state is checked after every
 * check_every-th accepted step (counted across calls by `phase`), and once
 * t >= t1 the origin moves to quantum * floor((t - t1) speed c0 / (dx quantum))
 * cells from the start (fvna_shift
 * by the difference; a move of nx cells or more leaves undisturbed medium in
 * the whole domain, and the path offset the recorder uses still advances by
 * the whole move).  The source's second stage (fvna_source .stage2_time,
 * normally t1) is set separately. */
typedef struct {
    double t1;                 /* [s], finite */
    int32_t check_every;       /* >= 1 */
    int32_t quantum;           /* cells, >= 1 */
    double speed;              /* domain speed along x1 in units of c0 (e.g. 1/cos(theta) for
                                  an oblique front's trace); 0 = 1 */
} fvna_window;
typedef struct {
    int64_t x_off;             /* cells the domain has moved (start at 0) */
    int64_t phase;             /* accepted steps since the last check, in [0, check_every) */
} fvna_window_state;

/* Advance nsteps accepted steps with the moving-domain rule above, updating
 * *st.  Synchronises the stream at every check (once per check_every steps)
 * and returns the first device status that is not FVNA_OK (the steps of the
 * failing chunk are not all taken).  FVNA_E_INVALID for bad arguments or x
 * sides that cannot move (as fvna_shift). */
fvna_status fvna_step_window(fvna_ctx* c, const fvna_window* w, fvna_window_state* st, int64_t nsteps);

/* Recorder of the on-axis quantities of Sec. 4.2 (pressure maxima over the
 * propagation axis, the time series at a probe) without a host round trip per
 * step.  While set, every attempt of fvna_step, fvna_sync and
 * fvna_step_window is followed by a small kernel that, once at least one step
 * has been accepted since fvna_set_recorder,
 *   row_max[x_off + i] = max(row_max[x_off + i], rho'(i, row))  for x_off + i < path_len,
 * with x_off the cells the domain has moved (fvna_shift) since the state was
 * set, and writes t and rho'(probe, row) of the latest accepted step k
 * (counted from 1 at fvna_set_recorder) to probe_t[k - 1], probe_rho[k - 1]
 * for k <= capacity while the probe column is inside the domain.  rho' in
 * kg/m^3 (p' = c0^2 rho'), t in s.  Rejected attempts leave everything as it
 * was (the kernel is idempotent).  The arrays are caller-owned device memory
 * and must outlive the recording; the caller initialises row_max (e.g. to
 * -inf) and the probe arrays.  fvna_set_recorder synchronises the stream;
 * NULL stops recording.  fvna_set_state and fvna_set_clock restart the step
 * count, and with it the probe index: the next accepted step is k = 1 again.  FVNA_E_INVALID for a row outside the grid, missing
 * arrays, path_len < 1 or probe_col < -1 (-1: no probe). */
typedef struct {
    int32_t row;
    int32_t probe_col;         /* path column, or -1 */
    int64_t path_len;
    double* row_max;           /* device, path_len doubles */
    double* probe_t;           /* device, capacity doubles (or NULL, capacity 0) */
    double* probe_rho;         /* device, capacity doubles */
    int64_t capacity;
} fvna_recorder;
fvna_status fvna_set_recorder(fvna_ctx* c, const fvna_recorder* r);

/* Synchronise and copy the current state out (same units and layout as set_state). */
fvna_status fvna_get_state(fvna_ctx* c, double* rho_p, double* mom_x, double* mom_y);

/* Synchronise and copy the window [i0, i0 + ni) x [j0, j0 + nj) of the current
 * state out, in the units of fvna_get_state, as arrays [nj][ni].  For probes
 * (e.g. a row of cells sampled every step) and sub-region comparisons without
 * exporting the whole grid.  The window must lie inside the grid. */
fvna_status fvna_get_window(fvna_ctx* c, int32_t i0, int32_t j0, int32_t ni, int32_t nj,
                            double* rho_p, double* mom_x, double* mom_y);

/* Synchronise and return the clock and CFL statistics. */
fvna_status fvna_get_stats(fvna_ctx* c, fvna_stats* s);

/* Synchronise and return FP64 sums over the grid of rho', rho u, rho v (SI),
 * computed on the device in a fixed order (identical on every run). */
fvna_status fvna_sums(fvna_ctx* c, double out[3]);

/* The errors E1 and Einf of eq. (error) (Sec. 4.1) of the current state
 * against the Taylor profile of fvna_set_taylor, computed on the device in
 * FP64: over the cells of the straight line along the propagation direction
 * (cos angle, sin angle) of length 2 half_length_m centred on the analytic
 * front at the current time t, whose point at t = 0 is (front0_x_m,
 * front0_y_m) (so the front is at that point + c0 t (cos, sin)),
 *   E1 = sum |R - R_ref| / sum |R_ref|,  Einf = max |R - R_ref| / max |R_ref|,
 * with R = rho'/rho0 and R_ref = -a tanh((xi - c0 t)/w) at the cell centres.
 * The line takes one cell per column when |cos| >= |sin| (columns i with
 * (i + 1/2) dx within half_length_m cos of the front, the cell of row
 * floor(y(i)/dx) the line crosses there), else one cell per row; cells
 * outside the domain are skipped.  Coordinates are path coordinates: on a
 * moving domain column i lies at path column x_off + i.  The sums run in a
 * fixed order (the same result on every run).  Synchronises the stream (steps
 * owed are taken first).  out[0] = E1, out[1] = Einf.  FVNA_E_INVALID without
 * Taylor data, for a non-positive half length or when no cell of the line is
 * in the domain. */
fvna_status fvna_taylor_errors(fvna_ctx* c, double front0_x_m, double front0_y_m, double half_length_m,
                               double out[2]);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the sums of
 * fvna_sums for one state buffer, with no context, no allocation and no
 * synchronisation.  p describes the buffer (grid, precision, store_scale,
 * rho0, c0; validated as by fvna_workspace_size); state is a device buffer
 * laid out as the library stores a state (fvna_workspace_size's state_bytes:
 * three planes R, M, N); out is device memory for 3 doubles, which receives
 * the sums of rho', rho u, rho v in SI, bitwise equal to what fvna_sums
 * returns for a context whose current state is that buffer.  Enqueued on
 * hip_stream (NULL = default stream); the result is valid once the stream
 * has reached it.  The partial sums live in a static device array of the
 * library, 512 x 3 doubles (12 KiB) per device, whatever the grid size (so
 * no grid fvna_workspace_size accepts is too large); it is found at the
 * first call on each device and kept until the process ends.  Every call on
 * one device uses the same array: calls that overlap on one device (two
 * streams, two threads) race and give wrong sums.  FVNA_E_INVALID for NULL
 * or misaligned (not 8-byte) pointers or invalid parameters. */
fvna_status fvna_sums_noalloc(const fvna_params* p, const void* state, void* hip_stream, double* out);

/* Time `reps` back-to-back launches of the fused step kernel alone on the
 * context's stream with HIP events; *ms_per_launch receives the mean.  The
 * launches recompute the attempt that the next fvna_step would make, so the
 * simulation state and its results are unchanged. */
fvna_status fvna_time_step_kernel(fvna_ctx* c, int32_t reps, double* ms_per_launch);

/* Pick tile_rows for this context by timing each candidate with
 * fvna_time_step_kernel; writes the chosen value to *tile_rows.  Results are
 * bitwise independent of the choice. */
fvna_status fvna_autotune(fvna_ctx* c, int32_t* tile_rows);

/* Rows per segment currently used by the step kernel. */
fvna_status fvna_get_tile_rows(fvna_ctx* c, int32_t* tile_rows);

/* Thread-local message of the last failing call (never NULL). */
const char* fvna_last_error(void);

/* Free the context (not the caller's buffers).  Synchronises the stream. */
void fvna_destroy(fvna_ctx* c);

/* ---- Batched form: many independent simulations, one launch per step ----
 * n simulations, each with its own parameters, state buffers and clock.
 * bufs holds 3 n device pointers: state_a, state_b, scratch of simulation k
 * at 3k, 3k+1, 3k+2, sized by fvna_workspace_size of per_sim[k].  All must use
 * the same precision and geometry.  Each step of fvna_batch_step is one
 * launch of the batched kernel over the tiles of every simulation followed by
 * one launch of the per-simulation controller; nsteps steps are replayed from
 * a captured HIP graph.  Results are bitwise those of n separate contexts. */
fvna_status fvna_batch_create(int32_t n, const fvna_params* per_sim, void* const* bufs,
                              void* hip_stream, fvna_batch** out);
fvna_status fvna_batch_set_state(fvna_batch* b, int32_t k, const double* rho_p,
                                 const double* mom_x, const double* mom_y);
fvna_status fvna_batch_step(fvna_batch* b, int64_t nsteps);
fvna_status fvna_batch_sync(fvna_batch* b);
fvna_status fvna_batch_get_state(fvna_batch* b, int32_t k, double* rho_p, double* mom_x,
                                 double* mom_y);
fvna_status fvna_batch_get_stats(fvna_batch* b, int32_t k, fvna_stats* s);
fvna_status fvna_batch_time_step_kernel(fvna_batch* b, int32_t reps, double* ms_per_launch);
/* Choose the segment height of the members by timing the batched step kernel
 * on the batch itself: members are grouped in size classes by ny (powers of
 * two); for each class in turn the heights 32, 48, 64, 96, 128, 192, 256 are
 * timed with the other classes fixed and the fastest kept.  Members created
 * with their own tile_rows keep it.  The choice is kept in-process for the
 * batch's composition (precision, geometry and every member's nx, ny in
 * order) and taken by later fvna_batch_create calls with the same
 * composition.  Results are bitwise independent of the heights.  Waits for
 * the stream; the timing launches recompute the attempt the next step makes,
 * so the simulations are unchanged.  tile_rows (may be NULL) receives n
 * heights. */
fvna_status fvna_batch_autotune(fvna_batch* b, int32_t* tile_rows);
/* The n members' segment heights. */
fvna_status fvna_batch_get_tile_rows(fvna_batch* b, int32_t* tile_rows);
void fvna_batch_destroy(fvna_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* FVNA_H */
