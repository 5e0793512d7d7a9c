/*
 * fvna3d.h -- C ABI of the three-dimensional step (the paper's equations in
 * three dimensions, which Sec. 5 says they allow): state (rho', rho u1,
 * rho u2, rho u3), Godunov splitting x1 -> x2 -> x3 -> source, each sweep the
 * high-resolution Roe scheme of Secs. 3.1-3.2 with a second shear wave, the
 * source delta times the 7-point Laplacian of each velocity component, the CFL
 * rule of Sec. 4 (max |s| over the interfaces of all three sweeps).
 *
 * Fields are [nz][ny][nx] doubles on the host, x1 contiguous, SI units as in
 * fvna.h.  Side kinds per side x-, x+, y-, y+, z-, z+: FVNA_BC_PERIODIC,
 * FVNA_BC_EXTRAP0, FVNA_BC_REFLECT (fvna.h).  Errors are fvna_status values,
 * with fvna3_last_error() describing the last failing call.
 *
 * On the device a step is three kernels and a controller: the x1 and x2
 * sweeps of z-plane tiles fused (lanes along x1, a register march along x2,
 * every interface solved once), the x3 sweep (a register march along x3),
 * the source, then the accept/reject decision and the next time step on one
 * device thread.  Attempts are replayed from a captured HIP graph; the host
 * waits once per fvna3_step call.
 */
#ifndef FVNA3D_H
#define FVNA3D_H
#include <stddef.h>
#include <stdint.h>
#include "fvna.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t nx, ny, nz;        /* cells, each >= 4 */
    double dx;                 /* [m] */
    double c0, rho0, beta, delta;
    int32_t precision;         /* FVNA_F64 or FVNA_F32 (state stored and computed in it) */
    int32_t bc[6];
    double cfl_target, cfl_max;
    int32_t max_retries;
    int32_t fixed_dt;          /* 1: never change dt, never reject */
    double dt0;                /* [s]; <= 0: from the initial state */
} fvna3_params;

typedef struct fvna3_ctx fvna3_ctx;

/* Bytes of each of the three state buffers (four fields of nz * ny rows,
 * rows padded to 256 bytes) and of the scratch buffer (device clock and a
 * staging area of nx * ny * nz doubles). */
fvna_status fvna3_workspace_size(const fvna3_params* p, size_t* state_bytes, size_t* scratch_bytes);

/* Borrow three device state buffers, a scratch buffer (sizes above) and a HIP
 * stream (NULL: the null stream); they must outlive the context. */
fvna_status fvna3_create(const fvna3_params* p, void* buf_a, void* buf_b, void* buf_c, void* scratch,
                         void* stream, fvna3_ctx** out);

/* Copy a host state in (SI, [nz][ny][nx] each); resets t, the counters and,
 * unless dt0 > 0, computes the first step from the state.  Synchronous. */
fvna_status fvna3_set_state(fvna3_ctx* c, const double* rho_p, const double* m1, const double* m2,
                            const double* m3);

/* Take nsteps accepted steps and wait for them (rejected attempts are redone
 * on the device with dt * nu_W / nu, at most max_retries in a row).
 * FVNA_E_NONHYPERBOLIC, FVNA_E_NONFINITE or FVNA_E_RETRIES stop the run with
 * the state of the last accepted step; they stay latched (further steps do
 * nothing and return them) until fvna3_set_state. */
fvna_status fvna3_step(fvna3_ctx* c, int64_t nsteps);

fvna_status fvna3_get_state(fvna3_ctx* c, double* rho_p, double* m1, double* m2, double* m3);
fvna_status fvna3_get_stats(fvna3_ctx* c, fvna_stats* st);

/* Mean duration in ms of the three kernels of one attempt without the
 * controller (reps recomputations back to back of the attempt the next step
 * makes; the state and the clock are unchanged). */
fvna_status fvna3_time_step_kernels(fvna3_ctx* c, int32_t reps, double* ms);

/* Thread-local message of the last failing call of this library. */
const char* fvna3_last_error(void);

void fvna3_destroy(fvna3_ctx* c);

#ifdef __cplusplus
}
#endif
#endif
