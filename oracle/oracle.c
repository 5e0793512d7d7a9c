/*
 * oracle.c -- plain, slow FP64 CPU reference for one time step of the
 * dimensionally split high-resolution finite-volume method for the
 * nonlinear thermoviscous acoustic balance laws of Velasco-Segura & Rendon,
 * "A Finite Volume Approach for the Simulation of Nonlinear Dissipative
 * Acoustic Wave Propagation" (arXiv:1311.3004).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the parity oracle: it is called by
 * the test-suite, by the smoke check and by the CPU-baseline leg of the
 * benchmark, never by the product library.  It shares no code, header, table
 * or helper with the HIP path.  Compile with -ffp-contract=off (no FMA
 * contraction) so that every operation below rounds exactly as written.
 * Serial by default; with -fopenmp and orc_set_threads(n) the rows of a sweep
 * (columns of the x2 sweep) and of the source are shared among n threads,
 * each row computed exactly as in the serial run, so the result is bitwise
 * independent of n.
 *
 * Units.  Lengths are measured in cells (the reference length L of the
 * paper's renormalisation, Sec. 3 eq. renorm, is taken as the mesh spacing,
 * so Delta x = 1) and time in units of Delta x / c0.  The state is stored in
 * perturbation form: R = q^1 - 1 = rho'/rho0, M = q^2, N = q^3 (eq. adim:q).
 * Carrying R instead of q^1 is an exact change of variable that keeps the
 * relative precision of small perturbations; every formula of the paper that
 * uses q^1 is written with q^1 = 1 + R.
 *
 * Step (Sec. 3, eqs. fs:cl1, fs:cl2, fs:source, applied one after another):
 *   ghosts(x) of Q^n -> x1 sweep -> ghosts(y) of Q* -> x2 sweep (components
 *   2 and 3 swapped) -> one ghost layer of Q** -> source -> Q^{n+1};
 *   then the CFL number of the step decides acceptance (Sec. 4 opening).
 *   In axisymmetric geometry the geometric terms enter as two half steps
 *   around the x2 sweep (geometric_half_step).
 *
 * Readings of points the paper leaves open are stated where they are used.
 * The pins that fix each function live in the test-suite; every side rule of
 * set_ghost is checked cell by cell through orc_ghost (the focused source's
 * momentum against the direction to the focus), and the reject-and-redo rule
 * of orc_run against single attempts at the two time steps involved.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { ORC_OK = 0, ORC_E_INVALID = 1, ORC_E_NOMEM = 2, ORC_E_NONHYPERBOLIC = 4,
       ORC_E_NONFINITE = 5, ORC_E_RETRIES = 6 };
enum { BC_PERIODIC = 0, BC_EXTRAP0 = 1, BC_REFLECT = 2, BC_TAYLOR = 3, BC_SOURCE = 4 };
enum { GEOM_PLANAR = 0, GEOM_AXISYM = 1 };

/* All quantities dimensionless (cells, Delta x / c0). */
typedef struct {
    int nx, ny;
    double beta;            /* coefficient of nonlinearity, beta = 1 + B/2A          */
    double delta;           /* delta~ = delta / (c0 Delta x)   (eq. phi-tdelta)       */
    int geometry;           /* GEOM_PLANAR or GEOM_AXISYM (x1 = z, x2 = r)            */
    int bc[4];              /* sides x-, x+, y-, y+                                   */
    double cfl_target;      /* nu_W                                                   */
    double cfl_max;         /* a step with nu > cfl_max is rejected and redone        */
    int max_retries;
    int fixed_dt;           /* 1: never change dt (parity runs); nu still recorded    */
    /* analytic Taylor shock-like profile used by BC_TAYLOR (eq. OurTaylorS) */
    double taylor_amp, taylor_width, taylor_x0, taylor_y0, taylor_angle;
    /* focused boundary source used by BC_SOURCE on side x- (eq. hifuBC)      */
    double src_amp, src_freq, src_focal, src_aperture, src_ramp_cycles;
    int src_envelope;         /* 0: sin^2 ramp over src_ramp_cycles periods from t = 0;
                                 1: the packet of eq. hifuBC:g, width src_packet_cycles */
    double src_packet_cycles;
    int src_stage2_on;        /* 1: from t >= src_stage2 on, the whole side x- is zero-order
                                 extrapolation (second stage of Sec. 4.2); 0: never */
    double src_stage2;
} orc_params;

typedef struct {
    double t, dt_next, nu_last, nu_mean, nu_std;
    long steps, rejected;
    int status;
    long status_step;
} orc_stats;

/* ------------------------------------------------------------------------- */
/* Flux and pressure-like function (eq. adim:q).  Exported for the pins.     */
/* ------------------------------------------------------------------------- */

/* phi(q^1) = q^1 + (beta-1)(q^1-1)^2, returned minus its ambient value 1 so
 * that flux differences keep the precision of the perturbations. */
static double phi_excess(double beta, double R) { return R + (beta - 1.0) * R * R; }

/* x1-flux f_1(q) = (q^2, (q^2)^2/(q^1)^2 + phi, q^2 q^3/(q^1)^2), with the
 * constant ambient part of phi removed (it cancels in every difference). */
void orc_flux(double beta, const double q[3], double f[3])
{
    double q1 = 1.0 + q[0];
    f[0] = q[1];
    f[1] = q[1] * q[1] / (q1 * q1) + phi_excess(beta, q[0]);
    f[2] = q[1] * q[2] / (q1 * q1);
}

/* ------------------------------------------------------------------------- */
/* Roe linearisation (Sec. 3.2).                                             */
/* ------------------------------------------------------------------------- */

/* Solve the 3x3 system A x = b by Gaussian elimination with partial pivoting.
 * Returns 0 if the matrix is singular. */
static int solve3(double A[3][3], double b[3], double x[3])
{
    double a[3][4];
    for (int i = 0; i < 3; i++) {
        for (int j = 0; j < 3; j++) a[i][j] = A[i][j];
        a[i][3] = b[i];
    }
    for (int c = 0; c < 3; c++) {
        int piv = c;
        for (int r = c + 1; r < 3; r++)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return 0;
        if (piv != c)
            for (int j = 0; j < 4; j++) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
        for (int r = c + 1; r < 3; r++) {
            double f = a[r][c] / a[c][c];
            for (int j = c; j < 4; j++) a[r][j] = a[r][j] - f * a[c][j];
        }
    }
    for (int r = 2; r >= 0; r--) {
        double s = a[r][3];
        for (int j = r + 1; j < 3; j++) s = s - a[r][j] * x[j];
        x[r] = s / a[r][r];
    }
    return 1;
}

/* Roe decomposition at one interface, for the x1 direction.
 * qL, qR: (R, M_normal, M_tangential) of the left and right cells.
 * Outputs: speeds s[p], eigenvectors r[p][c], strengths alpha[p], waves
 * W[p][c] = alpha[p] r[p][c], fluctuations amdq = sum_p min(s,0) W, apdq =
 * sum_p max(s,0) W (eqs. fluc:m, fluc:p).  Returns 1 if the eigenvalues are
 * real and distinct (discriminant > 0), 0 otherwise (outputs then undefined).
 *
 * Z-bar is the arithmetic mean of z = (q^1, q^2/q^1, q^3/q^1) of the two
 * cells; Phi = 1 + 2(beta-1)(Zbar^1 - 1); eigenvalues per eqs. lambda1-3.
 * Eigenvectors: the paper only says they follow directly; the form used here
 * is the kernel of (A-hat - s I): r = (1, s, Zbar^3 (s - 2 Zbar^2)/(Zbar^1 (s - Zbar^2/Zbar^1)))
 * for the two acoustic speeds, and (0, 0, 1) for s^3.  The strengths alpha
 * come from solving sum_p alpha^p r^p = Q_R - Q_L as a linear system. */
int orc_roe(double beta, const double qL[3], const double qR[3],
            double s[3], double r[3][3], double alpha[3], double W[3][3],
            double amdq[3], double apdq[3])
{
    double q1L = 1.0 + qL[0], q1R = 1.0 + qR[0];
    double z2L = qL[1] / q1L, z3L = qL[2] / q1L;
    double z2R = qR[1] / q1R, z3R = qR[2] / q1R;
    double Zb1m1 = 0.5 * (qL[0] + qR[0]);          /* Zbar^1 - 1 */
    double Zb1 = 1.0 + Zb1m1;
    double Zb2 = 0.5 * (z2L + z2R);
    double Zb3 = 0.5 * (z3L + z3R);
    double Phi = 1.0 + 2.0 * (beta - 1.0) * Zb1m1;
    double w = Zb2 / Zb1;
    double disc = (Zb2 * Zb2) / (Zb1 * Zb1) - 2.0 * (Zb2 * Zb2) / Zb1 + Phi;
    if (!(disc > 0.0)) return 0;
    double root = sqrt(disc);
    s[0] = w + root;
    s[1] = w - root;
    s[2] = w;
    for (int p = 0; p < 2; p++) {
        r[p][0] = 1.0;
        r[p][1] = s[p];
        r[p][2] = Zb3 * (s[p] - 2.0 * Zb2) / (Zb1 * (s[p] - w));
    }
    r[2][0] = 0.0; r[2][1] = 0.0; r[2][2] = 1.0;
    double Rm[3][3], dq[3];
    for (int c = 0; c < 3; c++) {
        for (int p = 0; p < 3; p++) Rm[c][p] = r[p][c];
        dq[c] = qR[c] - qL[c];
    }
    if (!solve3(Rm, dq, alpha)) return 0;
    for (int c = 0; c < 3; c++) { amdq[c] = 0.0; apdq[c] = 0.0; }
    for (int p = 0; p < 3; p++) {
        double sm = s[p] < 0.0 ? s[p] : 0.0;
        double sp = s[p] > 0.0 ? s[p] : 0.0;
        for (int c = 0; c < 3; c++) {
            W[p][c] = alpha[p] * r[p][c];
            amdq[c] = amdq[c] + sm * W[p][c];
            apdq[c] = apdq[c] + sp * W[p][c];
        }
    }
    return 1;
}

/* Monotonized central-difference limiter (Sec. 3.1, below eq. limiter). */
double orc_mc(double theta)
{
    double a = (1.0 + theta) / 2.0;
    double b = 2.0;
    double c = 2.0 * theta;
    double m = a < b ? a : b;
    m = m < c ? m : c;
    return m > 0.0 ? m : 0.0;
}

/* ------------------------------------------------------------------------- */
/* One-dimensional high-resolution sweep (Sec. 3.1, eq. fv-hr).              */
/* ------------------------------------------------------------------------- */

/* Per-interface data of one line. */
typedef struct { double s[3], W[3][3], amdq[3], apdq[3]; int ok; } iface_t;

/* Update n interior cells of one line.  Input arrays hold n + 4 values: two
 * ghost cells, the n interior cells, two ghost cells (index k = i + 2 for
 * cell i).  qn is the normal momentum, qt the tangential one.  Writes the
 * n updated interior values to the out arrays.  *smax is raised to the
 * largest |s^p| over the interfaces i - 1/2, i = 0..n (those adjacent to an
 * interior cell); *bad is set if one of them has non-real speeds. */
static int sweep_line(double beta, double dtdx, int n,
                      const double *qr, const double *qn, const double *qt,
                      double *outr, double *outn, double *outt,
                      iface_t *f, double *smax, int *bad)
{
    /* interface i - 1/2 for i = -1..n+1 stored at f[i + 1] */
    for (int i = -1; i <= n + 1; i++) {
        int kl = i + 1, kr = i + 2;     /* cells i-1 and i */
        double qL[3] = { qr[kl], qn[kl], qt[kl] };
        double qR[3] = { qr[kr], qn[kr], qt[kr] };
        double r[3][3], alpha[3];
        iface_t *F = &f[i + 1];
        F->ok = orc_roe(beta, qL, qR, F->s, r, alpha, F->W, F->amdq, F->apdq);
        if (!F->ok) {
            for (int p = 0; p < 3; p++) {
                F->s[p] = NAN;
                for (int c = 0; c < 3; c++) F->W[p][c] = NAN;
            }
            for (int c = 0; c < 3; c++) { F->amdq[c] = NAN; F->apdq[c] = NAN; }
        }
        if (i >= 0 && i <= n) {
            if (!F->ok) *bad = 1;
            for (int p = 0; p < 3; p++) {
                double a = fabs(F->s[p]);
                if (isnan(a) || a > *smax) *smax = a;
            }
        }
    }
    /* high-resolution correction F~_{i-1/2} for i = 0..n (eq. limiter) */
    double (*Ft)[3] = malloc(sizeof(double[3]) * (size_t)(n + 1));
    if (!Ft) return ORC_E_NOMEM;
    for (int i = 0; i <= n; i++) {
        const iface_t *F = &f[i + 1];
        for (int c = 0; c < 3; c++) Ft[i][c] = 0.0;
        for (int p = 0; p < 3; p++) {
            /* upwind interface I - 1/2: I = i - 1 if s > 0, i + 1 if s < 0.
             * When s = 0 the term is multiplied by |s| = 0; i - 1 is used. */
            const iface_t *U = (F->s[p] < 0.0) ? &f[i + 2] : &f[i];
            double num = 0.0, den = 0.0;
            for (int c = 0; c < 3; c++) {
                num = num + U->W[p][c] * F->W[p][c];
                den = den + F->W[p][c] * F->W[p][c];
            }
            double theta = (den == 0.0) ? 0.0 : num / den;
            double phi = orc_mc(theta);
            double as = fabs(F->s[p]);
            double coef = 0.5 * as * (1.0 - dtdx * as);
            for (int c = 0; c < 3; c++)
                Ft[i][c] = Ft[i][c] + coef * (phi * F->W[p][c]);
        }
    }
    /* cell update (eq. fv-hr), interface i-1/2 -> Ft[i], f[i+1] */
    for (int i = 0; i < n; i++) {
        const iface_t *Fl = &f[i + 1], *Fr = &f[i + 2];
        double q[3] = { qr[i + 2], qn[i + 2], qt[i + 2] };
        double o[3];
        for (int c = 0; c < 3; c++)
            o[c] = q[c] - dtdx * (Fr->amdq[c] + Fl->apdq[c]) - dtdx * (Ft[i + 1][c] - Ft[i][c]);
        outr[i] = o[0]; outn[i] = o[1]; outt[i] = o[2];
    }
    free(Ft);
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Grid with ghost frame and boundary conditions.                            */
/* ------------------------------------------------------------------------- */

#define GH 2
typedef struct { int nx, ny, pitch; double *R, *M, *N; } field_t;

static size_t idx(const field_t *g, int i, int j) { return (size_t)(j + GH) * (size_t)g->pitch + (size_t)(i + GH); }

static int field_alloc(field_t *g, int nx, int ny)
{
    g->nx = nx; g->ny = ny; g->pitch = nx + 2 * GH;
    size_t n = (size_t)g->pitch * (size_t)(ny + 2 * GH);
    g->R = calloc(n, sizeof(double));
    g->M = calloc(n, sizeof(double));
    g->N = calloc(n, sizeof(double));
    return (g->R && g->M && g->N) ? ORC_OK : ORC_E_NOMEM;
}

static void field_free(field_t *g) { free(g->R); free(g->M); free(g->N); }

/* Taylor shock-like profile (eq. OurTaylorS, rotated by the angle theta_T as
 * described in Sec. 4.1): R = -A tanh((xi - t)/w), momentum = R (cos, sin),
 * with xi the distance along the propagation direction. */
static void taylor_value(const orc_params *p, double x, double y, double t, double q[3])
{
    double ca = cos(p->taylor_angle), sa = sin(p->taylor_angle);
    double xi = (x - p->taylor_x0) * ca + (y - p->taylor_y0) * sa;
    double R = -p->taylor_amp * tanh((xi - t) / p->taylor_width);
    q[0] = R; q[1] = R * ca; q[2] = R * sa;
}

/* Focused boundary source (eq. hifuBC) at distance r from the symmetry line:
 * g = A sin(2 pi f tau) env, tau = t + r^2/(2F).  Envelope 1 is the paper's
 * packet of eq. hifuBC:g, read as exp(-(f tau / W)^10) with W periods (the
 * printed exponent -10 would make a hole around tau = 0 instead of a packet
 * centred there); envelope 0 replaces it by a sin^2 ramp in t over
 * src_ramp_cycles periods, for a continuous focused field. */
static double source_g(const orc_params *p, double r, double t)
{
    double f = p->src_freq;
    double tau = t + r * r / (2.0 * p->src_focal);
    double env;
    if (p->src_envelope == 1) {
        double x = f * tau / p->src_packet_cycles;
        env = exp(-pow(x, 10.0));
    } else {
        double tr = p->src_ramp_cycles / f;
        if (t <= 0.0) env = 0.0;
        else if (t < tr) { double s = sin(M_PI * f * t / (2.0 * p->src_ramp_cycles)); env = s * s; }
        else env = 1.0;
    }
    return p->src_amp * env * sin(2.0 * M_PI * f * tau);
}

/* Ghost cell (gi, gj) on the given side, layer g (1 = adjacent), at time t.
 * side 0: x-, 1: x+, 2: y-, 3: y+.  Source cell rules (Sec. 4.2 and the
 * periodic extension): periodic wrap; zero-order extrapolation copies the
 * nearest interior cell; reflection mirrors the interior and negates the
 * momentum normal to the side; Taylor and source are analytic. */
static void set_ghost(const orc_params *p, double t, field_t *g, int side, int gi, int gj, int layer)
{
    int nx = g->nx, ny = g->ny;
    int bc = p->bc[side];
    size_t d = idx(g, gi, gj);
    double x = gi + 0.5, y = gj + 0.5;
    if (bc == BC_TAYLOR) {
        double q[3];
        taylor_value(p, x, y, t, q);
        g->R[d] = q[0]; g->M[d] = q[1]; g->N[d] = q[2];
        return;
    }
    if (bc == BC_SOURCE) {   /* valid on side x- only (checked at entry) */
        double r = y;
        int first_stage = !(p->src_stage2_on && t >= p->src_stage2);
        if (first_stage && r <= p->src_aperture) {
            double gg = source_g(p, r, t);
            double h = sqrt(r * r + p->src_focal * p->src_focal);
            g->R[d] = gg;
            g->M[d] = p->src_focal * gg / h;
            g->N[d] = -r * gg / h;
            return;
        }
        bc = BC_EXTRAP0;
    }
    int si = gi, sj = gj;
    int xside = side < 2;
    if (bc == BC_PERIODIC) {
        if (side == 0) si = nx - layer;
        if (side == 1) si = layer - 1;
        if (side == 2) sj = ny - layer;
        if (side == 3) sj = layer - 1;
    } else if (bc == BC_EXTRAP0) {
        if (side == 0) si = 0;
        if (side == 1) si = nx - 1;
        if (side == 2) sj = 0;
        if (side == 3) sj = ny - 1;
    } else { /* BC_REFLECT */
        if (side == 0) si = layer - 1;
        if (side == 1) si = nx - layer;
        if (side == 2) sj = layer - 1;
        if (side == 3) sj = ny - layer;
    }
    size_t s = idx(g, si, sj);
    g->R[d] = g->R[s];
    g->M[d] = g->M[s];
    g->N[d] = g->N[s];
    if (bc == BC_REFLECT) {
        if (xside) g->M[d] = -g->M[d];
        else g->N[d] = -g->N[d];
    }
}

static void fill_ghosts_x(const orc_params *p, double t, field_t *g, int layers)
{
    for (int j = 0; j < g->ny; j++)
        for (int l = 1; l <= layers; l++) {
            set_ghost(p, t, g, 0, -l, j, l);
            set_ghost(p, t, g, 1, g->nx - 1 + l, j, l);
        }
}

static void fill_ghosts_y(const orc_params *p, double t, field_t *g, int layers)
{
    for (int i = 0; i < g->nx; i++)
        for (int l = 1; l <= layers; l++) {
            set_ghost(p, t, g, 2, i, -l, l);
            set_ghost(p, t, g, 3, i, g->ny - 1 + l, l);
        }
}

/* Ghost rows of the x1-swept state Q*: as fill_ghosts_y, except on sides with
 * analytic (Taylor) data, whose rows the step has already filled. */
static void fill_ghosts_y_q1(const orc_params *p, double t, field_t *g, int layers)
{
    for (int i = 0; i < g->nx; i++)
        for (int l = 1; l <= layers; l++) {
            if (p->bc[2] != BC_TAYLOR) set_ghost(p, t, g, 2, i, -l, l);
            if (p->bc[3] != BC_TAYLOR) set_ghost(p, t, g, 3, i, g->ny - 1 + l, l);
        }
}

/* ------------------------------------------------------------------------- */
/* Source step (eq. fs:source): forward Euler in time, second-order central  */
/* differences in space.                                                     */
/* ------------------------------------------------------------------------- */

/* Planar: psi = delta~ (0, lap(q^2/q^1), lap(q^3/q^1)) (eq. adim:q), read as
 * the Laplacian of the velocity u = q^2/q^1, as the physical right-hand side
 * rho0 delta lap(u) of eq. OurSystem requires.
 * Axisymmetric (x1 = z, x2 = r, r_j = j + 1/2; not in the paper, derived from
 * eq. OurSystem in cylindrical coordinates without swirl): the vector
 * Laplacian adds (1/r) d/dr of each velocity component and -v/r^2 to the
 * radial one.  The geometric (hoop) terms of the divergence are not part of
 * this step: see geometric_half_step. */
static int source_step(const orc_params *p, double dt, field_t *in, field_t *out, int nt)
{
    int nx = in->nx, ny = in->ny;
    size_t n = (size_t)in->pitch * (size_t)(ny + 2 * GH);
    double *u = malloc(n * sizeof(double));
    double *v = malloc(n * sizeof(double));
    if (!u || !v) { free(u); free(v); return ORC_E_NOMEM; }
#pragma omp parallel for schedule(static) num_threads(nt)
    for (long k = 0; k < (long)n; k++) {
        double q1 = 1.0 + in->R[k];
        u[k] = in->M[k] / q1;
        v[k] = in->N[k] / q1;
    }
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t c = idx(in, i, j);
            size_t xm = idx(in, i - 1, j), xp = idx(in, i + 1, j);
            size_t ym = idx(in, i, j - 1), yp = idx(in, i, j + 1);
            double lapu = u[xp] + u[xm] + u[yp] + u[ym] - 4.0 * u[c];
            double lapv = v[xp] + v[xm] + v[yp] + v[ym] - 4.0 * v[c];
            double sR = 0.0, sM, sN;
            if (p->geometry == GEOM_AXISYM) {
                double r = j + 0.5;
                double dur = (u[yp] - u[ym]) / 2.0;
                double dvr = (v[yp] - v[ym]) / 2.0;
                sM = p->delta * (lapu + dur / r);
                sN = p->delta * (lapv + dvr / r - v[c] / (r * r));
            } else {
                sM = p->delta * lapu;
                sN = p->delta * lapv;
            }
            out->R[c] = in->R[c] + dt * sR;
            out->M[c] = in->M[c] + dt * sM;
            out->N[c] = in->N[c] + dt * sN;
        }
    free(u);
    free(v);
    return ORC_OK;
}

/* Axisymmetric geometric terms (not in the paper; derived from eq.
 * OurSystem in cylindrical coordinates without swirl): the divergence of
 * rho u and of rho0 u(x)u + pI adds -N/r to the mass equation, -u v/r to the
 * axial and -v^2/r to the radial momentum (the pressure parts cancel).  They
 * are applied by forward Euler over half a time step, in place, on the
 * interior cells, once before and once after the x2 sweep (the sweep that
 * carries the radial flux): applied only after both sweeps the split step is
 * unstable near the axis above CFL ~0.8, applied symmetrically around the x2
 * sweep it is stable up to CFL 1 and second order in time.  Pinned by the
 * exact Bessel modes (the linear terms) and by a steady radial source flow
 * with axial drift (the quadratic terms -u v/r, -v^2/r). */
static void geometric_half_step(const orc_params *p, double h, field_t *f, int nt)
{
    (void)p;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int j = 0; j < f->ny; j++) {
        double r = j + 0.5;
        for (int i = 0; i < f->nx; i++) {
            size_t c = idx(f, i, j);
            double q1 = 1.0 + f->R[c];
            double u = f->M[c] / q1, v = f->N[c] / q1;
            double sR = -f->N[c] / r;
            double sM = -u * v / r;
            double sN = -v * v / r;
            f->R[c] = f->R[c] + h * sR;
            f->M[c] = f->M[c] + h * sM;
            f->N[c] = f->N[c] + h * sN;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Full step and driver.                                                     */
/* ------------------------------------------------------------------------- */

/* Scratch of one worker: the line being swept and its interfaces, and that
 * worker's share of the CFL maximum. */
typedef struct {
    double *lr, *ln, *lt, *or_, *on, *ot;
    iface_t *f;
    double smax;
    int bad, err;
    char pad[64];        /* keeps the workers' entries on separate cache lines */
} line_t;

typedef struct { field_t a, b, c, d; int nt; line_t *line; } work_t;

/* Worker threads of the sweeps and the source (OpenMP over rows, or over
 * columns for the x2 sweep).  Each row is computed by one thread with the
 * same operations as in a serial run, and the per-thread CFL maxima are
 * merged in thread order by the same rule, so the result does not depend on
 * the thread count.  Default 1. */
static int g_threads = 1;

void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void)
{
#ifdef _OPENMP
    return g_threads;
#else
    return 1;
#endif
}

static int work_alloc(work_t *w, int nx, int ny)
{
    memset(w, 0, sizeof(*w));
    int e = field_alloc(&w->a, nx, ny) | field_alloc(&w->b, nx, ny) |
            field_alloc(&w->c, nx, ny) | field_alloc(&w->d, nx, ny);
    int m = (nx > ny ? nx : ny) + 2 * GH;
    w->nt = orc_get_threads();
    w->line = calloc((size_t)w->nt, sizeof(line_t));
    if (e || !w->line) return ORC_E_NOMEM;
    for (int k = 0; k < w->nt; k++) {
        line_t *L = &w->line[k];
        L->lr = malloc(sizeof(double) * m); L->ln = malloc(sizeof(double) * m); L->lt = malloc(sizeof(double) * m);
        L->or_ = malloc(sizeof(double) * m); L->on = malloc(sizeof(double) * m); L->ot = malloc(sizeof(double) * m);
        L->f = malloc(sizeof(iface_t) * (size_t)(m + 1));
        if (!L->lr || !L->ln || !L->lt || !L->or_ || !L->on || !L->ot || !L->f) return ORC_E_NOMEM;
    }
    return ORC_OK;
}

static void work_free(work_t *w)
{
    field_free(&w->a); field_free(&w->b); field_free(&w->c); field_free(&w->d);
    if (w->line)
        for (int k = 0; k < w->nt; k++) {
            line_t *L = &w->line[k];
            free(L->lr); free(L->ln); free(L->lt); free(L->or_); free(L->on); free(L->ot); free(L->f);
        }
    free(w->line);
}

static int thread_id(void)
{
#ifdef _OPENMP
    return omp_get_thread_num();
#else
    return 0;
#endif
}

/* Merge the workers' CFL maxima into (*smax, *bad) in thread order, with the
 * rule of sweep_line (a NaN, once seen, stays). */
static int merge_lines(work_t *w, double *smax, int *bad)
{
    int e = ORC_OK;
    for (int k = 0; k < w->nt; k++) {
        const line_t *L = &w->line[k];
        double a = L->smax;
        if (isnan(a) || a > *smax) *smax = a;
        if (L->bad) *bad = 1;
        if (L->err) e = L->err;
    }
    return e;
}

static void clear_lines(work_t *w)
{
    for (int k = 0; k < w->nt; k++) { w->line[k].smax = 0.0; w->line[k].bad = 0; w->line[k].err = 0; }
}

/* One attempted step from w->a (interior holds Q^n) to w->d (Q^{n+1}) with
 * time step dt at time t.  Returns the largest |s^p| over both sweeps in
 * *smax and 1 in *bad if any counted interface had non-real speeds. */
static int attempt(const orc_params *p, work_t *w, double t, double dt, double *smax, int *bad)
{
    int nx = p->nx, ny = p->ny, e;
    *smax = 0.0; *bad = 0;
    /* x1 sweep on Q^n, one row per iteration */
    fill_ghosts_x(p, t, &w->a, 2);
    clear_lines(w);
#pragma omp parallel for schedule(static) num_threads(w->nt)
    for (int j = 0; j < ny; j++) {
        line_t *L = &w->line[thread_id()];
        for (int k = 0; k < nx + 2 * GH; k++) {
            size_t s = idx(&w->a, k - GH, j);
            L->lr[k] = w->a.R[s]; L->ln[k] = w->a.M[s]; L->lt[k] = w->a.N[s];
        }
        double sm = 0.0;
        int bd = 0;
        int er = sweep_line(p->beta, dt, nx, L->lr, L->ln, L->lt, L->or_, L->on, L->ot, L->f, &sm, &bd);
        if (er) L->err = er;
        if (isnan(sm) || sm > L->smax) L->smax = sm;
        if (bd) L->bad = 1;
        for (int i = 0; i < nx; i++) {
            size_t d = idx(&w->b, i, j);
            w->b.R[d] = L->or_[i]; w->b.M[d] = L->on[i]; w->b.N[d] = L->ot[i];
        }
    }
    e = merge_lines(w, smax, bad);
    if (e) return e;
    /* Ghost rows of Q* on sides with analytic (Taylor) data: the x1 sweep
     * applied to the analytic Q^n of those rows (their own x ghosts by the
     * x side rules), so that the x2 sweep meets ghost values that went through
     * the same first fractional step as the interior.  Their interfaces do not
     * enter the CFL maximum. */
    line_t *L0 = &w->line[0];
    for (int side = 2; side <= 3; side++) {
        if (p->bc[side] != BC_TAYLOR) continue;
        for (int l = 1; l <= 2; l++) {
            int j = side == 2 ? -l : ny - 1 + l;
            for (int i = 0; i < nx; i++) set_ghost(p, t, &w->a, side, i, j, l);
            for (int l2 = 1; l2 <= 2; l2++) {
                set_ghost(p, t, &w->a, 0, -l2, j, l2);
                set_ghost(p, t, &w->a, 1, nx - 1 + l2, j, l2);
            }
            for (int k = 0; k < nx + 2 * GH; k++) {
                size_t s = idx(&w->a, k - GH, j);
                L0->lr[k] = w->a.R[s]; L0->ln[k] = w->a.M[s]; L0->lt[k] = w->a.N[s];
            }
            double ghost_smax = 0.0;
            int ghost_bad = 0;
            e = sweep_line(p->beta, dt, nx, L0->lr, L0->ln, L0->lt, L0->or_, L0->on, L0->ot, L0->f,
                           &ghost_smax, &ghost_bad);
            if (e) return e;
            for (int i = 0; i < nx; i++) {
                size_t d = idx(&w->b, i, j);
                w->b.R[d] = L0->or_[i]; w->b.M[d] = L0->on[i]; w->b.N[d] = L0->ot[i];
            }
        }
    }
    if (p->geometry == GEOM_AXISYM) geometric_half_step(p, 0.5 * dt, &w->b, w->nt);
    /* x2 sweep on Q*: same scheme with components 2 and 3 swapped, one column
     * per iteration */
    fill_ghosts_y_q1(p, t, &w->b, 2);
    clear_lines(w);
#pragma omp parallel for schedule(static) num_threads(w->nt)
    for (int i = 0; i < nx; i++) {
        line_t *L = &w->line[thread_id()];
        for (int k = 0; k < ny + 2 * GH; k++) {
            size_t s = idx(&w->b, i, k - GH);
            L->lr[k] = w->b.R[s]; L->ln[k] = w->b.N[s]; L->lt[k] = w->b.M[s];
        }
        double sm = 0.0;
        int bd = 0;
        int er = sweep_line(p->beta, dt, ny, L->lr, L->ln, L->lt, L->or_, L->on, L->ot, L->f, &sm, &bd);
        if (er) L->err = er;
        if (isnan(sm) || sm > L->smax) L->smax = sm;
        if (bd) L->bad = 1;
        for (int j = 0; j < ny; j++) {
            size_t d = idx(&w->c, i, j);
            w->c.R[d] = L->or_[j]; w->c.N[d] = L->on[j]; w->c.M[d] = L->ot[j];
        }
    }
    e = merge_lines(w, smax, bad);
    if (e) return e;
    if (p->geometry == GEOM_AXISYM) geometric_half_step(p, 0.5 * dt, &w->c, w->nt);
    /* source on Q** with one ghost layer */
    fill_ghosts_x(p, t, &w->c, 1);
    fill_ghosts_y(p, t, &w->c, 1);
    return source_step(p, dt, &w->c, &w->d, w->nt);
}

static int check_params(const orc_params *p)
{
    if (p->nx < 4 || p->ny < 4) return ORC_E_INVALID;
    if (p->bc[1] == BC_SOURCE || p->bc[2] == BC_SOURCE || p->bc[3] == BC_SOURCE) return ORC_E_INVALID;
    for (int s = 0; s < 4; s++) if (p->bc[s] < 0 || p->bc[s] > BC_SOURCE) return ORC_E_INVALID;
    if ((p->bc[0] == BC_PERIODIC) != (p->bc[1] == BC_PERIODIC)) return ORC_E_INVALID;
    if ((p->bc[2] == BC_PERIODIC) != (p->bc[3] == BC_PERIODIC)) return ORC_E_INVALID;
    if (p->src_envelope < 0 || p->src_envelope > 1) return ORC_E_INVALID;
    if (p->src_envelope == 1 && !(p->src_packet_cycles > 0.0)) return ORC_E_INVALID;
    if (p->src_stage2_on != 0 && (p->src_stage2_on != 1 || !isfinite(p->src_stage2))) return ORC_E_INVALID;
    return ORC_OK;
}

/* Largest |s^p| over every interface adjacent to an interior cell of the
 * state, in both directions, with ghosts from the boundary rules at time t
 * (the dry pass that fixes the first time step).  Returns -1 if a counted
 * interface has non-real speeds. */
double orc_dry_smax(const orc_params *p, const double *R, const double *M, const double *N, double t)
{
    if (check_params(p)) return -1.0;
    work_t w;
    if (work_alloc(&w, p->nx, p->ny)) { work_free(&w); return -1.0; }
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t d = idx(&w.a, i, j), s = (size_t)j * p->nx + i;
            w.a.R[d] = R[s]; w.a.M[d] = M[s]; w.a.N[d] = N[s];
        }
    fill_ghosts_x(p, t, &w.a, 2);
    fill_ghosts_y(p, t, &w.a, 2);
    double smax = 0.0;
    int bad = 0;
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i <= p->nx; i++) {
            size_t l = idx(&w.a, i - 1, j), r = idx(&w.a, i, j);
            double qL[3] = { w.a.R[l], w.a.M[l], w.a.N[l] }, qR[3] = { w.a.R[r], w.a.M[r], w.a.N[r] };
            double s[3], rr[3][3], al[3], W[3][3], am[3], ap[3];
            if (!orc_roe(p->beta, qL, qR, s, rr, al, W, am, ap)) { bad = 1; continue; }
            for (int k = 0; k < 3; k++) { double a = fabs(s[k]); if (isnan(a) || a > smax) smax = a; }
        }
    for (int i = 0; i < p->nx; i++)
        for (int j = 0; j <= p->ny; j++) {
            size_t l = idx(&w.a, i, j - 1), r = idx(&w.a, i, j);
            double qL[3] = { w.a.R[l], w.a.N[l], w.a.M[l] }, qR[3] = { w.a.R[r], w.a.N[r], w.a.M[r] };
            double s[3], rr[3][3], al[3], W[3][3], am[3], ap[3];
            if (!orc_roe(p->beta, qL, qR, s, rr, al, W, am, ap)) { bad = 1; continue; }
            for (int k = 0; k < 3; k++) { double a = fabs(s[k]); if (isnan(a) || a > smax) smax = a; }
        }
    work_free(&w);
    return bad ? -1.0 : smax;
}

/* Advance the state (R, M, N: row-major [ny][nx], x1 contiguous) by nsteps
 * accepted steps.  *t is the time of the state; *dt the step to try next
 * (<= 0: nu_W / smax of the dry pass).  CFL control (Sec. 4 opening): after
 * each attempt nu = dt * smax; if nu > cfl_max the attempt is discarded and
 * redone with dt * nu_W / nu (at most max_retries times in a row), otherwise
 * it is accepted and the next step uses dt * nu_W / nu.  With fixed_dt the
 * step is never changed and never rejected.  nu_hist (may be NULL) receives
 * nu of each accepted step.  Returns ORC_OK or an error; on error the state
 * holds the last accepted step. */
int orc_run(const orc_params *p, double *R, double *M, double *N, long nsteps,
            double *t, double *dt, orc_stats *st, double *nu_hist)
{
    int e = check_params(p);
    if (e) return e;
    memset(st, 0, sizeof(*st));
    if (!(*dt > 0.0)) {
        double s0 = orc_dry_smax(p, R, M, N, *t);
        if (s0 < 0.0) { st->status = ORC_E_NONHYPERBOLIC; return ORC_E_NONHYPERBOLIC; }
        if (!(s0 > 0.0) || !isfinite(s0)) { st->status = ORC_E_NONFINITE; return ORC_E_NONFINITE; }
        *dt = p->cfl_target / s0;
    }
    work_t w;
    if (work_alloc(&w, p->nx, p->ny)) { work_free(&w); return ORC_E_NOMEM; }
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t d = idx(&w.a, i, j), s = (size_t)j * p->nx + i;
            w.a.R[d] = R[s]; w.a.M[d] = M[s]; w.a.N[d] = N[s];
        }
    double nu_mean = 0.0, nu_m2 = 0.0;    /* running mean and sum of squared deviations */
    int retries = 0;
    long accepted = 0;
    e = ORC_OK;
    while (accepted < nsteps) {
        double smax;
        int bad;
        e = attempt(p, &w, *t, *dt, &smax, &bad);
        if (e) break;
        if (bad) { e = ORC_E_NONHYPERBOLIC; break; }
        if (!isfinite(smax)) { e = ORC_E_NONFINITE; break; }
        double nu = *dt * smax;
        st->nu_last = nu;
        if (!p->fixed_dt && nu > p->cfl_max) {
            st->rejected++;
            if (++retries > p->max_retries) { e = ORC_E_RETRIES; break; }
            *dt = *dt * p->cfl_target / nu;
            continue;
        }
        retries = 0;
#pragma omp parallel for schedule(static) num_threads(w.nt)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++) {
                size_t d = idx(&w.a, i, j);
                w.a.R[d] = w.d.R[d]; w.a.M[d] = w.d.M[d]; w.a.N[d] = w.d.N[d];
            }
        *t = *t + *dt;
        if (nu_hist) nu_hist[accepted] = nu;
        accepted++;
        double dev = nu - nu_mean;
        nu_mean = nu_mean + dev / (double)accepted;
        nu_m2 = nu_m2 + dev * (nu - nu_mean);
        if (!p->fixed_dt && smax > 0.0) *dt = *dt * p->cfl_target / nu;
    }
    for (int j = 0; j < p->ny; j++)
        for (int i = 0; i < p->nx; i++) {
            size_t d = idx(&w.a, i, j), s = (size_t)j * p->nx + i;
            R[s] = w.a.R[d]; M[s] = w.a.M[d]; N[s] = w.a.N[d];
        }
    work_free(&w);
    st->t = *t;
    st->dt_next = *dt;
    st->steps = accepted;
    if (accepted > 0) {
        st->nu_mean = nu_mean;
        st->nu_std = sqrt(nu_m2 / (double)accepted);
    }
    st->status = e;
    st->status_step = e ? accepted : 0;
    return e;
}

/* Ghost cell (gi, gj) of ghost layer `layer` (1 = adjacent) on `side` (0: x-,
 * 1: x+, 2: y-, 3: y+) at time t, filled by the boundary rule of that side
 * from the interior state (R, M, N: row-major [ny][nx]) into q = (R, M, N).
 * Exported so that the pins can check every side rule cell by cell.  The
 * cell must lie on that side's ghost frame: gi = -layer (side 0) or
 * nx - 1 + layer (side 1) with 0 <= gj < ny, gj = -layer (side 2) or
 * ny - 1 + layer (side 3) with 0 <= gi < nx; else ORC_E_INVALID. */
int orc_ghost(const orc_params *p, const double *R, const double *M, const double *N, double t,
              int side, int gi, int gj, int layer, double q[3])
{
    if (check_params(p)) return ORC_E_INVALID;
    if (side < 0 || side > 3 || layer < 1 || layer > GH) return ORC_E_INVALID;
    int nx = p->nx, ny = p->ny;
    int ok = (side == 0 && gi == -layer && gj >= 0 && gj < ny) ||
             (side == 1 && gi == nx - 1 + layer && gj >= 0 && gj < ny) ||
             (side == 2 && gj == -layer && gi >= 0 && gi < nx) ||
             (side == 3 && gj == ny - 1 + layer && gi >= 0 && gi < nx);
    if (!ok) return ORC_E_INVALID;
    field_t g;
    if (field_alloc(&g, nx, ny)) { field_free(&g); return ORC_E_NOMEM; }
    for (int j = 0; j < ny; j++)
        for (int i = 0; i < nx; i++) {
            size_t d = idx(&g, i, j), s = (size_t)j * nx + i;
            g.R[d] = R[s]; g.M[d] = M[s]; g.N[d] = N[s];
        }
    set_ghost(p, t, &g, side, gi, gj, layer);
    size_t d = idx(&g, gi, gj);
    q[0] = g.R[d]; q[1] = g.M[d]; q[2] = g.N[d];
    field_free(&g);
    return ORC_OK;
}

/* Ghost value of the analytic Taylor profile and of the focused source, for
 * the pins (exported so the tests can sample the boundary data directly). */
void orc_taylor_value(const orc_params *p, double x, double y, double t, double q[3]) { taylor_value(p, x, y, t, q); }
double orc_source_g(const orc_params *p, double r, double t) { return source_g(p, r, t); }
