/*
 * oracle3d.c -- plain, slow FP64 CPU reference for the three-dimensional
 * extension of the finite-volume step of Velasco-Segura & Rendon
 * (arXiv:1311.3004), which the paper says its equations allow (Sec. 5).
 *
 * TEST INFRASTRUCTURE ONLY: called by the test-suite, never by the product
 * library; shares no code with the HIP path.  Compile with -ffp-contract=off.
 *
 * Same units and perturbation form as the 2-D oracle (lengths in cells, time
 * in dx/c0, R = q^1 - 1), with a fourth conserved component: the state is
 * (R, M1, M2, M3), M = rho u.  One step (Godunov splitting, the 3-D form of
 * eqs. fs:cl1, fs:cl2, fs:source): x1 sweep -> x2 sweep -> x3 sweep ->
 * source (delta~ times the 7-point Laplacian of each velocity component),
 * then the CFL decision as in 2-D.  Each 1-D sweep is the high-resolution
 * scheme of Sec. 3.1 with the Roe linearisation of Sec. 3.2 extended to a
 * second tangential component: a second shear wave at the speed w, and a
 * fourth entry of the acoustic eigenvectors built like the third.
 * Boundary kinds per side: periodic, zero-order extrapolation, reflection.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

enum { O3_OK = 0, O3_E_INVALID = 1, O3_E_NOMEM = 2, O3_E_NONHYPERBOLIC = 4, O3_E_NONFINITE = 5, O3_E_RETRIES = 6 };
enum { B3_PERIODIC = 0, B3_EXTRAP0 = 1, B3_REFLECT = 2 };

typedef struct {
    int nx, ny, nz;
    double beta, delta;     /* delta~ = delta / (c0 dx) */
    int bc[6];              /* x-, x+, y-, y+, z-, z+ */
    double cfl_target, cfl_max;
    int max_retries, fixed_dt;
} o3_params;

typedef struct {
    double t, dt_next, nu_last, nu_mean, nu_std;
    long steps, rejected;
    int status;
} o3_stats;

static double phi_excess(double beta, double R) { return R + (beta - 1.0) * R * R; }

/* normal-direction flux of (R, Mn, Mt1, Mt2): (Mn, un^2 + phi, un ut1, un ut2)
 * with u = M/(1+R) (the momentum flux of the model is rho0 u u + p). */
void o3_flux(double beta, const double q[4], double f[4])
{
    double q1 = 1.0 + q[0];
    f[0] = q[1];
    f[1] = q[1] * q[1] / (q1 * q1) + phi_excess(beta, q[0]);
    f[2] = q[1] * q[2] / (q1 * q1);
    f[3] = q[1] * q[3] / (q1 * q1);
}

static int solve4(double A[4][4], const double b[4], double x[4])
{
    double a[4][5];
    for (int i = 0; i < 4; i++) {
        for (int j = 0; j < 4; j++) a[i][j] = A[i][j];
        a[i][4] = b[i];
    }
    for (int c = 0; c < 4; c++) {
        int piv = c;
        for (int r = c + 1; r < 4; r++)
            if (fabs(a[r][c]) > fabs(a[piv][c])) piv = r;
        if (a[piv][c] == 0.0) return 0;
        if (piv != c)
            for (int j = 0; j < 5; j++) { double t = a[c][j]; a[c][j] = a[piv][j]; a[piv][j] = t; }
        for (int r = c + 1; r < 4; r++) {
            double f = a[r][c] / a[c][c];
            for (int j = c; j < 5; j++) a[r][j] = a[r][j] - f * a[c][j];
        }
    }
    for (int r = 3; r >= 0; r--) {
        double s = a[r][4];
        for (int j = r + 1; j < 4; j++) s = s - a[r][j] * x[j];
        x[r] = s / a[r][r];
    }
    return 1;
}

/* Roe decomposition in the normal direction.  Zbar = arithmetic mean of
 * z = (q^1, q^2/q^1, q^3/q^1, q^4/q^1); speeds w +- sqrt(disc), w, w; the
 * acoustic eigenvectors (1, s, Zb3 (s - 2 Zb2)/(Zb1 (s - w)), Zb4 (...)),
 * the shear ones (0,0,1,0), (0,0,0,1); strengths from sum alpha r = dQ. */
int o3_roe(double beta, const double qL[4], const double qR[4],
           double s[4], double alpha[4], double W[4][4], double amdq[4], double apdq[4])
{
    double q1L = 1.0 + qL[0], q1R = 1.0 + qR[0];
    double Zb1m1 = 0.5 * (qL[0] + qR[0]);
    double Zb1 = 1.0 + Zb1m1;
    double Zb2 = 0.5 * (qL[1] / q1L + qR[1] / q1R);
    double Zb3 = 0.5 * (qL[2] / q1L + qR[2] / q1R);
    double Zb4 = 0.5 * (qL[3] / q1L + qR[3] / q1R);
    double Phi = 1.0 + 2.0 * (beta - 1.0) * Zb1m1;
    double w = Zb2 / Zb1;
    double disc = (Zb2 * Zb2) / (Zb1 * Zb1) - 2.0 * (Zb2 * Zb2) / Zb1 + Phi;
    if (!(disc > 0.0)) return 0;
    double root = sqrt(disc);
    s[0] = w + root; s[1] = w - root; s[2] = w; s[3] = w;
    double r[4][4];
    for (int p = 0; p < 2; p++) {
        double g = (s[p] - 2.0 * Zb2) / (Zb1 * (s[p] - w));
        r[p][0] = 1.0; r[p][1] = s[p]; r[p][2] = Zb3 * g; r[p][3] = Zb4 * g;
    }
    for (int c = 0; c < 4; c++) { r[2][c] = 0.0; r[3][c] = 0.0; }
    r[2][2] = 1.0; r[3][3] = 1.0;
    double Rm[4][4], dq[4];
    for (int c = 0; c < 4; c++) {
        for (int p = 0; p < 4; p++) Rm[c][p] = r[p][c];
        dq[c] = qR[c] - qL[c];
    }
    if (!solve4(Rm, dq, alpha)) return 0;
    for (int c = 0; c < 4; c++) { amdq[c] = 0.0; apdq[c] = 0.0; }
    for (int p = 0; p < 4; p++) {
        double sm = s[p] < 0.0 ? s[p] : 0.0, sp = s[p] > 0.0 ? s[p] : 0.0;
        for (int c = 0; c < 4; c++) {
            W[p][c] = alpha[p] * r[p][c];
            amdq[c] = amdq[c] + sm * W[p][c];
            apdq[c] = apdq[c] + sp * W[p][c];
        }
    }
    return 1;
}

static double mc(double theta)
{
    double a = (1.0 + theta) / 2.0, m = a < 2.0 ? a : 2.0;
    m = m < 2.0 * theta ? m : 2.0 * theta;
    return m > 0.0 ? m : 0.0;
}

typedef struct { double s[4], W[4][4], amdq[4], apdq[4]; int ok; } if4_t;

/* One line of n interior cells, q[c][k] with k = i + 2 (two ghosts each side). */
static int sweep4(double beta, double dtdx, int n, double *const q[4], double *const out[4],
                  if4_t *f, double (*Ft)[4], double *smax, int *bad)
{
    for (int i = -1; i <= n + 1; i++) {
        double qL[4], qR[4], alpha[4];
        for (int c = 0; c < 4; c++) { qL[c] = q[c][i + 1]; qR[c] = q[c][i + 2]; }
        if4_t *F = &f[i + 1];
        F->ok = o3_roe(beta, qL, qR, F->s, alpha, F->W, F->amdq, F->apdq);
        if (!F->ok) {
            for (int p = 0; p < 4; p++) { F->s[p] = NAN; for (int c = 0; c < 4; c++) F->W[p][c] = NAN; }
            for (int c = 0; c < 4; c++) { F->amdq[c] = NAN; F->apdq[c] = NAN; }
        }
        if (i >= 0 && i <= n) {
            if (!F->ok) *bad = 1;
            for (int p = 0; p < 4; p++) {
                double a = fabs(F->s[p]);
                if (isnan(a) || a > *smax) *smax = a;
            }
        }
    }
    for (int i = 0; i <= n; i++) {
        const if4_t *F = &f[i + 1];
        for (int c = 0; c < 4; c++) Ft[i][c] = 0.0;
        for (int p = 0; p < 4; p++) {
            const if4_t *U = (F->s[p] < 0.0) ? &f[i + 2] : &f[i];
            double num = 0.0, den = 0.0;
            for (int c = 0; c < 4; c++) { num = num + U->W[p][c] * F->W[p][c]; den = den + F->W[p][c] * F->W[p][c]; }
            double theta = (den == 0.0) ? 0.0 : num / den;
            double as = fabs(F->s[p]);
            double coef = 0.5 * as * (1.0 - dtdx * as);
            double ph = mc(theta);
            for (int c = 0; c < 4; c++) Ft[i][c] = Ft[i][c] + coef * (ph * F->W[p][c]);
        }
    }
    for (int i = 0; i < n; i++) {
        const if4_t *Fl = &f[i + 1], *Fr = &f[i + 2];
        for (int c = 0; c < 4; c++)
            out[c][i] = q[c][i + 2] - dtdx * (Fr->amdq[c] + Fl->apdq[c]) - dtdx * (Ft[i + 1][c] - Ft[i][c]);
    }
    return O3_OK;
}

#define G3 2
typedef struct { int nx, ny, nz, px, py; double *q[4]; } f3_t;

static size_t at(const f3_t *g, int i, int j, int k)
{
    return ((size_t)(k + G3) * (size_t)g->py + (size_t)(j + G3)) * (size_t)g->px + (size_t)(i + G3);
}

static int f3_alloc(f3_t *g, int nx, int ny, int nz)
{
    g->nx = nx; g->ny = ny; g->nz = nz; g->px = nx + 2 * G3; g->py = ny + 2 * G3;
    size_t n = (size_t)g->px * (size_t)g->py * (size_t)(nz + 2 * G3);
    int ok = 1;
    for (int c = 0; c < 4; c++) { g->q[c] = calloc(n, sizeof(double)); ok = ok && g->q[c]; }
    return ok ? O3_OK : O3_E_NOMEM;
}

static void f3_free(f3_t *g) { for (int c = 0; c < 4; c++) free(g->q[c]); }

/* Ghost layers along axis a (0: x, 1: y, 2: z) by the side rules: periodic
 * wrap, zero-order extrapolation, or mirror with the normal momentum negated.
 * Filled over the whole extent of the other two axes including their ghosts. */
static void fill_ghosts(const o3_params *p, f3_t *g, int a)
{
    int n[3] = { g->nx, g->ny, g->nz };
    int lo[3] = { -G3, -G3, -G3 }, hi[3] = { g->nx + G3, g->ny + G3, g->nz + G3 };
    int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
    for (int u = lo[b0]; u < hi[b0]; u++)
        for (int v = lo[b1]; v < hi[b1]; v++)
            for (int side = 0; side < 2; side++)
                for (int l = 1; l <= G3; l++) {
                    int gi = side == 0 ? -l : n[a] - 1 + l, si;
                    int kind = p->bc[2 * a + side];
                    double sign = 1.0;
                    if (kind == B3_PERIODIC) si = side == 0 ? gi + n[a] : gi - n[a];
                    else if (kind == B3_REFLECT) { si = side == 0 ? l - 1 : n[a] - l; sign = -1.0; }
                    else si = side == 0 ? 0 : n[a] - 1;
                    int ig[3], is[3];
                    ig[a] = gi; is[a] = si; ig[b0] = is[b0] = u; ig[b1] = is[b1] = v;
                    size_t d = at(g, ig[0], ig[1], ig[2]), s = at(g, is[0], is[1], is[2]);
                    for (int c = 0; c < 4; c++) g->q[c][d] = g->q[c][s];
                    g->q[1 + a][d] = sign * g->q[1 + a][s];
                }
}

/* Sweep along axis a of in -> out (interior cells), components ordered
 * (R, M_a, the other two momenta). */
static int sweep_axis(const o3_params *p, double dt, int a, f3_t *in, f3_t *out, double *smax, int *bad)
{
    int n[3] = { in->nx, in->ny, in->nz };
    int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
    int m = n[a];
    int t1 = 1 + b0, t2 = 1 + b1;
    double *line[4], *res[4];
    for (int c = 0; c < 4; c++) { line[c] = malloc(sizeof(double) * (size_t)(m + 2 * G3)); res[c] = malloc(sizeof(double) * (size_t)m); }
    if4_t *f = malloc(sizeof(if4_t) * (size_t)(m + 3));
    double (*Ft)[4] = malloc(sizeof(double[4]) * (size_t)(m + 1));
    int e = O3_OK;
    for (int c = 0; c < 4; c++) if (!line[c] || !res[c]) e = O3_E_NOMEM;
    if (!f || !Ft) e = O3_E_NOMEM;
    int comp[4] = { 0, 1 + a, t1, t2 };
    for (int u = 0; u < n[b0] && !e; u++)
        for (int v = 0; v < n[b1] && !e; v++) {
            int ix[3];
            ix[b0] = u; ix[b1] = v;
            for (int k = -G3; k < m + G3; k++) {
                ix[a] = k;
                size_t s = at(in, ix[0], ix[1], ix[2]);
                for (int c = 0; c < 4; c++) line[c][k + G3] = in->q[comp[c]][s];
            }
            e = sweep4(p->beta, dt, m, line, res, f, Ft, smax, bad);
            for (int k = 0; k < m && !e; k++) {
                ix[a] = k;
                size_t d = at(out, ix[0], ix[1], ix[2]);
                for (int c = 0; c < 4; c++) out->q[comp[c]][d] = res[c][k];
            }
        }
    for (int c = 0; c < 4; c++) { free(line[c]); free(res[c]); }
    free(f); free(Ft);
    return e;
}

/* Source (3-D form of eq. fs:source): forward Euler, M_c += dt delta~ lap(u_c),
 * 7-point Laplacian, one ghost layer by the side rules. */
static void source3(const o3_params *p, double dt, f3_t *in, f3_t *out)
{
    for (int a = 0; a < 3; a++) fill_ghosts(p, in, a);
    for (int k = 0; k < in->nz; k++)
        for (int j = 0; j < in->ny; j++)
            for (int i = 0; i < in->nx; i++) {
                size_t c = at(in, i, j, k);
                size_t nb[6] = { at(in, i - 1, j, k), at(in, i + 1, j, k), at(in, i, j - 1, k),
                                 at(in, i, j + 1, k), at(in, i, j, k - 1), at(in, i, j, k + 1) };
                out->q[0][c] = in->q[0][c];
                for (int m = 1; m <= 3; m++) {
                    double uc = in->q[m][c] / (1.0 + in->q[0][c]);
                    double lap = -6.0 * uc;
                    for (int s = 0; s < 6; s++) lap = lap + in->q[m][nb[s]] / (1.0 + in->q[0][nb[s]]);
                    out->q[m][c] = in->q[m][c] + dt * (p->delta * lap);
                }
            }
}

static int attempt3(const o3_params *p, f3_t *a, f3_t *b, f3_t *c, double dt, double *smax, int *bad)
{
    *smax = 0.0; *bad = 0;
    int e;
    fill_ghosts(p, a, 0);
    if ((e = sweep_axis(p, dt, 0, a, b, smax, bad))) return e;
    fill_ghosts(p, b, 1);
    if ((e = sweep_axis(p, dt, 1, b, c, smax, bad))) return e;
    fill_ghosts(p, c, 2);
    if ((e = sweep_axis(p, dt, 2, c, b, smax, bad))) return e;
    source3(p, dt, b, c);
    return O3_OK;
}

/* Advance Q (arrays [nz][ny][nx]) by nsteps accepted steps; CFL control as
 * in the 2-D oracle: nu = dt max|s|, reject and redo with dt nu_W/nu if
 * nu > cfl_max, else accept and use dt nu_W/nu next (fixed_dt: never). */
int o3_run(const o3_params *p, double *Q0, double *Q1, double *Q2, double *Q3, long nsteps,
           double *t, double *dt, o3_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) return O3_E_INVALID;
    for (int a = 0; a < 3; a++)
        if ((p->bc[2 * a] == B3_PERIODIC) != (p->bc[2 * a + 1] == B3_PERIODIC)) return O3_E_INVALID;
    f3_t A, B, C;
    if (f3_alloc(&A, p->nx, p->ny, p->nz) || f3_alloc(&B, p->nx, p->ny, p->nz) || f3_alloc(&C, p->nx, p->ny, p->nz))
        return O3_E_NOMEM;
    double *Q[4] = { Q0, Q1, Q2, Q3 };
    for (int k = 0; k < p->nz; k++)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++)
                for (int c = 0; c < 4; c++)
                    A.q[c][at(&A, i, j, k)] = Q[c][((size_t)k * p->ny + j) * p->nx + i];
    int e = O3_OK, retries = 0;
    double sum = 0.0, sum2 = 0.0;
    if (!(*dt > 0.0)) {
        double smax; int bad;
        f3_t D;
        if (f3_alloc(&D, p->nx, p->ny, p->nz)) return O3_E_NOMEM;
        e = attempt3(p, &A, &B, &D, 0.0, &smax, &bad);     /* dt = 0: speeds of Q0 only */
        f3_free(&D);
        if (e) goto done;
        if (bad) { e = O3_E_NONHYPERBOLIC; goto done; }
        *dt = p->cfl_target / smax;
    }
    while (st->steps < nsteps) {
        double smax; int bad;
        if ((e = attempt3(p, &A, &B, &C, *dt, &smax, &bad))) goto done;
        if (bad) { e = O3_E_NONHYPERBOLIC; goto done; }
        if (!isfinite(smax)) { e = O3_E_NONFINITE; goto done; }
        double nu = *dt * smax;
        st->nu_last = nu;
        if (!p->fixed_dt && nu > p->cfl_max) {
            st->rejected++;
            if (++retries > p->max_retries) { e = O3_E_RETRIES; goto done; }
            *dt = *dt * p->cfl_target / nu;
            continue;
        }
        retries = 0;
        f3_t T = A; A = C; C = T;
        *t = *t + *dt;
        st->steps++;
        sum += nu; sum2 += nu * nu;
        if (!p->fixed_dt) *dt = *dt * p->cfl_target / nu;
    }
done:
    for (int k = 0; k < p->nz; k++)
        for (int j = 0; j < p->ny; j++)
            for (int i = 0; i < p->nx; i++)
                for (int c = 0; c < 4; c++)
                    Q[c][((size_t)k * p->ny + j) * p->nx + i] = A.q[c][at(&A, i, j, k)];
    st->t = *t; st->dt_next = *dt; st->status = e;
    if (st->steps) {
        st->nu_mean = sum / st->steps;
        double v = sum2 / st->steps - st->nu_mean * st->nu_mean;
        st->nu_std = v > 0 ? sqrt(v) : 0.0;
    }
    f3_free(&A); f3_free(&B); f3_free(&C);
    return e;
}
