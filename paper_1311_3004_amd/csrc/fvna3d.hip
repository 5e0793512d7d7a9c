// Three-dimensional step (the paper's equations in three dimensions): one
// thread per cell, one kernel per sweep and one for the source; the step is
// decided on the host.  Every neighbour index goes through the side rule of
// its axis and is then clamped to the grid, so no access leaves a buffer.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/fvna3d.h"

namespace {

thread_local std::string g_err3 = "no error";

fvna_status fail3(fvna_status s, const char* msg)
{
    g_err3 = msg;
    return s;
}

#define HIP3(x)                                                              \
    do {                                                                     \
        hipError_t e_ = (x);                                                 \
        if (e_ != hipSuccess) return fail3(FVNA_E_HIP, hipGetErrorString(e_)); \
    } while (0)

struct Desc3 {
    int n[3];                 // nx, ny, nz
    int bc[6];
    double beta, delta;       // delta~ = delta / (c0 dx)
};

struct Red3 {                 // device reduction of one attempt
    unsigned long long smax_bits;
    unsigned int flags;       // 1: non-real speeds, 2: non-finite
    unsigned int pad;
};

__device__ __forceinline__ size_t cell(const Desc3& d, int i, int j, int k)
{
    return ((size_t)k * d.n[1] + j) * d.n[0] + i;
}

// Map index m along axis a to a real index by the side rule; sign = -1 when
// the momentum normal to that axis is mirrored.  Clamped afterwards.
__device__ __forceinline__ int side_map(const Desc3& d, int a, int m, double& sign)
{
    const int n = d.n[a];
    sign = 1.0;
    if (m < 0) {
        const int b = d.bc[2 * a];
        if (b == FVNA_BC_PERIODIC) m += n;
        else if (b == FVNA_BC_REFLECT) { m = -m - 1; sign = -1.0; }
        else m = 0;
    } else if (m >= n) {
        const int b = d.bc[2 * a + 1];
        if (b == FVNA_BC_PERIODIC) m -= n;
        else if (b == FVNA_BC_REFLECT) { m = 2 * n - m - 1; sign = -1.0; }
        else m = n - 1;
    }
    return min(max(m, 0), n - 1);
}

template <typename T>
struct Roe4 {
    T s[4], W[4][4], amdq[4], apdq[4];
    bool ok;
};

// Roe decomposition in the normal direction of (R, Mn, Mt1, Mt2): speeds
// w +- c, w, w; acoustic eigenvectors (1, s, g Zb3, g Zb4) with
// g = (s - 2 Zb2)/(Zb1 (s - w)); strengths in closed form.
template <typename T>
__device__ __forceinline__ void roe4(const T* qL, const T* qR, T beta, Roe4<T>& o)
{
    const T q1L = T(1) + qL[0], q1R = T(1) + qR[0];
    const T Zb1m1 = T(0.5) * (qL[0] + qR[0]);
    const T Zb1 = T(1) + Zb1m1;
    const T Zb2 = T(0.5) * (qL[1] / q1L + qR[1] / q1R);
    const T Zb3 = T(0.5) * (qL[2] / q1L + qR[2] / q1R);
    const T Zb4 = T(0.5) * (qL[3] / q1L + qR[3] / q1R);
    const T Phi = T(1) + T(2) * (beta - T(1)) * Zb1m1;
    const T w = Zb2 / Zb1;
    const T disc = (Zb2 * Zb2) / (Zb1 * Zb1) - T(2) * (Zb2 * Zb2) / Zb1 + Phi;
    o.ok = disc > T(0);
    const T c = sqrt(o.ok ? disc : T(1));
    o.s[0] = w + c; o.s[1] = w - c; o.s[2] = w; o.s[3] = w;
    T dq[4];
    for (int m = 0; m < 4; ++m) dq[m] = qR[m] - qL[m];
    const T a1 = (dq[1] - o.s[1] * dq[0]) / (o.s[0] - o.s[1]);
    const T a2 = dq[0] - a1;
    const T g1 = (o.s[0] - T(2) * Zb2) / (Zb1 * c);
    const T g2 = (o.s[1] - T(2) * Zb2) / (Zb1 * -c);
    const T a3 = dq[2] - Zb3 * (a1 * g1 + a2 * g2);
    const T a4 = dq[3] - Zb4 * (a1 * g1 + a2 * g2);
    const T r[4][4] = {{T(1), o.s[0], g1 * Zb3, g1 * Zb4},
                       {T(1), o.s[1], g2 * Zb3, g2 * Zb4},
                       {T(0), T(0), T(1), T(0)},
                       {T(0), T(0), T(0), T(1)}};
    const T al[4] = {a1, a2, a3, a4};
    for (int m = 0; m < 4; ++m) { o.amdq[m] = T(0); o.apdq[m] = T(0); }
    for (int p = 0; p < 4; ++p) {
        const T sm = min(o.s[p], T(0)), sp = max(o.s[p], T(0));
        for (int m = 0; m < 4; ++m) {
            o.W[p][m] = al[p] * r[p][m];
            o.amdq[m] += sm * o.W[p][m];
            o.apdq[m] += sp * o.W[p][m];
        }
    }
}

template <typename T>
__device__ __forceinline__ T mc3(T th)
{
    return max(T(0), min(min(T(0.5) * (T(1) + th), T(2)), T(2) * th));
}

// F~ at the interface between the waves F and its upwind neighbour per family.
template <typename T>
__device__ __forceinline__ void corr(const Roe4<T>& F, const Roe4<T>& lo, const Roe4<T>& hi, T dt, T* out)
{
    for (int m = 0; m < 4; ++m) out[m] = T(0);
    for (int p = 0; p < 4; ++p) {
        const Roe4<T>& U = F.s[p] < T(0) ? hi : lo;
        T num = T(0), den = T(0);
        for (int m = 0; m < 4; ++m) { num += U.W[p][m] * F.W[p][m]; den += F.W[p][m] * F.W[p][m]; }
        const T th = den == T(0) ? T(0) : num / den;
        const T as = fabs(F.s[p]);
        const T coef = T(0.5) * as * (T(1) - dt * as);
        const T ph = mc3(th);
        for (int m = 0; m < 4; ++m) out[m] += coef * (ph * F.W[p][m]);
    }
}

template <typename T>
__device__ __forceinline__ void note_speed(const Roe4<T>& F, double& mloc, unsigned& fl)
{
    if (!F.ok) fl |= 1u;
    double m = 0.0;
    for (int p = 0; p < 4; ++p) m = fmax(m, (double)fabs(F.s[p]));
    if (!isfinite(m)) fl |= 2u;
    else mloc = fmax(mloc, m);
}

// One sweep along axis a: in -> out (4 planes each), dt in cells.
template <typename T>
__global__ __launch_bounds__(256) void k3_sweep(Desc3 d, int a, const T* __restrict__ in, T* __restrict__ out,
                                                T dt, Red3* red)
{
    const size_t cells = (size_t)d.n[0] * d.n[1] * d.n[2];
    double mloc = 0.0;
    unsigned fl = 0;
    // grid-stride over the cells, so that each wavefront folds many cells
    // into its single atomic (one atomic per cell wavefront serialises)
    for (size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x; id < cells;
         id += (size_t)gridDim.x * blockDim.x) {
        int ix[3];
        ix[0] = (int)(id % d.n[0]);
        ix[1] = (int)((id / d.n[0]) % d.n[1]);
        ix[2] = (int)(id / ((size_t)d.n[0] * d.n[1]));
        const int b0 = a == 0 ? 1 : 0, b1 = a == 2 ? 1 : 2;
        const int comp[4] = {0, 1 + a, 1 + b0, 1 + b1};
        T q[5][4];                                      // cells i-2 .. i+2 along the axis
        for (int o = -2; o <= 2; ++o) {
            double sg;
            int jx[3] = {ix[0], ix[1], ix[2]};
            jx[a] = side_map(d, a, ix[a] + o, sg);
            const size_t off = cell(d, jx[0], jx[1], jx[2]);
            for (int m = 0; m < 4; ++m) q[o + 2][m] = in[(size_t)comp[m] * cells + off];
            q[o + 2][1] *= (T)sg;
        }
        const T beta = (T)d.beta;
        Roe4<T> f[4];                                   // interfaces i-3/2, i-1/2, i+1/2, i+3/2
        for (int m = 0; m < 4; ++m) roe4<T>(q[m], q[m + 1], beta, f[m]);
        note_speed(f[1], mloc, fl);                     // i-1/2: adjacent to this real cell
        if (ix[a] == d.n[a] - 1) note_speed(f[2], mloc, fl);   // and the line's last interface
        T Fl[4], Fr[4];
        corr(f[1], f[0], f[2], dt, Fl);
        corr(f[2], f[1], f[3], dt, Fr);
        const size_t off = cell(d, ix[0], ix[1], ix[2]);
        for (int m = 0; m < 4; ++m)
            out[(size_t)comp[m] * cells + off] = q[2][m] - dt * (f[2].amdq[m] + f[1].apdq[m]) - dt * (Fr[m] - Fl[m]);
    }
    // fold the wavefront, one atomic per wavefront
    for (int off = 32; off >= 1; off >>= 1) mloc = fmax(mloc, __shfl_xor(mloc, off));
    const bool any_nh = __any(fl & 1u), any_nf = __any(fl & 2u);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&red->smax_bits, (unsigned long long)__double_as_longlong(mloc));
        if (any_nh || any_nf) atomicOr(&red->flags, (any_nh ? 1u : 0u) | (any_nf ? 2u : 0u));
    }
}

// Source: M_c += dt delta~ lap(u_c), 7-point, neighbours by the side rules.
template <typename T>
__global__ __launch_bounds__(256) void k3_source(Desc3 d, const T* __restrict__ in, T* __restrict__ out, T dt)
{
    const size_t cells = (size_t)d.n[0] * d.n[1] * d.n[2];
    const size_t id = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= cells) return;
    int ix[3];
    ix[0] = (int)(id % d.n[0]);
    ix[1] = (int)((id / d.n[0]) % d.n[1]);
    ix[2] = (int)(id / ((size_t)d.n[0] * d.n[1]));
    T lap[3], uc[3];
    const T rc = T(1) / (T(1) + in[id]);
    for (int m = 0; m < 3; ++m) { uc[m] = in[(size_t)(1 + m) * cells + id] * rc; lap[m] = T(-6) * uc[m]; }
    for (int a = 0; a < 3; ++a)
        for (int o = -1; o <= 1; o += 2) {
            double sg;
            int jx[3] = {ix[0], ix[1], ix[2]};
            jx[a] = side_map(d, a, ix[a] + o, sg);
            const size_t off = cell(d, jx[0], jx[1], jx[2]);
            const T rn = T(1) / (T(1) + in[off]);
            for (int m = 0; m < 3; ++m) {
                T v = in[(size_t)(1 + m) * cells + off] * rn;
                if (m == a) v *= (T)sg;
                lap[m] += v;
            }
        }
    out[id] = in[id];
    for (int m = 0; m < 3; ++m)
        out[(size_t)(1 + m) * cells + id] = in[(size_t)(1 + m) * cells + id] + dt * ((T)d.delta * lap[m]);
}

template <typename T>
__global__ void k3_import(const double* __restrict__ src, T* __restrict__ dst, size_t n, double denom)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (T)(src[i] / denom);
}

template <typename T>
__global__ void k3_export(const T* __restrict__ src, double* __restrict__ dst, size_t n, double factor)
{
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (double)src[i] * factor;
}

}  // namespace

struct fvna3_ctx {
    fvna3_params p;
    Desc3 d;
    char* buf[3];
    Red3* red;
    double* stage;
    hipStream_t s;
    int cur = 0;              // buffer holding Q^n
    double t = 0.0, dt = 0.0, nu_last = 0.0, nu_sum = 0.0, nu_sum2 = 0.0;
    long long steps = 0, rejected = 0;
    size_t cells = 0;
};

namespace {

size_t elem(const fvna3_params* p) { return p->precision == FVNA_F64 ? 8 : 4; }

fvna_status validate3(const fvna3_params* p)
{
    if (!p) return fail3(FVNA_E_INVALID, "params is NULL");
    if (p->nx < 4 || p->ny < 4 || p->nz < 4) return fail3(FVNA_E_INVALID, "grid must have at least 4 cells per axis");
    if ((long long)p->nx * p->ny * p->nz > (1ll << 31)) return fail3(FVNA_E_INVALID, "grid too large");
    if (!(p->dx > 0) || !(p->c0 > 0) || !(p->rho0 > 0) || !(p->beta >= 1) || !(p->delta >= 0))
        return fail3(FVNA_E_INVALID, "need dx, c0, rho0 > 0, beta >= 1, delta >= 0");
    if (p->precision != FVNA_F64 && p->precision != FVNA_F32) return fail3(FVNA_E_INVALID, "precision must be F64 or F32");
    for (int s = 0; s < 6; ++s)
        if (p->bc[s] != FVNA_BC_PERIODIC && p->bc[s] != FVNA_BC_EXTRAP0 && p->bc[s] != FVNA_BC_REFLECT)
            return fail3(FVNA_E_INVALID, "sides must be PERIODIC, EXTRAP0 or REFLECT");
    for (int a = 0; a < 3; ++a)
        if ((p->bc[2 * a] == FVNA_BC_PERIODIC) != (p->bc[2 * a + 1] == FVNA_BC_PERIODIC))
            return fail3(FVNA_E_INVALID, "both sides of an axis must be periodic together");
    if (!(p->cfl_target > 0) || !(p->cfl_target < p->cfl_max)) return fail3(FVNA_E_INVALID, "need 0 < cfl_target < cfl_max");
    if (p->max_retries < 0) return fail3(FVNA_E_INVALID, "max_retries must be >= 0");
    return FVNA_OK;
}

// One attempt from buf[cur] with dt (cells): x -> y -> z -> source into the
// last free buffer; returns smax and the flags.
template <typename T>
fvna_status attempt3(fvna3_ctx* c, double dt, int* out_buf, double* smax, unsigned* flags)
{
    const int a = c->cur, b = (a + 1) % 3, e = (a + 2) % 3;
    T* A = (T*)c->buf[a];
    T* B = (T*)c->buf[b];
    T* E = (T*)c->buf[e];
    HIP3(hipMemsetAsync(c->red, 0, sizeof(Red3), c->s));
    const int blocks = (int)((c->cells + 255) / 256);
    const int sweep_blocks = std::min(blocks, 4096);
    hipLaunchKernelGGL(k3_sweep<T>, dim3(sweep_blocks), dim3(256), 0, c->s, c->d, 0, A, B, (T)dt, c->red);
    hipLaunchKernelGGL(k3_sweep<T>, dim3(sweep_blocks), dim3(256), 0, c->s, c->d, 1, B, E, (T)dt, c->red);
    hipLaunchKernelGGL(k3_sweep<T>, dim3(sweep_blocks), dim3(256), 0, c->s, c->d, 2, E, B, (T)dt, c->red);
    hipLaunchKernelGGL(k3_source<T>, dim3(blocks), dim3(256), 0, c->s, c->d, B, E, (T)dt);
    HIP3(hipGetLastError());
    Red3 h;
    HIP3(hipMemcpyAsync(&h, c->red, sizeof(Red3), hipMemcpyDeviceToHost, c->s));
    HIP3(hipStreamSynchronize(c->s));
    *out_buf = e;
    double m;
    std::memcpy(&m, &h.smax_bits, sizeof(double));
    *smax = m;
    *flags = h.flags;
    return FVNA_OK;
}

fvna_status attempt_any(fvna3_ctx* c, double dt, int* out_buf, double* smax, unsigned* flags)
{
    return c->p.precision == FVNA_F64 ? attempt3<double>(c, dt, out_buf, smax, flags)
                                      : attempt3<float>(c, dt, out_buf, smax, flags);
}

}  // namespace

extern "C" {

const char* fvna3_last_error(void) { return g_err3.c_str(); }

fvna_status fvna3_workspace_size(const fvna3_params* p, size_t* state_bytes, size_t* scratch_bytes)
{
    fvna_status s = validate3(p);
    if (s) return s;
    if (!state_bytes || !scratch_bytes) return fail3(FVNA_E_INVALID, "NULL argument");
    const size_t cells = (size_t)p->nx * p->ny * p->nz;
    *state_bytes = 4 * cells * elem(p);
    *scratch_bytes = 256 + cells * sizeof(double);
    return FVNA_OK;
}

fvna_status fvna3_create(const fvna3_params* p, void* buf_a, void* buf_b, void* buf_c, void* scratch, void* stream,
                         fvna3_ctx** out)
{
    fvna_status s = validate3(p);
    if (s) return s;
    if (!buf_a || !buf_b || !buf_c || !scratch || !out) return fail3(FVNA_E_INVALID, "NULL buffer");
    fvna3_ctx* c = new (std::nothrow) fvna3_ctx;
    if (!c) return fail3(FVNA_E_NOMEM, "out of host memory");
    c->p = *p;
    c->d.n[0] = p->nx; c->d.n[1] = p->ny; c->d.n[2] = p->nz;
    for (int k = 0; k < 6; ++k) c->d.bc[k] = p->bc[k];
    c->d.beta = p->beta;
    c->d.delta = p->delta / (p->c0 * p->dx);
    c->buf[0] = (char*)buf_a; c->buf[1] = (char*)buf_b; c->buf[2] = (char*)buf_c;
    c->red = (Red3*)scratch;
    c->stage = (double*)((char*)scratch + 256);
    c->s = (hipStream_t)stream;
    c->cells = (size_t)p->nx * p->ny * p->nz;
    *out = c;
    return FVNA_OK;
}

fvna_status fvna3_set_state(fvna3_ctx* c, const double* rho_p, const double* m1, const double* m2, const double* m3)
{
    if (!c || !rho_p || !m1 || !m2 || !m3) return fail3(FVNA_E_INVALID, "NULL argument");
    const fvna3_params& p = c->p;
    const double* src[4] = {rho_p, m1, m2, m3};
    const double denom[4] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0, p.rho0 * p.c0};
    const size_t n = c->cells, es = elem(&p);
    const int blocks = (int)((n + 255) / 256);
    for (int f = 0; f < 4; ++f) {
        HIP3(hipMemcpyAsync(c->stage, src[f], n * sizeof(double), hipMemcpyHostToDevice, c->s));
        char* dst = c->buf[0] + (size_t)f * n * es;
        if (p.precision == FVNA_F64) hipLaunchKernelGGL(k3_import<double>, dim3(blocks), dim3(256), 0, c->s, c->stage, (double*)dst, n, denom[f]);
        else hipLaunchKernelGGL(k3_import<float>, dim3(blocks), dim3(256), 0, c->s, c->stage, (float*)dst, n, denom[f]);
        HIP3(hipGetLastError());
    }
    HIP3(hipStreamSynchronize(c->s));
    c->cur = 0; c->t = 0.0; c->steps = 0; c->rejected = 0; c->nu_last = c->nu_sum = c->nu_sum2 = 0.0;
    if (p.dt0 > 0) {
        c->dt = p.dt0 * p.c0 / p.dx;
        return FVNA_OK;
    }
    int ob; double smax; unsigned fl;
    fvna_status s = attempt_any(c, 0.0, &ob, &smax, &fl);   // dt = 0: speeds of Q^0 in all three sweeps
    if (s) return s;
    if (fl & 1u) return fail3(FVNA_E_NONHYPERBOLIC, "non-real Roe speeds in the initial state");
    if ((fl & 2u) || !(smax > 0)) return fail3(FVNA_E_NONFINITE, "no finite positive wave speed in the initial state");
    c->dt = p.cfl_target / smax;
    return FVNA_OK;
}

fvna_status fvna3_step(fvna3_ctx* c, int64_t nsteps)
{
    if (!c) return fail3(FVNA_E_INVALID, "ctx is NULL");
    if (nsteps < 0) return fail3(FVNA_E_INVALID, "nsteps must be >= 0");
    int retries = 0;
    for (int64_t k = 0; k < nsteps;) {
        int ob; double smax; unsigned fl;
        fvna_status s = attempt_any(c, c->dt, &ob, &smax, &fl);
        if (s) return s;
        if (fl & 1u) return fail3(FVNA_E_NONHYPERBOLIC, "non-real Roe speeds in a step");
        if (fl & 2u) return fail3(FVNA_E_NONFINITE, "non-finite wave speed in a step");
        const double nu = c->dt * smax;
        c->nu_last = nu;
        if (!c->p.fixed_dt && nu > c->p.cfl_max) {
            c->rejected++;
            if (++retries > c->p.max_retries) return fail3(FVNA_E_RETRIES, "too many rejected attempts in a row");
            c->dt *= c->p.cfl_target / nu;
            continue;
        }
        retries = 0;
        c->cur = ob;
        c->t += c->dt;
        c->steps++;
        ++k;
        c->nu_sum += nu; c->nu_sum2 += nu * nu;
        if (!c->p.fixed_dt) c->dt *= c->p.cfl_target / nu;
    }
    return FVNA_OK;
}

fvna_status fvna3_get_state(fvna3_ctx* c, double* rho_p, double* m1, double* m2, double* m3)
{
    if (!c || !rho_p || !m1 || !m2 || !m3) return fail3(FVNA_E_INVALID, "NULL argument");
    const fvna3_params& p = c->p;
    double* dst[4] = {rho_p, m1, m2, m3};
    const double fac[4] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0, p.rho0 * p.c0};
    const size_t n = c->cells, es = elem(&p);
    const int blocks = (int)((n + 255) / 256);
    for (int f = 0; f < 4; ++f) {
        const char* src = c->buf[c->cur] + (size_t)f * n * es;
        if (p.precision == FVNA_F64) hipLaunchKernelGGL(k3_export<double>, dim3(blocks), dim3(256), 0, c->s, (const double*)src, c->stage, n, fac[f]);
        else hipLaunchKernelGGL(k3_export<float>, dim3(blocks), dim3(256), 0, c->s, (const float*)src, c->stage, n, fac[f]);
        HIP3(hipGetLastError());
        HIP3(hipMemcpyAsync(dst[f], c->stage, n * sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIP3(hipStreamSynchronize(c->s));
    }
    return FVNA_OK;
}

fvna_status fvna3_get_stats(fvna3_ctx* c, fvna_stats* st)
{
    if (!c || !st) return fail3(FVNA_E_INVALID, "NULL argument");
    const double tu = c->p.dx / c->p.c0;
    std::memset(st, 0, sizeof(*st));
    st->t = c->t * tu;
    st->dt_next = c->dt * tu;
    st->nu_last = c->nu_last;
    if (c->steps) {
        st->nu_mean = c->nu_sum / c->steps;
        const double v = c->nu_sum2 / c->steps - st->nu_mean * st->nu_mean;
        st->nu_std = v > 0 ? std::sqrt(v) : 0.0;
    }
    st->steps = c->steps;
    st->rejected = c->rejected;
    st->status = FVNA_OK;
    return FVNA_OK;
}

fvna_status fvna3_time_step_kernels(fvna3_ctx* c, int32_t reps, double* ms)
{
    if (!c || !ms || reps < 1) return fail3(FVNA_E_INVALID, "bad argument");
    hipEvent_t e0, e1;
    HIP3(hipEventCreate(&e0));
    HIP3(hipEventCreate(&e1));
    int ob; double smax; unsigned fl;
    fvna_status s = attempt_any(c, c->dt, &ob, &smax, &fl);       // warm-up
    if (s) return s;
    float total = 0.0f;
    for (int r = 0; r < reps; ++r) {
        HIP3(hipEventRecord(e0, c->s));
        s = attempt_any(c, c->dt, &ob, &smax, &fl);
        if (s) return s;
        HIP3(hipEventRecord(e1, c->s));
        HIP3(hipEventSynchronize(e1));
        float t = 0.0f;
        HIP3(hipEventElapsedTime(&t, e0, e1));
        total += t;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = total / reps;
    return FVNA_OK;
}

void fvna3_destroy(fvna3_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    delete c;
}

}  // extern "C"
