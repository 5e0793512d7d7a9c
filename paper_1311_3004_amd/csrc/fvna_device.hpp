// fvna_device.hpp -- device code of libfvna for gfx950 (wave64).
//
// One fused kernel performs one attempted time step of the dimensionally
// split high-resolution finite-volume method of Velasco-Segura & Rendon
// (arXiv:1311.3004): x1 sweep, x2 sweep and source (Sec. 3, eqs. fs:cl1,
// fs:cl2, fs:source), reading the stored state once and writing it once.
//
// Work decomposition.  A wavefront owns a strip of 64 consecutive columns
// (lane l <-> column c0 - 3 + l) and a segment of rows.  It marches up the
// segment one row at a time:
//   * the x1 sweep of a row is lane-parallel; the left neighbour's cell, the
//     upwind neighbour's wave and the right neighbour's flux come from
//     cross-lane permutes (ds_bpermute), so every interface is solved once
//     and shared by the two cells it separates;
//   * the x2 sweep runs down each lane's column on rolling registers: each
//     new x1-swept row yields one x2 interface, one limited correction and
//     one x2-swept row;
//   * the source step of a row needs the x2-swept rows above and below it
//     (registers) and the lanes beside it (permutes); its result is the only
//     store.
// Lanes 3..60 produce the 58 output columns; lanes 0..2 and 61..63 are the
// halo the x1 stencil (two interfaces each side) and the source (one cell)
// need.  A segment starts three rows early and ends three rows late for the
// same reason.  Halo work is recomputed by the neighbouring wavefront, so
// results never depend on the strip or segment a cell falls in: every cell
// sees the same instruction sequence on the same operands.
//
// Boundaries.  Ghost values at a physical side are the boundary rule applied
// to the state of the stage that needs them (Q^n for the x1 sweep, the
// x1-swept state for the x2 sweep, the x2-swept state for the source), as
// the split method requires; they are synthesised in registers, never
// stored.
//
// Arithmetic: FP64 or FP32, with FP16/BF16 storage of scaled perturbations
// as an option.  Formulas use explicit fma() and the build disables FMA
// contraction, so every template instance rounds identically wherever it
// runs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fvna {

constexpr int WAVE = 64;
constexpr int HALO = 3;
constexpr int OUTW = WAVE - 2 * HALO;   // 58 output columns per wavefront
constexpr int WAVES_PER_BLOCK = 4;

enum { BC_PERIODIC = 0, BC_EXTRAP0 = 1, BC_REFLECT = 2, BC_TAYLOR = 3, BC_SOURCE = 4 };
enum { FLAG_NONHYP = 1u };
enum { ST_OK = 0, ST_NONHYP = 4, ST_NONFINITE = 5, ST_RETRIES = 6 };

// Device-resident clock and control word of one simulation.  Written only by
// the controller kernel (and the host between launches); the step kernel
// reads it and raises smax_bits / flags atomically.
struct Clock {
    double t;                    // time of the current state (dx/c0 units)
    double dt;                   // step of the next attempt
    long long accepted;          // accepted steps
    long long target;            // accepted steps requested
    long long rejected;          // rejected attempts
    long long attempts;
    long long status_step;
    unsigned long long smax_bits;  // max |s| of the running attempt (bits of a non-negative double)
    unsigned int flags;          // FLAG_* raised by the running attempt
    int cur;                     // buffer holding the current state (0 or 1)
    int status;                  // latched ST_* (0 = none)
    int retries;                 // consecutive rejections
    double nu_last, nu_mean, nu_m2;   // CFL statistics (Welford)
    long long nu_count;
    double pad[2];
};

// Everything a wavefront needs to know about its simulation.
struct SimDesc {
    int nx, ny, pitch, strips, segs, tile_rows;
    long long plane;             // elements per field plane = pitch * ny
    int bc[4];
    int fixed_dt, max_retries;
    double beta, delta, cfl_target, cfl_max;
    double ta_amp, ta_w, ta_x0, ta_y0, ta_cos, ta_sin;   // Taylor profile (cells)
    double sr_amp, sr_freq, sr_F, sr_ap, sr_ramp;        // focused source (cells, dx/c0)
    float scale[3], inv_scale[3];                        // half-width storage codec
    void* buf[2];                                        // state buffers: planes R, M, N
    Clock* clk;
};

// ---------------------------------------------------------------------------
// Storage codecs.
// ---------------------------------------------------------------------------
struct bf16 { uint16_t bits; };

template <typename S, typename T> struct Codec;
template <> struct Codec<double, double> {
    static __device__ __forceinline__ double ld(double s, float) { return s; }
    static __device__ __forceinline__ double st(double v, float) { return v; }
};
template <> struct Codec<float, float> {
    static __device__ __forceinline__ float ld(float s, float) { return s; }
    static __device__ __forceinline__ float st(float v, float) { return v; }
};
template <> struct Codec<_Float16, float> {
    static __device__ __forceinline__ float ld(_Float16 s, float scale) { return (float)s * scale; }
    static __device__ __forceinline__ _Float16 st(float v, float inv) { return (_Float16)(v * inv); }
};
template <> struct Codec<bf16, float> {
    static __device__ __forceinline__ float ld(bf16 s, float scale) {
        return __uint_as_float((uint32_t)s.bits << 16) * scale;
    }
    static __device__ __forceinline__ bf16 st(float v, float inv) {
        float x = v * inv;
        uint32_t b = __float_as_uint(x);
        bf16 r;
        if ((b & 0x7fffffffu) > 0x7f800000u) { r.bits = (uint16_t)((b >> 16) | 0x40u); return r; }  // quiet NaN
        b += 0x7fffu + ((b >> 16) & 1u);   // round to nearest, ties to even
        r.bits = (uint16_t)(b >> 16);
        return r;
    }
};

// ---------------------------------------------------------------------------
// Arithmetic helpers per compute type.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double abs_(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float abs_(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double min_(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float min_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double max_(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float max_(float a, float b) { return __builtin_fmaxf(a, b); }

// Cross-lane permutes (ds_bpermute; the source lane index wraps modulo 64).
__device__ __forceinline__ float perm(float v, int src) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src << 2, __float_as_int(v)));
}
__device__ __forceinline__ double perm(double v, int src) {
    long long b = __double_as_longlong(v);
    int lo = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b & 0xffffffffll));
    int hi = __builtin_amdgcn_ds_bpermute(src << 2, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

template <typename T> struct Cell { T R, M, N; };

// Roe wave structure of one interface in split-local components
// (density, normal momentum, tangential momentum).
template <typename T> struct Wave { T s1, s2, s3, a1, a2, a3, r1, r2; };

// Roe linearisation (Sec. 3.2).  Zbar is the arithmetic mean of
// z = (q^1, q^2/q^1, q^3/q^1); eigenvalues of eqs. lambda1-3; eigenvectors
// r^{1,2} = (1, s, zt (s - 2 zn)/(rho zbar (s - w))), r^3 = (0, 0, 1), where
// w = zn/rho and s - w = +-c; strengths from sum_p alpha^p r^p = Q_R - Q_L.
// L and R hold (density perturbation, normal momentum, tangential momentum)
// and the two velocities.  Returns false if the discriminant is not positive.
template <typename T>
__device__ __forceinline__ bool roe(T RL, T nL, T tL, T vnL, T vtL,
                                    T RR, T nR, T tR, T vnR, T vtR, T beta, Wave<T>& w)
{
    const T Rb = T(0.5) * (RL + RR);              // Zbar^1 - 1
    const T irb = rcp(T(1) + Rb);
    const T zn = T(0.5) * (vnL + vnR);
    const T zt = T(0.5) * (vtL + vtR);
    const T wv = zn * irb;
    const T Phi = fma_(T(2) * (beta - T(1)), Rb, T(1));
    const T D = fma_(wv, wv - T(2) * zn, Phi);    // w^2 - 2 zn^2/Zbar^1 + Phi
    const bool ok = D > T(0);
    const T c = sqrt_(D);
    const T ic = rcp(c);
    w.s1 = wv + c;
    w.s2 = wv - c;
    w.s3 = wv;
    const T k = zt * irb * ic;
    w.r1 = k * (w.s1 - T(2) * zn);
    w.r2 = -k * (w.s2 - T(2) * zn);
    const T d1 = RR - RL, d2 = nR - nL, d3 = tR - tL;
    w.a1 = T(0.5) * ic * fma_(-w.s2, d1, d2);
    w.a2 = d1 - w.a1;
    w.a3 = fma_(-w.a2, w.r2, fma_(-w.a1, w.r1, d3));
    return ok;
}

// MC limiter (Sec. 3.1): phi = max(0, min((1 + theta)/2, 2, 2 theta)).
template <typename T>
__device__ __forceinline__ T mc(T th)
{
    return max_(T(0), min_(min_(T(0.5) * (T(1) + th), T(2)), T(2) * th));
}

// theta = (W_up . W) / (W . W) with W = alpha (1, s, r) (theta = 0 when W = 0).
template <typename T>
__device__ __forceinline__ T theta_ac(T a, T s, T r, T au, T su, T ru)
{
    const T num = au * a * fma_(ru, r, fma_(su, s, T(1)));
    const T den = a * a * fma_(r, r, fma_(s, s, T(1)));
    return den != T(0) ? num * rcp(den) : T(0);
}

// From the interface's waves and its upwind neighbours' waves (per family),
// form Gm = A^- dQ + F~ (the part applied to the cell on the low side) and
// Gp = A^+ dQ - F~ (the part applied to the cell on the high side); eqs.
// fluc:m, fluc:p, limiter, fv-hr.  Components in split-local order.
template <typename T>
__device__ __forceinline__ void hr_split(const Wave<T>& w,
                                         T a1u, T s1u, T r1u, T a2u, T s2u, T r2u, T a3u,
                                         T dt, T Gm[3], T Gp[3])
{
    const T ph1 = mc(theta_ac(w.a1, w.s1, w.r1, a1u, s1u, r1u));
    const T ph2 = mc(theta_ac(w.a2, w.s2, w.r2, a2u, s2u, r2u));
    const T th3 = (w.a3 != T(0)) ? (a3u * w.a3) * rcp(w.a3 * w.a3) : T(0);
    const T ph3 = mc(th3);
    const T as1 = abs_(w.s1), as2 = abs_(w.s2), as3 = abs_(w.s3);
    // correction strengths c_p = 1/2 |s| (1 - dt |s|) phi alpha
    const T c1 = T(0.5) * as1 * fma_(-dt, as1, T(1)) * ph1 * w.a1;
    const T c2 = T(0.5) * as2 * fma_(-dt, as2, T(1)) * ph2 * w.a2;
    const T c3 = T(0.5) * as3 * fma_(-dt, as3, T(1)) * ph3 * w.a3;
    // e_p = min(s,0) alpha + c_p ; g_p = max(s,0) alpha - c_p
    const T e1 = fma_(min_(w.s1, T(0)), w.a1, c1);
    const T e2 = fma_(min_(w.s2, T(0)), w.a2, c2);
    const T e3 = fma_(min_(w.s3, T(0)), w.a3, c3);
    const T g1 = fma_(max_(w.s1, T(0)), w.a1, -c1);
    const T g2 = fma_(max_(w.s2, T(0)), w.a2, -c2);
    const T g3 = fma_(max_(w.s3, T(0)), w.a3, -c3);
    Gm[0] = e1 + e2;
    Gm[1] = fma_(e1, w.s1, e2 * w.s2);
    Gm[2] = fma_(e1, w.r1, fma_(e2, w.r2, e3));
    Gp[0] = g1 + g2;
    Gp[1] = fma_(g1, w.s1, g2 * w.s2);
    Gp[2] = fma_(g1, w.r1, fma_(g2, w.r2, g3));
}

// ---------------------------------------------------------------------------
// Analytic boundary data (always evaluated in FP64).
// ---------------------------------------------------------------------------

// Taylor shock-like profile, eq. OurTaylorS with the rotation of Sec. 4.1.
__device__ __forceinline__ void taylor_at(const SimDesc& d, double x, double y, double t,
                                          double& R, double& M, double& N)
{
    const double xi = (x - d.ta_x0) * d.ta_cos + (y - d.ta_y0) * d.ta_sin;
    R = -d.ta_amp * tanh((xi - t) / d.ta_w);
    M = R * d.ta_cos;
    N = R * d.ta_sin;
}

// Focused source, eq. hifuBC with a sin^2 ramp: the phase f (t + r^2/(2F)) is
// reduced modulo one period in FP64 before the sine.
template <typename T>
__device__ __forceinline__ void source_at(const SimDesc& d, double r, double t, T& R, T& M, T& N)
{
    const double f = d.sr_freq;
    double env;
    if (t <= 0.0) {
        env = 0.0;
    } else if (t < d.sr_ramp / f) {
        const double s = sin(M_PI * f * t / (2.0 * d.sr_ramp));
        env = s * s;
    } else {
        env = 1.0;
    }
    double ph = f * (t + r * r / (2.0 * d.sr_F));
    ph -= floor(ph);
    T g;
    if constexpr (sizeof(T) == 8) g = (T)(d.sr_amp * env * sin(2.0 * M_PI * ph));
    else g = (T)(d.sr_amp * env) * __sinf((float)(2.0 * M_PI * ph));
    const double h = sqrt(r * r + d.sr_F * d.sr_F);
    R = g;
    M = g * (T)(d.sr_F / h);
    N = g * (T)(-r / h);
}

// ---------------------------------------------------------------------------
// The fused step of one wavefront tile.
// ---------------------------------------------------------------------------

// x2-sweep pipeline state of one lane (its column).
template <typename T> struct Pipe {
    Cell<T> p1; T pu1, pv1;       // x1-swept row v-1 and its velocities
    Cell<T> p2;                   // x1-swept row v-2
    Wave<T> wB, wC;               // x2 interfaces v-3/2 and v-5/2
    T gpC[3];                     // Gp of interface v-5/2 (applied to row v-2)
    Cell<T> qc; T uc, vc;         // x2-swept row v-3 (its source comes next)
    T ub, vb;                     // velocities of x2-swept row v-4
    Cell<T> stash;                // x1-swept row ny-2 (reflecting top ghost)
};

template <typename S, typename T, int AXI>
__device__ __forceinline__ void march(const SimDesc& d, int strip, int seg, bool count)
{
    using C = Codec<S, T>;
    const int lane = threadIdx.x & (WAVE - 1);
    const int nx = d.nx, ny = d.ny;
    const int c0 = strip * OUTW;
    const int col = c0 - HALO + lane;
    const int r0 = seg * d.tile_rows;
    const int r1 = min(r0 + d.tile_rows, ny);
    const Clock* clk = d.clk;
    const double tn = clk->t;
    const T dt = (T)clk->dt;
    const int cur = clk->cur;
    const long long plane = d.plane;
    const size_t pitch = (size_t)d.pitch;
    const S* __restrict__ inR = (const S*)d.buf[cur];
    const S* __restrict__ inM = inR + plane;
    const S* __restrict__ inN = inM + plane;
    S* __restrict__ outR = (S*)d.buf[cur ^ 1];
    S* __restrict__ outM = outR + plane;
    S* __restrict__ outN = outM + plane;
    const bool perx = d.bc[0] == BC_PERIODIC;
    const bool pery = d.bc[2] == BC_PERIODIC;
    const T beta = (T)d.beta;
    const T delta = (T)d.delta;
    const float sc0 = d.scale[0], sc1 = d.scale[1], sc2 = d.scale[2];
    const float is0 = d.inv_scale[0], is1 = d.inv_scale[1], is2 = d.inv_scale[2];

    // ---- where this lane's Q^n comes from (x boundary rule) ----
    const bool incol = col >= 0 && col < nx;
    int scol = col;
    T msign = T(1);
    int xkind = 0;          // 0: load; 1: Taylor; 2: focused source (else extrapolate)
    if (perx) {
        scol = ((col % nx) + nx) % nx;
    } else if (col < 0) {
        const int g = -col;
        switch (d.bc[0]) {
        case BC_REFLECT: scol = g - 1; msign = T(-1); break;
        case BC_TAYLOR: xkind = 1; scol = 0; break;
        case BC_SOURCE: xkind = 2; scol = 0; break;
        default: scol = 0; break;
        }
    } else if (col >= nx) {
        const int g = col - nx + 1;
        switch (d.bc[1]) {
        case BC_REFLECT: scol = nx - g; msign = T(-1); break;
        case BC_TAYLOR: xkind = 1; scol = nx - 1; break;
        default: scol = nx - 1; break;
        }
    }
    scol = min(max(scol, 0), nx - 1);
    const bool real_col = perx || incol;
    const bool cnt_x = count && lane >= 1 && (perx || (col >= 0 && col <= nx));
    const bool cnt_y = count && lane >= 2 && lane <= WAVE - 3 && real_col;
    const bool out_lane = lane >= HALO && lane < WAVE - HALO && col < nx;
    const int lm1 = lane - 1, lp1 = lane + 1;

    T smax = T(0);
    bool bad = false;

    // ---- one x1-swept row (real row index vr in [0, ny)) ----
    auto xsweep = [&](int vr) -> Cell<T> {
        const size_t o = (size_t)vr * pitch + (size_t)scol;
        Cell<T> q;
        q.R = C::ld(inR[o], sc0);
        q.M = msign * C::ld(inM[o], sc1);
        q.N = C::ld(inN[o], sc2);
        if (xkind == 1) {
            double R, M, N;
            taylor_at(d, col + 0.5, vr + 0.5, tn, R, M, N);
            q.R = (T)R; q.M = (T)M; q.N = (T)N;
        } else if (xkind == 2) {
            const double r = vr + 0.5;
            if (r <= d.sr_ap) source_at<T>(d, r, tn, q.R, q.M, q.N);
        }
        const T irho = rcp(T(1) + q.R);
        const T u = q.M * irho, v = q.N * irho;
        const T RL = perm(q.R, lm1), ML = perm(q.M, lm1), NL = perm(q.N, lm1);
        const T uL = perm(u, lm1), vL = perm(v, lm1);
        Wave<T> w;
        const bool ok = roe(RL, ML, NL, uL, vL, q.R, q.M, q.N, u, v, beta, w);
        if (cnt_x) {
            bad |= !ok;
            smax = max_(smax, max_(abs_(w.s1), max_(abs_(w.s2), abs_(w.s3))));
        }
        const int u1 = w.s1 < T(0) ? lp1 : lm1;
        const int u2 = w.s2 < T(0) ? lp1 : lm1;
        const int u3 = w.s3 < T(0) ? lp1 : lm1;
        const T a1u = perm(w.a1, u1), s1u = perm(w.s1, u1), r1u = perm(w.r1, u1);
        const T a2u = perm(w.a2, u2), s2u = perm(w.s2, u2), r2u = perm(w.r2, u2);
        const T a3u = perm(w.a3, u3);
        T Gm[3], Gp[3];
        hr_split(w, a1u, s1u, r1u, a2u, s2u, r2u, a3u, dt, Gm, Gp);
        const T g0 = perm(Gm[0], lp1), g1 = perm(Gm[1], lp1), g2 = perm(Gm[2], lp1);
        Cell<T> o2;
        o2.R = fma_(-dt, g0 + Gp[0], q.R);
        o2.M = fma_(-dt, g1 + Gp[1], q.M);
        o2.N = fma_(-dt, g2 + Gp[2], q.N);
        return o2;
    };

    // ---- x2 pipeline ----
    Pipe<T> P;
    {
        const T z = T(0);
        P.p1 = {z, z, z}; P.pu1 = z; P.pv1 = z; P.p2 = {z, z, z};
        P.wB = {z, z, z, z, z, z, z, z}; P.wC = P.wB;
        P.gpC[0] = P.gpC[1] = P.gpC[2] = z;
        P.qc = {z, z, z}; P.uc = z; P.vc = z; P.ub = z; P.vb = z; P.stash = {z, z, z};
    }
    const int vfirst = r0 - HALO;

    // analytic (Taylor) velocities of a ghost cell
    auto taylor_uv = [&](double x, double y, T& uu, T& vv) {
        double R, M, N;
        taylor_at(d, x, y, tn, R, M, N);
        uu = (T)(M / (1.0 + R));
        vv = (T)(N / (1.0 + R));
    };

    auto push = [&](Cell<T> q, int v) {
        const T irho = rcp(T(1) + q.R);
        const T u = q.M * irho, vv = q.N * irho;
        // stage A: x2 interface v-1/2 between rows v-1 (low) and v (high); normal = N
        Wave<T> wA;
        const bool ok = roe(P.p1.R, P.p1.N, P.p1.M, P.pv1, P.pu1, q.R, q.N, q.M, vv, u, beta, wA);
        if (cnt_y && v > vfirst && (pery || (v >= 0 && v <= ny))) {
            bad |= !ok;
            smax = max_(smax, max_(abs_(wA.s1), max_(abs_(wA.s2), abs_(wA.s3))));
        }
        // stage B: limited correction at v-3/2 (upwind: v-5/2 if s >= 0, v-1/2 if s < 0)
        const Wave<T>& wB = P.wB;
        const bool f1 = wB.s1 < T(0), f2 = wB.s2 < T(0), f3 = wB.s3 < T(0);
        T Gm[3], Gp[3];
        hr_split(wB,
                 f1 ? wA.a1 : P.wC.a1, f1 ? wA.s1 : P.wC.s1, f1 ? wA.r1 : P.wC.r1,
                 f2 ? wA.a2 : P.wC.a2, f2 ? wA.s2 : P.wC.s2, f2 ? wA.r2 : P.wC.r2,
                 f3 ? wA.a3 : P.wC.a3, dt, Gm, Gp);
        // stage C: x2-swept row v-2 (split-local order R, N, M)
        Cell<T> qn;
        qn.R = fma_(-dt, Gm[0] + P.gpC[0], P.p2.R);
        qn.N = fma_(-dt, Gm[1] + P.gpC[1], P.p2.N);
        qn.M = fma_(-dt, Gm[2] + P.gpC[2], P.p2.M);
        const T irn = rcp(T(1) + qn.R);
        const T un = qn.M * irn, vn = qn.N * irn;
        // stage D: source of row j = v-3, then store
        const int j = v - 3;
        if (j >= r0 && j < r1) {
            T uxl = perm(P.uc, lm1), vxl = perm(P.vc, lm1);
            T uxr = perm(P.uc, lp1), vxr = perm(P.vc, lp1);
            T ubl = P.ub, vbl = P.vb, uab = un, vab = vn;
            if (!perx && col == 0) {
                const int b = d.bc[0];
                if (b == BC_REFLECT) { uxl = -P.uc; vxl = P.vc; }
                else if (b == BC_TAYLOR) taylor_uv(-0.5, j + 0.5, uxl, vxl);
                else if (b == BC_SOURCE && j + 0.5 <= d.sr_ap) {
                    T R, M, N;
                    source_at<T>(d, j + 0.5, tn, R, M, N);
                    const T ir = rcp(T(1) + R);
                    uxl = M * ir; vxl = N * ir;
                } else { uxl = P.uc; vxl = P.vc; }
            }
            if (!perx && col == nx - 1) {
                const int b = d.bc[1];
                if (b == BC_REFLECT) { uxr = -P.uc; vxr = P.vc; }
                else if (b == BC_TAYLOR) taylor_uv(nx + 0.5, j + 0.5, uxr, vxr);
                else { uxr = P.uc; vxr = P.vc; }
            }
            if (!pery && j == 0) {
                const int b = d.bc[2];
                if (b == BC_REFLECT) { ubl = P.uc; vbl = -P.vc; }
                else if (b == BC_TAYLOR) taylor_uv(col + 0.5, -0.5, ubl, vbl);
                else { ubl = P.uc; vbl = P.vc; }
            }
            if (!pery && j == ny - 1) {
                const int b = d.bc[3];
                if (b == BC_REFLECT) { uab = P.uc; vab = -P.vc; }
                else if (b == BC_TAYLOR) taylor_uv(col + 0.5, ny + 0.5, uab, vab);
                else { uab = P.uc; vab = P.vc; }
            }
            const T lapu = ((uxl + uxr) + (ubl + uab)) - T(4) * P.uc;
            const T lapv = ((vxl + vxr) + (vbl + vab)) - T(4) * P.vc;
            T oR = P.qc.R, oM, oN;
            if constexpr (AXI) {
                const T r = T(j) + T(0.5);
                const T ir = rcp(r);
                const T dur = T(0.5) * (uab - ubl), dvr = T(0.5) * (vab - vbl);
                const T sR = -P.qc.N * ir;
                const T sM = fma_(delta, fma_(dur, ir, lapu), -P.uc * P.vc * ir);
                const T sN = fma_(delta, fma_(-P.vc, ir * ir, fma_(dvr, ir, lapv)), -P.vc * P.vc * ir);
                oR = fma_(dt, sR, P.qc.R);
                oM = fma_(dt, sM, P.qc.M);
                oN = fma_(dt, sN, P.qc.N);
            } else {
                const T k = dt * delta;
                oM = fma_(k, lapu, P.qc.M);
                oN = fma_(k, lapv, P.qc.N);
            }
            if (out_lane) {
                const size_t o = (size_t)j * pitch + (size_t)col;
                outR[o] = C::st(oR, is0);
                outM[o] = C::st(oM, is1);
                outN[o] = C::st(oN, is2);
            }
        }
        // rotate
        P.ub = P.uc; P.vb = P.vc;
        P.qc = qn; P.uc = un; P.vc = vn;
        P.gpC[0] = Gp[0]; P.gpC[1] = Gp[1]; P.gpC[2] = Gp[2];
        P.wC = P.wB; P.wB = wA;
        P.p2 = P.p1; P.p1 = q; P.pu1 = u; P.pv1 = vv;
        if (v == ny - 2) P.stash = q;
    };

    // ghost row of the x1-swept state at the top (v >= ny, non-periodic)
    auto top_ghost = [&](int v) -> Cell<T> {
        const int b = d.bc[3];
        Cell<T> q = P.p1;
        if (b == BC_TAYLOR) {
            double R, M, N;
            taylor_at(d, col + 0.5, v + 0.5, tn, R, M, N);
            q.R = (T)R; q.M = (T)M; q.N = (T)N;
        } else if (b == BC_REFLECT) {
            if (v == ny) { q = P.p1; q.N = -q.N; }
            else if (v == ny + 1) { q = P.stash; q.N = -q.N; }
        }
        return q;
    };

    int v = vfirst;
    if (!pery && r0 == 0) {
        // bottom side: the ghost rows of the x1-swept state need rows 0 and 1 first
        const Cell<T> q0 = xsweep(0);
        const Cell<T> q1 = xsweep(1);
        const int b = d.bc[2];
        for (int g = HALO; g >= 1; --g) {       // rows -3, -2, -1
            Cell<T> q;
            if (b == BC_TAYLOR) {
                double R, M, N;
                taylor_at(d, col + 0.5, -g + 0.5, tn, R, M, N);
                q.R = (T)R; q.M = (T)M; q.N = (T)N;
            } else if (b == BC_REFLECT) {
                q = (g == 1) ? q0 : q1;
                q.N = -q.N;
            } else {
                q = q0;
            }
            push(q, -g);
        }
        push(q0, 0);
        push(q1, 1);
        v = 2;
    }
    const int vlast = r1 + HALO - 1;
    for (; v <= vlast; ++v) {
        Cell<T> q;
        if (pery) q = xsweep(((v % ny) + ny) % ny);
        else if (v < ny) q = xsweep(v);
        else q = top_ghost(v);
        push(q, v);
    }

    // ---- wave reductions: max |s| and the non-hyperbolic flag ----
    if (count) {
        T m = smax;
        for (int off = 32; off >= 1; off >>= 1) m = max_(m, perm(m, lane ^ off));
        const bool anybad = __any(bad);
        if (lane == 0) {
            const double md = (double)m;
            atomicMax(&d.clk->smax_bits, (unsigned long long)__double_as_longlong(md));
            if (anybad) atomicOr(&d.clk->flags, (unsigned int)FLAG_NONHYP);
        }
    }
}

}  // namespace fvna
