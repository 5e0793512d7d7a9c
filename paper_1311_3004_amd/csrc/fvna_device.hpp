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
//     whole-wave DPP shifts (no LDS round trip), so every interface is solved once
//     and shared by the two cells it separates;
//   * the x2 sweep runs down each lane's column on rolling registers: each
//     new x1-swept row yields one x2 interface, one limited correction and
//     one x2-swept row;
//   * the source step of a row needs the x2-swept rows above and below it
//     (registers) and the lanes beside it (DPP shifts); its result is the only
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
enum { FLAG_NONHYP = 1u, FLAG_NONFINITE = 2u };
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
    long long x_off;             // cells the domain has moved since the state was set
    double pad;
};

// Accept or reject the attempt just made, from its largest wave speed (the
// CFL rule of the opening of Sec. 4; rejection as stated in include/fvna.h):
// nu = dt max|s|; nu > cfl_max rejects (state kept, dt *= nu_W/nu, at most
// max_retries in a row), otherwise the step is accepted, t += dt, the buffer
// holding the new state (cur + 1 modulo nbuf) becomes current and, unless
// the time step is fixed, dt *= nu_W/nu.  All memory traffic is issued at
// once, so the launch costs one round trip: the attempt's largest speed and
// flags are taken (and cleared for the next attempt) whether or not the
// attempt counts -- a step launch that had nothing to do left them at zero.
// The decision itself, as a function: the clock state h an attempt ran with,
// the bits of its largest wave speed and its flags -> the state after it.
__device__ __forceinline__ Clock control_next(Clock h, unsigned long long sb, unsigned flags, int fixed_dt,
                                              double cfl_target, double cfl_max, int max_retries, int nbuf)
{
    h.smax_bits = 0;
    h.flags = 0;
    if (h.status != 0 || h.accepted >= h.target) return h;
    const double smax = __longlong_as_double((long long)sb);
    const long long step = h.accepted;
    h.attempts += 1;
    if (flags & FLAG_NONHYP) { h.status = ST_NONHYP; h.status_step = step; return h; }
    if ((flags & FLAG_NONFINITE) || !(smax <= 1.7976931348623157e308)) {
        h.status = ST_NONFINITE;
        h.status_step = step;
        return h;
    }
    const double dt = h.dt;
    const double nu = dt * smax;
    h.nu_last = nu;
    if (!fixed_dt && nu > cfl_max) {
        h.rejected += 1;
        h.retries += 1;
        if (h.retries > max_retries) { h.status = ST_RETRIES; h.status_step = step; return h; }
        h.dt = dt * cfl_target / nu;
        return h;
    }
    h.retries = 0;
    h.t = h.t + dt;
    h.accepted = step + 1;
    h.cur = h.cur + 1 == nbuf ? 0 : h.cur + 1;
    const long long n = h.nu_count + 1;
    h.nu_count = n;
    const double dev = nu - h.nu_mean;
    const double mean = h.nu_mean + dev / (double)n;
    h.nu_mean = mean;
    h.nu_m2 = h.nu_m2 + dev * (nu - mean);
    if (!fixed_dt && smax > 0.0) h.dt = dt * cfl_target / nu;
    return h;
}

__device__ __forceinline__ void control_attempt(Clock* c, int fixed_dt, double cfl_target, double cfl_max,
                                                int max_retries, int nbuf)
{
    const unsigned long long sb = atomicExch(&c->smax_bits, 0ull);
    const unsigned flags = atomicExch(&c->flags, 0u);
    const Clock h = *c;
    if (h.status != 0 || h.accepted >= h.target) return;
    *c = control_next(h, sb, flags, fixed_dt, cfl_target, cfl_max, max_retries, nbuf);
}

// Attempts that take the previous attempt's decision in their own prologue
// (k_step with pos >= 1): beside the clock, in the same allocation, two
// alternating copies of the clock state and two more CFL slots (slot 0 is the
// clock's own smax_bits / flags).
struct CflSlot { unsigned long long smax_bits; unsigned int flags, pad; };
struct ClockAux { Clock shadow[2]; CflSlot slot[2]; };
constexpr size_t CLOCK_AUX_OFFSET = 256;           // bytes after the clock
__device__ __forceinline__ ClockAux* clock_aux(Clock* c)
{
    return (ClockAux*)((char*)c + CLOCK_AUX_OFFSET);
}
__device__ __forceinline__ void cfl_slot(Clock* c, int k, unsigned long long*& sb, unsigned int*& fl)
{
    if (k == 0) { sb = &c->smax_bits; fl = &c->flags; }
    else { CflSlot& q = clock_aux(c)->slot[k - 1]; sb = &q.smax_bits; fl = &q.flags; }
}

// What one attempt runs with: the time, step, buffer and domain offset of
// its clock state, and where its largest wave speed and flags go.
struct Attempt {
    double t, dt;
    long long x_off;
    int cur;
    unsigned long long* smax;
    unsigned int* flags;
};
__device__ __forceinline__ Attempt attempt_of(const Clock& h, unsigned long long* sb, unsigned int* fl)
{
    return Attempt{h.t, h.dt, h.x_off, h.cur, sb, fl};
}

// Everything a wavefront needs to know about its simulation.
struct SimDesc {
    int nx, ny, pitch, strips, segs, tile_rows;
    int seg_edge, seg_mid;       // row segments: 0 = uniform tile_rows; else the first and last
                                 // segment have seg_edge rows, the others seg_mid (seg_bounds)
    long long plane;             // elements per field plane = pitch * ny
    int bc[4];
    int fixed_dt, max_retries;
    double beta, delta, cfl_target, cfl_max;
    double ta_amp, ta_w, ta_x0, ta_y0, ta_cos, ta_sin;   // Taylor profile (cells)
    double sr_amp, sr_freq, sr_F, sr_ap, sr_ramp;        // focused source (cells, dx/c0)
    float scale[3], inv_scale[3];                        // half-width storage codec
    void* buf[2];                                        // state buffers: planes R, M, N
    Clock* clk;
    const double* src_tab;       // focused source, per row j: frac(f r^2/(2F)), F/h, -r/h, f r^2/(2F) (null: none)
    int sr_env;                  // 0: sin^2 ramp in t; 1: packet exp(-(f tau / sr_W)^10)
    double sr_W;                 // packet half-width in periods
    double sr_t2;                // start of the second stage (+inf: none)
    const void* rinv;            // axisymmetric: 1/(j + 1/2) for rows j = -RINV_PAD .. ny + RINV_PAD - 1,
                                 // in the arithmetic type (rinv_at)
};

// 1/r at the centre of row j (r = j + 1/2 cells) from the per-row table the
// library fills when an axisymmetric grid is created (the correctly rounded
// quotient).  Read through the constant address space: a scalar load of a
// row-uniform value, where computing it took a conversion, an add and a
// reciprocal on the vector unit for each of the three uses per row.  Rows
// down to -RINV_PAD and up to ny + RINV_PAD - 1 are covered (the warm-up rows
// of the first and last segment push ghost rows, whose values are not used).
constexpr int RINV_PAD = 8;
template <typename T> __device__ __forceinline__ T rinv_at(const SimDesc& d, int j)
{
    typedef const __attribute__((address_space(4))) T* ConstT;
    return ((ConstT)d.rinv)[j + RINV_PAD];
}

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
    // round to nearest, ties to even, by gfx950's v_cvt_pk_bf16_f32
    static __device__ __forceinline__ bf16 st(float v, float inv) {
        bf16 r;
        r.bits = __builtin_bit_cast(uint16_t, (__bf16)(v * inv));
        return r;
    }
};

// ---------------------------------------------------------------------------
// Arithmetic helpers per compute type.
// ---------------------------------------------------------------------------
// FP64 reciprocal: the hardware estimate (relative error below 5e-8 on
// gfx950) refined by one third-order step, r += r (e + e^2) with
// e = 1 - x r: the same 1-ulp result as two Newton steps, in three FMAs
// instead of four (measured on 2M arguments over 1e-26 .. 1e26).  1/0 gives
// NaN instead of Inf, which the limiter treats exactly as it treats 0 * Inf
// (its wave strength is zero).
__device__ __forceinline__ double rcp(double x)
{
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, __builtin_fma(e, e, e), r);
}
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double sqrt_(double x) { return __builtin_sqrt(x); }
__device__ __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
// c = sqrt(D) and ic = 1/c from one reciprocal square root, then one step
// on c, c += (ic/2)(D - c^2).  c is the wave speed: a bias in it shifts the
// phase of every wave a little each step, which adds up (FP32 vs FP64 on the
// 4096^2 pulse after 2020 steps: max |dp|/p_peak 1.03e-5 without the step,
// 8.8e-6 with it).
// FP64: the hardware estimate (relative error below 6e-8) refined by one
// third-order step, ic += ic (e/2 + 3e^2/8) with e = 1 - D ic^2 (within an
// ulp), then c = D ic and the step on c: c and ic within an ulp of the
// correctly rounded values (measured on 2M arguments), in ten instructions
// where a correctly rounded square root and division take about 25.  For D
// not a positive finite number both come out NaN (D = +Inf and D = 0 through
// Inf * 0), which the CFL bookkeeping relies on.
__device__ __forceinline__ void sqrt_pair(double D, double& c, double& ic)
{
    const double q = __builtin_amdgcn_rsq(D);
    const double e = __builtin_fma(-(D * q), q, 1.0);
    ic = __builtin_fma(q, __builtin_fma(e, 0.375, 0.5) * e, q);
    const double c0 = D * ic;
    c = __builtin_fma(0.5 * ic, __builtin_fma(-c0, c0, D), c0);
}
__device__ __forceinline__ void sqrt_pair(float D, float& c, float& ic)
{
    ic = __builtin_amdgcn_rsqf(D);
    const float c0 = D * ic;
    c = __builtin_fmaf(0.5f * ic, __builtin_fmaf(-c0, c0, D), c0);
}
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

// Neighbour exchange along the wave with DPP whole-wave shifts (gfx9-family
// VALU, no LDS round trip): from_lo(v) gives lane l the value of lane l - 1,
// from_hi(v) the value of lane l + 1.  Lane 0 (from_lo) and lane 63
// (from_hi) receive 0; both are halo lanes whose results are never used.
constexpr int DPP_WAVE_SHL1 = 0x130;   // lane l reads lane l + 1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane l reads lane l - 1
template <int CTRL> __device__ __forceinline__ int dpp_(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, true);
}
template <int CTRL> __device__ __forceinline__ float shift_(float v)
{
    return __int_as_float(dpp_<CTRL>(__float_as_int(v)));
}
template <int CTRL> __device__ __forceinline__ double shift_(double v)
{
    const long long b = __double_as_longlong(v);
    const int lo = dpp_<CTRL>((int)(b & 0xffffffffll));
    const int hi = dpp_<CTRL>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
template <typename T> __device__ __forceinline__ T from_lo(T v) { return shift_<DPP_WAVE_SHR1>(v); }
template <typename T> __device__ __forceinline__ T from_hi(T v) { return shift_<DPP_WAVE_SHL1>(v); }

template <typename T> struct Cell { T R, M, N; };

// Roe wave structure of one interface in split-local components
// (density, normal momentum, tangential momentum).
template <typename T> struct Wave { T s1, s2, s3, a1, a2, a3, r1, r2; };

// Roe linearisation (Sec. 3.2).  Zbar is the arithmetic mean of
// z = (q^1, q^2/q^1, q^3/q^1); eigenvalues of eqs. lambda1-3; eigenvectors
// r^{1,2} = (1, s, zt (s - 2 zn)/(rho zbar (s - w))), r^3 = (0, 0, 1), where
// w = zn/rho and s - w = +-c; strengths from sum_p alpha^p r^p = Q_R - Q_L.
// L and R hold (density perturbation, normal momentum, tangential momentum)
// and the two velocities.
//
// Returns this interface's max_p |s^p| = c + |w| in a form the CFL reduction
// can carry exactly -- FP64 as is; FP32 as its excess over 1, (c - 1) + |w|
// with c - 1 = (D - 1)/(1 + c), which keeps ~1e-7 relative precision on the
// excess (so ~1e-10 on the speed itself) -- and the discriminant D in D.
// When D is not a positive finite number the returned value is meaningless
// (FP32: always NaN); Cfl::add sorts these cases out.
// roe_sh takes Sr = RL + RR and h = 1/(2 + Sr) from the caller (rcp_pair).
template <typename T>
__device__ __forceinline__ T roe_sh(T RL, T nL, T tL, T vnL, T vtL,
                                    T RR, T nR, T tR, T vnR, T vtR, T beta, T Sr, T h, Wave<T>& w, T& D)
{
    // Sums of the two sides stand for the means (Zbar^1 - 1 = Sr/2, zn = Sn/2,
    // zt = St/2); every factor of 2 they introduce cancels exactly.
    const T Sn = vnL + vnR;
    const T St = vtL + vtR;
    const T wv = Sn * h;                          // w = zn / Zbar^1, h = 1 / (2 Zbar^1)
    const T D1 = fma_(wv, wv - Sn, (beta - T(1)) * Sr);   // D - 1
    D = T(1) + D1;                                // w^2 - 2 zn^2/Zbar^1 + Phi
    T c, ic;
    sqrt_pair(D, c, ic);
    T spd;
    if constexpr (sizeof(T) == 8) spd = c + abs_(wv);
    else spd = fma_(D1, rcp(T(1) + c), abs_(wv));
    w.s1 = wv + c;
    w.s2 = wv - c;
    w.s3 = wv;
    const T k = St * h * ic;                      // zt / (Zbar^1 c)
    w.r1 = k * (w.s1 - Sn);
    w.r2 = -k * (w.s2 - Sn);
    const T d1 = RR - RL, d2 = nR - nL, d3 = tR - tL;
    w.a1 = T(0.5) * ic * fma_(-w.s2, d1, d2);
    w.a2 = d1 - w.a1;
    w.a3 = fma_(-w.a2, w.r2, fma_(-w.a1, w.r1, d3));
    return spd;
}
template <typename T>
__device__ __forceinline__ T roe(T RL, T nL, T tL, T vnL, T vtL,
                                 T RR, T nR, T tR, T vnR, T vtR, T beta, Wave<T>& w, T& D)
{
    const T Sr = RL + RR;
    return roe_sh(RL, nL, tL, vnL, vtL, RR, nR, tR, vnR, vtR, beta, Sr, rcp(T(2) + Sr), w, D);
}

// 1/a and 1/b for the two positive factors a = 1 + R of a cell and
// b = 2 + Sr of an interface it borders: FP64 from one reciprocal of a b
// (rounding of the product and the two multiplies aside, the same values; a
// reciprocal estimate holds the SIMD four times as long as an FMA), FP32 two
// estimates.
template <typename T>
__device__ __forceinline__ void rcp_pair(T a, T b, T& ia, T& ib)
{
    if constexpr (sizeof(T) == 8) {
        const T r = rcp(a * b);
        ia = r * b;
        ib = r * a;
    } else {
        ia = rcp(a);
        ib = rcp(b);
    }
}

// Value the CFL reduction starts from (no interface counted yet) and the
// largest wave speed a reduced value stands for.
template <typename T> __device__ __forceinline__ T cfl_floor() { return sizeof(T) == 8 ? T(0) : T(-1); }
template <typename T> __device__ __forceinline__ double cfl_speed(T m)
{
    if constexpr (sizeof(T) == 8) return m;
    else return 1.0 + (double)m;
}

// Running CFL bookkeeping of one lane over the interfaces it solves: the
// largest wave speed, and whether some discriminant D was <= 0 or NaN (no
// real wave speeds: non-hyperbolic) or else +Inf (non-finite).
//   FP32: a NaN-propagating maximum of the returned value (NaN exactly when
//   D is not a positive finite number) and a NaN-propagating minimum of D --
//   two instructions per interface, no branch.
//   FP64: the returned speed is NaN exactly when D is not a positive finite
//   number (sqrt_pair), and the IEEE maximum skips NaN, so the maximum
//   needs no mask; two class tests of D (one instruction each) record
//   D <= 0 or NaN, and D = +Inf.
template <typename T> struct Cfl;
template <> struct Cfl<float> {
    float m, dmin;
    __device__ __forceinline__ Cfl() : m(-1.0f), dmin(1.0f) {}
    __device__ __forceinline__ void add(float spd, float D)
    {
        m = __builtin_elementwise_maximum(m, spd);
        dmin = __builtin_elementwise_minimum(dmin, D);
    }
    // This lane's contribution if it holds real interfaces (else nothing).
    __device__ __forceinline__ void finish(bool counted, float& spd, bool& nonhyp, bool& nonfin) const
    {
        nonhyp = counted && !(dmin > 0.0f);
        nonfin = counted && !nonhyp && m != m;
        spd = (counted && m == m) ? m : -1.0f;
    }
};
template <> struct Cfl<double> {
    // v_cmp_class_f64 masks: -0, +0, -denormal, -normal, -Inf, quiet and
    // signalling NaN (D <= 0 or NaN); +Inf
    static constexpr int NOT_POSITIVE = 0x07f, POS_INF = 0x200;
    double m;
    bool h, f;
    __device__ __forceinline__ Cfl() : m(0.0), h(false), f(false) {}
    __device__ __forceinline__ void add(double spd, double D)
    {
        m = __builtin_fmax(m, spd);
        h = h || __builtin_amdgcn_class(D, NOT_POSITIVE);
        f = f || __builtin_amdgcn_class(D, POS_INF);
    }
    __device__ __forceinline__ void finish(bool counted, double& spd, bool& nonhyp, bool& nonfin) const
    {
        nonhyp = counted && h;
        nonfin = counted && !h && f;
        spd = (counted && !h && !f) ? m : 0.0;
    }
};

// MC limiter (Sec. 3.1), phi(theta) = max(0, min((1 + theta)/2, 2, 2 theta)),
// with theta = (W_up . W) / (W . W) for the waves W^p = alpha^p r^p,
// r^p = (1, s^p, r^p) of families p = 1, 2 and r^3 = (0, 0, 1).  The scheme
// needs theta only through the product phi(theta) alpha, and only half of it
// (hr_split doubles the factor it multiplies): psi alpha with psi = phi/2 =
// max(0, min((1 + theta)/4, 1, theta)).
//
// With X = r^p_up . r^p and n = r^p . r^p (>= 1), alpha cancels from the
// ratio: theta = t / (alpha n), t = alpha_up X.  The neighbour supplies t, so
// each lane ships t instead of the full product W_up . W.
//
// FP32, families 1 and 2: psi from theta = t / (alpha n), times alpha (one
// reciprocal estimate, a two-quad-cycle instruction in FP32; the shear family
// takes mc_unit below).  When alpha = 0 the quotient is x/0 or 0/0, psi is
// then 0 or 1 (min/max return the non-NaN operand), and the product with
// alpha is 0 -- the value the guard theta := 0 gives.  So no guard is
// evaluated.
template <typename T>
__device__ __forceinline__ T mc_half(T th)
{
    return max_(T(0), min_(min_(fma_(T(0.25), th, T(0.25)), T(1)), th));
}

// FP64: psi alpha directly from alpha and u = alpha theta = t / n, with no
// division by alpha.  Scaling the min/max by alpha (and flipping them when
// alpha < 0) gives, with g the sign of alpha,
//   psi alpha = g max(0, min((|alpha| + g u)/4, |alpha|, g u)),
// which is 0 for alpha = 0.  g u is formed as u * copysign(1, alpha), exact,
// and a multiply's result, which the compiler knows to be a canonical
// number (min/max in IEEE mode need canonical operands; a bit flip would
// cost a quieting instruction at each of them); the result takes alpha's
// sign by copysign; /4 is exact (ldexp).  1/n is needed for families 1 and 2
// only (n = 1 for family 3), and both come from one reciprocal of
// n1 n2 >= 1 (hr_split).  This saves the three reciprocals of alpha^p n^p --
// on this chip an FP64 reciprocal estimate occupies the SIMD four times as
// long as an FMA.
__device__ __forceinline__ double mc_scaled(double a, double u)
{
    const double gu = u * __builtin_copysign(1.0, a);
    const double aa = __builtin_fabs(a);
    const double m = max_(0.0, min_(min_(__builtin_ldexp(aa + gu, -2), aa), gu));
    return __builtin_copysign(m, a);
}

// FP32, a family whose eigenvector is a unit vector (n = 1, X = 1: the shear
// wave), so t = alpha_up and theta = t / alpha.  With q = (alpha + t)/4, the
// product psi alpha is max(0, min(q, alpha, t)) for alpha >= 0 and
// min(0, max(q, alpha, t)) for alpha < 0; both equal
// med3(0, min(q, alpha, t), max(q, alpha, t)) (when alpha and t differ in sign
// the minimum is negative and the maximum positive), and it is 0 for
// alpha = 0.  Five instructions (v_minimum3, v_maximum3 and v_med3 among them)
// and no reciprocal.  The NaN-propagating minimum and maximum take the
// neighbour's t as it comes off the lane shift (an IEEE min/max would need it
// quieted first); t and alpha are finite whenever the state is.
__device__ __forceinline__ float mc_unit(float a, float t)
{
    const float q = (a + t) * 0.25f;
    const float lo = __builtin_elementwise_minimum(__builtin_elementwise_minimum(q, a), t);
    const float hi = __builtin_elementwise_maximum(__builtin_elementwise_maximum(q, a), t);
    return __builtin_amdgcn_fmed3f(0.0f, lo, hi);
}

// The upwind values t of two neighbouring interfaces a (below) and b (above)
// for each other: ta = what b needs when a is its upwind interface (alpha_a X),
// tb = what a needs when b is upwind (alpha_b X), X = r^p_a . r^p_b for
// p = 1, 2; entry 2 is the neighbour's alpha^3 (X = 1 for family 3).
template <typename T>
__device__ __forceinline__ void wave_cross(const Wave<T>& a, const Wave<T>& b, T ta[3], T tb[3])
{
    const T x1 = fma_(a.r1, b.r1, fma_(a.s1, b.s1, T(1)));
    const T x2 = fma_(a.r2, b.r2, fma_(a.s2, b.s2, T(1)));
    ta[0] = a.a1 * x1; ta[1] = a.a2 * x2; ta[2] = a.a3;
    tb[0] = b.a1 * x1; tb[1] = b.a2 * x2; tb[2] = b.a3;
}

// From the waves of one interface and the upwind values t of the interface
// below (dlo) and above (dhi) (wave_cross), form
//   Gm = A^- dQ + F~   (applied to the cell on the low side) and
//   Gp = A^+ dQ - F~   (applied to the cell on the high side);
// eqs. fluc:m, fluc:p, limiter, fv-hr.  The upwind interface of family p is
// the one below when s^p >= 0 and the one above when s^p < 0.  Components in
// split-local order (density, normal, tangential momentum).
template <typename T>
__device__ __forceinline__ void hr_split(const Wave<T>& w, const T dlo[3], const T dhi[3], T dt,
                                         T Gm[3], T Gp[3])
{
    const T t1 = w.s1 < T(0) ? dhi[0] : dlo[0];
    const T t2 = w.s2 < T(0) ? dhi[1] : dlo[1];
    const T t3 = w.s3 < T(0) ? dhi[2] : dlo[2];
    const T n1 = fma_(w.r1, w.r1, fma_(w.s1, w.s1, T(1)));
    const T n2 = fma_(w.r2, w.r2, fma_(w.s2, w.s2, T(1)));
    // pa_p = psi^p alpha^p
    T pa1, pa2, pa3;
    if constexpr (sizeof(T) == 8) {
        const T ip = rcp(n1 * n2);
        pa1 = mc_scaled(w.a1, t1 * (ip * n2));
        pa2 = mc_scaled(w.a2, t2 * (ip * n1));
        pa3 = mc_scaled(w.a3, t3);
    } else {
        pa1 = mc_half(t1 * rcp(w.a1 * n1)) * w.a1;
        pa2 = mc_half(t2 * rcp(w.a2 * n2)) * w.a2;
        pa3 = mc_unit(w.a3, t3);
    }
    const T as1 = abs_(w.s1), as2 = abs_(w.s2), as3 = abs_(w.s3);
    // correction strengths c_p = 1/2 |s| (1 - dt |s|) phi alpha = |s| (1 - dt |s|) psi alpha
    const T c1 = (fma_(-dt, as1, T(1)) * as1) * pa1;
    const T c2 = (fma_(-dt, as2, T(1)) * as2) * pa2;
    const T c3 = (fma_(-dt, as3, T(1)) * as3) * pa3;
    // e_p = min(s,0) alpha + c_p ; g_p = max(s,0) alpha - c_p = s alpha - e_p
    const T e1 = fma_(min_(w.s1, T(0)), w.a1, c1);
    const T e2 = fma_(min_(w.s2, T(0)), w.a2, c2);
    const T e3 = fma_(min_(w.s3, T(0)), w.a3, c3);
    const T g1 = fma_(w.s1, w.a1, -e1);
    const T g2 = fma_(w.s2, w.a2, -e2);
    const T g3 = fma_(w.s3, w.a3, -e3);
    Gm[0] = e1 + e2;
    Gm[1] = fma_(e1, w.s1, e2 * w.s2);
    Gm[2] = fma_(e1, w.r1, fma_(e2, w.r2, e3));
    Gp[0] = g1 + g2;
    Gp[1] = fma_(g1, w.s1, g2 * w.s2);
    Gp[2] = fma_(g1, w.r1, fma_(g2, w.r2, g3));
}

// Axisymmetric geometric terms of the divergence (cylindrical coordinates,
// no swirl): d/dt (R, M, N) = -(N, u v, v^2)/r, applied by forward Euler over
// h = dt/2 on one cell in place; hr = h / r.  Used once on each x1-swept row
// before the x2 sweep and once on each x2-swept row after it (the symmetric
// placement keeps the split step stable near the axis up to CFL 1).
template <typename T>
__device__ __forceinline__ void geometric_half_step(Cell<T>& q, T hr)
{
    const T ir = rcp(T(1) + q.R);
    const T u = q.M * ir, v = q.N * ir;
    q.R = fma_(-hr, q.N, q.R);
    q.M = fma_(-hr, u * v, q.M);
    q.N = fma_(-hr, v * v, q.N);
}

// ---------------------------------------------------------------------------
// Analytic boundary data (always evaluated in FP64).
// ---------------------------------------------------------------------------

// Taylor shock-like profile, eq. OurTaylorS with the rotation of Sec. 4.1,
// at domain coordinates (x, y).  The profile is anchored on the path of a
// moving domain: x0 = ta_x0 - x_off, the profile's origin seen from a domain
// that has moved x_off cells (taylor_x0).
__device__ __forceinline__ double taylor_x0(const SimDesc& d, long long x_off)
{
    return d.ta_x0 - (double)x_off;
}
__device__ __forceinline__ void taylor_at(const SimDesc& d, double x0, double x, double y, double t,
                                          double& R, double& M, double& N)
{
    const double xi = (x - x0) * d.ta_cos + (y - d.ta_y0) * d.ta_sin;
    R = -d.ta_amp * tanh((xi - t) / d.ta_w);
    M = R * d.ta_cos;
    N = R * d.ta_sin;
}

// Focused source, eq. hifuBC.  The parts that depend on time only -- the
// ramp envelope and f t, whole and reduced modulo one period -- are evaluated
// once per wavefront and step (source_clock); the parts that depend on the
// row only -- the focusing delay f r^2/(2F), whole and reduced modulo one
// period, and the direction cosines F/h, -r/h with h = sqrt(r^2 + F^2) --
// come from a table filled when the source is set.  The sine's phase is the
// sum of the reduced parts reduced again, in FP64; the packet envelope of eq.
// hifuBC:g, exp(-(f tau / W)^10), takes the whole f tau.  `ap` is the
// aperture in cells during the first stage and -1 (no source row) in the
// second, when the whole side is zero-order extrapolation (Sec. 4.2).
struct SourceClock { double ft_frac, ft, env, ap; };

__device__ __forceinline__ SourceClock source_clock(const SimDesc& d, double t)
{
    SourceClock c;
    const double f = d.sr_freq;
    if (t <= 0.0) {
        c.env = 0.0;
    } else if (t < d.sr_ramp / f) {
        const double s = sin(M_PI * f * t / (2.0 * d.sr_ramp));
        c.env = s * s;
    } else {
        c.env = 1.0;
    }
    c.ft = f * t;
    c.ft_frac = c.ft - floor(c.ft);
    c.ap = t < d.sr_t2 ? d.sr_ap : -1.0;
    return c;
}

template <typename T>
__device__ __forceinline__ void source_at(const SimDesc& d, int j, const SourceClock& sc, T& R, T& M, T& N)
{
    if (!d.src_tab) { R = M = N = T(0); return; }
    // read-only during a step and indexed by a wave-uniform row: through the
    // constant address space these are scalar loads, which do not wait behind
    // the row loads in flight
    typedef const __attribute__((address_space(4))) double* ConstRow;
    const ConstRow e = (ConstRow)(d.src_tab + 4 * (size_t)j);
    double ph = sc.ft_frac + e[0];
    ph -= floor(ph);
    double env = sc.env;
    if (d.sr_env == 1) {
        const double x = (sc.ft + e[3]) / d.sr_W;
        const double x2 = x * x, x4 = x2 * x2, x8 = x4 * x4;
        env = exp(-(x8 * x2));
    }
    T g;
    if constexpr (sizeof(T) == 8) g = (T)(d.sr_amp * env * sin(2.0 * M_PI * ph));
    else g = (T)(d.sr_amp * env) * __sinf((float)(2.0 * M_PI * ph));
    R = g;
    M = g * (T)e[1];
    N = g * (T)e[2];
}

// ---------------------------------------------------------------------------
// Raw buffer access.  The lean path (tiles whose rows are all real rows) reads
// and writes through one buffer resource per field plane covering exactly the
// rows the tile touches: the row goes in the scalar offset, the column in the
// lane's vector offset, so a row costs no vector address arithmetic.  The
// byte count of a resource stays below 2^31; a lane whose vector offset is
// OFF_NONE lies outside it whatever the scalar offset, and the hardware range
// check discards its store.
// ---------------------------------------------------------------------------
using Rsrc = __amdgpu_buffer_rsrc_t;
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int RAW_BUFFER_DWORD3 = 0x00020000;   // raw (unformatted, stride 0) buffer on gfx9-family parts
constexpr int OFF_NONE = (int)0x80000000u;

__device__ __forceinline__ Rsrc make_rsrc(const void* base, int bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, bytes, RAW_BUFFER_DWORD3);
}
__device__ __forceinline__ void bld(Rsrc r, int vo, int so, double& x)
{
    x = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
__device__ __forceinline__ void bld(Rsrc r, int vo, int so, float& x)
{
    x = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ __forceinline__ void bld(Rsrc r, int vo, int so, _Float16& x)
{
    x = __builtin_bit_cast(_Float16, (unsigned short)__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0));
}
__device__ __forceinline__ void bld(Rsrc r, int vo, int so, bf16& x)
{
    x.bits = (uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0);
}
__device__ __forceinline__ void bst(Rsrc r, int vo, int so, double x)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, vo, so, 0);
}
__device__ __forceinline__ void bst(Rsrc r, int vo, int so, float x)
{
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(x), r, vo, so, 0);
}
__device__ __forceinline__ void bst(Rsrc r, int vo, int so, _Float16 x)
{
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, vo, so, 0);
}
__device__ __forceinline__ void bst(Rsrc r, int vo, int so, bf16 x)
{
    __builtin_amdgcn_raw_buffer_store_b16(x.bits, r, vo, so, 0);
}

// ---------------------------------------------------------------------------
// The fused step of one wavefront tile.
// ---------------------------------------------------------------------------

// Rows [r0, r1) of row segment `seg`.  Uniform segments of tile_rows rows, or
// (seg_edge > 0) a first and a last segment of seg_edge rows and seg_mid rows
// in each of the others: the first and last segment of a strip take the
// general path (ghost rows, boundary rows in the source), which costs more
// per row than the lean path, so they are given fewer rows.
__device__ __forceinline__ void seg_bounds(const SimDesc& d, int seg, int& r0, int& r1)
{
    if (d.seg_edge == 0) {
        r0 = seg * d.tile_rows;
        r1 = min(r0 + d.tile_rows, d.ny);
    } else if (seg == 0) {
        r0 = 0;
        r1 = d.seg_edge;
    } else if (seg == d.segs - 1) {
        r0 = d.ny - d.seg_edge;
        r1 = d.ny;
    } else {
        r0 = d.seg_edge + (seg - 1) * d.seg_mid;
        r1 = min(r0 + d.seg_mid, d.ny - d.seg_edge);
    }
}

// State one lane carries from one x2 row to the next.  Every entry is
// consumed by the very next row, so two copies alternated by a two-row
// unrolled loop need no register moves.
template <typename T> struct Carry {
    Cell<T> q; T u, v;      // last x1-swept row Q*_v pushed, and its velocities
    Wave<T> w;              // x2 interface v - 1/2
    T dlo[3];               // upwind values t of x2 interface v-3/2 for v-1/2 (wave_cross)
    Cell<T> part;           // Q*_{v-1} - dt Gp_{v-3/2}: row v-1 awaiting its upper flux
    Cell<T> qs; T us, vs;   // x2-swept row v-2 awaiting its source, and its velocities
    T ub, vb;               // velocities of x2-swept row v-3
};

template <typename T>
__device__ __forceinline__ void carry_zero(Carry<T>& c)
{
    const T z = T(0);
    c.q = {z, z, z}; c.u = z; c.v = z;
    c.w = {z, z, z, z, z, z, z, z};
    c.dlo[0] = c.dlo[1] = c.dlo[2] = z;
    c.part = {z, z, z};
    c.qs = {z, z, z}; c.us = z; c.vs = z;
    c.ub = z; c.vb = z;
}

template <bool B> struct Flag { static constexpr bool value = B; };

// Issue priority from progress.  Among waves of equal priority the SIMD
// arbiter favours the oldest, so the waves that start together on a SIMD
// would finish one after another and leave it with one or two waves (and a
// fraction of its issue rate) for the last part of the step.  A wave lowers
// its priority as it advances -- 3 for the first half of its rows, 2 to three
// quarters, 1 to nine tenths, 0 after -- so the waves of a SIMD stay level and
// keep it full until they all finish.  Priority changes timing only.
struct Pace {
    int b1, b2, b3;          // row counts at which the priority drops
    int level;
    __device__ __forceinline__ explicit Pace(int total)
        : b1(total / 2), b2((3 * total) / 4), b3((9 * total) / 10), level(3)
    {
        __builtin_amdgcn_s_setprio(3);
    }
    __device__ __forceinline__ void update(int done)
    {
        const int want = done < b1 ? 3 : done < b2 ? 2 : done < b3 ? 1 : 0;
        if (want != level) {
            level = want;
            if (want == 2) __builtin_amdgcn_s_setprio(2);
            else if (want == 1) __builtin_amdgcn_s_setprio(1);
            else __builtin_amdgcn_s_setprio(0);
        }
    }
};

// One wavefront tile of the fused step.
//   EDGE: the strip touches a non-periodic x side (ghost columns and x
//         overrides needed); interior strips compile without that logic.
//   LEAN: every row the tile touches (three below the segment to three above)
//         is a real row: no ghost rows, no periodic wrap, no boundary rows in
//         the source, and the main loop has no branches at all.  Other
//         segments take the general path.  Both paths evaluate every cell
//         with the same arithmetic, so results do not depend on the path.
template <typename S, typename T, int AXI, bool EDGE, bool LEAN>
__device__ __forceinline__ void march(const SimDesc& d, int strip, int seg, const Attempt& at)
{
    using C = Codec<S, T>;
    const int lane = threadIdx.x & (WAVE - 1);
    const int nx = d.nx, ny = d.ny;
    const int c0 = strip * OUTW;
    const int col = c0 - HALO + lane;
    int r0, r1;
    seg_bounds(d, seg, r0, r1);
    const double tn = at.t;
    const double tx0 = taylor_x0(d, at.x_off);
    const T dt = (T)at.dt;
    const int cur = at.cur;
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
    const T hdt = T(0.5) * dt;
    const float sc0 = d.scale[0], sc1 = d.scale[1], sc2 = d.scale[2];
    const float is0 = d.inv_scale[0], is1 = d.inv_scale[1], is2 = d.inv_scale[2];
    SourceClock src_clk = {0.0, 0.0, 0.0, -1.0}; // focused source at this step's time
    if (EDGE && d.bc[0] == BC_SOURCE) src_clk = source_clock(d, tn);

    // ---- where this lane's Q^n comes from (x boundary rule) ----
    const bool incol = col >= 0 && col < nx;
    int scol = col;
    T msign = T(1);
    int xkind = 0;          // 0: load; 1: Taylor; 2: focused source (else extrapolate)
    if (perx) {
        scol = ((col % nx) + nx) % nx;
    } else if (EDGE) {
        if (col < 0) {
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
    }
    const bool real_col = perx || incol;
    const bool out_lane = lane >= HALO && lane < WAVE - HALO && col < nx;
    const bool ghost_lo = EDGE && !perx && col == 0;        // left neighbour of this output cell is a ghost
    const bool ghost_hi = EDGE && !perx && col == nx - 1;   // right neighbour is a ghost

    // Per-lane CFL bookkeeping, x1 and x2 interfaces apart; which lanes hold
    // real interfaces is applied once at the end (maxima and minima are
    // indifferent to order and repetition).
    Cfl<T> xacc, yacc;

    // ---- lean path: buffer resources over rows rs .. vlast ----
    const int rs = r0 - HALO;
    const int vlast = r1 + HALO - 1;
    const int pb = d.pitch * (int)sizeof(S);
    const int tile_bytes = (vlast - rs + 1) * pb;
    const size_t rso = (size_t)(LEAN ? rs : 0) * pitch;
    const Rsrc iR = make_rsrc(inR + rso, tile_bytes), iM = make_rsrc(inM + rso, tile_bytes),
               iN = make_rsrc(inN + rso, tile_bytes);
    const Rsrc oR = make_rsrc(outR + rso, tile_bytes), oM = make_rsrc(outM + rso, tile_bytes),
               oN = make_rsrc(outN + rso, tile_bytes);
    const int vld = scol * (int)sizeof(S);
    const int vst = out_lane ? col * (int)sizeof(S) : OFF_NONE;

    // ---- raw loads of one row of Q^n (real row index) ----
    auto load_row = [&](int vr, S& a, S& b, S& c) {
        if constexpr (LEAN) {
            const int so = (min(vr, vlast) - rs) * pb;     // rows past the tile: harmless repeat
            bld(iR, vld, so, a);
            bld(iM, vld, so, b);
            bld(iN, vld, so, c);
        } else {
            const size_t o = (size_t)vr * pitch + (size_t)scol;
            a = inR[o];
            b = inM[o];
            c = inN[o];
        }
    };

    // ---- x1 sweep of one row (lane-parallel) ----
    // GHOST: a ghost row of a side with analytic data (its Q^n analytic, the
    // x side rules applied to it as to a real row); its interfaces do not
    // enter the CFL maximum and it takes no geometric term.
    auto xsweep_core = [&](auto ghost, int vr, Cell<T> q) -> Cell<T> {
        constexpr bool GHOST = decltype(ghost)::value;
        if (EDGE) {
            q.M *= msign;
            if (xkind == 1) {
                double R, M, N;
                taylor_at(d, tx0, col + 0.5, vr + 0.5, tn, R, M, N);
                q.R = (T)R; q.M = (T)M; q.N = (T)N;
            } else if (xkind == 2) {
                const bool row_ok = !GHOST || (unsigned)vr < (unsigned)ny;
                if (row_ok && vr + 0.5 <= src_clk.ap) source_at<T>(d, vr, src_clk, q.R, q.M, q.N);
            }
        }
        const T RL = from_lo(q.R);
        const T Sr = RL + q.R;
        T irho, h;
        rcp_pair(T(1) + q.R, T(2) + Sr, irho, h);
        const T u = q.M * irho, v = q.N * irho;
        const T ML = from_lo(q.M), NL = from_lo(q.N);
        const T uL = from_lo(u), vL = from_lo(v);
        Wave<T> w;
        T D;
        const T spd = roe_sh(RL, ML, NL, uL, vL, q.R, q.M, q.N, u, v, beta, Sr, h, w, D);
        if constexpr (!GHOST) xacc.add(spd, D);
        // waves of the interface to the right -> products with it; the lane
        // to the left supplies the products with the interface below
        Wave<T> wr;
        wr.a1 = from_hi(w.a1); wr.s1 = from_hi(w.s1); wr.r1 = from_hi(w.r1);
        wr.a2 = from_hi(w.a2); wr.s2 = from_hi(w.s2); wr.r2 = from_hi(w.r2);
        wr.a3 = from_hi(w.a3);
        T tup[3], dhi[3], dlo[3];
        wave_cross(w, wr, tup, dhi);
        dlo[0] = from_lo(tup[0]); dlo[1] = from_lo(tup[1]); dlo[2] = from_lo(tup[2]);
        T Gm[3], Gp[3];
        hr_split(w, dlo, dhi, dt, Gm, Gp);
        const T g0 = from_hi(Gm[0]), g1 = from_hi(Gm[1]), g2 = from_hi(Gm[2]);
        Cell<T> o2;
        o2.R = fma_(-dt, g0 + Gp[0], q.R);
        o2.M = fma_(-dt, g1 + Gp[1], q.M);
        o2.N = fma_(-dt, g2 + Gp[2], q.N);
        if constexpr (AXI && !GHOST) geometric_half_step(o2, hdt * rinv_at<T>(d, vr));
        return o2;
    };
    auto xsweep = [&](int vr, S ra, S rb, S rc) -> Cell<T> {
        Cell<T> q;
        q.R = C::ld(ra, sc0);
        q.M = C::ld(rb, sc1);
        q.N = C::ld(rc, sc2);
        return xsweep_core(Flag<false>{}, vr, q);
    };
    // Q* of ghost row vr of a side with analytic (Taylor) data: the x1 sweep
    // of the analytic Q^n of that row, so that the x2 sweep meets ghost values
    // that went through the same first fractional step as the interior
    auto xsweep_taylor_ghost = [&](int vr) -> Cell<T> {
        double R, M, N;
        taylor_at(d, tx0, scol + 0.5, vr + 0.5, tn, R, M, N);
        return xsweep_core(Flag<true>{}, vr, Cell<T>{(T)R, (T)M, (T)N});
    };

    // analytic (Taylor) velocities of a ghost cell
    auto taylor_uv = [&](double x, double y, T& uu, T& vv) {
        double R, M, N;
        taylor_at(d, tx0, x, y, tn, R, M, N);
        uu = (T)(M / (1.0 + R));
        vv = (T)(N / (1.0 + R));
    };

    const int vfirst = rs;

    // ---- push x1-swept row v through the x2 sweep and the source ----
    // src (lean path): whether row v - 3 is an output row of this tile.
    auto push = [&](const Cell<T>& q, int v, const Carry<T>& in, Carry<T>& out, auto src) {
        const T Sr = in.q.R + q.R;
        T irho, h;
        rcp_pair(T(1) + q.R, T(2) + Sr, irho, h);
        const T u = q.M * irho, vv = q.N * irho;
        // x2 interface v-1/2 between rows v-1 (low) and v (high); normal = N
        Wave<T> wA;
        T D;
        const T spd = roe_sh(in.q.R, in.q.N, in.q.M, in.v, in.u, q.R, q.N, q.M, vv, u, beta, Sr, h, wA, D);
        if (LEAN || (v > vfirst && (pery || (v >= 0 && v <= ny)))) yacc.add(spd, D);
        T tup[3], dhi[3];
        wave_cross(in.w, wA, tup, dhi);
        // limited correction and fluctuations at v-3/2
        T Gm[3], Gp[3];
        hr_split(in.w, in.dlo, dhi, dt, Gm, Gp);
        // row v-2 completes; row v-1 receives its lower flux (split-local order R, N, M)
        Cell<T> qn;
        qn.R = fma_(-dt, Gm[0], in.part.R);
        qn.N = fma_(-dt, Gm[1], in.part.N);
        qn.M = fma_(-dt, Gm[2], in.part.M);
        out.part.R = fma_(-dt, Gp[0], in.q.R);
        out.part.N = fma_(-dt, Gp[1], in.q.N);
        out.part.M = fma_(-dt, Gp[2], in.q.M);
        if constexpr (AXI) geometric_half_step(qn, hdt * rinv_at<T>(d, v - 2));
        const T irn = rcp(T(1) + qn.R);
        const T un = qn.M * irn, vn = qn.N * irn;
        // source of row j = v-3 (x2-swept rows j-1, j, j+1), then store
        const int j = v - 3;
        bool do_src;
        if constexpr (LEAN) do_src = decltype(src)::value;
        else do_src = j >= r0 && j < r1;
        if (do_src) {
            T uxl = from_lo(in.us), vxl = from_lo(in.vs);
            T uxr = from_hi(in.us), vxr = from_hi(in.vs);
            T ubl = in.ub, vbl = in.vb, uab = un, vab = vn;
            if (EDGE) {
                if (ghost_lo) {
                    const int b = d.bc[0];
                    if (b == BC_REFLECT) { uxl = -in.us; vxl = in.vs; }
                    else if (b == BC_TAYLOR) taylor_uv(-0.5, j + 0.5, uxl, vxl);
                    else if (b == BC_SOURCE && j + 0.5 <= src_clk.ap) {
                        T R, M, N;
                        source_at<T>(d, j, src_clk, R, M, N);
                        const T ir = rcp(T(1) + R);
                        uxl = M * ir; vxl = N * ir;
                    } else { uxl = in.us; vxl = in.vs; }
                }
                if (ghost_hi) {
                    const int b = d.bc[1];
                    if (b == BC_REFLECT) { uxr = -in.us; vxr = in.vs; }
                    else if (b == BC_TAYLOR) taylor_uv(nx + 0.5, j + 0.5, uxr, vxr);
                    else { uxr = in.us; vxr = in.vs; }
                }
            }
            if constexpr (!LEAN) {
                if (!pery && j == 0) {
                    const int b = d.bc[2];
                    if (b == BC_REFLECT) { ubl = in.us; vbl = -in.vs; }
                    else if (b == BC_TAYLOR) taylor_uv(col + 0.5, -0.5, ubl, vbl);
                    else { ubl = in.us; vbl = in.vs; }
                }
                if (!pery && j == ny - 1) {
                    const int b = d.bc[3];
                    if (b == BC_REFLECT) { uab = in.us; vab = -in.vs; }
                    else if (b == BC_TAYLOR) taylor_uv(col + 0.5, ny + 0.5, uab, vab);
                    else { uab = in.us; vab = in.vs; }
                }
            }
            const T lapu = fma_(T(-4), in.us, (uxl + uxr) + (ubl + uab));
            const T lapv = fma_(T(-4), in.vs, (vxl + vxr) + (vbl + vab));
            const T oRv = in.qs.R;
            T oMv, oNv;
            if constexpr (AXI) {
                // cylindrical vector Laplacian: + (1/r) d/dr of each velocity, - v/r^2
                const T ir = rinv_at<T>(d, j);
                const T dur = T(0.5) * (uab - ubl), dvr = T(0.5) * (vab - vbl);
                const T k = dt * delta;
                oMv = fma_(k, fma_(dur, ir, lapu), in.qs.M);
                oNv = fma_(k, fma_(-in.vs, ir * ir, fma_(dvr, ir, lapv)), in.qs.N);
            } else {
                const T k = dt * delta;
                oMv = fma_(k, lapu, in.qs.M);
                oNv = fma_(k, lapv, in.qs.N);
            }
            if constexpr (LEAN) {
                const int so = (j - rs) * pb;
                bst(oR, vst, so, C::st(oRv, is0));
                bst(oM, vst, so, C::st(oMv, is1));
                bst(oN, vst, so, C::st(oNv, is2));
            } else if (out_lane) {
                const size_t o = (size_t)j * pitch + (size_t)col;
                outR[o] = C::st(oRv, is0);
                outM[o] = C::st(oMv, is1);
                outN[o] = C::st(oNv, is2);
            }
        }
        out.q = q; out.u = u; out.v = vv;
        out.w = wA;
        out.dlo[0] = tup[0]; out.dlo[1] = tup[1]; out.dlo[2] = tup[2];
        out.qs = qn; out.us = un; out.vs = vn;
        out.ub = in.us; out.vb = in.vs;
    };

    Carry<T> A, B;
    carry_zero(A);

    if constexpr (LEAN) {
        // two rows of Q^n in flight ahead of the one being swept
        S a0, b0, e0, a1, b1, e1;
        load_row(rs, a0, b0, e0);
        load_row(rs + 1, a1, b1, e1);
        int v = rs;
        // six warm-up rows, no source; the lowest x2 interface borders the
        // zeroed carry and is dropped from the CFL maximum
#pragma unroll 1
        for (int k = 0; k < 3; ++k, v += 2) {
            S a = a0, b = b0, e = e0;
            load_row(v + 2, a0, b0, e0);
            push(xsweep(v, a, b, e), v, A, B, Flag<false>{});
            if (k == 0) yacc = Cfl<T>();
            a = a1; b = b1; e = e1;
            load_row(v + 3, a1, b1, e1);
            push(xsweep(v + 1, a, b, e), v + 1, B, A, Flag<false>{});
        }
        // output rows r0 .. r1-1 (pushed rows r0+3 .. r1+2)
        Pace pace(vlast - rs + 1);
#pragma unroll 1
        for (; v + 1 <= vlast; v += 2) {
            pace.update(v - rs);
            S a = a0, b = b0, e = e0;
            load_row(v + 2, a0, b0, e0);
            push(xsweep(v, a, b, e), v, A, B, Flag<true>{});
            a = a1; b = b1; e = e1;
            load_row(v + 3, a1, b1, e1);
            push(xsweep(v + 1, a, b, e), v + 1, B, A, Flag<true>{});
        }
        if (v <= vlast) push(xsweep(v, a0, b0, e0), v, A, B, Flag<true>{});
    } else {
        carry_zero(B);
        Cell<T> stash = {T(0), T(0), T(0)};    // x1-swept row ny-2 (reflecting top ghost)
        auto keep = [&](const Cell<T>& q, int v) { if (v == ny - 2) stash = q; };
        const Flag<true> any;

        int v = vfirst;
        if (!pery && r0 == 0) {
            // bottom side: the ghost rows of the x1-swept state need rows 0 and 1 first
            S a0, b0, c0_, a1, b1, c1;
            load_row(0, a0, b0, c0_);
            load_row(1, a1, b1, c1);
            const Cell<T> q0 = xsweep(0, a0, b0, c0_);
            const Cell<T> q1 = xsweep(1, a1, b1, c1);
            const int b = d.bc[2];
            Cell<T> g[HALO];
            for (int k = HALO; k >= 1; --k) {       // rows -3, -2, -1
                Cell<T> q;
                if (b == BC_TAYLOR) {
                    q = xsweep_taylor_ghost(-k);
                } else if (b == BC_REFLECT) {
                    q = (k == 1) ? q0 : q1;
                    q.N = -q.N;
                } else {
                    q = q0;
                }
                g[k - 1] = q;
            }
            push(g[2], -3, A, B, any);
            push(g[1], -2, B, A, any);
            push(g[0], -1, A, B, any);
            push(q0, 0, B, A, any); keep(q0, 0);
            push(q1, 1, A, B, any); keep(q1, 1);
            A = B;
            v = 2;
        }
        // real rows, two per iteration, loads one row ahead
        const int vreal = pery ? vlast : min(vlast, ny - 1);
        auto wrap = [&](int vv) { return pery ? ((vv % ny) + ny) % ny : vv; };
        if (v <= vreal) {
            S na, nb, nc;
            load_row(wrap(v), na, nb, nc);
            Pace pace(vlast - vfirst + 1);
            for (; v + 1 <= vreal; v += 2) {
                pace.update(v - vfirst);
                S a = na, b = nb, c = nc;
                load_row(wrap(v + 1), na, nb, nc);
                const Cell<T> q = xsweep(wrap(v), a, b, c);
                push(q, v, A, B, any); keep(q, v);
                a = na; b = nb; c = nc;
                if (v + 2 <= vreal) load_row(wrap(v + 2), na, nb, nc);
                const Cell<T> q2 = xsweep(wrap(v + 1), a, b, c);
                push(q2, v + 1, B, A, any); keep(q2, v + 1);
            }
            if (v <= vreal) {
                const Cell<T> q = xsweep(wrap(v), na, nb, nc);
                push(q, v, A, B, any); keep(q, v);
                A = B;
                ++v;
            }
        }
        // ghost rows above a non-periodic top side
        for (; v <= vlast; ++v) {
            const int b = d.bc[3];
            Cell<T> q = A.q;                           // zero-order extrapolation of Q*_{ny-1}
            if (b == BC_TAYLOR) {
                q = xsweep_taylor_ghost(v);
            } else if (b == BC_REFLECT) {
                if (v == ny) { q = A.q; q.N = -q.N; }
                else if (v == ny + 1) { q = stash; q.N = -q.N; }
            }
            push(q, v, A, B, any);
            A = B;
        }
    }

    // ---- wave reduction of the CFL entries over real interfaces ----
    // x1 interface of lane l: between columns col-1 and col (lane 0 has no
    // left neighbour); x2 interfaces: lanes whose x1-swept values are exact.
    const bool cnt_x = lane >= 1 && (perx || (col >= 0 && col <= nx));
    const bool cnt_y = lane >= 2 && lane <= WAVE - 3 && real_col;
    T sx, sy;
    bool hx, hy, fx, fy;
    xacc.finish(cnt_x, sx, hx, fx);
    yacc.finish(cnt_y, sy, hy, fy);
    T m = max_(sx, sy);
    for (int off = 32; off >= 1; off >>= 1) m = max_(m, perm(m, lane ^ off));
    const bool anyh = __any(hx || hy);
    const bool anyf = __any(fx || fy);
    if (lane == 0) {
        atomicMax(at.smax, (unsigned long long)__double_as_longlong(cfl_speed<T>(m)));
        const unsigned fl = (anyh ? FLAG_NONHYP : 0u) | (anyf ? FLAG_NONFINITE : 0u);
        if (fl) atomicOr(at.flags, fl);
    }
}

// Interior strips (no ghost column, no x override) take the EDGE = false
// variant; segments whose rows are all real rows take the lean path.
template <typename S, typename T, int AXI>
__device__ __forceinline__ void march_tile(const SimDesc& d, int strip, int seg, const Attempt& at)
{
    const int c0 = strip * OUTW;
    const bool interior = d.bc[0] == BC_PERIODIC || (c0 - HALO >= 0 && c0 + OUTW + HALO - 1 <= d.nx - 1);
    int r0, r1;
    seg_bounds(d, seg, r0, r1);
    const bool lean = r0 >= HALO && r1 + HALO <= d.ny &&
                      (long long)(r1 - r0 + 2 * HALO) * d.pitch * (long long)sizeof(S) < (1ll << 31);
    if (interior) {
        if (lean) march<S, T, AXI, false, true>(d, strip, seg, at);
        else march<S, T, AXI, false, false>(d, strip, seg, at);
    } else {
        if (lean) march<S, T, AXI, true, true>(d, strip, seg, at);
        else march<S, T, AXI, true, false>(d, strip, seg, at);
    }
}

}  // namespace fvna
