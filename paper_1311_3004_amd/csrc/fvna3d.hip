// fvna3d.hip -- the three-dimensional step (the paper's equations in three
// dimensions, which Sec. 5 says they allow) and its C ABI (include/fvna3d.h).
//
// State (R, M1, M2, M3) = (rho'/rho0, rho u1/(rho0 c0), ...), dimensionless
// with the mesh spacing as length unit.  One step: x1 sweep -> x2 sweep ->
// x3 sweep -> source (Godunov splitting, each sweep the high-resolution Roe
// scheme of Secs. 3.1-3.2 with a second passive shear wave), then the CFL
// decision of the opening of Sec. 4, all on the device:
//   k3_sweep12  x1 and x2 sweeps of one z-plane tile: lanes along x1 (the
//               left cell, the neighbour waves and the right flux over DPP
//               lane shifts, every x1 interface solved once), a register
//               march along x2 (every x2 interface solved once);
//   k3_sweep3   x3 sweep: a register march along x3, one lane per column;
//   k3_source   7-point Laplacian of each velocity component: x3 neighbours
//               carried in registers, x1 neighbours over DPP, x2 neighbours
//               loaded;
//   k3_ctrl     accept or reject (control_attempt), one thread.
// Three state buffers X0, X1, X2 and the device clock's cur = c.  The source
// leaves the density as the x3 sweep made it, so a state keeps its density
// and its momenta in different buffers: density in X[1-c], momenta in X[-c]
// (indices modulo 3).  The x1-x2 sweep writes all four fields to the third
// buffer X[2-c]; the x3 sweep writes its density into X[-c] and its momenta
// into X[1-c] (planes the current state does not use); the source writes the
// momenta into X[2-c] and no density.  An accepted step advances c by one,
// which makes exactly these the new state's buffers; a rejected one leaves
// the current state untouched.  Steps are replayed from a captured HIP graph;
// the host waits once per fvna3_step call.
// Ghost values follow the side rule of their axis applied to the state of
// the stage that needs them (Q^n for x1, the x1-swept state for x2, the
// x2-swept state for x3, the x3-swept state for the source).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "../../include/fvna3d.h"
#include "fvna_device.hpp"
#include "fvna_step.hpp"

using namespace fvna;

namespace {

constexpr int HALO12 = 2;                      // x1 stencil: two interfaces each side
constexpr int OUT12 = WAVE - 2 * HALO12;       // 60 output columns per x1-x2 wavefront

// Buffer roles for clock cur = c (see the file's header).
__device__ __forceinline__ int buf_rho(int c) { return c == 0 ? 1 : c == 1 ? 0 : 2; }
__device__ __forceinline__ int buf_mom(int c) { return c == 0 ? 0 : c == 1 ? 2 : 1; }
__device__ __forceinline__ int buf_x12(int c) { return c == 0 ? 2 : c == 1 ? 1 : 0; }

struct Desc3 {
    int n[3];                  // nx, ny, nz
    int pitch;                 // elements per x1 row (padded to 256 bytes)
    int strips12, segs12, rows12;   // x1-x2 tiles: 60-column strips, row segments of rows12
    int tailw12, tailp12, tailk12;  // packed tail (tailw12 > 0): the last nx mod 60 columns of
                                    // tailp12 planes per wavefront, lanes in segments of
                                    // tailw12 = that + 4; tailk12 plane groups
    int strips64, segs3, planes3;   // x3 tiles: 64-column strips, z segments of planes3
    int segs4, planes4;             // source tiles: z segments of planes4 (blocks of four rows)
    long long plane;           // elements per field = pitch * ny * nz
    int bc[6];
    int fixed_dt, max_retries;
    double beta, delta;        // delta~ = delta / (c0 dx)
    double cfl_target, cfl_max;
    void* buf[3];
    Clock* clk;
};

// Index m along axis a mapped to a stored index by the side rule of that
// axis; *neg is set when the momentum normal to the axis is mirrored.
__device__ __forceinline__ int side_map(const Desc3& d, int a, int m, bool& neg)
{
    const int n = d.n[a];
    neg = false;
    if (m < 0) {
        const int b = d.bc[2 * a];
        if (b == FVNA_BC_PERIODIC) m += n;
        else if (b == FVNA_BC_REFLECT) { m = -m - 1; neg = true; }
        else m = 0;
    } else if (m >= n) {
        const int b = d.bc[2 * a + 1];
        if (b == FVNA_BC_PERIODIC) m -= n;
        else if (b == FVNA_BC_REFLECT) { m = 2 * n - m - 1; neg = true; }
        else m = n - 1;
    }
    return min(max(m, 0), n - 1);
}

// ---------------------------------------------------------------------------
// Roe solver of one interface with two tangential momenta (a, b).
// ---------------------------------------------------------------------------
template <typename T> struct W4 { T s1, s2, s3, a1, a2, a3, a4, r1a, r2a, r1b, r2b; };
template <typename T> struct Q4 { T R, n, a, b; };

// Eigenvalues w + c, w - c, w, w; acoustic eigenvectors (1, s, ra, rb) with
// ra = za (s - 2 zn)/(Zbar^1 (s - w)) (likewise rb), shear eigenvectors
// (0, 0, 1, 0) and (0, 0, 0, 1); strengths from sum_p alpha^p r^p = Q_R - Q_L.
// The means are carried as sums of the two sides (every factor 2 cancels).
// Returns the interface's largest |s| in the form Cfl<T> reduces (FP32 as an
// excess over 1) and the discriminant in D.
// h = 1/(2 + L.R + R.R) comes from the caller (rcp_pair).
template <typename T>
__device__ __forceinline__ T roe4(const Q4<T>& L, T unL, T uaL, T ubL, const Q4<T>& R, T unR, T uaR, T ubR,
                                  T beta, T h, W4<T>& w, T& D)
{
    const T Sr = L.R + R.R, Sn = unL + unR, Sa = uaL + uaR, Sb = ubL + ubR;
    const T wv = Sn * h;
    const T D1 = fma_(wv, wv - Sn, (beta - T(1)) * Sr);
    D = T(1) + D1;
    T c, ic;
    sqrt_pair(D, c, ic);
    T spd;
    if constexpr (sizeof(T) == 8) spd = c + abs_(wv);
    else spd = fma_(D1, rcp(T(1) + c), abs_(wv));
    w.s1 = wv + c;
    w.s2 = wv - c;
    w.s3 = wv;
    const T hic = h * ic;
    const T ka = Sa * hic, kb = Sb * hic;
    const T e1 = w.s1 - Sn, e2 = w.s2 - Sn;
    w.r1a = ka * e1;
    w.r2a = -ka * e2;
    w.r1b = kb * e1;
    w.r2b = -kb * e2;
    const T d1 = R.R - L.R, d2 = R.n - L.n, d3 = R.a - L.a, d4 = R.b - L.b;
    w.a1 = T(0.5) * ic * fma_(-w.s2, d1, d2);
    w.a2 = d1 - w.a1;
    w.a3 = fma_(-w.a2, w.r2a, fma_(-w.a1, w.r1a, d3));
    w.a4 = fma_(-w.a2, w.r2b, fma_(-w.a1, w.r1b, d4));
    return spd;
}

// Upwind values of two neighbouring interfaces x (below) and y (above) for
// each other, as wave_cross in two dimensions: tx = alpha_x X for y, ty =
// alpha_y X for x, X = r^p_x . r^p_y for the acoustic families (entries 0, 1);
// entries 2, 3: the shear strengths alpha^3, alpha^4 (X = 1).
template <typename T>
__device__ __forceinline__ void cross4(const W4<T>& x, const W4<T>& y, T tx[4], T ty[4])
{
    const T x1 = fma_(x.r1b, y.r1b, fma_(x.r1a, y.r1a, fma_(x.s1, y.s1, T(1))));
    const T x2 = fma_(x.r2b, y.r2b, fma_(x.r2a, y.r2a, fma_(x.s2, y.s2, T(1))));
    tx[0] = x.a1 * x1; tx[1] = x.a2 * x2; tx[2] = x.a3; tx[3] = x.a4;
    ty[0] = y.a1 * x1; ty[1] = y.a2 * x2; ty[2] = y.a3; ty[3] = y.a4;
}

// Fluctuations plus limited corrections of one interface (eqs. fluc:m,
// fluc:p, limiter, fv-hr): Gm = A^- dQ + F~ for the cell on the low side,
// Gp = A^+ dQ - F~ for the cell on the high side.  lo/hi: upwind values t of
// the interface below/above (cross4).  The upwind interface is the one below
// for s >= 0.  The limited products psi alpha as in two dimensions (hr_split):
// FP64 from u = t / n with one reciprocal of n1 n2, FP32 from
// theta = t / (alpha n).
template <typename T>
__device__ __forceinline__ void hr_split4(const W4<T>& w, const T lo[4], const T hi[4], T dt, T Gm[4], T Gp[4])
{
    const bool n1 = w.s1 < T(0), n2 = w.s2 < T(0), n3 = w.s3 < T(0);
    const T t1 = n1 ? hi[0] : lo[0], t2 = n2 ? hi[1] : lo[1];
    const T t3 = n3 ? hi[2] : lo[2], t4 = n3 ? hi[3] : lo[3];
    const T q1 = fma_(w.r1b, w.r1b, fma_(w.r1a, w.r1a, fma_(w.s1, w.s1, T(1))));
    const T q2 = fma_(w.r2b, w.r2b, fma_(w.r2a, w.r2a, fma_(w.s2, w.s2, T(1))));
    T pa1, pa2, pa3, pa4;
    if constexpr (sizeof(T) == 8) {
        const T ip = rcp(q1 * q2);
        pa1 = mc_scaled(w.a1, t1 * (ip * q2));
        pa2 = mc_scaled(w.a2, t2 * (ip * q1));
        pa3 = mc_scaled(w.a3, t3);
        pa4 = mc_scaled(w.a4, t4);
    } else {
        pa1 = mc_half(t1 * rcp(w.a1 * q1)) * w.a1;
        pa2 = mc_half(t2 * rcp(w.a2 * q2)) * w.a2;
        pa3 = mc_unit(w.a3, t3);
        pa4 = mc_unit(w.a4, t4);
    }
    const T as1 = abs_(w.s1), as2 = abs_(w.s2), as3 = abs_(w.s3);
    const T f1 = fma_(-dt, as1, T(1)) * as1, f2 = fma_(-dt, as2, T(1)) * as2, f3 = fma_(-dt, as3, T(1)) * as3;
    const T c1 = f1 * pa1, c2 = f2 * pa2, c3 = f3 * pa3, c4 = f3 * pa4;
    const T m3 = min_(w.s3, T(0));
    const T e1 = fma_(min_(w.s1, T(0)), w.a1, c1);
    const T e2 = fma_(min_(w.s2, T(0)), w.a2, c2);
    const T e3 = fma_(m3, w.a3, c3);
    const T e4 = fma_(m3, w.a4, c4);
    const T g1 = fma_(w.s1, w.a1, -e1);
    const T g2 = fma_(w.s2, w.a2, -e2);
    const T g3 = fma_(w.s3, w.a3, -e3);
    const T g4 = fma_(w.s3, w.a4, -e4);
    Gm[0] = e1 + e2;
    Gm[1] = fma_(e1, w.s1, e2 * w.s2);
    Gm[2] = fma_(e1, w.r1a, fma_(e2, w.r2a, e3));
    Gm[3] = fma_(e1, w.r1b, fma_(e2, w.r2b, e4));
    Gp[0] = g1 + g2;
    Gp[1] = fma_(g1, w.s1, g2 * w.s2);
    Gp[2] = fma_(g1, w.r1a, fma_(g2, w.r2a, g3));
    Gp[3] = fma_(g1, w.r1b, fma_(g2, w.r2b, g4));
}

// State carried by a register march from one cell of the marching axis to
// the next (split-local components: R, normal, tangential a, tangential b).
template <typename T> struct March4 {
    Q4<T> q; T un, ua, ub;     // last cell pushed and its velocities
    W4<T> w;                   // interface below it
    T lo[4];                   // upwind values t of the interface below it for it (cross4)
    Q4<T> part;                // previous cell minus dt Gp of its lower interface (awaiting its upper flux)
};

template <typename T>
__device__ __forceinline__ void march_zero(March4<T>& m)
{
    const T z = T(0);
    m.q = {z, z, z, z};
    m.un = m.ua = m.ub = z;
    m.w = {z, z, z, z, z, z, z, z, z, z, z};
    m.lo[0] = m.lo[1] = m.lo[2] = m.lo[3] = z;
    m.part = {z, z, z, z};
}

// Push cell v (split-local q) through a march: solve interface v - 1/2,
// correct interface v - 3/2, and return cell v - 2 completed in `done`.
// Adds the speed of interface v - 1/2 to acc when `count`.
template <typename T>
__device__ __forceinline__ void march_push(const Q4<T>& q, const March4<T>& in, March4<T>& out, T beta, T dt,
                                           bool count, Cfl<T>& acc, Q4<T>& done)
{
    T ir, h;
    rcp_pair(T(1) + q.R, T(2) + (in.q.R + q.R), ir, h);
    const T un = q.n * ir, ua = q.a * ir, ub = q.b * ir;
    W4<T> wA;
    T D;
    const T spd = roe4(in.q, in.un, in.ua, in.ub, q, un, ua, ub, beta, h, wA, D);
    if (count) acc.add(spd, D);
    T tup[4], hi[4];
    cross4(in.w, wA, tup, hi);
    T Gm[4], Gp[4];
    hr_split4(in.w, in.lo, hi, dt, Gm, Gp);
    done.R = fma_(-dt, Gm[0], in.part.R);
    done.n = fma_(-dt, Gm[1], in.part.n);
    done.a = fma_(-dt, Gm[2], in.part.a);
    done.b = fma_(-dt, Gm[3], in.part.b);
    out.part.R = fma_(-dt, Gp[0], in.q.R);
    out.part.n = fma_(-dt, Gp[1], in.q.n);
    out.part.a = fma_(-dt, Gp[2], in.q.a);
    out.part.b = fma_(-dt, Gp[3], in.q.b);
    out.q = q;
    out.un = un; out.ua = ua; out.ub = ub;
    out.w = wA;
    out.lo[0] = tup[0];
    out.lo[1] = tup[1];
    out.lo[2] = tup[2];
    out.lo[3] = tup[3];
}

// Fold a lane's CFL bookkeeping into the clock (one atomic per wavefront).
template <typename T>
__device__ __forceinline__ void cfl_commit(const Desc3& d, const Cfl<T>& acc, bool counted)
{
    T m;
    bool nh, nf;
    acc.finish(counted, m, nh, nf);
    const int lane = threadIdx.x & (WAVE - 1);
    for (int off = 32; off >= 1; off >>= 1) m = max_(m, perm(m, lane ^ off));
    const bool anyh = __any(nh), anyf = __any(nf);
    if (lane == 0) {
        atomicMax(&d.clk->smax_bits, (unsigned long long)__double_as_longlong(cfl_speed<T>(m)));
        const unsigned fl = (anyh ? FLAG_NONHYP : 0u) | (anyf ? FLAG_NONFINITE : 0u);
        if (fl) atomicOr(&d.clk->flags, fl);
    }
}

__device__ __forceinline__ bool step_owed(const Clock* c, int force)
{
    return force || (c->status == 0 && c->accepted < c->target);
}

// ---------------------------------------------------------------------------
// x1 and x2 sweeps of one tile: 64 lanes over columns c0 - 2 .. c0 + 61 (the
// 60 outputs in lanes 2..61), rows r0 .. r1 - 1 of plane k.  Rows r0 - 2 ..
// r1 + 1 go through the x1 sweep and the x2 march; a row outside the grid is
// the x1 sweep of the row its side rule names (mirrored rows with M2
// negated), which is the side rule applied to the x1-swept state.
//
// Packed tail: the last nx mod 60 columns (rem) would fill a 60-column strip
// only in part (256 columns: 16 of 60).  Their tiles instead pack tailp12
// planes into one wavefront: lane segments of w = rem + 4 lanes, segment s
// holding columns c0 - 2 .. c0 + rem + 1 of plane kg tailp12 + s (a full
// strip is the case of one 64-lane segment, sweep12_lanes).  The lane shifts
// run across segment ends; what crosses them reaches only the two end lanes
// of a segment, which are its halo, exactly as at the ends of a full strip.
// Lanes of no segment or past the last plane read a real cell and store and
// count nothing.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sweep12_lanes(const Desc3& d, int tile, int& seg, int& k, int& col, int& loc,
                                              int& w, bool& lane_ok)
{
    const int lane = threadIdx.x & (WAVE - 1);
    const int nfull = d.strips12 * d.segs12 * d.n[2];
    int c0, k0, np;
    if (tile < nfull) {
        const int strip = tile % d.strips12;
        seg = (tile / d.strips12) % d.segs12;
        k0 = tile / (d.strips12 * d.segs12);
        c0 = strip * OUT12;
        w = WAVE;
        np = 1;
    } else {
        const int t = tile - nfull;
        seg = t % d.segs12;
        k0 = (t / d.segs12) * d.tailp12;
        c0 = d.strips12 * OUT12;
        w = d.tailw12;
        np = d.tailp12;
    }
    const int sgm = lane / w;
    loc = lane - sgm * w;
    const int kk = k0 + sgm;
    lane_ok = sgm < np && kk < d.n[2];
    k = lane_ok ? kk : d.n[2] - 1;
    col = c0 - HALO12 + loc;
}

template <typename T>
__device__ __forceinline__ void sweep12_tile(const Desc3& d, int tile, const Clock* clk)
{
    const int nx = d.n[0], ny = d.n[1];
    const int lane = threadIdx.x & (WAVE - 1);
    int seg, k, col, loc, w;
    bool lane_ok;
    sweep12_lanes(d, tile, seg, k, col, loc, w, lane_ok);
    const int r0 = seg * d.rows12, r1 = min(r0 + d.rows12, ny);
    const T dt = (T)clk->dt;
    const int cur = clk->cur;
    const T* inR = (const T*)d.buf[buf_rho(cur)];
    const T* inM = (const T*)d.buf[buf_mom(cur)];
    T* out = (T*)d.buf[buf_x12(cur)];
    const T beta = (T)d.beta;
    const bool perx = d.bc[0] == FVNA_BC_PERIODIC, pery = d.bc[2] == FVNA_BC_PERIODIC;
    bool xneg;
    const int scol = side_map(d, 0, col, xneg);
    const T xs = xneg ? T(-1) : T(1);
    const size_t pl = (size_t)d.plane;
    const size_t zoff = (size_t)k * (size_t)ny * (size_t)d.pitch;
    const bool out_lane = lane_ok && loc >= HALO12 && loc < w - HALO12 && col < nx;
    Cfl<T> xacc, yacc;

    // x1 sweep of stored row sr (lane-parallel), components (R, M1, M2, M3)
    // raw Q^n of the row that row v stands for (side rule along x2)
    // this lane's plane and column, fixed over the march (the row offset
    // added per row is the same for every lane)
    const T* __restrict__ inR_l = inR + (zoff + (size_t)scol);
    const T* __restrict__ inM_l = inM + (zoff + (size_t)scol);
    T* __restrict__ out_l = out + (zoff + (size_t)(out_lane ? col : 0));
    auto load_row = [&](int v) -> Q4<T> {
        bool yneg;
        const int sr = side_map(d, 1, v, yneg);
        const size_t ro = (size_t)sr * (size_t)d.pitch;
        const T* m = inM_l + ro;
        return Q4<T>{inR_l[ro], m[pl], m[2 * pl], m[3 * pl]};
    };
    auto xsweep = [&](Q4<T> q) -> Q4<T> {
        q.n = xs * q.n;
        Q4<T> L;
        L.R = from_lo(q.R);
        T ir, h;
        rcp_pair(T(1) + q.R, T(2) + (L.R + q.R), ir, h);
        const T un = q.n * ir, ua = q.a * ir, ub = q.b * ir;
        L.n = from_lo(q.n); L.a = from_lo(q.a); L.b = from_lo(q.b);
        const T unL = from_lo(un), uaL = from_lo(ua), ubL = from_lo(ub);
        W4<T> wv;
        T D;
        const T spd = roe4(L, unL, uaL, ubL, q, un, ua, ub, beta, h, wv, D);
        xacc.add(spd, D);
        W4<T> wr;
        wr.a1 = from_hi(wv.a1); wr.s1 = from_hi(wv.s1); wr.r1a = from_hi(wv.r1a); wr.r1b = from_hi(wv.r1b);
        wr.a2 = from_hi(wv.a2); wr.s2 = from_hi(wv.s2); wr.r2a = from_hi(wv.r2a); wr.r2b = from_hi(wv.r2b);
        wr.a3 = from_hi(wv.a3);
        wr.a4 = from_hi(wv.a4);
        T tup[4], hi[4], lo[4];
        cross4(wv, wr, tup, hi);
        lo[0] = from_lo(tup[0]); lo[1] = from_lo(tup[1]); lo[2] = from_lo(tup[2]); lo[3] = from_lo(tup[3]);
        T Gm[4], Gp[4];
        hr_split4(wv, lo, hi, dt, Gm, Gp);
        Q4<T> o2;
        o2.R = fma_(-dt, from_hi(Gm[0]) + Gp[0], q.R);
        o2.n = fma_(-dt, from_hi(Gm[1]) + Gp[1], q.n);
        o2.a = fma_(-dt, from_hi(Gm[2]) + Gp[2], q.a);
        o2.b = fma_(-dt, from_hi(Gm[3]) + Gp[3], q.b);
        return o2;
    };

    // x2 march over rows v = r0 - 2 .. r1 + 1; components (R, M2, M1, M3)
    March4<T> A, B;
    march_zero(A);
    const int v0 = r0 - HALO12, v1 = r1 + HALO12;
    auto step_row = [&](int v, const Q4<T>& raw, const March4<T>& mi, March4<T>& mo) {
        bool yneg;
        (void)side_map(d, 1, v, yneg);
        const Q4<T> x = xsweep(raw);
        Q4<T> q;                                   // split-local for x2: normal = M2
        q.R = x.R;
        q.n = yneg ? -x.a : x.a;
        q.a = x.n;
        q.b = x.b;
        const bool cnt = v > v0 && (pery || (v >= 0 && v <= ny));
        Q4<T> dn;
        march_push(q, mi, mo, beta, dt, cnt, yacc, dn);
        const int j = v - 2;
        if (j >= r0 && out_lane) {
            T* o = out_l + (size_t)j * (size_t)d.pitch;
            o[0] = dn.R;
            o[pl] = dn.a;
            o[2 * pl] = dn.n;
            o[3 * pl] = dn.b;
        }
    };
    // two rows of loads in flight ahead of the row being swept (rows past
    // v1 - 1 are clamped by the side rule and never used)
    Q4<T> p0 = load_row(v0), p1 = load_row(v0 + 1);
    int v = v0;
#pragma unroll 1
    for (; v + 1 < v1; v += 2) {
        Q4<T> r = p0;
        p0 = load_row(v + 2);
        step_row(v, r, A, B);
        r = p1;
        p1 = load_row(v + 3);
        step_row(v + 1, r, B, A);
    }
    if (v < v1) step_row(v, p0, A, B);

    // x1 interfaces: a lane's lies between columns col - 1 and col (the
    // first lane of a segment has no left neighbour); x2 interfaces: lanes
    // with exact x1-swept values
    const bool real_col = perx || (col >= 0 && col < nx);
    const bool cnt_x = lane_ok && loc >= 1 && (perx || (col >= 0 && col <= nx));
    const bool cnt_y = lane_ok && loc >= HALO12 && loc < w - HALO12 && real_col;
    T sx, sy;
    bool hx, hy, fx, fy;
    xacc.finish(cnt_x, sx, hx, fx);
    yacc.finish(cnt_y, sy, hy, fy);
    T m = max_(sx, sy);
    for (int off = 32; off >= 1; off >>= 1) m = max_(m, perm(m, lane ^ off));
    const bool anyh = __any(hx || hy), anyf = __any(fx || fy);
    if (lane == 0) {
        atomicMax(&d.clk->smax_bits, (unsigned long long)__double_as_longlong(cfl_speed<T>(m)));
        const unsigned fl = (anyh ? FLAG_NONHYP : 0u) | (anyf ? FLAG_NONFINITE : 0u);
        if (fl) atomicOr(&d.clk->flags, fl);
    }
}

template <typename T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occupancy<T>::waves)))
void k3_sweep12(Desc3 d, int force)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wave;
    const int nfull = d.strips12 * d.segs12 * d.n[2];
    if (tile >= nfull + d.tailk12 * d.segs12) return;
    const Clock* clk = d.clk;
    if (!step_owed(clk, force)) return;
    sweep12_tile<T>(d, tile, clk);
}

// ---------------------------------------------------------------------------
// x3 sweep: lane = column strip * 64 + lane, row j, planes k0 .. k1 - 1 of
// the output; planes k0 - 2 .. k1 + 1 are pushed through the march, those
// outside the grid by the x3 side rule applied to the x2-swept state.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(256) void k3_sweep3(Desc3 d, int force)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wave;
    const int ntiles = d.strips64 * d.n[1] * d.segs3;
    if (tile >= ntiles) return;
    const Clock* clk = d.clk;
    if (!step_owed(clk, force)) return;
    const int strip = tile % d.strips64;
    const int j = (tile / d.strips64) % d.n[1];
    const int seg = tile / (d.strips64 * d.n[1]);
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int lane = threadIdx.x & (WAVE - 1);
    const int col = strip * WAVE + lane;
    const int scol = min(col, nx - 1);
    const int k0 = seg * d.planes3, k1 = min(k0 + d.planes3, nz);
    const T dt = (T)clk->dt;
    const int cur = clk->cur;
    const T* in = (const T*)d.buf[buf_x12(cur)];
    T* outR = (T*)d.buf[buf_mom(cur)];          // density plane of the momentum buffer
    T* outM = (T*)d.buf[buf_rho(cur)];          // momentum planes of the density buffer
    const T beta = (T)d.beta;
    const bool perz = d.bc[4] == FVNA_BC_PERIODIC;
    const size_t pl = (size_t)d.plane;
    const size_t zstride = (size_t)ny * (size_t)d.pitch;
    const size_t rowoff = (size_t)j * (size_t)d.pitch + (size_t)scol;
    Cfl<T> acc;
    March4<T> A, B;
    march_zero(A);
    const int v0 = k0 - 2, v1 = k1 + 2;
    // raw x2-swept cell of the plane that plane v stands for, split-local
    // for x3 (normal = M3), the mirror applied
    auto load_plane = [&](int v) -> Q4<T> {
        bool zneg;
        const int sk = side_map(d, 2, v, zneg);
        const size_t o = (size_t)sk * zstride + rowoff;
        Q4<T> q{in[o], in[3 * pl + o], in[pl + o], in[2 * pl + o]};
        if (zneg) q.n = -q.n;
        return q;
    };
    auto step_plane = [&](int v, const Q4<T>& q, const March4<T>& mi, March4<T>& mo) {
        const bool cnt = v > v0 && (perz || (v >= 0 && v <= nz));
        Q4<T> dn;
        march_push(q, mi, mo, beta, dt, cnt, acc, dn);
        const int kk = v - 2;
        if (kk >= k0 && col < nx) {
            const size_t w = (size_t)kk * zstride + (size_t)j * (size_t)d.pitch + (size_t)col;
            outR[w] = dn.R;
            outM[pl + w] = dn.a;
            outM[2 * pl + w] = dn.b;
            outM[3 * pl + w] = dn.n;
        }
    };
    Q4<T> p0 = load_plane(v0), p1 = load_plane(v0 + 1);
    int v = v0;
#pragma unroll 1
    for (; v + 1 < v1; v += 2) {
        Q4<T> r = p0;
        p0 = load_plane(v + 2);
        step_plane(v, r, A, B);
        r = p1;
        p1 = load_plane(v + 3);
        step_plane(v + 1, r, B, A);
    }
    if (v < v1) step_plane(v, p0, A, B);
    cfl_commit(d, acc, col < nx);
}

// ---------------------------------------------------------------------------
// Source (3-D form of eq. fs:source, forward Euler): M_c += dt delta~ lap(u_c),
// 7-point Laplacian of u_c = M_c / (1 + R); the density is not rewritten (it
// stays where the x3 sweep put it).  A block of
// SRC_ROWS (= s) wavefronts takes rows s g .. s g + s - 1 of one 64-column
// strip over planes k0 .. k1 - 1: lane = column, wave = row.  Per plane each
// wave publishes its row's velocities in LDS (the first and last waves also
// the rows s g - 1 and s g + s),
// and after one barrier reads its x2 neighbours there; x3 neighbours are
// carried in registers, x1 neighbours come over DPP (the strip's end lanes
// load theirs).  Neighbours outside the grid follow the side rules (mirrored
// normal velocity); rows past ny are such ghost rows and are never stored.
// Every wave of a block runs the same number of barriers: the only early
// exits come before the loop and hold for the whole block.
// ---------------------------------------------------------------------------
template <typename T> struct Vel { T u1, u2, u3; };

// Rows (wavefronts) per source block.  Eight rows read fewer halo rows (10
// per 8 instead of 6 per 4) but measured level: 256^3 per step FP32 0.451 ms
// with 4 or 8, FP64 0.783 / 0.775 ms.
#ifndef FVNA3_SRC_ROWS
#define FVNA3_SRC_ROWS 4
#endif
constexpr int SRC_ROWS = FVNA3_SRC_ROWS;

template <typename T>
__global__ __launch_bounds__(WAVE * SRC_ROWS) void k3_source(Desc3 d, int force)
{
    // [plane parity][row g SRC_ROWS - 1 .. (g + 1) SRC_ROWS][component][lane]
    __shared__ T ys[2][SRC_ROWS + 2][3][WAVE];
    const int ngroups = (d.n[1] + SRC_ROWS - 1) / SRC_ROWS;
    const int b = xcd_block(blockIdx.x, gridDim.x);
    if (b >= d.strips64 * ngroups * d.segs4) return;        // the whole block
    const Clock* clk = d.clk;
    if (!step_owed(clk, force)) return;                       // the whole block (same clock)
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int strip = b % d.strips64;
    const int g = (b / d.strips64) % ngroups;
    const int seg = b / (d.strips64 * ngroups);
    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const int lane = threadIdx.x & (WAVE - 1);
    const int col = strip * WAVE + lane;
    const int j = SRC_ROWS * g + wave;
    // lanes past the last column hold the x+ ghost by the side rule (the
    // lane after the last column is that column's right neighbour); rows past
    // the last row likewise hold the y+ ghost
    bool oneg, jneg;
    const int scol = side_map(d, 0, col, oneg);
    const int sj = side_map(d, 1, j, jneg);
    const int k0 = seg * d.planes4, k1 = min(k0 + d.planes4, nz);
    const T dt = (T)clk->dt;
    const int cur = clk->cur;
    const T* inR = (const T*)d.buf[buf_mom(cur)];     // the x3 sweep's density ...
    const T* inM = (const T*)d.buf[buf_rho(cur)];     // ... and momenta
    T* out = (T*)d.buf[buf_x12(cur)];                 // momenta only
    const T kd = dt * (T)d.delta;
    const size_t pl = (size_t)d.plane;
    const size_t zstride = (size_t)ny * (size_t)d.pitch;
    const bool edge = lane == 0 || lane == WAVE - 1;
    bool eneg = false;
    int ecol = scol;
    if (lane == 0) ecol = side_map(d, 0, col - 1, eneg);
    else if (lane == WAVE - 1) ecol = side_map(d, 0, col + 1, eneg);
    // halo rows: wave 0 publishes row 4g - 1, wave 3 row 4g + 4
    const bool halo = wave == 0 || wave == SRC_ROWS - 1;
    bool hneg = false;
    const int hj = halo ? side_map(d, 1, wave == 0 ? SRC_ROWS * g - 1 : SRC_ROWS * (g + 1), hneg) : sj;
    const int hslot = wave == 0 ? 0 : SRC_ROWS + 1;
    // raw cell at element offset o with the mirrored components negated
    auto raw = [&](size_t o, bool neg1, bool neg2, bool neg3) -> Q4<T> {
        Q4<T> q{inR[o], inM[pl + o], inM[2 * pl + o], inM[3 * pl + o]};
        if (neg1) q.n = -q.n;
        if (neg2) q.a = -q.a;
        if (neg3) q.b = -q.b;
        return q;
    };
    auto vel = [&](const Q4<T>& q) -> Vel<T> {
        const T ir = rcp(T(1) + q.R);
        return Vel<T>{q.n * ir, q.a * ir, q.b * ir};
    };
    // this lane's cell in plane v (side rule along x3)
    auto own = [&](int v) -> Q4<T> {
        bool zneg;
        const int sk = side_map(d, 2, v, zneg);
        return raw((size_t)sk * zstride + (size_t)sj * (size_t)d.pitch + (size_t)scol, oneg, jneg, zneg);
    };
    // the halo row (waves 0, 3) and the end lanes' x neighbours in plane v
    // (v inside the grid when used; clamped otherwise)
    const Q4<T> zero{T(0), T(0), T(0), T(0)};
    auto side_cells = [&](int v, Q4<T>& h, Q4<T>& e) {
        const size_t zo = (size_t)min(max(v, 0), nz - 1) * zstride;
        h = zero;
        e = zero;
        if (halo) h = raw(zo + (size_t)hj * (size_t)d.pitch + (size_t)scol, oneg, hneg, false);
        if (edge) e = raw(zo + (size_t)sj * (size_t)d.pitch + (size_t)ecol, eneg, jneg, false);
    };
    // loads run ahead: this lane's cells two planes, the side cells one plane
    Q4<T> q0 = own(k0), q1 = own(k0 + 1), hq, eq;
    side_cells(k0, hq, eq);
    Vel<T> ub = vel(own(k0 - 1)), uc = vel(q0);
#pragma unroll 1
    for (int k = k0; k < k1; ++k) {
        const Q4<T> q2 = own(k + 2);
        Q4<T> hq1, eq1;
        side_cells(k + 1, hq1, eq1);
        const Vel<T> ua = vel(q1);
        // publish plane k's velocities of this wave's row (and the halo row)
        T (*slot)[3][WAVE] = ys[k & 1];
        slot[wave + 1][0][lane] = uc.u1;
        slot[wave + 1][1][lane] = uc.u2;
        slot[wave + 1][2][lane] = uc.u3;
        if (halo) {
            const Vel<T> hv = vel(hq);
            slot[hslot][0][lane] = hv.u1;
            slot[hslot][1][lane] = hv.u2;
            slot[hslot][2][lane] = hv.u3;
        }
        // every wave has published plane k; the slot written next (plane
        // k + 1) was last read before the previous barrier
        __syncthreads();
        const Vel<T> yl{slot[wave][0][lane], slot[wave][1][lane], slot[wave][2][lane]};
        const Vel<T> yh{slot[wave + 2][0][lane], slot[wave + 2][1][lane], slot[wave + 2][2][lane]};
        const Vel<T> e = vel(eq);
        Vel<T> xl, xh;
        xl.u1 = from_lo(uc.u1); xl.u2 = from_lo(uc.u2); xl.u3 = from_lo(uc.u3);
        xh.u1 = from_hi(uc.u1); xh.u2 = from_hi(uc.u2); xh.u3 = from_hi(uc.u3);
        if (lane == 0) xl = e;
        if (lane == WAVE - 1) xh = e;
        // the oracle's order: -6 u_c, then x-, x+, y-, y+, z-, z+
        auto lap = [&](T c, T a0, T a1, T a2, T a3, T a4, T a5) {
            return ((((((T(-6) * c + a0) + a1) + a2) + a3) + a4) + a5);
        };
        const T l1 = lap(uc.u1, xl.u1, xh.u1, yl.u1, yh.u1, ub.u1, ua.u1);
        const T l2 = lap(uc.u2, xl.u2, xh.u2, yl.u2, yh.u2, ub.u2, ua.u2);
        const T l3 = lap(uc.u3, xl.u3, xh.u3, yl.u3, yh.u3, ub.u3, ua.u3);
        if (col < nx && j < ny) {
            const size_t o = (size_t)k * zstride + (size_t)j * (size_t)d.pitch + (size_t)col;
            out[pl + o] = fma_(kd, l1, q0.n);
            out[2 * pl + o] = fma_(kd, l2, q0.a);
            out[3 * pl + o] = fma_(kd, l3, q0.b);
        }
        ub = uc;
        uc = ua;
        q0 = q1;
        q1 = q2;
        hq = hq1;
        eq = eq1;
    }
}

__global__ void k3_ctrl(Desc3 d)
{
    if (threadIdx.x == 0) control_attempt(d.clk, d.fixed_dt, d.cfl_target, d.cfl_max, d.max_retries, 3);
}

__global__ void k3_bump(Clock* c, long long n)
{
    if (threadIdx.x == 0) c->target += n;
}

// First time step from the speeds of every interface of the current state in
// all three directions (the sweeps run with dt = 0, which leaves the state
// unchanged, so each sweep sees Q^0).
__global__ void k3_dt0(Desc3 d)
{
    if (threadIdx.x != 0) return;
    Clock* c = d.clk;
    const double smax = __longlong_as_double((long long)c->smax_bits);
    const unsigned flags = c->flags;
    c->smax_bits = 0ull;
    c->flags = 0u;
    if (flags & FLAG_NONHYP) { c->status = ST_NONHYP; c->status_step = 0; return; }
    if ((flags & FLAG_NONFINITE) || !(smax > 0.0) || !(smax <= 1.7976931348623157e308)) {
        c->status = ST_NONFINITE;
        c->status_step = 0;
        return;
    }
    c->dt = d.cfl_target / smax;
}

__global__ void k3_clock(Clock* c, double t, double dt, int cur)
{
    if (threadIdx.x != 0) return;
    Clock h;
    __builtin_memset(&h, 0, sizeof(h));
    h.t = t;
    h.dt = dt;
    h.cur = cur;
    *c = h;
}

// Host doubles (SI, staged) <-> stored dimensionless field; rows r over
// ny * nz, grid-strided (gridDim.y is at most 65535).
template <typename T>
__global__ void k3_import(Desc3 d, const double* __restrict__ src, int field, double denom)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.pitch) return;
    const int rows = d.n[1] * d.n[2];
    for (int r = blockIdx.y; r < rows; r += gridDim.y) {
        // the state of clock cur = 0 (set after the import)
        T* dst = (T*)d.buf[field == 0 ? buf_rho(0) : buf_mom(0)] + (size_t)field * (size_t)d.plane +
                 (size_t)r * (size_t)d.pitch;
        dst[i] = i < d.n[0] ? (T)(src[(size_t)r * d.n[0] + i] / denom) : T(0);
    }
}

template <typename T>
__global__ void k3_export(Desc3 d, double* __restrict__ dst, int field, double factor)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.n[0]) return;
    const int rows = d.n[1] * d.n[2];
    const int cur = d.clk->cur;
    const T* base = (const T*)d.buf[field == 0 ? buf_rho(cur) : buf_mom(cur)] + (size_t)field * (size_t)d.plane;
    for (int r = blockIdx.y; r < rows; r += gridDim.y)
        dst[(size_t)r * d.n[0] + i] = (double)base[(size_t)r * (size_t)d.pitch + i] * factor;
}

thread_local std::string g_err3 = "no error";

fvna_status fail3(fvna_status s, const std::string& msg)
{
    g_err3 = msg;
    return s;
}

#define HIP3(x)                                                                        \
    do {                                                                               \
        hipError_t e_ = (x);                                                           \
        if (e_ != hipSuccess) return fail3(FVNA_E_HIP, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int GRAPH3_CHUNK = 32;    // attempts per captured graph

size_t elem(const fvna3_params* p) { return p->precision == FVNA_F64 ? 8 : 4; }
int pitch3(const fvna3_params* p) { const int per = 256 / (int)elem(p); return (p->nx + per - 1) / per * per; }

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

// scratch layout: [Clock][staging of one field]
constexpr size_t OFF3_STAGE = 256;

int cu_count3()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

// Segment lengths: enough tiles to fill every wavefront slot of the device
// once (CUs x 4 SIMDs x `waves`) where the grid allows, never shorter than 16
// cells (the two warm-up cells at each end are repeated work).
int seg_len(long long tiles_per_seg_unit, int n, int cus, int waves)
{
    const long long slots = (long long)cus * 4 * waves;
    const long long per = std::max(1ll, slots / std::max(1ll, tiles_per_seg_unit));
    const long long len = (n + per - 1) / per;
    return (int)std::max(16ll, std::min(len, (long long)n));
}

}  // namespace

struct fvna3_ctx {
    fvna3_params p;
    Desc3 d;
    hipStream_t s;
    hipStream_t cap;
    char* scratch;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    void (*launch)(const Desc3&, int force, hipStream_t) = nullptr;
};

namespace {

template <typename T>
void launch_sweeps(const Desc3& d, int force, hipStream_t s, bool source)
{
    const int t12 = (d.strips12 * d.n[2] + d.tailk12) * d.segs12;
    const int t3 = d.strips64 * d.n[1] * d.segs3;
    hipLaunchKernelGGL(k3_sweep12<T>, dim3((t12 + 3) / 4), dim3(256), 0, s, d, force);
    hipLaunchKernelGGL(k3_sweep3<T>, dim3((t3 + 3) / 4), dim3(256), 0, s, d, force);
    const int tsrc = d.strips64 * ((d.n[1] + SRC_ROWS - 1) / SRC_ROWS) * d.segs4;    // blocks of SRC_ROWS rows
    if (source) hipLaunchKernelGGL(k3_source<T>, dim3(tsrc), dim3(WAVE * SRC_ROWS), 0, s, d, force);
}

template <typename T>
void launch_attempt(const Desc3& d, int force, hipStream_t s)
{
    launch_sweeps<T>(d, force, s, true);
    hipLaunchKernelGGL(k3_ctrl, dim3(1), dim3(64), 0, s, d);
}

void drop_graph3(fvna3_ctx* c)
{
    if (c->exec || c->graph) (void)hipStreamSynchronize(c->s);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

fvna_status build_graph3(fvna3_ctx* c)
{
    if (c->exec) return FVNA_OK;
    HIP3(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH3_CHUNK; ++k) c->launch(c->d, 0, c->cap);
    hipGraph_t g = nullptr;
    HIP3(hipStreamEndCapture(c->cap, &g));
    c->graph = g;
    HIP3(hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0));
    return FVNA_OK;
}

fvna_status enqueue3(fvna3_ctx* c, long long attempts)
{
    fvna_status s = build_graph3(c);
    if (s) return s;
    for (long long k = 0; k < attempts / GRAPH3_CHUNK; ++k) HIP3(hipGraphLaunch(c->exec, c->s));
    for (long long k = 0; k < attempts % GRAPH3_CHUNK; ++k) c->launch(c->d, 0, c->s);
    HIP3(hipGetLastError());
    return FVNA_OK;
}

fvna_status read_clock3(fvna3_ctx* c, Clock* h)
{
    HIP3(hipStreamSynchronize(c->s));
    HIP3(hipMemcpy(h, c->d.clk, sizeof(Clock), hipMemcpyDeviceToHost));
    return FVNA_OK;
}

fvna_status status3(int st)
{
    switch (st) {
    case 0: return FVNA_OK;
    case ST_NONHYP: return fail3(FVNA_E_NONHYPERBOLIC, "non-real Roe speeds (discriminant <= 0) in a step");
    case ST_NONFINITE: return fail3(FVNA_E_NONFINITE, "non-finite wave speed in a step");
    case ST_RETRIES: return fail3(FVNA_E_RETRIES, "too many rejected attempts in a row");
    default: return fail3(FVNA_E_STATE, "unknown device status");
    }
}

// Wait for the stream and top up the steps rejected attempts left owed.
fvna_status sync3(fvna3_ctx* c)
{
    Clock h;
    for (int guard = 0; guard < 1000; ++guard) {
        fvna_status s = read_clock3(c, &h);
        if (s) return s;
        if (h.status != 0 || h.accepted >= h.target) return status3(h.status);
        s = enqueue3(c, h.target - h.accepted);
        if (s) return s;
    }
    return fail3(FVNA_E_STATE, "steps still owed after many top-up rounds");
}

}  // namespace

extern "C" {

const char* fvna3_last_error(void) { return g_err3.c_str(); }

fvna_status fvna3_workspace_size(const fvna3_params* p, size_t* state_bytes, size_t* scratch_bytes)
{
    fvna_status s = validate3(p);
    if (s) return s;
    if (!state_bytes || !scratch_bytes) return fail3(FVNA_E_INVALID, "NULL argument");
    *state_bytes = 4 * (size_t)pitch3(p) * (size_t)p->ny * (size_t)p->nz * elem(p);
    *scratch_bytes = OFF3_STAGE + (size_t)p->nx * (size_t)p->ny * (size_t)p->nz * sizeof(double);
    return FVNA_OK;
}

fvna_status fvna3_create(const fvna3_params* p, void* buf_a, void* buf_b, void* buf_c, void* scratch, void* stream,
                         fvna3_ctx** out)
{
    if (!out) return fail3(FVNA_E_INVALID, "out is NULL");
    *out = nullptr;
    fvna_status s = validate3(p);
    if (s) return s;
    if (!buf_a || !buf_b || !buf_c || !scratch) return fail3(FVNA_E_INVALID, "NULL buffer");
    if (((uintptr_t)buf_a | (uintptr_t)buf_b | (uintptr_t)buf_c | (uintptr_t)scratch) % 256)
        return fail3(FVNA_E_INVALID, "device buffers must be 256-byte aligned");
    fvna3_ctx* c = new (std::nothrow) fvna3_ctx;
    if (!c) return fail3(FVNA_E_NOMEM, "out of host memory");
    c->p = *p;
    Desc3& d = c->d;
    std::memset(&d, 0, sizeof(d));
    d.n[0] = p->nx; d.n[1] = p->ny; d.n[2] = p->nz;
    d.pitch = pitch3(p);
    d.plane = (long long)d.pitch * p->ny * p->nz;
    const int cus = cu_count3();
    // resident waves per SIMD the kernels' registers allow: FP32 5-6, FP64 3-4
#ifndef FVNA3_WAVES
#define FVNA3_WAVES 4
#endif
    const int waves = p->precision == FVNA_F64 ? 2 : FVNA3_WAVES;
    // x1-x2 tiles: full 60-column strips, and the remaining nx mod 60
    // columns packed several planes to a wavefront when at least two fit
    // (256^3 FP32: 3330 wavefronts instead of 3840)
    const int rem12 = p->nx % OUT12, tw = rem12 + 2 * HALO12;
#ifndef FVNA3_PACK_TAIL
#define FVNA3_PACK_TAIL 1
#endif
    if (FVNA3_PACK_TAIL && rem12 > 0 && WAVE / tw >= 2) {
        d.strips12 = p->nx / OUT12;
        d.tailw12 = tw;
        d.tailp12 = WAVE / tw;
        d.tailk12 = (p->nz + d.tailp12 - 1) / d.tailp12;
    } else {
        d.strips12 = (p->nx + OUT12 - 1) / OUT12;
        d.tailw12 = 0;
        d.tailp12 = 1;
        d.tailk12 = 0;
    }
    // row segments for about six x1-x2 tiles per SIMD: several rounds of
    // wavefronts let the dispatcher even out the load of the SIMDs, where
    // one round leaves some with a wavefront more than others (256^3, per
    // step: FP32 0.470 ms with one round of 86-row tiles, 0.448 with 43-row
    // tiles; FP64 0.918 with whole 256-row columns, 0.762 with 43 rows;
    // 64 / 52 / 37 rows measured 0.459 / 0.453 / 0.450 and 0.769 / 0.773 /
    // 0.764 ms); never fewer than 16 rows (two warm-up rows at each end)
    {
        const long long units = (long long)d.strips12 * p->nz + d.tailk12;
        const long long want = 6ll * cus * 4;
        const long long nseg = std::max(1ll, (want + units - 1) / units);
        d.rows12 = (int)std::max(16ll, std::min((long long)p->ny, ((long long)p->ny + nseg - 1) / nseg));
        d.rows12 = std::min(d.rows12, p->ny);
    }
    d.segs12 = (p->ny + d.rows12 - 1) / d.rows12;
    d.strips64 = (p->nx + WAVE - 1) / WAVE;
    d.planes3 = seg_len((long long)d.strips64 * p->ny, p->nz, cus, waves);
    d.segs3 = (p->nz + d.planes3 - 1) / d.planes3;
    // the source kernel's blocks hold one plane's rows in LDS and are light:
    // half the x3 sweep's z-segments, twice its waves (256^3 FP32: source
    // blocks over 64 / 32 / 16 planes 0.486 / 0.469 / 0.473 ms per step)
    d.planes4 = std::max(8, (d.planes3 + 1) / 2);
    d.segs4 = (p->nz + d.planes4 - 1) / d.planes4;
    for (int k = 0; k < 6; ++k) d.bc[k] = p->bc[k];
    d.fixed_dt = p->fixed_dt ? 1 : 0;
    d.max_retries = p->max_retries;
    d.beta = p->beta;
    d.delta = p->delta / (p->c0 * p->dx);
    d.cfl_target = p->cfl_target;
    d.cfl_max = p->cfl_max;
    d.buf[0] = buf_a; d.buf[1] = buf_b; d.buf[2] = buf_c;
    d.clk = (Clock*)scratch;
    c->scratch = (char*)scratch;
    c->s = (hipStream_t)stream;
    c->launch = p->precision == FVNA_F64 ? launch_attempt<double> : launch_attempt<float>;
    if (hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail3(FVNA_E_HIP, "cannot create the capture stream");
    }
    const size_t sb = 4 * (size_t)d.plane * elem(p);
    for (int b = 0; b < 3; ++b)
        if (hipMemsetAsync(d.buf[b], 0, sb, c->s) != hipSuccess) {
            (void)hipStreamDestroy(c->cap);
            delete c;
            return fail3(FVNA_E_HIP, "cannot clear the state buffers");
        }
    hipLaunchKernelGGL(k3_clock, dim3(1), dim3(64), 0, c->s, d.clk, 0.0, 0.0, 0);
    if (hipStreamSynchronize(c->s) != hipSuccess) {
        (void)hipStreamDestroy(c->cap);
        delete c;
        return fail3(FVNA_E_HIP, "cannot initialise the clock");
    }
    *out = c;
    return FVNA_OK;
}

fvna_status fvna3_set_state(fvna3_ctx* c, const double* rho_p, const double* m1, const double* m2, const double* m3)
{
    if (!c || !rho_p || !m1 || !m2 || !m3) return fail3(FVNA_E_INVALID, "NULL argument");
    const fvna3_params& p = c->p;
    const Desc3& d = c->d;
    const double* src[4] = {rho_p, m1, m2, m3};
    const double denom[4] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0, p.rho0 * p.c0};
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    double* stage = (double*)(c->scratch + OFF3_STAGE);
    HIP3(hipStreamSynchronize(c->s));
    const dim3 grid((d.pitch + 255) / 256, std::min(p.ny * p.nz, 65535));
    for (int f = 0; f < 4; ++f) {
        HIP3(hipMemcpyAsync(stage, src[f], n * sizeof(double), hipMemcpyHostToDevice, c->s));
        if (p.precision == FVNA_F64) hipLaunchKernelGGL(k3_import<double>, grid, dim3(256), 0, c->s, d, stage, f, denom[f]);
        else hipLaunchKernelGGL(k3_import<float>, grid, dim3(256), 0, c->s, d, stage, f, denom[f]);
        HIP3(hipGetLastError());
        HIP3(hipStreamSynchronize(c->s));
    }
    const double dt0 = p.dt0 > 0 ? p.dt0 * p.c0 / p.dx : 0.0;
    hipLaunchKernelGGL(k3_clock, dim3(1), dim3(64), 0, c->s, d.clk, 0.0, dt0, 0);
    HIP3(hipGetLastError());
    if (!(dt0 > 0)) {
        // dt = 0: the x1, x2 and x3 sweeps see Q^0 (the source is not needed)
        if (p.precision == FVNA_F64) launch_sweeps<double>(d, 1, c->s, false);
        else launch_sweeps<float>(d, 1, c->s, false);
        hipLaunchKernelGGL(k3_dt0, dim3(1), dim3(64), 0, c->s, d);
        HIP3(hipGetLastError());
    }
    Clock h;
    fvna_status s = read_clock3(c, &h);
    if (s) return s;
    if (h.status == ST_NONHYP) return fail3(FVNA_E_NONHYPERBOLIC, "non-real Roe speeds in the initial state");
    if (h.status) return fail3(FVNA_E_NONFINITE, "no finite positive wave speed in the initial state");
    return FVNA_OK;
}

fvna_status fvna3_step(fvna3_ctx* c, int64_t nsteps)
{
    if (!c) return fail3(FVNA_E_INVALID, "ctx is NULL");
    if (nsteps < 0) return fail3(FVNA_E_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return FVNA_OK;
    hipLaunchKernelGGL(k3_bump, dim3(1), dim3(64), 0, c->s, c->d.clk, (long long)nsteps);
    HIP3(hipGetLastError());
    fvna_status s = enqueue3(c, nsteps);
    if (s) return s;
    return sync3(c);
}

fvna_status fvna3_get_state(fvna3_ctx* c, double* rho_p, double* m1, double* m2, double* m3)
{
    if (!c || !rho_p || !m1 || !m2 || !m3) return fail3(FVNA_E_INVALID, "NULL argument");
    const fvna3_params& p = c->p;
    const Desc3& d = c->d;
    double* dst[4] = {rho_p, m1, m2, m3};
    const double fac[4] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0, p.rho0 * p.c0};
    const size_t n = (size_t)p.nx * p.ny * p.nz;
    double* stage = (double*)(c->scratch + OFF3_STAGE);
    HIP3(hipStreamSynchronize(c->s));
    const dim3 grid((p.nx + 255) / 256, std::min(p.ny * p.nz, 65535));
    for (int f = 0; f < 4; ++f) {
        if (p.precision == FVNA_F64) hipLaunchKernelGGL(k3_export<double>, grid, dim3(256), 0, c->s, d, stage, f, fac[f]);
        else hipLaunchKernelGGL(k3_export<float>, grid, dim3(256), 0, c->s, d, stage, f, fac[f]);
        HIP3(hipGetLastError());
        HIP3(hipMemcpyAsync(dst[f], stage, n * sizeof(double), hipMemcpyDeviceToHost, c->s));
        HIP3(hipStreamSynchronize(c->s));
    }
    return FVNA_OK;
}

fvna_status fvna3_get_stats(fvna3_ctx* c, fvna_stats* st)
{
    if (!c || !st) return fail3(FVNA_E_INVALID, "NULL argument");
    Clock h;
    fvna_status s = read_clock3(c, &h);
    if (s) return s;
    const double tu = c->p.dx / c->p.c0;
    std::memset(st, 0, sizeof(*st));
    st->t = h.t * tu;
    st->dt_next = h.dt * tu;
    st->nu_last = h.nu_last;
    st->nu_mean = h.nu_mean;
    st->nu_std = h.nu_count > 0 ? std::sqrt(h.nu_m2 / (double)h.nu_count) : 0.0;
    st->steps = h.accepted;
    st->rejected = h.rejected;
    st->status = h.status;
    st->status_step = h.status_step;
    return FVNA_OK;
}

fvna_status fvna3_time_step_kernels(fvna3_ctx* c, int32_t reps, double* ms)
{
    if (!c || !ms || reps < 1) return fail3(FVNA_E_INVALID, "bad argument");
    // back-to-back recomputations of the attempt the next step would make
    // (forced, no controller): the state and the clock are unchanged apart
    // from the attempt's speed maximum, which the next controller run clears
    auto sweeps = c->p.precision == FVNA_F64 ? launch_sweeps<double> : launch_sweeps<float>;
    hipEvent_t e0, e1;
    HIP3(hipEventCreate(&e0));
    HIP3(hipEventCreate(&e1));
    sweeps(c->d, 1, c->s, true);
    HIP3(hipEventRecord(e0, c->s));
    for (int r = 0; r < reps; ++r) sweeps(c->d, 1, c->s, true);
    HIP3(hipGetLastError());
    HIP3(hipEventRecord(e1, c->s));
    HIP3(hipEventSynchronize(e1));
    float t = 0.0f;
    HIP3(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = (double)t / reps;
    return FVNA_OK;
}

void fvna3_destroy(fvna3_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->s);
    drop_graph3(c);
    (void)hipStreamDestroy(c->cap);
    delete c;
}

}  // extern "C"
