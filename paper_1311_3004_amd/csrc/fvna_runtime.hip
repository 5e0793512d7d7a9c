// fvna_runtime.hip -- host runtime and C ABI of libfvna (declared in include/fvna.h).
//
// Responsibilities: validate parameters, convert SI to the dimensionless
// variables of the paper's renormalisation with the mesh spacing as length
// unit (Sec. 3, eqs. renorm and phi-tdelta), bind caller-owned device
// buffers, launch the fused step kernel and the device-side time-step
// controller, replay them from a captured HIP graph, and surface the device
// status word at synchronisation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fvna.h"
#include "fvna_device.hpp"
#include "fvna_step.hpp"

using namespace fvna;

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------

// Accept or reject the attempt just made (control_attempt of
// fvna_device.hpp); one thread per simulation, in its own launch after the
// step kernel.  (Deciding in the step kernel's last wavefront instead needs an
// agent-scope release fence in every wavefront, which writes back the L2 and
// cost more than the launch it saves.)
__device__ __forceinline__ void control(const SimDesc& d)
{
    control_attempt(d.clk, d.fixed_dt, d.cfl_target, d.cfl_max, d.max_retries, 2);
}

__global__ void k_ctrl(SimDesc d)
{
    if (threadIdx.x == 0) control(d);
}

// Closing decision of a captured graph whose attempts 1 .. last took the one
// before them in their prologue (k_step, pos >= 1): the decision on attempt
// `last` from its shadow state and CFL slot goes into the clock, and every
// CFL slot is cleared for the next graph.
#ifndef FVNA_FOLD_CONTROL
#define FVNA_FOLD_CONTROL 1
#endif
__global__ void k_ctrl_fold(SimDesc d, int last)
{
    if (threadIdx.x != 0) return;
    Clock* c = d.clk;
    ClockAux* aux = clock_aux(c);
    const Clock prev = last == 0 ? *c : aux->shadow[last & 1];
    unsigned long long* sb;
    unsigned int* fl;
    cfl_slot(c, last % 3, sb, fl);
    const unsigned long long s = *sb;
    const unsigned int f = *fl;
    *c = control_next(prev, s, f, d.fixed_dt, d.cfl_target, d.cfl_max, d.max_retries, 2);
    aux->slot[0].smax_bits = 0ull;
    aux->slot[0].flags = 0u;
    aux->slot[1].smax_bits = 0ull;
    aux->slot[1].flags = 0u;
}

__global__ void k_ctrl_batch(const SimDesc* __restrict__ descs, int n)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) control(descs[k]);
}

__global__ void k_bump(Clock* c, long long n)
{
    if (threadIdx.x == 0) c->target += n;
}

__global__ void k_bump_batch(const SimDesc* __restrict__ descs, int n, long long steps)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) descs[k].clk->target += steps;
}

// Cell (i, j) of the state in buffer `cur`, with at most one index one step
// outside the grid; ghost values follow the boundary rules at time t.
template <typename S, typename T>
__device__ Cell<T> cell_at(const SimDesc& d, int i, int j, double t)
{
    using C = Codec<S, T>;
    const int nx = d.nx, ny = d.ny;
    int si = i, sj = j;
    T sgnM = T(1), sgnN = T(1);
    int side = -1;
    if (i < 0) side = 0;
    else if (i >= nx) side = 1;
    else if (j < 0) side = 2;
    else if (j >= ny) side = 3;
    if (side >= 0) {
        const int b = d.bc[side];
        if (b == BC_TAYLOR) {
            double R, M, N;
            taylor_at(d, taylor_x0(d, d.clk->x_off), i + 0.5, j + 0.5, t, R, M, N);
            return Cell<T>{(T)R, (T)M, (T)N};
        }
        if (b == BC_SOURCE) {
            const SourceClock sc = source_clock(d, t);
            if ((j + 0.5) <= sc.ap) {
                Cell<T> q;
                source_at<T>(d, j, sc, q.R, q.M, q.N);
                return q;
            }
        }
        if (b == BC_PERIODIC) {
            if (side == 0) si = i + nx;
            if (side == 1) si = i - nx;
            if (side == 2) sj = j + ny;
            if (side == 3) sj = j - ny;
        } else if (b == BC_REFLECT) {
            if (side == 0) { si = -1 - i; sgnM = T(-1); }
            if (side == 1) { si = 2 * nx - 1 - i; sgnM = T(-1); }
            if (side == 2) { sj = -1 - j; sgnN = T(-1); }
            if (side == 3) { sj = 2 * ny - 1 - j; sgnN = T(-1); }
        } else {
            si = min(max(i, 0), nx - 1);
            sj = min(max(j, 0), ny - 1);
        }
    }
    const S* R = (const S*)d.buf[d.clk->cur];
    const size_t o = (size_t)sj * (size_t)d.pitch + (size_t)si;
    Cell<T> q;
    q.R = C::ld(R[o], d.scale[0]);
    q.M = sgnM * C::ld(R[d.plane + o], d.scale[1]);
    q.N = sgnN * C::ld(R[2 * d.plane + o], d.scale[2]);
    return q;
}

// Dry pass over every interface adjacent to an interior cell, both
// directions: largest |s^p| of the current state (fixes the first step).
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_dry(SimDesc d)
{
    // rows j = blockIdx.y, + gridDim.y, ... (j = ny: the top x2 interfaces);
    // each wavefront folds its rows before its single atomic, so one launch
    // issues a few thousand atomics instead of one per 64 interfaces
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const double t = d.clk->t;
    const T beta = (T)d.beta;
    Cfl<T> acc;
    for (int j = blockIdx.y; j <= d.ny && i <= d.nx; j += gridDim.y) {
        if (j < d.ny) {
            const Cell<T> a = cell_at<S, T>(d, i - 1, j, t), b = cell_at<S, T>(d, i, j, t);
            const T ia = rcp(T(1) + a.R), ib = rcp(T(1) + b.R);
            Wave<T> w;
            T D;
            const T spd = roe(a.R, a.M, a.N, a.M * ia, a.N * ia, b.R, b.M, b.N, b.M * ib, b.N * ib, beta, w, D);
            acc.add(spd, D);
        }
        if (i < d.nx) {
            const Cell<T> a = cell_at<S, T>(d, i, j - 1, t), b = cell_at<S, T>(d, i, j, t);
            const T ia = rcp(T(1) + a.R), ib = rcp(T(1) + b.R);
            Wave<T> w;
            T D;
            const T spd = roe(a.R, a.N, a.M, a.N * ia, a.M * ia, b.R, b.N, b.M, b.N * ib, b.M * ib, beta, w, D);
            acc.add(spd, D);
        }
    }
    T sm;
    bool nh, nf;
    acc.finish(true, sm, nh, nf);
    const int lane = threadIdx.x & 63;
    for (int off = 32; off >= 1; off >>= 1) sm = max_(sm, perm(sm, lane ^ off));
    const bool anyh = __any(nh), anyf = __any(nf);
    if (lane == 0) {
        atomicMax(&d.clk->smax_bits, (unsigned long long)__double_as_longlong(cfl_speed<T>(sm)));
        const unsigned fl = (anyh ? FLAG_NONHYP : 0u) | (anyf ? FLAG_NONFINITE : 0u);
        if (fl) atomicOr(&d.clk->flags, fl);
    }
}

__global__ void k_dt0(SimDesc d)
{
    if (threadIdx.x != 0) return;
    Clock* c = d.clk;
    const double smax = __longlong_as_double((long long)c->smax_bits);
    const unsigned flags = c->flags;
    c->smax_bits = 0ull;
    c->flags = 0u;
    if (flags & FLAG_NONHYP) { c->status = ST_NONHYP; c->status_step = 0; return; }
    if ((flags & FLAG_NONFINITE) || !(smax > 0.0) || !(smax <= DBL_MAX)) {
        c->status = ST_NONFINITE;
        c->status_step = 0;
        return;
    }
    c->dt = d.cfl_target / smax;
}

// Per-row table of the focused source (eq. hifuBC), rows r = j + 1/2: the
// focusing delay f r^2/(2F) reduced modulo one period, the direction cosines
// F/h and -r/h with h = sqrt(r^2 + F^2), and the whole delay.  FP64 with
// correctly rounded division and square root.
__global__ void k_src_table(double* __restrict__ tab, int ny, double f, double F)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ny) return;
    const double r = j + 0.5;
    const double delay = f * (r * r / (2.0 * F));
    const double h = sqrt(r * r + F * F);
    tab[4 * (size_t)j] = delay - floor(delay);
    tab[4 * (size_t)j + 1] = F / h;
    tab[4 * (size_t)j + 2] = -r / h;
    tab[4 * (size_t)j + 3] = delay;
}

// Per-row 1/r of an axisymmetric grid, r = j + 1/2 for rows j = -RINV_PAD ..
// ny + RINV_PAD - 1 (entry j + RINV_PAD): the correctly rounded FP64
// quotient, in the arithmetic type of the step.
template <typename T>
__global__ void k_rinv_table(T* __restrict__ tab, int ny)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= ny + 2 * RINV_PAD) return;
    tab[k] = (T)(1.0 / ((double)(k - RINV_PAD) + 0.5));
}

// Whole clock of one simulation written from its arguments (every field the
// controller and the step kernel read starts defined, counters at zero).
__global__ void k_clock_init(Clock* __restrict__ c, double t, double dt, int cur, long long target)
{
    if (threadIdx.x != 0) return;
    Clock h;
    __builtin_memset(&h, 0, sizeof(h));
    h.t = t;
    h.dt = dt;
    h.cur = cur;
    h.target = target;
    *c = h;
}

// Host doubles (SI, staged on the device) -> stored dimensionless field.
template <typename S, typename T>
__global__ void k_import(SimDesc d, const double* __restrict__ src, int field, int row0, int nrows,
                         double denom, int buf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= d.pitch || r >= nrows) return;
    S* dst = (S*)d.buf[buf] + (size_t)field * d.plane + (size_t)(row0 + r) * d.pitch;
    const T v = (i < d.nx) ? (T)(src[(size_t)r * d.nx + i] / denom) : T(0);
    dst[i] = Codec<S, T>::st(v, d.inv_scale[field]);
}

template <typename S, typename T>
__global__ void k_export(SimDesc d, double* __restrict__ dst, int field, int row0, int nrows, int col0,
                         int ncols, double factor)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int r = blockIdx.y;
    if (i >= ncols || r >= nrows) return;
    const S* src = (const S*)d.buf[d.clk->cur] + (size_t)field * d.plane + (size_t)(row0 + r) * d.pitch + col0;
    dst[(size_t)r * ncols + i] = (double)Codec<S, T>::ld(src[i], d.scale[field]) * factor;
}

// Moving domain (Sec. 4): the current state moved `ncols` cells along +x1 into
// the other buffer.  Entering on the right: undisturbed medium (stored zero,
// whatever the scale), or, when side x+ holds Taylor data, the profile at the
// new path columns at the time of the move (the medium ahead of the front);
// the row padding stays zero.  Kept columns are raw copies of the stored
// values: no conversion, so a move is exact in every precision.  k_flip then
// makes the moved state current; it runs after every block of k_shift has
// read `cur` and x_off.
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_shift(SimDesc d, int ncols)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= d.pitch) return;
    const Clock* clk = d.clk;
    const int cur = clk->cur;
    const S* __restrict__ src = (const S*)d.buf[cur];
    S* __restrict__ dst = (S*)d.buf[cur ^ 1];
    const bool inside = i < d.nx - ncols;
    const bool fill = !inside && i < d.nx && d.bc[1] == BC_TAYLOR;
    const double x0 = taylor_x0(d, clk->x_off + ncols), t = clk->t;
    for (int r = blockIdx.y; r < 3 * d.ny; r += gridDim.y) {
        const int field = r / d.ny, row = r - field * d.ny;
        const size_t base = (size_t)field * d.plane + (size_t)row * d.pitch;
        S v;
        if (inside) {
            v = src[base + i + ncols];
        } else if (fill) {
            double q[3];
            taylor_at(d, x0, i + 0.5, row + 0.5, t, q[0], q[1], q[2]);
            v = Codec<S, T>::st((T)q[field], d.inv_scale[field]);
        } else {
            __builtin_memset(&v, 0, sizeof(S));
        }
        dst[base + i] = v;
    }
}

__global__ void k_flip(Clock* c, int ncols)
{
    if (threadIdx.x == 0) {
        c->cur ^= 1;
        c->x_off += ncols;
    }
}

// Recorder: after an attempt, the running maximum of rho' along one grid row,
// kept per column of the path the (possibly moving) domain covers, and rho'
// and t at one probe column after every accepted step.  Idempotent: after a
// rejected or empty attempt it sees the state and step count it saw before,
// so it can follow every attempt without knowing which were accepted.
struct RecDesc {
    int row, probe_col;
    long long path_len, base, capacity;
    double* row_max;
    double* probe_t;
    double* probe_rho;
    double rho0, t_unit;
};

// Controller and recorder in one launch (one block): thread 0 decides the
// attempt (control), hands the updated clock to the block through LDS, and
// the block records the row (a separate recorder launch after k_ctrl cost as
// much as the controller itself, 4.6 us per attempt).
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_ctrl_record(SimDesc d, RecDesc r)
{
    __shared__ long long s_acc, s_xoff;
    __shared__ int s_cur;
    __shared__ double s_t;
    if (threadIdx.x == 0) {
        control_attempt(d.clk, d.fixed_dt, d.cfl_target, d.cfl_max, d.max_retries, 2);
        const Clock* clk = d.clk;
        s_acc = clk->accepted;
        s_xoff = clk->x_off;
        s_cur = clk->cur;
        s_t = clk->t;
    }
    __syncthreads();
    const long long k = s_acc - r.base - 1;             // index of the latest accepted step
    if (k < 0) return;
    const S* R = (const S*)d.buf[s_cur] + (size_t)r.row * d.pitch;
    for (int i = threadIdx.x; i < d.nx; i += blockDim.x) {
        const double rho = (double)Codec<S, T>::ld(R[i], d.scale[0]) * r.rho0;
        const long long pc = s_xoff + i;
        if (pc < r.path_len) r.row_max[pc] = fmax(r.row_max[pc], rho);
        if (pc == r.probe_col && k < r.capacity) {
            r.probe_t[k] = s_t * r.t_unit;
            r.probe_rho[k] = rho;
        }
    }
}

// Fixed-order FP64 sums: block b sums rows b, b + NB, ... with a fixed
// thread stride and a fixed tree; the final pass sums the NB partials.
constexpr int SUM_BLOCKS = 512;

// `state` is the buffer to sum, or null for the simulation's current one.
template <typename S, typename T>
__global__ __launch_bounds__(256) void k_sums_partial(SimDesc d, const void* state, double* __restrict__ part)
{
    __shared__ double sh[3][256];
    const int b = blockIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    const S* base = (const S*)(state ? state : d.buf[d.clk->cur]);
    for (int j = b; j < d.ny; j += SUM_BLOCKS)
        for (int i = threadIdx.x; i < d.nx; i += 256)
            for (int f = 0; f < 3; ++f)
                acc[f] += (double)Codec<S, T>::ld(base[(size_t)f * d.plane + (size_t)j * d.pitch + i], d.scale[f]);
    for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int f = 0; f < 3; ++f) part[(size_t)b * 3 + f] = sh[f][0];
}

// out[f] = (sum of the partials of field f) * factor_f: the SI sums.
__global__ __launch_bounds__(256) void k_sums_final(const double* __restrict__ part, double* __restrict__ out,
                                                    double f0, double f1, double f2)
{
    __shared__ double sh[3][256];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int b = threadIdx.x; b < SUM_BLOCKS; b += 256)
        for (int f = 0; f < 3; ++f) acc[f] += part[(size_t)b * 3 + f];
    for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] = acc[f];
    __syncthreads();
    for (int s = 128; s >= 1; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int f = 0; f < 3; ++f) sh[f][threadIdx.x] += sh[f][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0] * f0;
        out[1] = sh[1][0] * f1;
        out[2] = sh[2][0] * f2;
    }
}

// Errors of eq. (error) on a line of cells (fvna_taylor_errors): one block of
// 256 threads, thread k takes line cells k, k + 256, ...; a fixed tree
// reduces the four FP64 accumulators (sum |R - R_ref|, sum |R_ref|, and the
// two maxima).  Line geometry in SI metres, as the host describes it: cells
// a0 .. a0 + n - 1 along the line's main axis (columns, or rows when steep),
// the other index the floor of the line's coordinate there.
struct ErrLine {
    double fx, fy;       // front point at time t [m]
    double c, s;         // propagation direction
    double dx, x0;       // mesh spacing, Taylor origin on the path [m]
    double c0t, w, amp;  // c0 t [m], tanh width [m], amplitude (dimensionless)
    long long a0, n, x_off;
    int steep;
};

template <typename S, typename T>
__global__ __launch_bounds__(256) void k_taylor_err(SimDesc d, ErrLine L, double* __restrict__ out)
{
    __shared__ double sh[4][256];
    double se = 0.0, sr = 0.0, me = 0.0, mr = 0.0;
    const S* R = (const S*)d.buf[d.clk->cur];
    for (long long k = threadIdx.x; k < L.n; k += 256) {
        const long long a = L.a0 + k;
        long long ip, jp;
        if (!L.steep) {
            ip = a;
            jp = (long long)floor((L.fy + (((double)a + 0.5) * L.dx - L.fx) * L.s / L.c) / L.dx);
        } else {
            jp = a;
            ip = (long long)floor((L.fx + (((double)a + 0.5) * L.dx - L.fy) * L.c / L.s) / L.dx);
        }
        const long long i = ip - L.x_off;
        if (i < 0 || i >= d.nx || jp < 0 || jp >= d.ny) continue;
        const double xi = (((double)ip + 0.5) * L.dx - L.x0) * L.c + ((double)jp + 0.5) * L.dx * L.s;
        const double ref = -L.amp * tanh((xi - L.c0t) / L.w);
        const double v = (double)Codec<S, T>::ld(R[(size_t)jp * (size_t)d.pitch + (size_t)i], d.scale[0]);
        const double e = fabs(v - ref);
        se += e;
        sr += fabs(ref);
        me = fmax(me, e);
        mr = fmax(mr, fabs(ref));
    }
    sh[0][threadIdx.x] = se;
    sh[1][threadIdx.x] = sr;
    sh[2][threadIdx.x] = me;
    sh[3][threadIdx.x] = mr;
    __syncthreads();
    for (int h = 128; h >= 1; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sh[0][threadIdx.x] += sh[0][threadIdx.x + h];
            sh[1][threadIdx.x] += sh[1][threadIdx.x + h];
            sh[2][threadIdx.x] = fmax(sh[2][threadIdx.x], sh[2][threadIdx.x + h]);
            sh[3][threadIdx.x] = fmax(sh[3][threadIdx.x], sh[3][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = sh[0][0] / sh[1][0];
        out[1] = sh[2][0] / sh[3][0];
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

namespace {

thread_local std::string g_err = "no error";

fvna_status fail(fvna_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(FVNA_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
    } while (0)

constexpr size_t ALIGN = 256;
constexpr size_t STAGE_CELLS = size_t(1) << 20;   // staging chunk for set/get state
constexpr int GRAPH_CHUNK = 32;                   // attempts per captured graph
// Segment height of batched simulations without their own: the batch runs in
// several rounds of wavefronts, so the one-round rule of a single grid does not
// apply; 128 rows measured best on 64 uneven grids (48..256 tried).
constexpr int BATCH_TILE_ROWS = 128;

constexpr size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

size_t elem_size(int precision)
{
    switch (precision) {
    case FVNA_F64: return 8;
    case FVNA_F32: return 4;
    default: return 2;
    }
}

int pitch_of(const fvna_params* p)
{
    // rows padded to a multiple of 256 bytes
    const size_t es = elem_size(p->precision);
    const size_t per = ALIGN / es;
    return (int)align_up((size_t)p->nx, per);
}

fvna_status validate(const fvna_params* p)
{
    if (!p) return fail(FVNA_E_INVALID, "params is NULL");
    if (p->nx < 4 || p->ny < 4) return fail(FVNA_E_INVALID, "grid must have at least 4 cells per axis");
    if ((long long)p->nx * (long long)p->ny > (1ll << 34)) return fail(FVNA_E_INVALID, "grid too large");
    if (!(p->dx > 0) || !(p->c0 > 0) || !(p->rho0 > 0))
        return fail(FVNA_E_INVALID, "dx, c0 and rho0 must be positive");
    if (!(p->beta >= 1.0)) return fail(FVNA_E_INVALID, "beta must be >= 1");
    if (!(p->delta >= 0.0)) return fail(FVNA_E_INVALID, "delta must be >= 0");
    if (p->geometry != FVNA_CARTESIAN && p->geometry != FVNA_AXISYMMETRIC)
        return fail(FVNA_E_INVALID, "unknown geometry");
    if (p->precision < FVNA_F64 || p->precision > FVNA_F32_BF16STORE)
        return fail(FVNA_E_INVALID, "unknown precision");
    if (!(p->cfl_target > 0.0) || !(p->cfl_target < p->cfl_max))
        return fail(FVNA_E_INVALID, "need 0 < cfl_target < cfl_max");
    if (p->max_retries < 0) return fail(FVNA_E_INVALID, "max_retries must be >= 0");
    if (p->tile_rows != 0 && (p->tile_rows < 8 || p->tile_rows > 65536))
        return fail(FVNA_E_INVALID, "tile_rows must be 0 or in [8, 65536]");
    for (int s = 0; s < 4; ++s)
        if (p->bc[s] < FVNA_BC_PERIODIC || p->bc[s] > FVNA_BC_SOURCE)
            return fail(FVNA_E_INVALID, "unknown boundary kind");
    if ((p->bc[0] == FVNA_BC_PERIODIC) != (p->bc[1] == FVNA_BC_PERIODIC) ||
        (p->bc[2] == FVNA_BC_PERIODIC) != (p->bc[3] == FVNA_BC_PERIODIC))
        return fail(FVNA_E_INVALID, "periodic must be set on both sides of an axis");
    if (p->bc[1] == FVNA_BC_SOURCE || p->bc[2] == FVNA_BC_SOURCE || p->bc[3] == FVNA_BC_SOURCE)
        return fail(FVNA_E_INVALID, "the focused source is only available on side x-");
    if (p->geometry == FVNA_AXISYMMETRIC && p->bc[2] != FVNA_BC_REFLECT)
        return fail(FVNA_E_INVALID, "axisymmetric geometry needs REFLECT on side y- (the axis)");
    for (int f = 0; f < 3; ++f)
        if (!(p->store_scale[f] >= 0.0)) return fail(FVNA_E_INVALID, "store_scale must be >= 0");
    return FVNA_OK;
}

size_t state_bytes_of(const fvna_params* p)
{
    return align_up((size_t)3 * (size_t)pitch_of(p) * (size_t)p->ny * elem_size(p->precision), ALIGN);
}

// scratch layout: [Clock, ClockAux][sum partials][sum out][source table][1/r table][staging]
constexpr size_t OFF_CLOCK = 0;
constexpr size_t OFF_PART = 768;
static_assert(CLOCK_AUX_OFFSET >= sizeof(Clock) && CLOCK_AUX_OFFSET + sizeof(ClockAux) <= OFF_PART,
              "clock and its shadow states must fit before the partial sums");
constexpr size_t OFF_SUMOUT = OFF_PART + align_up(SUM_BLOCKS * 3 * sizeof(double), ALIGN);
constexpr size_t OFF_SRCTAB = OFF_SUMOUT + 256;

size_t rinv_off_of(const fvna_params* p)
{
    return OFF_SRCTAB + align_up(4 * (size_t)p->ny * sizeof(double), ALIGN);
}

size_t stage_off_of(const fvna_params* p)
{
    return rinv_off_of(p) + align_up(((size_t)p->ny + 2 * RINV_PAD) * sizeof(double), ALIGN);
}

// The per-row 1/r table of an axisymmetric grid (nothing for a Cartesian one).
static fvna_status fill_rinv(SimDesc& d, const fvna_params* p, char* scratch, hipStream_t stream)
{
    d.rinv = nullptr;
    if (p->geometry != FVNA_AXISYMMETRIC) return FVNA_OK;
    void* tab = scratch + rinv_off_of(p);
    const int n = p->ny + 2 * RINV_PAD;
    if (p->precision == FVNA_F64)
        hipLaunchKernelGGL(k_rinv_table<double>, dim3((n + 255) / 256), dim3(256), 0, stream, (double*)tab, p->ny);
    else
        hipLaunchKernelGGL(k_rinv_table<float>, dim3((n + 255) / 256), dim3(256), 0, stream, (float*)tab, p->ny);
    HIP_TRY(hipGetLastError());
    d.rinv = tab;
    return FVNA_OK;
}

size_t stage_cells_of(const fvna_params* p)
{
    const size_t cells = (size_t)p->nx * (size_t)p->ny;
    return std::min(cells, std::max(STAGE_CELLS, (size_t)p->nx));
}

size_t scratch_bytes_of(const fvna_params* p)
{
    return stage_off_of(p) + align_up(stage_cells_of(p) * sizeof(double), ALIGN);
}

// Row segments of a grid for a nominal height tr (device side: seg_bounds).
// The first and last segment of a strip take the general path, which issues
// more instructions per row than the lean one (FP64: 13% more VALU); they get
// about FVNA_EDGE_PERMILLE/1000 of tr rows, the others share the rest evenly
// in segments of at most tr rows.  Small grids keep uniform segments.  With
// every wavefront resident at once, the slowest tile ends the step: measured
// step kernel at 100 / 85 / 70 / 55% edge rows, FP64 4096^2 0.275 / 0.271 /
// 0.261 / 0.263 ms, axisymmetric FP32 8192 x 2048 0.197 / 0.189 / 0.186 /
// 0.186 ms, FP32 4096^2 unchanged (0.160 ms).
#ifndef FVNA_EDGE_PERMILLE
#define FVNA_EDGE_PERMILLE 700
#endif
struct Segments { int segs, edge, mid; };
static Segments segments_of(int ny, int tr, bool short_edges = true)
{
    const int e = std::max(8, (int)(((long long)tr * FVNA_EDGE_PERMILLE + 999) / 1000));
    if (!short_edges || FVNA_EDGE_PERMILLE >= 1000 || ny - 2 * e < tr) return Segments{(ny + tr - 1) / tr, 0, tr};
    const int m = (ny - 2 * e + tr - 1) / tr;    // >= 1; (m - 1) tr < ny - 2e, so none is empty
    return Segments{m + 2, e, (ny - 2 * e + m - 1) / m};
}
// Batch members run in many rounds of wavefronts, where the end of the step
// is not set by one slow tile: they keep uniform segments (short_edges =
// false; measured on the 64 uneven grids: 0.95 ms per launch with short edge
// segments against 0.83 ms uniform at 128 rows).
static void set_segments(SimDesc& d, int tr, bool short_edges = true)
{
    const Segments g = segments_of(d.ny, tr, short_edges);
    d.tile_rows = tr;
    d.segs = g.segs;
    d.seg_edge = g.edge;
    d.seg_mid = g.mid;
}

// Rows per wavefront segment when none is given: enough segments that the
// grid's wavefronts fill every resident slot of the device (CUs x 4 SIMDs x
// the occupancy the step kernel is compiled for) in one round without
// spilling a few into a second round, and never fewer than 16 rows (the six
// warm-up rows of a segment are redundant work).
int default_tile_rows(const fvna_params* p, int cu_count)
{
    const int waves_per_simd = p->precision == FVNA_F64 ? Occupancy<double>::waves : Occupancy<float>::waves;
    const long long slots = (long long)std::max(cu_count, 1) * 4 * waves_per_simd;
    const long long strips = (p->nx + OUTW - 1) / OUTW;
    const long long per_strip = std::max(1ll, slots / strips);
    long long tr = (p->ny + per_strip - 1) / per_strip;
    tr = std::max(16ll, std::min(tr, 65536ll));
    // shorter first and last segments: the smallest height whose segments
    // still fit the slots (at most per_strip of them)
    if (FVNA_EDGE_PERMILLE < 1000 && per_strip >= 3) {
        const double f = FVNA_EDGE_PERMILLE / 1000.0;
        long long t2 = std::max(16ll, (long long)std::ceil(p->ny / (per_strip - 2 + 2 * f)));
        while (t2 < 65536 && segments_of(p->ny, (int)t2).segs > per_strip) ++t2;
        tr = t2;
    }
    return (int)tr;
}

int device_cu_count()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) return 256;
    return n;
}

// in-process autotune cache keyed by (precision, geometry, nx, ny)
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int>, int> g_tune;

}  // namespace

struct Launcher {
    void (*step)(const SimDesc&, int force, int pos, hipStream_t);
    void (*step_batch)(const SimDesc*, const TileRef*, int ntiles, int force, hipStream_t);
    void (*dry)(const SimDesc&, hipStream_t);
    void (*imp)(const SimDesc&, const double*, int, int, int, double, int, hipStream_t);
    void (*exp)(const SimDesc&, double*, int, int, int, int, int, double, hipStream_t);
    void (*sums)(const SimDesc&, const void* state, double* part, double* out, const double* factor, hipStream_t);
    void (*shift)(const SimDesc&, int, hipStream_t);
    void (*ctrl_record)(const SimDesc&, const RecDesc&, hipStream_t);
    void (*taylor_err)(const SimDesc&, const ErrLine&, double*, hipStream_t);
};

template <typename S, typename T, int AXI>
Launcher make_launcher()
{
    Launcher L;
    L.step = [](const SimDesc& d, int force, int pos, hipStream_t s) {
        const int tiles = d.strips * d.segs;
        const int blocks = (tiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        hipLaunchKernelGGL((k_step<S, T, AXI>), dim3(blocks), dim3(256), 0, s, d, force, pos);
    };
    L.step_batch = [](const SimDesc* descs, const TileRef* tiles, int ntiles, int force, hipStream_t s) {
        const int blocks = (ntiles + WAVES_PER_BLOCK - 1) / WAVES_PER_BLOCK;
        hipLaunchKernelGGL((k_step_batch<S, T, AXI>), dim3(blocks), dim3(256), 0, s, descs, tiles, ntiles, force);
    };
    L.dry = [](const SimDesc& d, hipStream_t s) {
        hipLaunchKernelGGL((k_dry<S, T>), dim3((d.nx + 1 + 255) / 256, std::min(d.ny + 1, 64)), dim3(256), 0, s, d);
    };
    L.imp = [](const SimDesc& d, const double* src, int field, int row0, int nrows, double denom, int buf,
               hipStream_t s) {
        hipLaunchKernelGGL((k_import<S, T>), dim3((d.pitch + 255) / 256, nrows), dim3(256), 0, s, d, src, field,
                           row0, nrows, denom, buf);
    };
    L.exp = [](const SimDesc& d, double* dst, int field, int row0, int nrows, int col0, int ncols, double factor,
               hipStream_t s) {
        hipLaunchKernelGGL((k_export<S, T>), dim3((ncols + 255) / 256, nrows), dim3(256), 0, s, d, dst, field, row0,
                           nrows, col0, ncols, factor);
    };
    L.sums = [](const SimDesc& d, const void* state, double* part, double* out, const double* factor,
                hipStream_t s) {
        hipLaunchKernelGGL((k_sums_partial<S, T>), dim3(SUM_BLOCKS), dim3(256), 0, s, d, state, part);
        hipLaunchKernelGGL(k_sums_final, dim3(1), dim3(256), 0, s, part, out, factor[0], factor[1], factor[2]);
    };
    L.shift = [](const SimDesc& d, int ncols, hipStream_t s) {
        const int rows = std::min(3 * d.ny, 65535);
        hipLaunchKernelGGL((k_shift<S, T>), dim3((d.pitch + 255) / 256, rows), dim3(256), 0, s, d, ncols);
        hipLaunchKernelGGL(k_flip, dim3(1), dim3(64), 0, s, d.clk, ncols);
    };
    L.ctrl_record = [](const SimDesc& d, const RecDesc& r, hipStream_t s) {
        hipLaunchKernelGGL((k_ctrl_record<S, T>), dim3(1), dim3(256), 0, s, d, r);
    };
    L.taylor_err = [](const SimDesc& d, const ErrLine& e, double* out, hipStream_t s) {
        hipLaunchKernelGGL((k_taylor_err<S, T>), dim3(1), dim3(256), 0, s, d, e, out);
    };
    return L;
}

static Launcher pick_launcher(int precision, int geometry)
{
    const bool a = geometry == FVNA_AXISYMMETRIC;
    switch (precision) {
    case FVNA_F64: return a ? make_launcher<double, double, 1>() : make_launcher<double, double, 0>();
    case FVNA_F32: return a ? make_launcher<float, float, 1>() : make_launcher<float, float, 0>();
    case FVNA_F32_F16STORE: return a ? make_launcher<_Float16, float, 1>() : make_launcher<_Float16, float, 0>();
    default: return a ? make_launcher<bf16, float, 1>() : make_launcher<bf16, float, 0>();
    }
}

// Fill the simulation descriptor (everything dimensionless) from SI params.
static void fill_desc(SimDesc& d, const fvna_params* p, void* a, void* b, Clock* clk, int tile_rows,
                      bool short_edges = true)
{
    std::memset(&d, 0, sizeof(d));
    d.nx = p->nx;
    d.ny = p->ny;
    d.pitch = pitch_of(p);
    d.plane = (long long)d.pitch * (long long)p->ny;
    d.strips = (p->nx + OUTW - 1) / OUTW;
    set_segments(d, tile_rows, short_edges);
    for (int s = 0; s < 4; ++s) d.bc[s] = p->bc[s];
    d.fixed_dt = p->fixed_dt ? 1 : 0;
    d.max_retries = p->max_retries;
    d.beta = p->beta;
    d.delta = p->delta / (p->c0 * p->dx);
    d.cfl_target = p->cfl_target;
    d.cfl_max = p->cfl_max;
    d.ta_amp = 0.0; d.ta_w = 1.0; d.ta_cos = 1.0; d.ta_sin = 0.0;
    d.sr_freq = 1.0; d.sr_F = 1e30; d.sr_ramp = 3.0; d.sr_t2 = INFINITY;
    for (int f = 0; f < 3; ++f) {
        const bool half = p->precision == FVNA_F32_F16STORE || p->precision == FVNA_F32_BF16STORE;
        const double sc = (half && p->store_scale[f] > 0.0) ? p->store_scale[f] : 1.0;
        d.scale[f] = (float)sc;
        d.inv_scale[f] = (float)(1.0 / sc);
    }
    d.buf[0] = a;
    d.buf[1] = b;
    d.clk = clk;
}

struct fvna_ctx {
    fvna_params p;
    SimDesc d;
    Launcher L;
    hipStream_t stream;         // caller's stream (borrowed)
    hipStream_t cap;            // private stream used only to capture graphs
    char* scratch;
    Clock* clk;
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    int device = 0;
    bool recording = false;     // a recorder follows every attempt
    RecDesc rec{};
    bool taylor = false;        // fvna_set_taylor was called
    double ta_amp_pa = 0.0, ta_x0_m = 0.0;
};

// One attempt on stream s: the step, then the CFL decision (and the recorder,
// in the same launch, if any).
static void launch_attempt(fvna_ctx* c, hipStream_t s)
{
    c->L.step(c->d, 0, 0, s);
    if (c->recording) c->L.ctrl_record(c->d, c->rec, s);
    else hipLaunchKernelGGL(k_ctrl, dim3(1), dim3(64), 0, s, c->d);
}

// Destroy the captured graph after every launch of it already enqueued on the
// context's stream has finished (a graph replay may still be in flight when a
// setter changes what the next capture must hold).
static void drop_graph(fvna_ctx* c)
{
    if (c->exec || c->graph) (void)hipStreamSynchronize(c->stream);
    if (c->exec) (void)hipGraphExecDestroy(c->exec);
    if (c->graph) (void)hipGraphDestroy(c->graph);
    c->exec = nullptr;
    c->graph = nullptr;
}

static fvna_status build_graph(fvna_ctx* c)
{
    if (c->exec) return FVNA_OK;
    HIP_TRY(hipStreamBeginCapture(c->cap, hipStreamCaptureModeThreadLocal));
    if (c->recording || !FVNA_FOLD_CONTROL) {
        for (int k = 0; k < GRAPH_CHUNK; ++k) launch_attempt(c, c->cap);
    } else {
        // attempts 1 .. GRAPH_CHUNK-1 take the decision on the attempt before
        // them in their prologue; one controller launch closes the graph
        for (int k = 0; k < GRAPH_CHUNK; ++k) c->L.step(c->d, 0, k, c->cap);
        hipLaunchKernelGGL(k_ctrl_fold, dim3(1), dim3(64), 0, c->cap, c->d, GRAPH_CHUNK - 1);
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(c->cap, &g));
    c->graph = g;
    HIP_TRY(hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0));
    return FVNA_OK;
}

// Host copy of the clock.
static fvna_status read_clock(fvna_ctx* c, Clock* h)
{
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(h, c->clk, sizeof(Clock), hipMemcpyDeviceToHost));
    return FVNA_OK;
}

static fvna_status status_of(int st)
{
    switch (st) {
    case 0: return FVNA_OK;
    case ST_NONHYP: return fail(FVNA_E_NONHYPERBOLIC, "non-real Roe speeds (discriminant <= 0) in a step");
    case ST_NONFINITE: return fail(FVNA_E_NONFINITE, "non-finite wave speed in a step");
    case ST_RETRIES: return fail(FVNA_E_RETRIES, "too many rejected attempts in a row");
    default: return fail(FVNA_E_STATE, "unknown device status");
    }
}

// Reset the clock to (t, dt) and recompute dt from the state if dt <= 0.
static fvna_status reset_clock(fvna_ctx* c, double t_dimless, double dt_dimless, int cur,
                               long long x_off = 0)
{
    Clock h;
    std::memset(&h, 0, sizeof(h));
    h.t = t_dimless;
    h.dt = dt_dimless > 0.0 ? dt_dimless : 0.0;
    h.cur = cur;
    h.x_off = x_off;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->clk, &h, sizeof(Clock), hipMemcpyHostToDevice));
    if (c->recording) {
        // the step count restarts at 0: the recorder counts from here on
        // (its descriptor is a kernel argument of the captured graph)
        c->rec.base = 0;
        drop_graph(c);
    }
    if (!(dt_dimless > 0.0)) {
        c->L.dry(c->d, c->stream);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_dt0, dim3(1), dim3(64), 0, c->stream, c->d);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(c->stream));
    }
    return FVNA_OK;
}

extern "C" {

fvna_status fvna_workspace_size(const fvna_params* p, size_t* state_bytes, size_t* scratch_bytes)
{
    fvna_status s = validate(p);
    if (s) return s;
    if (state_bytes) *state_bytes = state_bytes_of(p);
    if (scratch_bytes) *scratch_bytes = scratch_bytes_of(p);
    return FVNA_OK;
}

fvna_status fvna_create(const fvna_params* p, void* state_a, void* state_b, void* scratch, void* hip_stream,
                        fvna_ctx** out)
{
    if (!out) return fail(FVNA_E_INVALID, "out is NULL");
    *out = nullptr;
    fvna_status s = validate(p);
    if (s) return s;
    if (!state_a || !state_b || !scratch) return fail(FVNA_E_INVALID, "device buffer is NULL");
    if (((uintptr_t)state_a | (uintptr_t)state_b | (uintptr_t)scratch) % ALIGN)
        return fail(FVNA_E_INVALID, "device buffers must be 256-byte aligned");
    if (state_a == state_b) return fail(FVNA_E_INVALID, "state_a and state_b must differ");
    fvna_ctx* c = new (std::nothrow) fvna_ctx();
    if (!c) return fail(FVNA_E_NOMEM, "out of host memory");
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    c->scratch = (char*)scratch;
    c->clk = (Clock*)(c->scratch + OFF_CLOCK);
    c->L = pick_launcher(p->precision, p->geometry);
    int tr = p->tile_rows;
    if (tr == 0) {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune.find(std::make_tuple(p->precision, p->geometry, p->nx, p->ny));
        tr = it != g_tune.end() ? it->second : default_tile_rows(p, device_cu_count());
    }
    fill_desc(c->d, p, state_a, state_b, c->clk, tr);
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(FVNA_E_HIP, "cannot create the capture stream");
    }
    // zero state, t = 0
    const size_t sb = state_bytes_of(p);
    if (hipMemsetAsync(state_a, 0, sb, c->stream) != hipSuccess ||
        hipMemsetAsync(state_b, 0, sb, c->stream) != hipSuccess) {
        (void)hipStreamDestroy(c->cap);
        delete c;
        return fail(FVNA_E_HIP, "cannot clear the state buffers");
    }
    s = fill_rinv(c->d, p, c->scratch, c->stream);
    if (s) {
        (void)hipStreamDestroy(c->cap);
        delete c;
        return s;
    }
    s = reset_clock(c, 0.0, p->dt0 > 0 ? p->dt0 * p->c0 / p->dx : 0.0, 0);
    if (s) {
        (void)hipStreamDestroy(c->cap);
        delete c;
        return s;
    }
    *out = c;
    return FVNA_OK;
}

fvna_status fvna_set_bc(fvna_ctx* c, int32_t side, int32_t bc)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    if (side < 0 || side > 3) return fail(FVNA_E_INVALID, "side must be 0..3");
    fvna_params q = c->p;
    q.bc[side] = bc;
    fvna_status s = validate(&q);
    if (s) return s;
    c->p = q;
    c->d.bc[side] = bc;
    drop_graph(c);
    return FVNA_OK;
}

// Check a focused-source description and put it into a simulation
// descriptor (dimensionless); the per-row table goes to `tab` on `stream`.
static fvna_status apply_source(SimDesc& d, const fvna_params& p, const fvna_source* s, double* tab,
                                hipStream_t stream)
{
    if (!(s->freq > 0) || !(s->focal_length > 0) || !(s->aperture >= 0))
        return fail(FVNA_E_INVALID, "need freq > 0, focal_length > 0, aperture >= 0");
    if (s->envelope == FVNA_ENV_RAMP) {
        if (!(s->ramp_cycles > 0)) return fail(FVNA_E_INVALID, "the ramp envelope needs ramp_cycles > 0");
    } else if (s->envelope == FVNA_ENV_PACKET) {
        if (!(s->packet_cycles > 0)) return fail(FVNA_E_INVALID, "the packet envelope needs packet_cycles > 0");
    } else {
        return fail(FVNA_E_INVALID, "unknown source envelope");
    }
    if (s->second_stage != 0 && (s->second_stage != 1 || !std::isfinite(s->stage2_time)))
        return fail(FVNA_E_INVALID, "second_stage must be 0 or 1, with a finite stage2_time");
    d.sr_amp = s->p_surface / (p.rho0 * p.c0 * p.c0);
    d.sr_freq = s->freq * p.dx / p.c0;
    d.sr_F = s->focal_length / p.dx;
    d.sr_ap = s->aperture / p.dx;
    d.sr_ramp = s->envelope == FVNA_ENV_RAMP ? s->ramp_cycles : 1.0;
    d.sr_env = s->envelope;
    d.sr_W = s->envelope == FVNA_ENV_PACKET ? s->packet_cycles : 1.0;
    d.sr_t2 = s->second_stage ? s->stage2_time * p.c0 / p.dx : INFINITY;
    hipLaunchKernelGGL(k_src_table, dim3((p.ny + 255) / 256), dim3(256), 0, stream, tab, p.ny, d.sr_freq, d.sr_F);
    HIP_TRY(hipGetLastError());
    d.src_tab = tab;
    return FVNA_OK;
}

fvna_status fvna_set_source(fvna_ctx* c, int32_t side, const fvna_source* s)
{
    if (!c || !s) return fail(FVNA_E_INVALID, "NULL argument");
    if (side != 0) return fail(FVNA_E_INVALID, "the focused source is only available on side x-");
    drop_graph(c);
    HIP_TRY(hipStreamSynchronize(c->stream));
    SimDesc d = c->d;
    fvna_status st = apply_source(d, c->p, s, (double*)(c->scratch + OFF_SRCTAB), c->stream);
    if (st) return st;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->d = d;
    return FVNA_OK;
}

fvna_status fvna_set_taylor(fvna_ctx* c, double amplitude_pa, double x0_m, double angle)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    const fvna_params& p = c->p;
    if (!(amplitude_pa != 0.0) || !(p.delta > 0.0))
        return fail(FVNA_E_INVALID, "the Taylor profile needs a non-zero amplitude and delta > 0");
    const double a = amplitude_pa / (p.rho0 * p.c0 * p.c0);
    c->d.ta_amp = a;
    c->d.ta_w = (p.delta / p.c0) / (p.beta * a) / p.dx;
    c->d.ta_x0 = x0_m / p.dx;
    c->d.ta_y0 = 0.0;
    c->d.ta_cos = std::cos(angle);
    c->d.ta_sin = std::sin(angle);
    c->taylor = true;
    c->ta_amp_pa = amplitude_pa;
    c->ta_x0_m = x0_m;
    drop_graph(c);
    return FVNA_OK;
}

fvna_status fvna_set_state(fvna_ctx* c, const double* rho_p, const double* mom_x, const double* mom_y)
{
    if (!c || !rho_p || !mom_x || !mom_y) return fail(FVNA_E_INVALID, "NULL argument");
    const fvna_params& p = c->p;
    double* stage = (double*)(c->scratch + stage_off_of(&c->p));
    const size_t chunk_rows = std::max<size_t>(1, stage_cells_of(&p) / (size_t)p.nx);
    const double denom[3] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0};
    const double* src[3] = {rho_p, mom_x, mom_y};
    HIP_TRY(hipStreamSynchronize(c->stream));
    // the state goes into buffer 0; buffer 1 is cleared so padding stays zero
    HIP_TRY(hipMemsetAsync(c->d.buf[1], 0, state_bytes_of(&p), c->stream));
    for (int f = 0; f < 3; ++f)
        for (size_t r0 = 0; r0 < (size_t)p.ny; r0 += chunk_rows) {
            const size_t nr = std::min(chunk_rows, (size_t)p.ny - r0);
            HIP_TRY(hipMemcpyAsync(stage, src[f] + r0 * (size_t)p.nx, nr * (size_t)p.nx * sizeof(double),
                                   hipMemcpyHostToDevice, c->stream));
            c->L.imp(c->d, stage, f, (int)r0, (int)nr, denom[f], 0, c->stream);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    return reset_clock(c, 0.0, p.dt0 > 0 ? p.dt0 * p.c0 / p.dx : 0.0, 0);
}

fvna_status fvna_set_clock(fvna_ctx* c, double t, double dt_next)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    Clock h;
    fvna_status s = read_clock(c, &h);
    if (s) return s;
    const fvna_params& p = c->p;
    return reset_clock(c, t * p.c0 / p.dx, dt_next > 0 ? dt_next * p.c0 / p.dx : 0.0, h.cur, h.x_off);
}

// Enqueue exactly `attempts` attempts: whole captured chunks, then single launches.
static fvna_status enqueue_attempts(fvna_ctx* c, long long attempts)
{
    fvna_status s = build_graph(c);
    if (s) return s;
    for (long long k = 0; k < attempts / GRAPH_CHUNK; ++k) HIP_TRY(hipGraphLaunch(c->exec, c->stream));
    for (long long k = 0; k < attempts % GRAPH_CHUNK; ++k) launch_attempt(c, c->stream);
    HIP_TRY(hipGetLastError());
    return FVNA_OK;
}

fvna_status fvna_step(fvna_ctx* c, int64_t nsteps)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    if (nsteps < 0) return fail(FVNA_E_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return FVNA_OK;
    hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, c->stream, c->clk, (long long)nsteps);
    HIP_TRY(hipGetLastError());
    return enqueue_attempts(c, nsteps);
}

fvna_status fvna_sync(fvna_ctx* c)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    Clock h;
    for (int guard = 0; guard < 1000; ++guard) {
        fvna_status s = read_clock(c, &h);
        if (s) return s;
        if (h.status != 0 || h.accepted >= h.target) return status_of(h.status);
        // rejected attempts left steps owed: run more attempts
        s = enqueue_attempts(c, h.target - h.accepted);
        if (s) return s;
    }
    return fail(FVNA_E_STATE, "steps still owed after many top-up rounds");
}

fvna_status fvna_set_recorder(fvna_ctx* c, const fvna_recorder* r)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    if (!r) {
        HIP_TRY(hipStreamSynchronize(c->stream));
        c->recording = false;
        drop_graph(c);
        return FVNA_OK;
    }
    if (r->row < 0 || r->row >= c->p.ny) return fail(FVNA_E_INVALID, "recorder row outside the grid");
    if (r->path_len < 1 || !r->row_max) return fail(FVNA_E_INVALID, "recorder needs row_max and path_len >= 1");
    if (r->capacity < 0 || (r->capacity > 0 && (!r->probe_t || !r->probe_rho)))
        return fail(FVNA_E_INVALID, "recorder probe arrays missing for capacity > 0");
    if (r->probe_col < -1) return fail(FVNA_E_INVALID, "probe_col must be >= -1");
    Clock h;
    fvna_status s = read_clock(c, &h);
    if (s) return s;
    RecDesc d{};
    d.row = r->row;
    d.probe_col = r->probe_col;
    d.path_len = r->path_len;
    d.base = h.accepted;
    d.capacity = r->probe_col >= 0 ? r->capacity : 0;
    d.row_max = r->row_max;
    d.probe_t = r->probe_t;
    d.probe_rho = r->probe_rho;
    d.rho0 = c->p.rho0;
    d.t_unit = c->p.dx / c->p.c0;
    c->rec = d;
    c->recording = true;
    drop_graph(c);
    return FVNA_OK;
}

fvna_status fvna_shift(fvna_ctx* c, int32_t ncols)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    if (ncols < 0 || ncols > c->p.nx) return fail(FVNA_E_INVALID, "ncols must be in [0, nx]");
    if (c->p.bc[0] == FVNA_BC_PERIODIC)
        return fail(FVNA_E_INVALID, "a periodic x axis cannot move");
    if (ncols == 0) return FVNA_OK;
    c->L.shift(c->d, ncols, c->stream);
    HIP_TRY(hipGetLastError());
    return FVNA_OK;
}

fvna_status fvna_step_window(fvna_ctx* c, const fvna_window* w, fvna_window_state* st, int64_t nsteps)
{
    if (!c || !w || !st) return fail(FVNA_E_INVALID, "NULL argument");
    if (nsteps < 0) return fail(FVNA_E_INVALID, "nsteps must be >= 0");
    if (w->check_every < 1 || w->quantum < 1 || !std::isfinite(w->t1))
        return fail(FVNA_E_INVALID, "need check_every >= 1, quantum >= 1 and a finite t1");
    if (!(w->speed >= 0.0) || !std::isfinite(w->speed)) return fail(FVNA_E_INVALID, "speed must be finite and >= 0");
    if (st->x_off < 0 || st->phase < 0 || st->phase >= w->check_every)
        return fail(FVNA_E_INVALID, "window state out of range");
    if (c->p.bc[0] == FVNA_BC_PERIODIC) return fail(FVNA_E_INVALID, "a periodic x axis cannot move");
    const fvna_params& p = c->p;
    const double t1 = w->t1 * p.c0 / p.dx;        // cells travelled at c0 per unit time
    const double speed = w->speed > 0.0 ? w->speed : 1.0;
    while (nsteps > 0) {
        const int64_t k = std::min<int64_t>(nsteps, w->check_every - st->phase);
        fvna_status s = fvna_step(c, k);
        if (s) return s;
        s = fvna_sync(c);
        if (s) return s;
        nsteps -= k;
        st->phase += k;
        if (st->phase < w->check_every) continue;
        st->phase = 0;
        Clock h;
        s = read_clock(c, &h);
        if (s) return s;
        if (!(h.t >= t1)) continue;
        const int64_t target = (int64_t)w->quantum * (int64_t)std::floor((h.t - t1) * speed / w->quantum);
        if (target <= st->x_off) continue;
        // a move of nx or more columns leaves undisturbed medium everywhere;
        // the device offset still advances by the whole move, so that path
        // columns (recorder) and st->x_off stay equal
        const int64_t move = target - st->x_off;
        if (move > (int64_t)INT32_MAX - (int64_t)p.nx)
            return fail(FVNA_E_INVALID, "moving-domain jump too large");
        c->L.shift(c->d, (int)move, c->stream);
        HIP_TRY(hipGetLastError());
        st->x_off = target;
    }
    return FVNA_OK;
}

// Copy a window of the current state of a context out (no synchronisation of
// owed steps).
static fvna_status export_window(fvna_ctx* c, int i0, int j0, int ni, int nj, double* rho_p, double* mom_x,
                                 double* mom_y)
{
    const fvna_params& p = c->p;
    double* stage = (double*)(c->scratch + stage_off_of(&c->p));
    const size_t chunk_rows = std::max<size_t>(1, stage_cells_of(&p) / (size_t)ni);
    const double factor[3] = {p.rho0, p.rho0 * p.c0, p.rho0 * p.c0};
    double* dst[3] = {rho_p, mom_x, mom_y};
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int f = 0; f < 3; ++f)
        for (size_t r0 = 0; r0 < (size_t)nj; r0 += chunk_rows) {
            const size_t nr = std::min(chunk_rows, (size_t)nj - r0);
            c->L.exp(c->d, stage, f, (int)(j0 + r0), (int)nr, i0, ni, factor[f], c->stream);
            HIP_TRY(hipGetLastError());
            HIP_TRY(hipMemcpyAsync(dst[f] + r0 * (size_t)ni, stage, nr * (size_t)ni * sizeof(double),
                                   hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
    return FVNA_OK;
}

static fvna_status export_state(fvna_ctx* c, double* rho_p, double* mom_x, double* mom_y)
{
    return export_window(c, 0, 0, c->p.nx, c->p.ny, rho_p, mom_x, mom_y);
}

static void stats_from_clock(const Clock& h, const fvna_params& p, fvna_stats* st)
{
    const double tu = p.dx / p.c0;
    st->t = h.t * tu;
    st->dt_next = h.dt * tu;
    st->nu_last = h.nu_last;
    st->nu_mean = h.nu_mean;
    st->nu_std = h.nu_count > 0 ? std::sqrt(h.nu_m2 / (double)h.nu_count) : 0.0;
    st->steps = h.accepted;
    st->rejected = h.rejected;
    st->status = h.status;
    st->status_step = h.status_step;
}

static fvna_status stats_of(fvna_ctx* c, fvna_stats* st)
{
    Clock h;
    fvna_status r = read_clock(c, &h);
    if (r) return r;
    const double tu = c->p.dx / c->p.c0;
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

static bool is_device_error(fvna_status s)
{
    return s == FVNA_E_NONHYPERBOLIC || s == FVNA_E_NONFINITE || s == FVNA_E_RETRIES;
}

fvna_status fvna_get_state(fvna_ctx* c, double* rho_p, double* mom_x, double* mom_y)
{
    if (!c || !rho_p || !mom_x || !mom_y) return fail(FVNA_E_INVALID, "NULL argument");
    const fvna_status dev = fvna_sync(c);
    if (dev != FVNA_OK && !is_device_error(dev)) return dev;
    const std::string msg = g_err;
    fvna_status s = export_state(c, rho_p, mom_x, mom_y);
    if (s) return s;
    if (dev != FVNA_OK) g_err = msg;
    return dev;
}

fvna_status fvna_get_window(fvna_ctx* c, int32_t i0, int32_t j0, int32_t ni, int32_t nj, double* rho_p,
                            double* mom_x, double* mom_y)
{
    if (!c || !rho_p || !mom_x || !mom_y) return fail(FVNA_E_INVALID, "NULL argument");
    if (ni < 1 || nj < 1 || i0 < 0 || j0 < 0 || (long long)i0 + ni > c->p.nx || (long long)j0 + nj > c->p.ny)
        return fail(FVNA_E_INVALID, "window outside the grid");
    const fvna_status dev = fvna_sync(c);
    if (dev != FVNA_OK && !is_device_error(dev)) return dev;
    const std::string msg = g_err;
    fvna_status s = export_window(c, i0, j0, ni, nj, rho_p, mom_x, mom_y);
    if (s) return s;
    if (dev != FVNA_OK) g_err = msg;
    return dev;
}

fvna_status fvna_get_stats(fvna_ctx* c, fvna_stats* st)
{
    if (!c || !st) return fail(FVNA_E_INVALID, "NULL argument");
    const fvna_status dev = fvna_sync(c);
    if (dev != FVNA_OK && !is_device_error(dev)) return dev;
    const std::string msg = g_err;
    fvna_status s = stats_of(c, st);
    if (s) return s;
    if (dev != FVNA_OK) g_err = msg;
    return dev;
}

fvna_status fvna_sums(fvna_ctx* c, double out[3])
{
    if (!c || !out) return fail(FVNA_E_INVALID, "NULL argument");
    fvna_status s = fvna_sync(c);
    if (s != FVNA_OK && !is_device_error(s)) return s;
    double* part = (double*)(c->scratch + OFF_PART);
    double* res = (double*)(c->scratch + OFF_SUMOUT);
    const double factor[3] = {c->p.rho0, c->p.rho0 * c->p.c0, c->p.rho0 * c->p.c0};
    c->L.sums(c->d, nullptr, part, res, factor, c->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(out, res, 3 * sizeof(double), hipMemcpyDeviceToHost));
    return FVNA_OK;
}

fvna_status fvna_taylor_errors(fvna_ctx* c, double front0_x_m, double front0_y_m, double half_length_m,
                               double out[2])
{
    if (!c || !out) return fail(FVNA_E_INVALID, "NULL argument");
    if (!c->taylor) return fail(FVNA_E_INVALID, "no Taylor profile set (fvna_set_taylor)");
    if (!(half_length_m > 0.0) || !std::isfinite(front0_x_m) || !std::isfinite(front0_y_m))
        return fail(FVNA_E_INVALID, "need a positive half length and a finite front point");
    fvna_status s = fvna_sync(c);
    if (s != FVNA_OK && !is_device_error(s)) return s;
    Clock h;
    s = read_clock(c, &h);
    if (s) return s;
    const fvna_params& p = c->p;
    ErrLine L;
    L.c = c->d.ta_cos;
    L.s = c->d.ta_sin;
    L.dx = p.dx;
    L.x0 = c->ta_x0_m;
    const double t = h.t * (p.dx / p.c0);
    L.c0t = p.c0 * t;
    L.fx = front0_x_m + L.c0t * L.c;
    L.fy = front0_y_m + L.c0t * L.s;
    L.w = c->d.ta_w * p.dx;
    L.amp = c->d.ta_amp;
    L.x_off = h.x_off;
    L.steep = std::fabs(L.c) < std::fabs(L.s) ? 1 : 0;
    const double f = L.steep ? L.fy : L.fx, cs = L.steep ? L.s : L.c;
    const double lo = std::ceil((f - half_length_m * cs) / p.dx - 0.5);
    const double hi = std::floor((f + half_length_m * cs) / p.dx - 0.5);
    if (!(hi >= lo) || !(std::fabs(hi) < 4.0e18) || !(std::fabs(lo) < 4.0e18))
        return fail(FVNA_E_INVALID, "the line has no cells");
    L.a0 = (long long)lo;
    L.n = (long long)hi - (long long)lo + 1;
    double* res = (double*)(c->scratch + OFF_SUMOUT);
    c->L.taylor_err(c->d, L, res, c->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(out, res, 2 * sizeof(double), hipMemcpyDeviceToHost));
    if (!std::isfinite(out[0]) || !std::isfinite(out[1]))
        return fail(FVNA_E_INVALID, "no cell of the line lies in the domain");
    return FVNA_OK;
}

// Scratch of fvna_sums_noalloc: the partial sums of k_sums_partial, in a
// static device array rather than caller or library allocations.  Each device
// holds its own copy at its own address, found once per device with
// hipGetSymbolAddress and kept in noalloc_ptr (the array's name is not a
// device address in host code).  Every call on a device shares that copy.
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) double noalloc_scratch[SUM_BLOCKS * 3];
static std::mutex g_noalloc_mu;
static void* g_noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

static fvna_status noalloc_ptr(void** ptr)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(FVNA_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> g(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
        void* p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)));
        if (!p) return fail(FVNA_E_HIP, "hipGetSymbolAddress returned no address for the static scratch");
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return FVNA_OK;
}

fvna_status fvna_sums_noalloc(const fvna_params* p, const void* state, void* hip_stream, double* out)
{
    if (!state || !out) return fail(FVNA_E_INVALID, "NULL argument");
    fvna_status s = validate(p);
    if (s) return s;
    if (((uintptr_t)state | (uintptr_t)out) % 8) return fail(FVNA_E_INVALID, "state and out must be 8-byte aligned");
    void* part = nullptr;
    s = noalloc_ptr(&part);
    if (s) return s;
    SimDesc d;
    fill_desc(d, p, const_cast<void*>(state), const_cast<void*>(state), nullptr, 16);
    const Launcher L = pick_launcher(p->precision, p->geometry);
    const double factor[3] = {p->rho0, p->rho0 * p->c0, p->rho0 * p->c0};
    L.sums(d, state, (double*)part, out, factor, (hipStream_t)hip_stream);
    HIP_TRY(hipGetLastError());
    return FVNA_OK;
}

fvna_status fvna_time_step_kernel(fvna_ctx* c, int32_t reps, double* ms_per_launch)
{
    if (!c || !ms_per_launch || reps < 1) return fail(FVNA_E_INVALID, "bad argument");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, c->stream));
    for (int k = 0; k < reps; ++k) c->L.step(c->d, 1, 0, c->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    return FVNA_OK;
}

fvna_status fvna_get_tile_rows(fvna_ctx* c, int32_t* tile_rows)
{
    if (!c || !tile_rows) return fail(FVNA_E_INVALID, "NULL argument");
    *tile_rows = c->d.tile_rows;
    return FVNA_OK;
}

fvna_status fvna_autotune(fvna_ctx* c, int32_t* tile_rows)
{
    if (!c) return fail(FVNA_E_INVALID, "ctx is NULL");
    // candidates: segments that fill the device in 1, 2 or 3 whole rounds, and
    // a few fixed heights
    std::vector<int> cand = {32, 48, 64, 96, 128};
    {
        const int w = c->p.precision == FVNA_F64 ? 2 : 4;
        const long long slots = (long long)device_cu_count() * 4 * w;
        const long long strips = c->d.strips;
        for (int rounds = 1; rounds <= 3; ++rounds) {
            const long long per = std::max(1ll, rounds * slots / strips);
            const long long tr = (c->p.ny + per - 1) / per;
            if (tr >= 16) cand.push_back((int)tr);
        }
    }
    double best = 1e30;
    int best_tr = c->d.tile_rows;
    for (int tr : cand) {
        if (tr > 2 * c->p.ny) continue;
        set_segments(c->d, tr);
        double ms = 0.0;
        fvna_status s = fvna_time_step_kernel(c, 1, &ms);       // warm-up
        if (!s) s = fvna_time_step_kernel(c, 5, &ms);
        if (s) return s;
        if (ms < best) { best = ms; best_tr = tr; }
    }
    set_segments(c->d, best_tr);
    // the timing launches left this attempt's speeds in the clock; they are
    // exactly what the next real attempt computes, so nothing to undo
    drop_graph(c);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        g_tune[std::make_tuple(c->p.precision, c->p.geometry, c->p.nx, c->p.ny)] = best_tr;
    }
    if (tile_rows) *tile_rows = best_tr;
    return FVNA_OK;
}

const char* fvna_last_error(void) { return g_err.c_str(); }

void fvna_destroy(fvna_ctx* c)
{
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graph(c);
    (void)hipStreamDestroy(c->cap);
    delete c;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batched form
// ---------------------------------------------------------------------------

struct fvna_batch {
    int n = 0;
    std::vector<fvna_params> p;
    std::vector<SimDesc> d;
    std::vector<char*> scratch;
    Launcher L;
    hipStream_t stream;
    hipStream_t cap;
    SimDesc* d_desc = nullptr;      // device copy of the descriptors
    TileRef* d_tiles = nullptr;
    int ntiles = 0;
    int tile_cap = 0;               // TileRefs d_tiles can hold
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
};

namespace {

// Batch autotune cache: (precision, geometry, the members' (nx, ny) in order)
// -> the chosen segment height of each member.
typedef std::tuple<int, int, std::vector<std::pair<int, int>>> BatchKey;
std::mutex g_btune_mu;
std::map<BatchKey, std::vector<int>> g_btune;

BatchKey batch_key(const fvna_params* p, int n)
{
    std::vector<std::pair<int, int>> g;
    for (int k = 0; k < n; ++k) g.emplace_back(p[k].nx, p[k].ny);
    return BatchKey(p[0].precision, p[0].geometry, g);
}

void batch_tiles(const fvna_batch* b, std::vector<TileRef>& tiles)
{
    tiles.clear();
    for (int k = 0; k < b->n; ++k)
        for (int sg = 0; sg < b->d[k].segs; ++sg)
            for (int st = 0; st < b->d[k].strips; ++st) tiles.push_back(TileRef{k, st, sg, 0});
}

}  // namespace

static fvna_status batch_graph(fvna_batch* b)
{
    if (b->exec) return FVNA_OK;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    for (int k = 0; k < GRAPH_CHUNK; ++k) {
        b->L.step_batch(b->d_desc, b->d_tiles, b->ntiles, 0, b->cap);
        hipLaunchKernelGGL(k_ctrl_batch, dim3((b->n + 63) / 64), dim3(64), 0, b->cap, b->d_desc, b->n);
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(b->cap, &g));
    b->graph = g;
    HIP_TRY(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    return FVNA_OK;
}

// A batch member seen as a single context (shares kernels and conversions).
static fvna_ctx member_ctx(fvna_batch* b, int k)
{
    fvna_ctx c;
    c.p = b->p[k];
    c.d = b->d[k];
    c.L = b->L;
    c.stream = b->stream;
    c.cap = b->cap;
    c.scratch = b->scratch[k];
    c.clk = (Clock*)(b->scratch[k] + OFF_CLOCK);
    return c;
}

extern "C" {

fvna_status fvna_batch_create(int32_t n, const fvna_params* per_sim, void* const* bufs, void* hip_stream,
                              fvna_batch** out)
{
    if (!out || !per_sim || !bufs || n < 1) return fail(FVNA_E_INVALID, "bad argument");
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        fvna_status s = validate(&per_sim[k]);
        if (s) return fail(s, "simulation " + std::to_string(k) + ": " + g_err);
        if (per_sim[k].precision != per_sim[0].precision || per_sim[k].geometry != per_sim[0].geometry)
            return fail(FVNA_E_INVALID, "all simulations of a batch need the same precision and geometry");
        for (int j = 0; j < 3; ++j)
            if (!bufs[3 * k + j] || ((uintptr_t)bufs[3 * k + j]) % ALIGN)
                return fail(FVNA_E_INVALID, "device buffers must be non-NULL and 256-byte aligned");
    }
    fvna_batch* b = new (std::nothrow) fvna_batch();
    if (!b) return fail(FVNA_E_NOMEM, "out of host memory");
    b->n = n;
    b->stream = (hipStream_t)hip_stream;
    b->L = pick_launcher(per_sim[0].precision, per_sim[0].geometry);
    std::vector<int> tuned;
    {
        std::lock_guard<std::mutex> g(g_btune_mu);
        auto it = g_btune.find(batch_key(per_sim, n));
        if (it != g_btune.end()) tuned = it->second;
    }
    for (int k = 0; k < n; ++k) {
        const fvna_params& p = per_sim[k];
        b->p.push_back(p);
        SimDesc d;
        // many simulations fill the device in many rounds: moderate segments
        // (or the heights fvna_batch_autotune chose for this composition)
        int tr = p.tile_rows ? p.tile_rows : (tuned.empty() ? BATCH_TILE_ROWS : tuned[k]);
        char* sc = (char*)bufs[3 * k + 2];
        fill_desc(d, &p, bufs[3 * k], bufs[3 * k + 1], (Clock*)(sc + OFF_CLOCK), tr, false);
        const fvna_status sr = fill_rinv(d, &p, sc, b->stream);
        if (sr) {
            delete b;
            return sr;
        }
        b->d.push_back(d);
        b->scratch.push_back(sc);
    }
    std::vector<TileRef> tiles;
    batch_tiles(b, tiles);
    b->ntiles = (int)tiles.size();
    b->tile_cap = b->ntiles;
    auto cleanup = [&]() {
        if (b->d_desc) (void)hipFree(b->d_desc);
        if (b->d_tiles) (void)hipFree(b->d_tiles);
        delete b;
    };
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return fail(FVNA_E_HIP, "cannot create the capture stream");
    }
    if (hipMalloc(&b->d_desc, sizeof(SimDesc) * n) != hipSuccess ||
        hipMalloc(&b->d_tiles, sizeof(TileRef) * tiles.size()) != hipSuccess) {
        (void)hipStreamDestroy(b->cap);
        cleanup();
        return fail(FVNA_E_HIP, "cannot allocate the batch tables");
    }
    if (hipMemcpy(b->d_desc, b->d.data(), sizeof(SimDesc) * n, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->d_tiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipStreamDestroy(b->cap);
        cleanup();
        return fail(FVNA_E_HIP, "cannot upload the batch tables");
    }
    for (int k = 0; k < n; ++k) {
        fvna_ctx c = member_ctx(b, k);
        const fvna_params& p = per_sim[k];
        const size_t sb = state_bytes_of(&p);
        if (hipMemsetAsync(c.d.buf[0], 0, sb, b->stream) != hipSuccess ||
            hipMemsetAsync(c.d.buf[1], 0, sb, b->stream) != hipSuccess ||
            reset_clock(&c, 0.0, p.dt0 > 0 ? p.dt0 * p.c0 / p.dx : 0.0, 0) != FVNA_OK) {
            (void)hipStreamDestroy(b->cap);
            cleanup();
            return fail(FVNA_E_HIP, "cannot initialise simulation " + std::to_string(k));
        }
    }
    *out = b;
    return FVNA_OK;
}

fvna_status fvna_batch_set_state(fvna_batch* b, int32_t k, const double* rho_p, const double* mom_x,
                                 const double* mom_y)
{
    if (!b || k < 0 || k >= b->n) return fail(FVNA_E_INVALID, "bad simulation index");
    fvna_ctx c = member_ctx(b, k);
    return fvna_set_state(&c, rho_p, mom_x, mom_y);
}

static fvna_status batch_enqueue(fvna_batch* b, long long attempts)
{
    fvna_status s = batch_graph(b);
    if (s) return s;
    for (long long k = 0; k < attempts / GRAPH_CHUNK; ++k) HIP_TRY(hipGraphLaunch(b->exec, b->stream));
    for (long long k = 0; k < attempts % GRAPH_CHUNK; ++k) {
        b->L.step_batch(b->d_desc, b->d_tiles, b->ntiles, 0, b->stream);
        hipLaunchKernelGGL(k_ctrl_batch, dim3((b->n + 63) / 64), dim3(64), 0, b->stream, b->d_desc, b->n);
    }
    HIP_TRY(hipGetLastError());
    return FVNA_OK;
}

fvna_status fvna_batch_step(fvna_batch* b, int64_t nsteps)
{
    if (!b) return fail(FVNA_E_INVALID, "batch is NULL");
    if (nsteps < 0) return fail(FVNA_E_INVALID, "nsteps must be >= 0");
    if (nsteps == 0) return FVNA_OK;
    hipLaunchKernelGGL(k_bump_batch, dim3((b->n + 63) / 64), dim3(64), 0, b->stream, b->d_desc, b->n,
                       (long long)nsteps);
    HIP_TRY(hipGetLastError());
    return batch_enqueue(b, nsteps);
}

fvna_status fvna_batch_sync(fvna_batch* b)
{
    if (!b) return fail(FVNA_E_INVALID, "batch is NULL");
    for (int guard = 0; guard < 1000; ++guard) {
        HIP_TRY(hipStreamSynchronize(b->stream));
        long long owed = 0;
        int worst = 0;
        for (int k = 0; k < b->n; ++k) {
            Clock h;
            HIP_TRY(hipMemcpy(&h, b->scratch[k] + OFF_CLOCK, sizeof(Clock), hipMemcpyDeviceToHost));
            if (h.status) worst = worst ? worst : h.status;
            else owed = std::max(owed, h.target - h.accepted);
        }
        if (owed <= 0) return status_of(worst);
        fvna_status s = batch_enqueue(b, owed);
        if (s) return s;
    }
    return fail(FVNA_E_STATE, "steps still owed after many top-up rounds");
}

// Device status of one member, as a status code (message set).
static fvna_status member_status(fvna_ctx* c)
{
    Clock h;
    fvna_status r = read_clock(c, &h);
    if (r) return r;
    return status_of(h.status);
}

fvna_status fvna_batch_get_state(fvna_batch* b, int32_t k, double* rho_p, double* mom_x, double* mom_y)
{
    if (!b || k < 0 || k >= b->n || !rho_p || !mom_x || !mom_y) return fail(FVNA_E_INVALID, "bad argument");
    const fvna_status bs = fvna_batch_sync(b);
    if (bs != FVNA_OK && !is_device_error(bs)) return bs;
    fvna_ctx c = member_ctx(b, k);
    const fvna_status dev = member_status(&c);
    if (dev != FVNA_OK && !is_device_error(dev)) return dev;
    const std::string msg = g_err;
    fvna_status s = export_state(&c, rho_p, mom_x, mom_y);
    if (s) return s;
    if (dev != FVNA_OK) g_err = msg;
    return dev;
}

fvna_status fvna_batch_get_stats(fvna_batch* b, int32_t k, fvna_stats* st)
{
    if (!b || k < 0 || k >= b->n || !st) return fail(FVNA_E_INVALID, "bad argument");
    const fvna_status bs = fvna_batch_sync(b);
    if (bs != FVNA_OK && !is_device_error(bs)) return bs;
    fvna_ctx c = member_ctx(b, k);
    const fvna_status dev = member_status(&c);
    if (dev != FVNA_OK && !is_device_error(dev)) return dev;
    const std::string msg = g_err;
    fvna_status s = stats_of(&c, st);
    if (s) return s;
    if (dev != FVNA_OK) g_err = msg;
    return dev;
}

// Upload the descriptors and tile table after a change of segment heights
// (the captured graph holds the old tile count: dropped).
static fvna_status batch_retile(fvna_batch* b)
{
    if (b->exec || b->graph) {
        HIP_TRY(hipStreamSynchronize(b->stream));
        if (b->exec) (void)hipGraphExecDestroy(b->exec);
        if (b->graph) (void)hipGraphDestroy(b->graph);
        b->exec = nullptr;
        b->graph = nullptr;
    }
    std::vector<TileRef> tiles;
    batch_tiles(b, tiles);
    HIP_TRY(hipStreamSynchronize(b->stream));
    if ((int)tiles.size() > b->tile_cap) {
        TileRef* t = nullptr;
        HIP_TRY(hipMalloc(&t, sizeof(TileRef) * tiles.size()));
        (void)hipFree(b->d_tiles);
        b->d_tiles = t;
        b->tile_cap = (int)tiles.size();
    }
    HIP_TRY(hipMemcpy(b->d_tiles, tiles.data(), sizeof(TileRef) * tiles.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(b->d_desc, b->d.data(), sizeof(SimDesc) * b->n, hipMemcpyHostToDevice));
    b->ntiles = (int)tiles.size();
    return FVNA_OK;
}

fvna_status fvna_batch_autotune(fvna_batch* b, int32_t* tile_rows)
{
    if (!b) return fail(FVNA_E_INVALID, "batch is NULL");
    // size classes by ny (powers of two); members with their own tile_rows keep it
    std::map<int, std::vector<int>> cls;
    for (int k = 0; k < b->n; ++k)
        if (b->p[k].tile_rows == 0) {
            int c = 0;
            while ((2 << c) <= b->p[k].ny) ++c;
            cls[c].push_back(k);
        }
    const int cand[] = {32, 48, 64, 96, 128, 192, 256};
    auto time_it = [&](double* ms) -> fvna_status {
        fvna_status s = fvna_batch_time_step_kernel(b, 1, ms);      // warm-up
        if (!s) s = fvna_batch_time_step_kernel(b, 5, ms);
        return s;
    };
    // one pass of coordinate descent over the classes, smallest grids first
    for (auto& kv : cls) {
        const int cur = b->d[kv.second[0]].tile_rows;
        double best = 1e30;
        int best_tr = cur;
        for (int tr : cand) {
            bool useful = false;
            for (int k : kv.second) useful = useful || tr < 2 * b->p[k].ny;
            if (!useful) continue;
            for (int k : kv.second) set_segments(b->d[k], tr, false);
            fvna_status s = batch_retile(b);
            double ms = 0.0;
            if (!s) s = time_it(&ms);
            if (s) return s;
            if (ms < best) { best = ms; best_tr = tr; }
        }
        for (int k : kv.second) set_segments(b->d[k], best_tr, false);
    }
    fvna_status s = batch_retile(b);
    if (s) return s;
    std::vector<int> chosen(b->n);
    for (int k = 0; k < b->n; ++k) chosen[k] = b->d[k].tile_rows;
    {
        std::lock_guard<std::mutex> g(g_btune_mu);
        g_btune[batch_key(b->p.data(), b->n)] = chosen;
    }
    if (tile_rows)
        for (int k = 0; k < b->n; ++k) tile_rows[k] = chosen[k];
    return FVNA_OK;
}

fvna_status fvna_batch_get_tile_rows(fvna_batch* b, int32_t* tile_rows)
{
    if (!b || !tile_rows) return fail(FVNA_E_INVALID, "NULL argument");
    for (int k = 0; k < b->n; ++k) tile_rows[k] = b->d[k].tile_rows;
    return FVNA_OK;
}

fvna_status fvna_batch_time_step_kernel(fvna_batch* b, int32_t reps, double* ms_per_launch)
{
    if (!b || !ms_per_launch || reps < 1) return fail(FVNA_E_INVALID, "bad argument");
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, b->stream));
    for (int k = 0; k < reps; ++k) b->L.step_batch(b->d_desc, b->d_tiles, b->ntiles, 1, b->stream);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms_per_launch = (double)ms / reps;
    return FVNA_OK;
}

void fvna_batch_destroy(fvna_batch* b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    (void)hipStreamDestroy(b->cap);
    (void)hipFree(b->d_desc);
    (void)hipFree(b->d_tiles);
    delete b;
}

}  // extern "C"

