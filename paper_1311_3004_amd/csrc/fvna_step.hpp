// fvna_step.hpp -- the step kernels of libfvna: one launch = one attempted
// time step over every tile of one simulation (k_step) or of many
// simulations (k_step_batch).  The per-tile work is march_tile of
// fvna_device.hpp.
#pragma once

#include "fvna_device.hpp"

namespace fvna {

// Waves per SIMD the register allocation must allow: three for FP32 compute
// (168 VGPRs, no spills; with tiles that fill every slot in one round this
// measured 9% faster than four waves at 128 VGPRs on a 4096^2 grid and level
// on 8192^2), two for FP64.
#ifndef FVNA_F32_WAVES_PER_SIMD
#define FVNA_F32_WAVES_PER_SIMD 3
#endif
template <typename T> struct Occupancy { static constexpr int waves = sizeof(T) == 8 ? 2 : FVNA_F32_WAVES_PER_SIMD; };

// One attempted step over the whole grid.  force = 1 (timing): run even when
// no step is owed.
// Workgroups are handed to the XCDs round-robin (block b to XCD b mod 8,
// each with its own L2).  Block b is given logical block start(x) + b / 8 of
// XCD x = b mod 8, so every XCD works on one contiguous run of tiles, which
// in row-major tile order is a band of whole segment rows: the halo columns
// of side-by-side strips and the warm-up rows of stacked segments are then
// read into the same L2.  A bijection of block indices; results do not
// depend on it.
constexpr int XCDS = 8;
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
    const int x = b % XCDS, k = b / XCDS;
    const int per = nblocks / XCDS, rem = nblocks % XCDS;
    return x * per + min(x, rem) + k;
}

// pos = 0: the attempt runs with the clock as it stands and its CFL maximum
// goes to the clock (a controller launch decides after it).  pos >= 1 (the
// attempts of a captured graph after its first): the attempt first takes the
// decision on the attempt before it itself.  Every wavefront computes it
// (control_next) from that attempt's clock state -- the clock for pos = 1,
// shadow copy (pos - 1) mod 2 after -- and its CFL slot (pos - 1) mod 3,
// none of which this launch writes; the grid's first wavefront stores the
// result as shadow copy pos mod 2; this attempt's maximum goes to slot
// pos mod 3.  Every attempt (pos 0 included) clears slot (pos + 1) mod 3
// for the one after it.  A closing k_ctrl_fold takes the last decision of
// the graph into the clock.
template <typename S, typename T, int AXI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occupancy<T>::waves)))
void k_step(SimDesc d, int force, int pos)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wave;
    if (tile >= d.strips * d.segs) return;
    Clock* clk = d.clk;
    ClockAux* aux = clock_aux(clk);
    pos = max(pos, 0);
    Clock h;
    if (pos == 0) {
        h = *clk;
    } else {
        const Clock& prev = pos == 1 ? *clk : aux->shadow[(pos - 1) & 1];
        unsigned long long* psb;
        unsigned int* pfl;
        cfl_slot(clk, (pos - 1) % 3, psb, pfl);
        h = control_next(prev, *psb, *pfl, d.fixed_dt, d.cfl_target, d.cfl_max, d.max_retries, 2);
    }
    // the grid's first wavefront: this attempt's state for the next one, and
    // a cleared CFL slot for the next one to accumulate into (slot 1 after an
    // attempt at pos 0, which the others of its graph then follow)
    if (tile == 0 && (threadIdx.x & (WAVE - 1)) == 0) {
        if (pos >= 1) aux->shadow[pos & 1] = h;
        unsigned long long* nsb;
        unsigned int* nfl;
        cfl_slot(clk, (pos + 1) % 3, nsb, nfl);
        *nsb = 0ull;
        *nfl = 0u;
    }
    unsigned long long* sb;
    unsigned int* fl;
    cfl_slot(clk, pos % 3, sb, fl);
    if (!force && (h.status != 0 || h.accepted >= h.target)) return;
    march_tile<S, T, AXI>(d, tile % d.strips, tile / d.strips, attempt_of(h, sb, fl));
}

struct TileRef { int sim, strip, seg, pad; };

template <typename S, typename T, int AXI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Occupancy<T>::waves)))
void k_step_batch(const SimDesc* __restrict__ descs, const TileRef* __restrict__ tiles, int ntiles, int force)
{
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = xcd_block(blockIdx.x, gridDim.x) * WAVES_PER_BLOCK + wave;
    if (tile >= ntiles) return;
    const TileRef tr = tiles[tile];
    const SimDesc& d = descs[tr.sim];
    Clock* clk = d.clk;
    const Clock h = *clk;
    if (!force && (h.status != 0 || h.accepted >= h.target)) return;
    march_tile<S, T, AXI>(d, tr.strip, tr.seg, attempt_of(h, &clk->smax_bits, &clk->flags));
}

}  // namespace fvna
