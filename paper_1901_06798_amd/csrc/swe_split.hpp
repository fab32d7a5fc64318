// swe_split.hpp -- the split step kernel (one wave64 per strip task) and the
// CFL rule fused into its last wave.  Included by swe_step.hip, which
// instantiates the FP64 kernels (and the FP32-storage, FP64-arithmetic
// ones), and by swe_step_f32.hip, which instantiates the FP32
// surface-deviation kernels in a unit of their own (built with contracted
// multiply-adds: that path is held to its surface bar in metres, not to the
// FP64 path's rounding).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "swe.h"
#include "swe_common.hpp"
#include "swe_march.hpp"
#include "swe_math.hpp"

namespace swe {

// Arguments of one patch step.  Planes hold doubles (FP64: h, hu, hv, b) or
// floats (surface-deviation path: eta', hu, hv, b).
struct StepArgs {
    const void* qin;
    void* qout;
    const void* b;
    const double* dt;
    double* smax;
    uint32_t* status;
    int64_t off, ps;
    double dx, dy;
    int pitch, mx, my, H, nstrips, nitems;
    int8_t bc[4];
    DevParams P;
    const uint32_t* gate;  // retake launch: run only if *gate != 0; NULL: always
    // launch order (NULL: task k at position k): position k runs task
    // order[k] - 1, or task k where order[k] is 0 or out of range
    const uint32_t* order;
    uint32_t* cost;  // per task, the march's solved row sweeps (NULL: not kept)
    const double* metric;  // latitude-longitude patch: capacities, edge lengths
    int xcd_run;           // ranks dealt to an XCD in runs of this many (1: in turn)
    // CFL rule in the launch's last wave (NULL done: none): done counts the
    // finished waves; the rule writes *dt_next, flags[0] (NULL: no retake
    // flag), status
    uint32_t* done;
    double* dt_next;
    uint32_t* flags;
    uint32_t* status_out;  // status the settled conditions join (status then holds
                           // the launch's pending pair)
    double cfl_desired, cfl_max;
    int tref;
};

// The CFL rule of one group (swe_cfl_reduce with the group's one patch) in
// the launch's last wave to finish.  Every wave's speeds reach smax by
// device-scope atomics, which are performed coherently across the XCDs'
// caches; a wave waits for its atomics to complete (a workgroup-scope release
// fence: no cache write-back) before it counts itself, so the wave that
// counts last finds every speed in smax, and reads it with atomic exchanges.
// The counter and smax are left at 0 for the next launch.
__device__ __forceinline__ void cfl_tail(const StepArgs& a, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(a.done, 1u);
    prev = __builtin_amdgcn_readfirstlane(prev);
    if (prev + 1 != (uint32_t)a.nitems || lane != 0) return;
    unsigned long long* sm = reinterpret_cast<unsigned long long*>(a.smax);
    const double sx = __longlong_as_double(static_cast<long long>(atomicExch(&sm[0], 0ull)));
    const double sy = __longlong_as_double(static_cast<long long>(atomicExch(&sm[1], 0ull)));
    const double rx = sx / a.dx, ry = sy / a.dy;
    double r = rx > ry ? rx : ry;
    r = r / (double)a.tref;
    if (isnan(rx) || isnan(ry)) r = rx + ry;
    const double rate = (r > 0.0 || isnan(r)) ? r : 0.0;
    const double dt = *a.dt;
    uint32_t f = 0;
    if (isnan(rate)) f |= SWE_STATUS_NONFINITE;
    const bool over = rate > 0.0 && dt * rate > a.cfl_max;
    if (over) f |= a.flags ? SWE_STATUS_RETAKEN : SWE_STATUS_CFL_EXCEEDED;
    if (a.flags) atomicExch(a.flags, over ? 1u : 0u);
    if (rate > 0.0 && isfinite(rate)) atomicExch(reinterpret_cast<unsigned long long*>(a.dt_next),
                                                 static_cast<unsigned long long>(
                                                     __double_as_longlong(a.cfl_desired / rate)));
    if (f) atomicOr(a.status_out, f);
    // the launch's own conditions count when its step stands; a step to be
    // redone reports nothing (the redo reports its own)
    const uint32_t pf = atomicExch(&a.status[0], 0u), pc = atomicExch(&a.status[1], 0u);
    if (!(a.flags && over)) {
        if (pf) atomicOr(a.status_out, pf);
        if (pc) atomicAdd(&a.status_out[1], pc);
    }
    atomicExch(a.done, 0u);
}

// Rank in the launch order of launch position `pos` (one wave per
// workgroup).  Workgroups go to the eight XCDs in turn (workgroup i to XCD
// i mod 8), each XCD with its own L2.  The ranks are dealt to the XCDs in runs
// of G consecutive ranks, which in index order, and within a cost bin of the
// heaviest-first order, are neighbouring strips of one row chunk: the cache
// lines two neighbouring strips share (their rows are 60 columns apart, not a
// multiple of a 128-byte line) are then fetched into one L2.  The XCDs still
// take ranks in turn, so the launch stays heaviest first in blocks of 8 G
// ranks; positions past the last whole block keep their rank.
__device__ __forceinline__ int rank_at(int pos, int n, int G) {
    const int block = 8 * G;
    if (G <= 1 || pos >= n / block * block) return pos;
    const int xcd = pos & 7, slot = pos >> 3;
    return ((slot / G) * 8 + xcd) * G + slot % G;
}

// Task at launch position `pos` (wave-uniform).
__device__ __forceinline__ int task_at(const StepArgs& a, int pos) {
    const int k = rank_at(pos, a.nitems, a.xcd_run);
    if (!a.order) return k;
    const uint32_t v = a.order[k];
    return (v != 0 && v <= (uint32_t)a.nitems) ? (int)v - 1 : k;
}

// Depth of the LDS row ring of the split step (0: rows loaded into registers
// one iteration ahead).  Two rows ahead measured 4.7 % faster than the
// register path in FP32 and 0.8 % in FP64 on the 4096^2 shelf; four rows
// ahead gained less.
#ifndef SWE_RING_DEPTH
#define SWE_RING_DEPTH 2
#endif
constexpr int kRing = SWE_RING_DEPTH;

// LDS bytes of one wave's row ring.
constexpr size_t ring_bytes(bool f64) {
    return (size_t)kRing * 4 * kWave * (f64 ? sizeof(double) : sizeof(float));
}

// One patch, one wave64 per (strip, chunk of H rows).
// Waves per SIMD the register budget is fitted to, without spilling: the
// FP32 march takes four (at most 128 VGPRs), the FP64 one three (168); with
// the friction step compiled in, one fewer.
template <bool DEV, bool FRIC, bool SPH, bool WIDE = false>
__device__ __forceinline__ void split_task(const StepArgs& a) {
    const int lane = threadIdx.x & (kWave - 1);
    // the task, and with it the row loop's trip count, is the same for the
    // whole wave: keep it in scalar registers
    const int pos = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) +
                                                   (threadIdx.x / kWave));
    if (pos >= a.nitems) return;  // whole wave leaves together
    if (a.gate && *a.gate == 0) return;  // no step to retake
    const int item = __builtin_amdgcn_readfirstlane(task_at(a, pos));
    Task tk;
    tk.qin = a.qin;
    tk.qout = a.qout;
    tk.b = a.b;
    tk.off = a.off;
    tk.ps = a.ps;
    tk.dt = *a.dt;
    tk.dx = a.dx;
    tk.dy = a.dy;
    tk.pitch = a.pitch;
    tk.mx = a.mx;
    tk.my = a.my;
    tk.c0 = (item % a.nstrips) * kStripOut;
    tk.segw = kWave;
    tk.U0 = 2 + (item / a.nstrips) * a.H;
    tk.U1 = min(tk.U0 + a.H - 1, a.my + 1);
    for (int s = 0; s < 4; ++s) tk.bc[s] = a.bc[s];
    tk.active = true;
    tk.metric = a.metric;
    using S = typename Prec<DEV>::S;
    extern __shared__ __align__(16) unsigned char swe_step_lds[];
    S* ring = reinterpret_cast<S*>(swe_step_lds) + (threadIdx.x / kWave) * (kRing * 4 * kWave);
    const MarchOut o =
        march<DEV, kWave, FRIC, kRing, SPH, WIDE>(tk, a.P, lane, tk.U1 - tk.U0 + 5, ring);
    const double wx = wave_max_nonneg(o.smx);
    const double wy = wave_max_nonneg(o.smy);
    if (lane == 0) {
        atomic_max_nonneg(&a.smax[0], wx);
        atomic_max_nonneg(&a.smax[1], wy);
        if (a.cost) a.cost[item] = o.work;
    }
    if (o.clamps) atomicAdd(&a.status[1], o.clamps);
    if (o.flags) atomicOr(&a.status[0], o.flags);
    if (a.done) cfl_tail(a, lane);
}

// WIDE: FP32 surface-deviation planes, FP64 arithmetic (SWE_F32_STORE).
template <bool DEV, bool FRIC, bool WIDE = false>
__global__ void __launch_bounds__(256, (DEV && !WIDE ? 4 : 3) - (FRIC ? 1 : 0))
    k_split(StepArgs a) {
    split_task<DEV, FRIC, false, WIDE>(a);
}

}  // namespace swe
