// swe_step.hip -- the per-patch split step on gfx950 (FP64), and the small
// kernels around it: ghost fill, speed scan, CFL reduction, mass.
//
// Split step (Qin, LeVeque & Motley, Sec. 2, dimensionally split x/y forms):
// one wave64 owns a strip of 64 adjacent columns (60 of which it updates) and
// a chunk of rows, and marches down the rows.  For every row it loads
// (h, hu, hv, b) once from HBM (coalesced along x), solves the x-edges of the
// row with one lane per edge, exchanges neighbour data across lanes for the
// limiter and the update, and obtains Q* of the row in registers.  The
// y-sweep is a per-lane pipeline over the rows of Q*: each lane keeps the
// waves of the last y-edges, so every y-edge of the column is solved once, and
// the cell two rows behind is finished and written.  Every cell of the state is
// read once and written once; no LDS and no barriers are needed.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "swe.h"
#include "swe_common.hpp"
#include "swe_march.hpp"
#include "swe_unsplit.hpp"
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

// The same on a latitude-longitude patch (FP64).
template <bool FRIC>
__global__ void __launch_bounds__(256, FRIC ? 2 : 3) k_split_sphere(StepArgs a) {
    split_task<false, FRIC, true>(a);
}

template __global__ void k_split<false, false>(StepArgs);
template __global__ void k_split<true, false>(StepArgs);
template __global__ void k_split<false, true>(StepArgs);
template __global__ void k_split<true, true>(StepArgs);
template __global__ void k_split<true, false, true>(StepArgs);
template __global__ void k_split<true, true, true>(StepArgs);
template __global__ void k_split_sphere<false>(StepArgs);
template __global__ void k_split_sphere<true>(StepArgs);

// One patch, unsplit with transverse waves (FP64).
template <bool FRIC>
__global__ void __launch_bounds__(256) k_unsplit(StepArgs a, int transverse_order) {
    const int lane = threadIdx.x & (kWave - 1);
    const int pos = __builtin_amdgcn_readfirstlane(blockIdx.x * (blockDim.x / kWave) +
                                                   (threadIdx.x / kWave));
    if (pos >= a.nitems) return;
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
    tk.metric = nullptr;
    const MarchOut o =
        march_unsplit<kWave, FRIC>(tk, a.P, lane, tk.U1 - tk.U0 + 5, transverse_order);
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

template __global__ void k_unsplit<false>(StepArgs, int);
template __global__ void k_unsplit<true>(StepArgs, int);

// Launch order of the next step of a patch: its tasks by the work their
// marches recorded, largest first, ties by task index (the order is a
// function of the work alone).  Tasks over water at rest or dry land skip
// their solves and finish several times faster than tasks under a moving
// wave; launched in index order, some long tasks start late and the launch
// ends on them.  Heaviest first, it ends on short tasks.
//
// A counting sort over kOrderBins bins of `width` work units, in one
// workgroup.  A round covers up to kOrderRound tasks, kOrderPer consecutive
// ones per thread.  C[b][t] counts the tasks of bin b held by thread t; an
// exclusive scan of C read bins descending, then threads ascending, gives
// every (bin, thread) pair the number of tasks placed before its first one
// within the round.  Patches with more than one round first count every bin
// over all tasks (start[]) and carry a per-bin cursor across rounds.
constexpr int kOrderBins = 16;
constexpr int kOrderThreads = 1024;
constexpr int kOrderPer = 16;
constexpr int kOrderRound = kOrderThreads * kOrderPer;
constexpr int kOrderWaves = kOrderThreads / kWave;
constexpr int kOrderRowThreads = kOrderThreads / kOrderPer;  // threads per bin row
static_assert(kOrderWaves == kOrderBins, "one wave per bin in the count pass");

__device__ __forceinline__ int order_bin(uint32_t c, uint32_t width) {
    const uint32_t q = c / width;
    return q < (uint32_t)kOrderBins ? (int)q : kOrderBins - 1;
}

__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

__global__ void __launch_bounds__(kOrderThreads) k_order(uint32_t* __restrict__ order,
                                                         const uint32_t* __restrict__ cost,
                                                         int n, uint32_t width) {
    __shared__ uint16_t C[kOrderBins][kOrderThreads];
    __shared__ uint32_t wsum[kOrderWaves];
    __shared__ uint32_t start[kOrderBins], cursor[kOrderBins], rowbase[kOrderBins];
    const int t = threadIdx.x, lane = t & (kWave - 1), wv = t / kWave;
    const bool multi = n > kOrderRound;
    if (multi) {
        for (int bn = 0; bn < kOrderBins; ++bn) C[bn][t] = 0;
        for (int i = t; i < n; i += kOrderThreads) {
            const int bn = order_bin(cost[i], width);
            C[bn][t] = (uint16_t)(C[bn][t] + 1);
        }
        __syncthreads();
        uint32_t sum = 0;  // wave wv totals bin wv
        for (int k = lane; k < kOrderThreads; k += kWave) sum += C[wv][k];
        sum = wave_inclusive_sum(sum);
        if (lane == kWave - 1) wsum[wv] = sum;
        __syncthreads();
        if (t == 0) {
            uint32_t run = 0;
            for (int bn = kOrderBins - 1; bn >= 0; --bn) {
                start[bn] = run;
                run += wsum[bn];
            }
        }
    }
    if (t < kOrderBins) cursor[t] = 0;
    for (int r0 = 0; r0 < n; r0 += kOrderRound) {
        const int R = min(n - r0, kOrderRound);
        const int K = (R + kOrderThreads - 1) / kOrderThreads;
        int bins[kOrderPer];
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            const int i = t * K + j;
            bins[j] = (j < K && i < R) ? order_bin(cost[r0 + i], width) : -1;
        }
        __syncthreads();  // the last pass over C has ended
#pragma unroll
        for (int bn = 0; bn < kOrderBins; ++bn) C[bn][t] = 0;
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j)
            if (bins[j] >= 0) C[bins[j]][t] = (uint16_t)(C[bins[j]][t] + 1);
        __syncthreads();
        // thread t scans kOrderPer consecutive entries of bin row fb
        const int fb = kOrderBins - 1 - t / kOrderRowThreads;
        const int c0 = (t % kOrderRowThreads) * kOrderPer;
        uint32_t v[kOrderPer], own = 0;
#pragma unroll
        for (int e = 0; e < kOrderPer; ++e) {
            v[e] = C[fb][c0 + e];
            own += v[e];
        }
        const uint32_t incl = wave_inclusive_sum(own);
        if (lane == kWave - 1) wsum[wv] = incl;
        __syncthreads();
        uint32_t run = incl - own;
        for (int w = 0; w < wv; ++w) run += wsum[w];
#pragma unroll
        for (int e = 0; e < kOrderPer; ++e) {
            C[fb][c0 + e] = (uint16_t)run;
            run += v[e];
        }
        __syncthreads();
        if (t < kOrderBins) rowbase[t] = C[t][0];
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOrderPer; ++j) {
            const int bn = bins[j];
            if (bn < 0) continue;
            const uint32_t within = (uint32_t)C[bn][t] - (multi ? rowbase[bn] : 0u);
            const uint32_t pos = (multi ? start[bn] + cursor[bn] : 0u) + within;
            C[bn][t] = (uint16_t)(C[bn][t] + 1);
            order[pos] = (uint32_t)(r0 + t * K + j) + 1u;
        }
        __syncthreads();
        if (t < kOrderBins) cursor[t] += (uint32_t)C[t][kOrderThreads - 1] - rowbase[t];
    }
}

// ---------------------------------------------------------------------------
// Batched helpers: one block row (blockIdx.y) per patch.

struct PatchView {
    int64_t off, ps;
    int mx, my, pitch;
    int8_t bc[4];
};

__device__ __forceinline__ PatchView view(const swe_patch& p) {
    PatchView v;
    v.off = p.off;
    v.ps = p.plane_stride;
    v.mx = p.mx;
    v.my = p.my;
    v.pitch = p.pitch;
    v.bc[0] = p.bc[0];
    v.bc[1] = p.bc[1];
    v.bc[2] = p.bc[2];
    v.bc[3] = p.bc[3];
    return v;
}

// Ghost cells of a patch written into memory by the synthesis rule.
template <typename S>
__global__ void __launch_bounds__(256) k_ghost_fill(const swe_patch* __restrict__ patches, S* q,
                                                    S* b, int fill_b) {
    const PatchView v = view(patches[blockIdx.y]);
    const int nx = v.mx + 4;
    const int nperim = 4 * nx + 4 * v.my;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nperim; k += gridDim.x * blockDim.x) {
        int R, c;
        if (k < 2 * nx) { R = k / nx; c = k % nx; }
        else if (k < 4 * nx) { R = v.my + 2 + (k - 2 * nx) / nx; c = (k - 2 * nx) % nx; }
        else {
            const int r = k - 4 * nx;
            R = 2 + r / 4;
            const int s = r % 4;
            c = s < 2 ? s : v.mx + s;
        }
        bool write;
        if (R < 2) write = v.bc[2] != SWE_BC_USER;
        else if (R > v.my + 1) write = v.bc[3] != SWE_BC_USER;
        else write = (c < 2) ? v.bc[0] != SWE_BC_USER : v.bc[1] != SWE_BC_USER;
        if (!write) continue;
        const Src s = map_cell(R, c, v.mx, v.my, v.pitch, v.off, v.bc);
        const int64_t dst = v.off + (int64_t)R * v.pitch + c;
        const S h = q[s.idx], hu = S(s.sx) * q[s.idx + v.ps], hv = S(s.sy) * q[s.idx + 2 * v.ps];
        q[dst] = h;
        q[dst + v.ps] = hu;
        q[dst + 2 * v.ps] = hv;
        if (fill_b) b[dst] = b[s.idx];
    }
}

// Largest speeds over the x- and y-edges of the interior cells of each patch.
// metric (latitude-longitude patch, FP64): each speed is scaled as the
// split step reports it, by 1 / kappa of the row for an x-edge and by the
// mean of its two rows' 1 / kappa for a y-edge.
template <bool DEV>
__global__ void __launch_bounds__(256) k_speed_scan(const swe_patch* __restrict__ patches,
                                                    const void* qv, const void* bv, double* smax,
                                                    DevParams P, const double* metric) {
    using S = typename Prec<DEV>::S;
    const S* __restrict__ q = static_cast<const S*>(qv);
    const S* __restrict__ b = static_cast<const S*>(bv);
    const int pk = blockIdx.y;
    const PatchView v = view(patches[pk]);
    double sx = 0.0, sy = 0.0;
    const int64_t ncell = (int64_t)v.mx * v.my;
    for (int64_t k = blockIdx.x * blockDim.x + threadIdx.x; k < ncell;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int c = 2 + (int)(k % v.mx);
        const int R = 2 + (int)(k / v.mx);
        struct Cell {
            Side<S> s;
            S m, t;
        };
        auto load = [&](int RR, int CC, bool ydir) {
            const Src s = map_cell(RR, CC, v.mx, v.my, v.pitch, v.off, v.bc);
            const S q0 = q[s.idx], hu = S(s.sx) * q[s.idx + v.ps], hv = S(s.sy) * q[s.idx + 2 * v.ps];
            Cell cl;
            cl.m = ydir ? hv : hu;
            cl.t = ydir ? hu : hv;
            cl.s = side_from<DEV, S, S>(q0, cl.m, cl.t, b[s.idx], P);
            return cl;
        };
        // 1 / kappa of rows R - 1, R, R + 1 (1 without a metric)
        double ik[3] = {1.0, 1.0, 1.0};
        if (metric) {
            ik[0] = 1.0 / metric[R - 1];
            ik[1] = 1.0 / metric[R];
            ik[2] = 1.0 / metric[R + 1];
        }
        auto scaled = [&](const Waves<S>& w, double f) {
            const double s = double(max_speed(w));
            return metric ? s * f : s;
        };
        Waves<S> w;
        const Cell me = load(R, c, false);
        Cell o = load(R, c - 1, false);
        solve_edge<DEV, S>(o.s, me.s, o.m, o.t, me.m, me.t, P, w);
        sx = fmax(sx, scaled(w, ik[1]));
        if (c == v.mx + 1) {
            o = load(R, c + 1, false);
            solve_edge<DEV, S>(me.s, o.s, me.m, me.t, o.m, o.t, P, w);
            sx = fmax(sx, scaled(w, ik[1]));
        }
        const Cell mey = load(R, c, true);
        o = load(R - 1, c, true);
        solve_edge<DEV, S>(o.s, mey.s, o.m, o.t, mey.m, mey.t, P, w);
        sy = fmax(sy, scaled(w, 0.5 * (ik[0] + ik[1])));
        if (R == v.my + 1) {
            o = load(R + 1, c, true);
            solve_edge<DEV, S>(mey.s, o.s, mey.m, mey.t, o.m, o.t, P, w);
            sy = fmax(sy, scaled(w, 0.5 * (ik[1] + ik[2])));
        }
    }
    sx = wave_max_nonneg(sx);
    sy = wave_max_nonneg(sy);
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomic_max_nonneg(&smax[2 * pk], sx);
        atomic_max_nonneg(&smax[2 * pk + 1], sy);
    }
}

// CFL rule per group; one block per group.
// Step sizes of the levels of a hierarchy from the coarse one, each the one
// below divided by the refinement ratio.
__global__ void k_level_steps(const double* dt_coarse, int ratio, int nlevels, double* dt_levels) {
    if (threadIdx.x != 0) return;
    double v = dt_coarse[0];
    dt_levels[0] = v;
    for (int l = 1; l < nlevels; ++l) {
        v = v / (double)ratio;
        dt_levels[l] = v;
    }
}

// pending (NULL: none): per group, the (flags, clamps) the step just taken
// reported; they join status and group_status when the step stands and are
// dropped when it is to be redone (the redo reports its own), so only
// accepted steps count.
__global__ void __launch_bounds__(256) k_cfl_reduce(const swe_patch* __restrict__ patches, int n,
                                                    double* smax, double* dt_group,
                                                    uint32_t* status, uint32_t* group_flags,
                                                    uint32_t* retake, double cfl_desired,
                                                    double cfl_max, int initial,
                                                    uint32_t* pending, uint32_t* group_status) {
    const int g = blockIdx.x;
    __shared__ unsigned long long red[256 / kWave];
    double rate = 0.0;
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const swe_patch& p = patches[k];
        if (p.group != g) continue;
        const double rx = smax[2 * k] / p.dx, ry = smax[2 * k + 1] / p.dy;
        double r = rx > ry ? rx : ry;
        r = r / (double)p.tref;
        if (isnan(rx) || isnan(ry)) r = rx + ry;
        rate = (r > rate || isnan(r)) ? r : rate;
        smax[2 * k] = 0.0;
        smax[2 * k + 1] = 0.0;
    }
    rate = wave_max_nonneg(rate);
    if ((threadIdx.x & (kWave - 1)) == 0)
        red[threadIdx.x / kWave] = static_cast<unsigned long long>(__double_as_longlong(rate));
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = 0;
        for (int i = 0; i < (int)(blockDim.x / kWave); ++i) m = red[i] > m ? red[i] : m;
        const double r = __longlong_as_double(static_cast<long long>(m));
        const double dt = dt_group[g];
        uint32_t f = 0;
        if (isnan(r)) f |= SWE_STATUS_NONFINITE;
        const bool over = !initial && r > 0.0 && dt * r > cfl_max;
        if (over) f |= retake ? SWE_STATUS_RETAKEN : SWE_STATUS_CFL_EXCEEDED;
        if (retake) retake[g] = over ? 1u : 0u;
        if (r > 0.0 && isfinite(r)) dt_group[g] = cfl_desired / r;
        if (f) {
            atomicOr(status, f);
            if (group_flags) atomicOr(&group_flags[g], f);
        }
        if (pending) {
            const uint32_t pf = pending[2 * g], pc = pending[2 * g + 1];
            pending[2 * g] = 0u;
            pending[2 * g + 1] = 0u;
            if (!(retake && over)) {
                if (pf) atomicOr(status, pf);
                if (pc) atomicAdd(&status[1], pc);
                if (group_status && pf) atomicOr(&group_status[2 * g], pf);
                if (group_status && pc) atomicAdd(&group_status[2 * g + 1], pc);
            }
        }
    }
}

// Water volume per patch, FP64, fixed reduction order.  On the deviation
// path the depth is eta' + sea_level - b, formed in FP64.  metric
// (latitude-longitude patch): each depth weighted by its row's capacity.
template <bool DEV>
__global__ void __launch_bounds__(256) k_mass(const swe_patch* __restrict__ patches,
                                              const void* qv, const void* bv,
                                              double* __restrict__ mass, double sea_level,
                                              const double* metric) {
    using S = typename Prec<DEV>::S;
    const S* __restrict__ q = static_cast<const S*>(qv);
    const S* __restrict__ b = static_cast<const S*>(bv);
    const int pk = blockIdx.x;
    const swe_patch p = patches[pk];
    __shared__ double red[256];
    double s = 0.0;
    const int64_t ncell = (int64_t)p.mx * p.my;
    for (int64_t k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int c = 2 + (int)(k % p.mx);
        const int R = 2 + (int)(k / p.mx);
        const int64_t i = p.off + (int64_t)R * p.pitch + c;
        const double h = DEV ? (double(q[i]) + sea_level) - double(b[i]) : double(q[i]);
        s += metric ? h * metric[R] : h;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) mass[pk] = red[0] * p.dx * p.dy;
}

// Interior cells of each patch from FP64 planes into the precision's planes
// (copy, or the surface deviation formed in FP64 and rounded once).
template <bool DEV>
__global__ void __launch_bounds__(256) k_state_import(const swe_patch* __restrict__ patches,
                                                      const double* __restrict__ src,
                                                      const double* __restrict__ src_b,
                                                      int64_t shift, int64_t stride, void* qv,
                                                      void* bv, double sea_level) {
    using S = typename Prec<DEV>::S;
    S* __restrict__ q = static_cast<S*>(qv);
    S* __restrict__ b = static_cast<S*>(bv);
    const swe_patch p = patches[blockIdx.y];
    const int64_t ss = stride ? stride : p.plane_stride;
    const int64_t ncell = (int64_t)p.mx * p.my;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ncell;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p.off + (2 + k / p.mx) * (int64_t)p.pitch + 2 + k % p.mx;
        const int64_t j = i - shift;
        const double h = src[j], bed = src_b[j];
        q[i] = DEV ? S((h > 0.0 ? h + bed : bed) - sea_level) : S(h);
        q[i + p.plane_stride] = S(src[j + ss]);
        q[i + 2 * p.plane_stride] = S(src[j + 2 * ss]);
        b[i] = S(bed);
    }
}

// Interior (h, hu, hv) of each patch as FP64 planes.
template <bool DEV>
__global__ void __launch_bounds__(256) k_state_export(const swe_patch* __restrict__ patches,
                                                      const void* qv, const void* bv,
                                                      double* __restrict__ dst, int64_t shift,
                                                      int64_t stride, double sea_level) {
    using S = typename Prec<DEV>::S;
    const S* __restrict__ q = static_cast<const S*>(qv);
    const S* __restrict__ b = static_cast<const S*>(bv);
    const swe_patch p = patches[blockIdx.y];
    const int64_t ds = stride ? stride : p.plane_stride;
    const int64_t ncell = (int64_t)p.mx * p.my;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < ncell;
         k += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = p.off + (2 + k / p.mx) * (int64_t)p.pitch + 2 + k % p.mx;
        const int64_t j = i - shift;
        const double h = DEV ? fmax((double(q[i]) + sea_level) - double(b[i]), 0.0) : double(q[i]);
        dst[j] = h;
        dst[j + ds] = double(q[i + p.plane_stride]);
        dst[j + 2 * ds] = double(q[i + 2 * p.plane_stride]);
    }
}

}  // namespace swe

// ===========================================================================
// C ABI

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(SWE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return SWE_OK;
}

swe::DevParams dev_params(const swe_params* p) {
    swe::DevParams d;
    d.g = p->g;
    d.drytol = p->drytol;
    d.h_corr = p->h_corr;
    d.manning_n = p->manning_n;
    d.sea_level = p->sea_level;
    d.h_fp64 = p->h_fp64;
    d.order = p->order;
    return d;
}

int check_params(const swe_params* p) {
    if (!p) return fail(SWE_EINVAL, "params is NULL");
    if (!(p->g > 0.0) || !(p->drytol >= 0.0) || !(p->h_corr >= 0.0) || !(p->manning_n >= 0.0) ||
        !(p->cfl_desired > 0.0) || !(p->cfl_max > 0.0))
        return fail(SWE_EINVAL, "params: g, cfl_desired, cfl_max must be > 0; drytol, h_corr, "
                                "manning_n must be >= 0");
    if (p->order != 1 && p->order != 2) return fail(SWE_EINVAL, "params: order must be 1 or 2");
    if (p->method != SWE_SPLIT && p->method != SWE_UNSPLIT)
        return fail(SWE_EINVAL, "params: unknown method");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV && p->precision != SWE_F32_STORE)
        return fail(SWE_EINVAL, "params: unknown precision");
    return SWE_OK;
}

int check_patch(const swe_patch* pt) {
    if (!pt) return fail(SWE_EINVAL, "patch is NULL");
    if (pt->mx < 1 || pt->my < 1) return fail(SWE_EINVAL, "patch: mx and my must be >= 1");
    if (pt->pitch < pt->mx + 4) return fail(SWE_EINVAL, "patch: pitch must be >= mx + 4");
    if (pt->off < 0 || pt->plane_stride < (int64_t)pt->pitch * (pt->my + 4))
        return fail(SWE_EINVAL, "patch: off must be >= 0 and plane_stride >= pitch * (my + 4)");
    if (!(pt->dx > 0.0) || !(pt->dy > 0.0)) return fail(SWE_EINVAL, "patch: dx, dy must be > 0");
    if (pt->tref < 1) return fail(SWE_EINVAL, "patch: tref must be >= 1");
    for (int s = 0; s < 4; ++s)
        if (pt->bc[s] != SWE_BC_WALL && pt->bc[s] != SWE_BC_EXTRAP && pt->bc[s] != SWE_BC_USER)
            return fail(SWE_EINVAL, "patch: unknown boundary code");
    if ((pt->bc[0] == SWE_BC_WALL || pt->bc[1] == SWE_BC_WALL) && pt->mx < 2)
        return fail(SWE_EINVAL, "patch: a wall in x needs mx >= 2");
    if ((pt->bc[2] == SWE_BC_WALL || pt->bc[3] == SWE_BC_WALL) && pt->my < 2)
        return fail(SWE_EINVAL, "patch: a wall in y needs my >= 2");
    return SWE_OK;
}

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const char* pa = static_cast<const char*>(a);
    const char* pb = static_cast<const char*>(b);
    return pa < pb + nb && pb < pa + na;
}

// Launch shape of the patch step with the defaults filled in, or an error.
// Rows per strip task: a wave marches H rows plus 4 rows of pipeline fill.
// Waves over water at rest skip their Riemann solves and finish early, so
// tasks must be many more than the device holds at once for the launch to
// balance; in index order 32 rows did best, and with the heaviest tasks
// launched first 40-56 rows are 7-8 % faster than 32 on the 4096^2 shelf (the
// fill overhead drops from 1/8 to 1/12 at 48).  At most kWave - 4 rows: the
// task's rows with their two ghost rows either side then fit one wave's lanes,
// which the latitude-longitude march uses to hold its per-row values.  Runs of
// 8 ranks per XCD fetch 13 % fewer bytes on the 4096^2 FP64 step than ranks
// dealt in turn; only one-wave workgroups map positions to XCDs one to one.
struct Shape {
    int H, wpb, xcd_run;
};

int launch_shape(const swe_launch* l, int my, Shape* out) {
    int H = 48, wpb = 1, run = 8;
    if (l) {
        if (l->rows_per_task < 0 || l->rows_per_task > swe::kWave - 4)
            return fail(SWE_EINVAL, "launch: rows_per_task must be 0 (default) or 1 .. 60");
        if (l->waves_per_block != 0 && l->waves_per_block != 1 && l->waves_per_block != 2 &&
            l->waves_per_block != 4)
            return fail(SWE_EINVAL, "launch: waves_per_block must be 0 (default), 1, 2 or 4");
        if (l->xcd_run < 0) return fail(SWE_EINVAL, "launch: xcd_run must be >= 0");
        if (l->rows_per_task) H = l->rows_per_task;
        if (l->waves_per_block) wpb = l->waves_per_block;
        if (l->xcd_run) run = l->xcd_run;
    }
    out->H = H < my ? H : my;
    out->wpb = wpb;
    out->xcd_run = wpb == 1 && run > 1 ? run : 1;
    return SWE_OK;
}

}  // namespace

extern "C" {

// error slot shared by the library's translation units (not part of the ABI)
__attribute__((visibility("hidden"))) int swe_internal_set_error(int code, const char* msg) {
    g_err = msg;
    return code;
}

const char* swe_last_error(void) { return g_err.c_str(); }

const char* swe_version(void) { return "swe-gfx950 0.1"; }

// Strip tasks of one patch step (the launch's waves) for a given task height.
static int patch_tasks(const swe_patch* patch, int H) {
    const int nstrips = (patch->mx + swe::kStripOut - 1) / swe::kStripOut;
    return nstrips * ((patch->my + H - 1) / H);
}

// The CFL rule fused into a launch (swe_patch_step_cfl, swe_patch_retake_cfl).
struct FusedCfl {
    uint32_t* counter;
    double* dt;
    uint32_t* flags;  // the group's retake flag to write, or NULL
};

static int patch_step(const swe_params* p, const swe_patch* patch, const void* q_in, void* q_out,
                      const void* b, const double* dt, double* smax, uint32_t* status,
                      const uint32_t* gate, uint32_t* sched, int64_t sched_len,
                      const swe_launch* launch, void* stream, const double* metric = nullptr,
                      const FusedCfl* fused = nullptr) {
    int rc = check_params(p);
    if (rc) return rc;
    if ((rc = check_patch(patch))) return rc;
    Shape sh;
    if ((rc = launch_shape(launch, patch->my, &sh))) return rc;
    // a gated retake launch, which mostly ends at once, takes four waves per
    // workgroup (fewer workgroups to dispatch; results do not depend on it)
    if (gate) {
        sh.wpb = 4;
        sh.xcd_run = 1;
    }
    if (sched && sched_len < 2 * (int64_t)patch_tasks(patch, sh.H))
        return fail(SWE_EINVAL, "swe_patch_step: schedule buffer shorter than 2 x tasks");
    if (!q_in || !q_out || !b || !dt || !smax || !status)
        return fail(SWE_EINVAL, "swe_patch_step: null pointer");
    if (p->method == SWE_UNSPLIT && p->precision != SWE_F64)
        return fail(SWE_EINVAL, "swe_patch_step: the unsplit step is available in FP64 only");
    if (p->method == SWE_UNSPLIT && p->transverse_order != 1 && p->transverse_order != 2)
        return fail(SWE_EINVAL, "params: transverse_order must be 1 or 2");
    const size_t esz = p->precision == SWE_F64 ? sizeof(double) : sizeof(float);
    const size_t span = (size_t)(patch->off + 2 * patch->plane_stride +
                                 (int64_t)patch->pitch * (patch->my + 4)) * esz;
    if (overlap(q_in, span, q_out, span))
        return fail(SWE_EINVAL, "swe_patch_step: q_in and q_out overlap");
    swe::StepArgs a;
    a.qin = q_in;
    a.qout = q_out;
    a.b = b;
    a.dt = dt;
    a.smax = smax;
    a.status = status;
    a.off = patch->off;
    a.ps = patch->plane_stride;
    a.dx = patch->dx;
    a.dy = patch->dy;
    a.pitch = patch->pitch;
    a.mx = patch->mx;
    a.my = patch->my;
    // one wave per workgroup by default: the finest unit the dispatcher can
    // balance
    const int waves_per_block = sh.wpb;
    const bool fric = p->manning_n > 0.0;
    const bool f64 = p->precision == SWE_F64;
    a.H = sh.H;
    a.nstrips = (patch->mx + swe::kStripOut - 1) / swe::kStripOut;
    const int nchunks = (patch->my + a.H - 1) / a.H;
    a.nitems = a.nstrips * nchunks;
    for (int s = 0; s < 4; ++s) a.bc[s] = patch->bc[s];
    a.P = dev_params(p);
    a.gate = gate;
    a.order = sched;
    a.cost = sched ? sched + a.nitems : nullptr;
    a.metric = metric;
    a.xcd_run = sh.xcd_run;
    a.done = fused ? fused->counter : nullptr;
    a.dt_next = fused ? fused->dt : nullptr;
    a.flags = fused ? fused->flags : nullptr;
    a.status_out = status;
    if (fused) a.status = fused->counter + 1;  // the launch's pending (flags, clamps)
    a.cfl_desired = p->cfl_desired;
    a.cfl_max = p->cfl_max;
    a.tref = patch->tref;
    const int blocks = (a.nitems + waves_per_block - 1) / waves_per_block;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    const dim3 grid(blocks), block(64 * waves_per_block);
    const int tord = (int)p->transverse_order;
    if (p->method == SWE_UNSPLIT) {
        if (fric) hipLaunchKernelGGL(swe::k_unsplit<true>, grid, block, 0, st, a, tord);
        else hipLaunchKernelGGL(swe::k_unsplit<false>, grid, block, 0, st, a, tord);
    } else if (f64 && metric) {
        const size_t lds = waves_per_block * swe::ring_bytes(true);
        if (fric) hipLaunchKernelGGL(swe::k_split_sphere<true>, grid, block, lds, st, a);
        else hipLaunchKernelGGL(swe::k_split_sphere<false>, grid, block, lds, st, a);
    } else if (f64) {
        const size_t lds = waves_per_block * swe::ring_bytes(true);
        if (fric) hipLaunchKernelGGL((swe::k_split<false, true>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((swe::k_split<false, false>), grid, block, lds, st, a);
    } else if (p->precision == SWE_F32_STORE) {
        const size_t lds = waves_per_block * swe::ring_bytes(false);
        if (fric) hipLaunchKernelGGL((swe::k_split<true, true, true>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((swe::k_split<true, false, true>), grid, block, lds, st, a);
    } else {
        const size_t lds = waves_per_block * swe::ring_bytes(false);
        if (fric) hipLaunchKernelGGL((swe::k_split<true, true>), grid, block, lds, st, a);
        else hipLaunchKernelGGL((swe::k_split<true, false>), grid, block, lds, st, a);
    }
    return check_launch("swe_patch_step");
}

int swe_patch_step(const swe_params* p, const swe_patch* patch, const void* q_in, void* q_out,
                   const void* b, const double* dt, double* smax, uint32_t* status,
                   void* stream) {
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status, nullptr, nullptr, 0, nullptr,
                      stream);
}

int swe_patch_step_sphere(const swe_params* p, const swe_patch* patch, const void* q_in,
                          void* q_out, const void* b, const double* dt, double* smax,
                          uint32_t* status, const double* metric, uint32_t* sched,
                          int64_t sched_len, const swe_launch* launch, void* stream) {
    if (!metric) return fail(SWE_EINVAL, "swe_patch_step_sphere: null metric");
    if (p && (p->method != SWE_SPLIT || p->precision != SWE_F64))
        return fail(SWE_EINVAL, "swe_patch_step_sphere: FP64 split step only");
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status, nullptr, sched, sched_len,
                      launch, stream, metric);
}

int32_t swe_patch_tasks(const swe_patch* patch, const swe_launch* launch) {
    int rc = check_patch(patch);
    if (rc) return rc;
    Shape sh;
    if ((rc = launch_shape(launch, patch->my, &sh))) return rc;
    return patch_tasks(patch, sh.H);
}

size_t swe_workspace_bytes(const swe_patch* patch, const swe_launch* launch) {
    const int32_t n = swe_patch_tasks(patch, launch);
    return n < 0 ? 0 : 2 * (size_t)n * sizeof(uint32_t);
}

int swe_patch_step_sched(const swe_params* p, const swe_patch* patch, const void* q_in,
                         void* q_out, const void* b, const double* dt, double* smax,
                         uint32_t* status, uint32_t* sched, int64_t sched_len,
                         const swe_launch* launch, void* stream) {
    if (!sched) return fail(SWE_EINVAL, "swe_patch_step_sched: null schedule buffer");
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status, nullptr, sched, sched_len,
                      launch, stream);
}

int swe_patch_order(const swe_patch* patch, uint32_t* sched, int64_t sched_len,
                    const swe_launch* launch, void* stream) {
    int rc = check_patch(patch);
    if (rc) return rc;
    if (!sched) return fail(SWE_EINVAL, "swe_patch_order: null schedule buffer");
    Shape sh;
    if ((rc = launch_shape(launch, patch->my, &sh))) return rc;
    const int n = patch_tasks(patch, sh.H);
    if (sched_len < 2 * (int64_t)n)
        return fail(SWE_EINVAL, "swe_patch_order: schedule buffer shorter than 2 x tasks");
    // a task marches H + 5 rows, each with an x- and a y-sweep
    const int most = 2 * (sh.H + 5);
    const uint32_t width = (uint32_t)((most + swe::kOrderBins) / swe::kOrderBins);
    hipLaunchKernelGGL(swe::k_order, dim3(1), dim3(swe::kOrderThreads), 0,
                       static_cast<hipStream_t>(stream), sched, sched + n, n, width);
    return check_launch("swe_patch_order");
}

int swe_patch_retake(const swe_params* p, const swe_patch* patch, const void* q_in, void* q_out,
                     const void* b, const double* dt, double* smax, uint32_t* status,
                     const uint32_t* retake, void* stream) {
    if (!retake) return fail(SWE_EINVAL, "swe_patch_retake: null retake flags");
    if (patch && patch->group < 0) return fail(SWE_EINVAL, "swe_patch_retake: negative group");
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status,
                      patch ? retake + patch->group : retake, nullptr, 0, nullptr, stream);
}

int swe_patch_retake_sphere(const swe_params* p, const swe_patch* patch, const void* q_in,
                            void* q_out, const void* b, const double* dt, double* smax,
                            uint32_t* status, const double* metric, const uint32_t* retake,
                            void* stream) {
    if (!retake) return fail(SWE_EINVAL, "swe_patch_retake_sphere: null retake flags");
    if (!metric) return fail(SWE_EINVAL, "swe_patch_retake_sphere: null metric");
    if (patch && patch->group < 0)
        return fail(SWE_EINVAL, "swe_patch_retake_sphere: negative group");
    if (p && (p->method != SWE_SPLIT || p->precision != SWE_F64))
        return fail(SWE_EINVAL, "swe_patch_retake_sphere: FP64 split step only");
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status,
                      patch ? retake + patch->group : retake, nullptr, 0, nullptr, stream,
                      metric);
}

int swe_patch_step_cfl(const swe_params* p, const swe_patch* patch, const void* q_in, void* q_out,
                       const void* b, double* dt, double* smax, uint32_t* status,
                       uint32_t* retake, uint32_t* counter, const double* metric,
                       uint32_t* sched, int64_t sched_len, const swe_launch* launch,
                       void* stream) {
    if (!dt || !retake || !counter)
        return fail(SWE_EINVAL, "swe_patch_step_cfl: null dt, retake flags or counter");
    if (patch && patch->group < 0) return fail(SWE_EINVAL, "swe_patch_step_cfl: negative group");
    if (patch && patch->tref < 1) return fail(SWE_EINVAL, "swe_patch_step_cfl: tref < 1");
    if (metric && p && (p->method != SWE_SPLIT || p->precision != SWE_F64))
        return fail(SWE_EINVAL, "swe_patch_step_cfl: a metric needs the FP64 split step");
    const FusedCfl f{counter, dt, patch ? retake + patch->group : retake};
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status, nullptr, sched,
                      sched ? sched_len : 0, launch, stream, metric, &f);
}

int swe_patch_retake_cfl(const swe_params* p, const swe_patch* patch, const void* q_in,
                         void* q_out, const void* b, double* dt, double* smax, uint32_t* status,
                         uint32_t* retake, uint32_t* counter, const double* metric, int32_t last,
                         void* stream) {
    if (!dt || !retake || !counter)
        return fail(SWE_EINVAL, "swe_patch_retake_cfl: null dt, retake flags or counter");
    if (patch && patch->group < 0) return fail(SWE_EINVAL, "swe_patch_retake_cfl: negative group");
    if (patch && patch->tref < 1) return fail(SWE_EINVAL, "swe_patch_retake_cfl: tref < 1");
    if (metric && p && (p->method != SWE_SPLIT || p->precision != SWE_F64))
        return fail(SWE_EINVAL, "swe_patch_retake_cfl: a metric needs the FP64 split step");
    // not the last redo: a redone step still above the limit sets the flag
    // again for the next one; the last one's stands, flagged
    uint32_t* flag = patch ? retake + patch->group : retake;
    const FusedCfl f{counter, dt, last ? nullptr : flag};
    return patch_step(p, patch, q_in, q_out, b, dt, smax, status, flag, nullptr, 0, nullptr,
                      stream, metric, &f);
}

int swe_ghost_fill(const swe_params* p, const swe_patch* patches, int32_t n, int32_t max_mx,
                   int32_t max_my, void* q, void* b, int32_t fill_b, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !q || (fill_b && !b) || n < 0 || max_mx < 1 || max_my < 1)
        return fail(SWE_EINVAL, "swe_ghost_fill: bad arguments");
    if (n == 0) return SWE_OK;
    const int nperim = 4 * (max_mx + 4) + 4 * max_my;
    const int bx = (nperim + 255) / 256;
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_ghost_fill<double>, dim3(bx, n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, static_cast<double*>(q),
                           static_cast<double*>(b), fill_b);
    else
        hipLaunchKernelGGL(swe::k_ghost_fill<float>, dim3(bx, n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, static_cast<float*>(q),
                           static_cast<float*>(b), fill_b);
    return check_launch("swe_ghost_fill");
}

int swe_speed_scan(const swe_params* p, const swe_patch* patches, int32_t n, int32_t max_mx,
                   int32_t max_my, const void* q, const void* b, double* smax_patch,
                   void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !q || !b || !smax_patch || n < 0 || max_mx < 1 || max_my < 1)
        return fail(SWE_EINVAL, "swe_speed_scan: bad arguments");
    if (n == 0) return SWE_OK;
    const int64_t ncell = (int64_t)max_mx * max_my;
    int bx = (int)((ncell + 255) / 256);
    if (bx > 4096) bx = 4096;
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_speed_scan<false>, dim3(bx, n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, q, b, smax_patch,
                           dev_params(p), nullptr);
    else
        hipLaunchKernelGGL(swe::k_speed_scan<true>, dim3(bx, n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, q, b, smax_patch,
                           dev_params(p), nullptr);
    return check_launch("swe_speed_scan");
}

int swe_cfl_reduce(const swe_params* p, const swe_patch* patches, int32_t n, int32_t ngroups,
                   double* smax_patch, double* dt_group, uint32_t* status,
                   uint32_t* group_flags, uint32_t* retake, int32_t initial, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !smax_patch || !dt_group || !status || n < 0 || ngroups < 1)
        return fail(SWE_EINVAL, "swe_cfl_reduce: bad arguments");
    hipLaunchKernelGGL(swe::k_cfl_reduce, dim3(ngroups), dim3(256), 0,
                       static_cast<hipStream_t>(stream), patches, n, smax_patch, dt_group,
                       status, group_flags, retake, p->cfl_desired, p->cfl_max, initial,
                       nullptr, nullptr);
    return check_launch("swe_cfl_reduce");
}

// The parameter check, for swe_batched_advance's fused CFL rule (not part of
// the ABI).
__attribute__((visibility("hidden"))) int swe_internal_check_params(const swe_params* p) {
    return check_params(p);
}

// swe_cfl_reduce that also settles the steps' pending conditions (for
// swe_batched_advance; not part of the ABI).
__attribute__((visibility("hidden"))) int swe_internal_cfl_reduce_pending(
    const swe_params* p, const swe_patch* patches, int32_t n, int32_t ngroups,
    double* smax_patch, double* dt_group, uint32_t* status, uint32_t* group_flags,
    uint32_t* retake, uint32_t* pending, uint32_t* group_status, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !smax_patch || !dt_group || !status || !pending || n < 0 || ngroups < 1)
        return fail(SWE_EINVAL, "swe_cfl_reduce: bad arguments");
    hipLaunchKernelGGL(swe::k_cfl_reduce, dim3(ngroups), dim3(256), 0,
                       static_cast<hipStream_t>(stream), patches, n, smax_patch, dt_group,
                       status, group_flags, retake, p->cfl_desired, p->cfl_max, 0, pending,
                       group_status);
    return check_launch("swe_cfl_reduce");
}

int swe_level_steps(const double* dt_coarse, int32_t ratio, int32_t nlevels, double* dt_levels,
                    void* stream) {
    if (!dt_coarse || !dt_levels || ratio < 1 || nlevels < 1)
        return fail(SWE_EINVAL, "swe_level_steps: null pointer, ratio < 1 or nlevels < 1");
    hipLaunchKernelGGL(swe::k_level_steps, dim3(1), dim3(64), 0, static_cast<hipStream_t>(stream),
                       dt_coarse, ratio, nlevels, dt_levels);
    return check_launch("swe_level_steps");
}

int swe_mass(const swe_params* p, const swe_patch* patches, int32_t n, const void* q,
             const void* b, double* mass_patch, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !q || !mass_patch || n < 0 || (p->precision != SWE_F64 && !b))
        return fail(SWE_EINVAL, "swe_mass: bad arguments");
    if (n == 0) return SWE_OK;
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_mass<false>, dim3(n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, q, b, mass_patch,
                           p->sea_level, nullptr);
    else
        hipLaunchKernelGGL(swe::k_mass<true>, dim3(n), dim3(256), 0,
                           static_cast<hipStream_t>(stream), patches, q, b, mass_patch,
                           p->sea_level, nullptr);
    return check_launch("swe_mass");
}

static int sphere_args(const swe_params* p, const char* what) {
    int rc = check_params(p);
    if (rc) return rc;
    if (p->method != SWE_SPLIT || p->precision != SWE_F64)
        return fail(SWE_EINVAL, std::string(what) + ": FP64 split step only");
    return SWE_OK;
}

int swe_speed_scan_sphere(const swe_params* p, const swe_patch* patch, int32_t max_mx,
                          int32_t max_my, const void* q, const void* b, const double* metric,
                          double* smax, void* stream) {
    int rc = sphere_args(p, "swe_speed_scan_sphere");
    if (rc) return rc;
    if (!patch || !q || !b || !metric || !smax || max_mx < 1 || max_my < 1)
        return fail(SWE_EINVAL, "swe_speed_scan_sphere: bad arguments");
    const int64_t ncell = (int64_t)max_mx * max_my;
    int bx = (int)((ncell + 255) / 256);
    if (bx > 4096) bx = 4096;
    hipLaunchKernelGGL(swe::k_speed_scan<false>, dim3(bx, 1), dim3(256), 0,
                       static_cast<hipStream_t>(stream), patch, q, b, smax, dev_params(p),
                       metric);
    return check_launch("swe_speed_scan_sphere");
}

int swe_mass_sphere(const swe_params* p, const swe_patch* patch, const void* q,
                    const double* metric, double* mass, void* stream) {
    int rc = sphere_args(p, "swe_mass_sphere");
    if (rc) return rc;
    if (!patch || !q || !metric || !mass) return fail(SWE_EINVAL, "swe_mass_sphere: bad arguments");
    hipLaunchKernelGGL(swe::k_mass<false>, dim3(1), dim3(256), 0,
                       static_cast<hipStream_t>(stream), patch, q, nullptr, mass, p->sea_level,
                       metric);
    return check_launch("swe_mass_sphere");
}

static int state_grid(int32_t n, int32_t max_mx, int32_t max_my, dim3* grid) {
    if (n < 0 || max_mx < 1 || max_my < 1) return fail(SWE_EINVAL, "bad patch count or bounds");
    int64_t bx = ((int64_t)max_mx * max_my + 255) / 256;
    if (bx > 4096) bx = 4096;
    *grid = dim3((unsigned)bx, (unsigned)n);
    return SWE_OK;
}

int swe_state_import(const swe_params* p, const swe_patch* patches, int32_t n, int32_t max_mx,
                     int32_t max_my, const double* src, const double* src_b, int64_t src_shift,
                     int64_t src_stride, void* q, void* b, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !src || !src_b || !q || !b)
        return fail(SWE_EINVAL, "swe_state_import: null pointer");
    if (src_stride < 0) return fail(SWE_EINVAL, "swe_state_import: src_stride must be >= 0");
    dim3 grid;
    if ((rc = state_grid(n, max_mx, max_my, &grid))) return rc;
    if (n == 0) return SWE_OK;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_state_import<false>, grid, dim3(256), 0, st, patches, src,
                           src_b, src_shift, src_stride, q, b, p->sea_level);
    else
        hipLaunchKernelGGL(swe::k_state_import<true>, grid, dim3(256), 0, st, patches, src,
                           src_b, src_shift, src_stride, q, b, p->sea_level);
    return check_launch("swe_state_import");
}

int swe_state_export(const swe_params* p, const swe_patch* patches, int32_t n, int32_t max_mx,
                     int32_t max_my, const void* q, const void* b, double* dst, int64_t dst_shift,
                     int64_t dst_stride, void* stream) {
    int rc = check_params(p);
    if (rc) return rc;
    if (!patches || !q || !dst || (p->precision != SWE_F64 && !b))
        return fail(SWE_EINVAL, "swe_state_export: null pointer");
    if (dst_stride < 0) return fail(SWE_EINVAL, "swe_state_export: dst_stride must be >= 0");
    dim3 grid;
    if ((rc = state_grid(n, max_mx, max_my, &grid))) return rc;
    if (n == 0) return SWE_OK;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_state_export<false>, grid, dim3(256), 0, st, patches, q, b, dst,
                           dst_shift, dst_stride, p->sea_level);
    else
        hipLaunchKernelGGL(swe::k_state_export<true>, grid, dim3(256), 0, st, patches, q, b, dst,
                           dst_shift, dst_stride, p->sea_level);
    return check_launch("swe_state_export");
}

}  // extern "C"
