// swe_batched_kern.hpp -- the batched step kernels (items, plain tasks,
// packed strips) and the CFL rule fused into one-launch steps.  Included by
// swe_batched.hip, which instantiates the FP64 kernels, and by
// swe_batched_f32.hip, which instantiates the FP32 surface-deviation kernels
// in a unit of their own (built with contracted multiply-adds: that path is
// held to its surface bar in metres, not to the FP64 path's rounding).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "swe.h"
#include "swe_common.hpp"
#include "swe_march.hpp"

namespace swe {

// The CFL rule of swe_cfl_reduce with the steps' pending conditions, fused
// into the last workgroup of a step that is one launch (one wave per
// workgroup).  ctr[0] counts the finished workgroups and is left at 0;
// ctr[1] says whether the rule flagged a group for a redo, so that a gated
// redo launch with nothing to redo ends in every workgroup at once.
constexpr int kTailGroups = 256;
struct CflTail {
    uint32_t* ctr;           // NULL: no fused rule
    int npatches;            // the table's patches
    int ngroups;             // groups of dt_next, retake_out, group_flags (<= kTailGroups)
    double* dt_next;         // dt_group, written where the rate is finite and positive
    uint32_t* retake_out;    // redo flags; NULL: no further redo (a step above the limit stands)
    uint32_t* status_out;    // (flags, clamps) of the accepted steps
    uint32_t* gstatus_out;   // per group (flags, clamps); may be NULL
    uint32_t* group_flags;   // per group flags of the rule; may be NULL
    double cfl_desired, cfl_max;
};

struct BatchArgs {
    const swe_patch* patches;
    const swe_item* items;
    const swe_task* tasks;
    const void* pin;
    void* pout;
    void* pwork;
    const void* pb;
    const double* dt_group;
    double* smax;
    uint32_t* status;        // (flags, clamps) of all patches; NULL: not kept
    uint32_t* group_status;  // per group (flags, clamps) pairs; NULL: not kept
    uint32_t* queue;  // [0] next item, [1] finished workgroups
    int nitems;
    DevParams P;
    const uint32_t* retake;  // retake launch: only groups with retake[g] != 0; NULL: all
    int ngroups;             // entries of retake
    int sub;                 // plain launches: the substep this launch runs
    CflTail t;               // the CFL rule fused into one-launch steps
};

// Whether a fused redo launch has nothing to redo (wave-uniform): the rule
// of the launch before wrote ctr[1].
__device__ __forceinline__ bool tail_idle_redo(const BatchArgs& a) {
    return a.t.ctr && a.retake &&
           __hip_atomic_load(&a.t.ctr[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
}

// The last workgroup to finish takes the rate of every patch (its speed
// maxima over dx and dy, over its substeps), the largest per group, and
// from it the group's next step size, its redo flag and its flags; the
// groups' pending conditions join the status where the step stands.  The
// arithmetic is swe_cfl_reduce's.  Speeds and pending pairs are read with
// atomic exchanges (the other workgroups wrote them with atomics) and left
// at 0.
__device__ __forceinline__ void cfl_tail(const BatchArgs& a, int lane) {
    const CflTail& t = a.t;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&t.ctr[0], 1u);
    prev = __builtin_amdgcn_readfirstlane(prev);
    if (prev + 1 != gridDim.x) return;
    __shared__ unsigned long long rate[kTailGroups];
    for (int g = lane; g < t.ngroups; g += kWave) rate[g] = 0ull;
    __syncthreads();
    unsigned long long* sm = reinterpret_cast<unsigned long long*>(a.smax);
    for (int k = lane; k < t.npatches; k += kWave) {
        const swe_patch& p = a.patches[k];
        if (p.group < 0 || p.group >= t.ngroups) continue;
        const double sx = __longlong_as_double(static_cast<long long>(atomicExch(&sm[2 * k], 0ull)));
        const double sy =
            __longlong_as_double(static_cast<long long>(atomicExch(&sm[2 * k + 1], 0ull)));
        const double rx = sx / p.dx, ry = sy / p.dy;
        double r = rx > ry ? rx : ry;
        r = r / (double)p.tref;
        if (isnan(rx) || isnan(ry)) r = rx + ry;
        atomicMax(&rate[p.group], static_cast<unsigned long long>(__double_as_longlong(r)));
    }
    __syncthreads();
    bool redo = false;
    for (int g = lane; g < t.ngroups; g += kWave) {
        const double r = __longlong_as_double(static_cast<long long>(rate[g]));
        const double dt = t.dt_next[g];
        uint32_t f = 0;
        if (isnan(r)) f |= SWE_STATUS_NONFINITE;
        const bool over = r > 0.0 && dt * r > t.cfl_max;
        if (over) f |= t.retake_out ? SWE_STATUS_RETAKEN : SWE_STATUS_CFL_EXCEEDED;
        if (t.retake_out) t.retake_out[g] = over ? 1u : 0u;
        if (r > 0.0 && isfinite(r)) t.dt_next[g] = t.cfl_desired / r;
        if (f) {
            atomicOr(t.status_out, f);
            if (t.group_flags) atomicOr(&t.group_flags[g], f);
        }
        const uint32_t pf = atomicExch(&a.group_status[2 * g], 0u);
        const uint32_t pc = atomicExch(&a.group_status[2 * g + 1], 0u);
        const bool stands = !(t.retake_out && over);
        if (stands) {
            if (pf) atomicOr(t.status_out, pf);
            if (pc) atomicAdd(&t.status_out[1], pc);
            if (t.gstatus_out && pf) atomicOr(&t.gstatus_out[2 * g], pf);
            if (t.gstatus_out && pc) atomicAdd(&t.gstatus_out[2 * g + 1], pc);
        }
        redo = redo || !stands;
    }
    const uint32_t any = __any(redo) ? 1u : 0u;
    if (lane == 0) {
        atomicExch(&t.ctr[1], any);
        atomicExch(&t.ctr[0], 0u);
    }
}

// The FP32 march fits three waves per SIMD (at most 168 VGPRs) without
// spilling, which 256-thread workgroups can use; the FP64 one, and the
// variants with friction, two.
template <bool DEV, int SEG, bool FRIC>
__global__ void __launch_bounds__(512, (DEV && !FRIC) ? 3 : 2) k_batched(BatchArgs a) {
    constexpr int kSegPerWave = kWave / SEG;
    __shared__ int s_item;
    const int wave = threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int seg_in_wave = lane / SEG;
    const int lane_in_seg = lane % SEG;
    const int nseg = (blockDim.x / kWave) * kSegPerWave;
    const int seg_id = wave * kSegPerWave + seg_in_wave;
    if (a.retake) {
        // a retake launch with no flagged group ends at once; every workgroup
        // reads the same flags, so all of them leave and the queue stays at 0
        uint32_t any = 0;
        for (int g = 0; g < a.ngroups; ++g) any |= a.retake[g];
        if (!any) return;
    }

    for (;;) {
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&a.queue[0], 1u);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= a.nitems) break;
        const swe_item it = a.items[item];
        const swe_patch pt = a.patches[it.patch];
        if (a.retake && a.retake[pt.group] == 0) continue;  // the group's step stands
        const double dt_sub = a.dt_group[pt.group] / (double)pt.tref;
        double smx = 0.0, smy = 0.0;
        uint32_t clamps = 0, flags = 0;
        const void* src = a.pin;
        for (int s = 0; s < it.substeps; ++s) {
            // the last substep lands in pool_out; earlier ones alternate so that
            // no substep reads the buffer it writes
            void* dst = ((it.substeps - 1 - s) % 2 == 0) ? a.pout : a.pwork;
            for (int base = it.task_begin; base < it.task_end; base += nseg) {
                // with one segment per wave the task is the wave's: scalar
                const int tid = SEG == kWave ? __builtin_amdgcn_readfirstlane(base + seg_id)
                                             : base + seg_id;
                const bool active = tid < it.task_end;
                const swe_task tsk = a.tasks[active ? tid : it.task_begin];
                Task tk;
                tk.qin = src;
                tk.qout = dst;
                tk.b = a.pb;
                tk.off = pt.off;
                tk.ps = pt.plane_stride;
                tk.dt = dt_sub;
                tk.dx = pt.dx;
                tk.dy = pt.dy;
                tk.pitch = pt.pitch;
                tk.mx = pt.mx;
                tk.my = pt.my;
                tk.c0 = tsk.strip * (SEG - 4);
                tk.segw = SEG;
                tk.U0 = tsk.row0;
                tk.U1 = tsk.row0 + tsk.rows - 1;
                tk.bc[0] = pt.bc[0];
                tk.bc[1] = pt.bc[1];
                tk.bc[2] = pt.bc[2];
                tk.bc[3] = pt.bc[3];
                tk.active = active;
                tk.metric = nullptr;
                // every lane of the wave runs the same number of row iterations
                int steps = tsk.rows + 4;
#pragma unroll
                for (int o = kWave / 2; o >= 1; o >>= 1) {
                    const int other = __shfl_xor(steps, o, kWave);
                    steps = other > steps ? other : steps;
                }
                // the same for every lane after the reduction: a scalar trip count
                steps = __builtin_amdgcn_readfirstlane(steps);
                const MarchOut r = march<DEV, SEG, FRIC>(tk, a.P, lane_in_seg, steps);
                smx = r.smx > smx ? r.smx : smx;
                smy = r.smy > smy ? r.smy : smy;
                clamps += r.clamps;
                flags |= r.flags;
            }
            if (s + 1 < it.substeps) {
                // the next substep reads what this one wrote, across the waves
                __threadfence_block();
                __syncthreads();
            }
            src = dst;
        }
        // NaN propagates through the bit-pattern maximum
        const double wx = wave_max_nonneg(smx);
        const double wy = wave_max_nonneg(smy);
        if (lane == 0) {
            atomic_max_nonneg(&a.smax[2 * it.patch], wx);
            atomic_max_nonneg(&a.smax[2 * it.patch + 1], wy);
        }
        if (a.status && clamps) atomicAdd(&a.status[1], clamps);
        if (a.status && flags) atomicOr(&a.status[0], flags);
        if (a.group_status && clamps) atomicAdd(&a.group_status[2 * pt.group + 1], clamps);
        if (a.group_status && flags) atomicOr(&a.group_status[2 * pt.group], flags);
    }
    // the last workgroup to finish rewinds the queue for the next launch
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&a.queue[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&a.queue[0], 0u);
            atomicExch(&a.queue[1], 0u);
        }
    }
}

// Plain tasks (`tasks` is the plan's plain part, `nitems` its length): one
// wave per workgroup, SEG = 64 one task per wave, SEG = 32 two.  The launch
// runs substep `sub` of each task's patch (a patch with tref <= sub has no
// such substep); substeps alternate between pool_out and pool_work so that
// the last one lands in pool_out, as in the item kernel.
// Register budget as for the single-patch step (FP32 four waves per SIMD,
// FP64 three), one wave fewer with friction or with two segments per wave
// (whose tasks are per lane rather than scalar).
template <bool DEV, int SEG, bool FRIC>
__device__ __forceinline__ void plain_task(const BatchArgs& a) {
    constexpr int kSegPerWave = kWave / SEG;
    const int lane = threadIdx.x & (kWave - 1);
    const int seg_in_wave = lane / SEG;
    const int lane_in_seg = lane % SEG;
    const int t0 = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kSegPerWave);
    const int tid = SEG == kWave ? t0 : t0 + seg_in_wave;
    const bool exists = tid < a.nitems;
    const swe_task tsk = a.tasks[exists ? tid : t0];
    const swe_patch pt = a.patches[tsk.patch];
    // on a retake launch only the tasks of flagged groups run
    const bool run =
        exists && a.sub < pt.tref && (!a.retake || a.retake[pt.group] != 0);
    if (!__any(run)) return;
    const int last = pt.tref - 1;
    Task tk;
    tk.qin = a.sub == 0 ? a.pin : ((last - (a.sub - 1)) % 2 == 0 ? a.pout : a.pwork);
    tk.qout = (last - a.sub) % 2 == 0 ? a.pout : a.pwork;
    tk.b = a.pb;
    tk.off = pt.off;
    tk.ps = pt.plane_stride;
    tk.dt = a.dt_group[pt.group] / (double)pt.tref;
    tk.dx = pt.dx;
    tk.dy = pt.dy;
    tk.pitch = pt.pitch;
    tk.mx = pt.mx;
    tk.my = pt.my;
    tk.c0 = tsk.strip * (SEG - 4);
    tk.segw = SEG;
    tk.U0 = tsk.row0;
    tk.U1 = tsk.row0 + tsk.rows - 1;
    tk.bc[0] = pt.bc[0];
    tk.bc[1] = pt.bc[1];
    tk.bc[2] = pt.bc[2];
    tk.bc[3] = pt.bc[3];
    tk.active = run;
    tk.metric = nullptr;
    int steps = tsk.rows + 4;
    if (SEG != kWave) {
        const int other = __shfl_xor(steps, SEG, kWave);
        steps = other > steps ? other : steps;
    }
    steps = __builtin_amdgcn_readfirstlane(steps);
    const MarchOut r = march<DEV, SEG, FRIC>(tk, a.P, lane_in_seg, steps);
    // each segment reports to its own patch (NaN propagates through the
    // bit-pattern maximum)
    const double wx = wave_max_nonneg<SEG>(r.smx);
    const double wy = wave_max_nonneg<SEG>(r.smy);
    if (lane_in_seg == 0 && run) {
        atomic_max_nonneg(&a.smax[2 * tsk.patch], wx);
        atomic_max_nonneg(&a.smax[2 * tsk.patch + 1], wy);
    }
    if (a.status && r.clamps) atomicAdd(&a.status[1], r.clamps);
    if (a.status && r.flags) atomicOr(&a.status[0], r.flags);
    if (a.group_status && run && r.clamps) atomicAdd(&a.group_status[2 * pt.group + 1], r.clamps);
    if (a.group_status && run && r.flags) atomicOr(&a.group_status[2 * pt.group], r.flags);
}

template <bool DEV, int SEG, bool FRIC>
__global__ void __launch_bounds__(64, (DEV ? 4 : 3) - (FRIC ? 1 : 0) - (SEG == kWave ? 0 : 1))
    k_plain(BatchArgs a) {
    if (tail_idle_redo(a)) return;
    plain_task<DEV, SEG, FRIC>(a);
    if (a.t.ctr) cfl_tail(a, threadIdx.x & (kWave - 1));
}

// Packed tasks (seg = 0): one wave per pack (an entry of `items`), its tasks
// side by side from lane 0, each lane marching the task whose lanes hold it
// (lanes past the last task only take part in the cross-lane moves).  The
// launch runs substep `sub` of the pack's patches, which share one tref;
// buffers alternate as in k_plain.  Each task reports to its own patch: a
// suffix maximum within the segment leaves the segment's maximum in its
// first lane.
template <bool DEV, bool FRIC>
__device__ __forceinline__ void pack_task(const BatchArgs& a) {
    const int lane = threadIdx.x & (kWave - 1);
    const swe_item pk = a.items[blockIdx.x];
    if (a.sub >= pk.substeps) return;
    int tid = pk.task_begin, seg_l0 = 0, lane0 = 0, maxrows = 0;
    bool have = false;
    for (int j = pk.task_begin; j < pk.task_end; ++j) {
        const int w = a.tasks[j].lanes;
        const int rows = a.tasks[j].rows;
        if (!have && lane < lane0 + w) {
            tid = j;
            seg_l0 = lane0;
            have = true;
        }
        lane0 += w;
        maxrows = rows > maxrows ? rows : maxrows;
    }
    const swe_task tsk = a.tasks[tid];
    const swe_patch pt = a.patches[tsk.patch];
    const bool run = have && (!a.retake || a.retake[pt.group] != 0);
    if (!__any(run)) return;
    const int last = pk.substeps - 1;
    Task tk;
    tk.qin = a.sub == 0 ? a.pin : ((last - (a.sub - 1)) % 2 == 0 ? a.pout : a.pwork);
    tk.qout = (last - a.sub) % 2 == 0 ? a.pout : a.pwork;
    tk.b = a.pb;
    tk.off = pt.off;
    tk.ps = pt.plane_stride;
    tk.dt = a.dt_group[pt.group] / (double)pt.tref;
    tk.dx = pt.dx;
    tk.dy = pt.dy;
    tk.pitch = pt.pitch;
    tk.mx = pt.mx;
    tk.my = pt.my;
    tk.c0 = tsk.col0;
    tk.segw = tsk.lanes;
    tk.U0 = tsk.row0;
    tk.U1 = tsk.row0 + tsk.rows - 1;
    tk.bc[0] = pt.bc[0];
    tk.bc[1] = pt.bc[1];
    tk.bc[2] = pt.bc[2];
    tk.bc[3] = pt.bc[3];
    tk.active = run;
    tk.metric = nullptr;
    const int steps = __builtin_amdgcn_readfirstlane(maxrows + 4);
    const MarchOut r = march<DEV, 0, FRIC>(tk, a.P, have ? lane - seg_l0 : 0, steps);
    // suffix maximum of the bit patterns within each segment (NaN propagates)
    unsigned long long bx = run ? static_cast<unsigned long long>(__double_as_longlong(r.smx)) : 0ull;
    unsigned long long by = run ? static_cast<unsigned long long>(__double_as_longlong(r.smy)) : 0ull;
    const int seg_end = have ? seg_l0 + tsk.lanes : 0;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const unsigned long long ox = static_cast<unsigned long long>(
            __shfl_down(static_cast<long long>(bx), d, kWave));
        const unsigned long long oy = static_cast<unsigned long long>(
            __shfl_down(static_cast<long long>(by), d, kWave));
        const bool in = lane + d < seg_end;
        bx = in && ox > bx ? ox : bx;
        by = in && oy > by ? oy : by;
    }
    if (run && lane == seg_l0) {
        atomic_max_nonneg(&a.smax[2 * tsk.patch], __longlong_as_double(static_cast<long long>(bx)));
        atomic_max_nonneg(&a.smax[2 * tsk.patch + 1],
                          __longlong_as_double(static_cast<long long>(by)));
    }
    if (a.status && r.clamps) atomicAdd(&a.status[1], r.clamps);
    if (a.status && r.flags) atomicOr(&a.status[0], r.flags);
    if (a.group_status && run && r.clamps) atomicAdd(&a.group_status[2 * pt.group + 1], r.clamps);
    if (a.group_status && run && r.flags) atomicOr(&a.group_status[2 * pt.group], r.flags);
}

template <bool DEV, bool FRIC>
__global__ void __launch_bounds__(64, (DEV ? 3 : 2) - (FRIC ? 1 : 0)) k_pack(BatchArgs a) {
    if (tail_idle_redo(a)) return;
    pack_task<DEV, FRIC>(a);
    if (a.t.ctr) cfl_tail(a, threadIdx.x & (kWave - 1));
}

}  // namespace swe
