// swe_batched.hip -- many patches in one persistent launch (gfx950).
//
// Patches of an AMR hierarchy (Qin, LeVeque & Motley, Sec. 3: levels refined
// in space and time by integer ratios) or the grids of several scenarios are
// advanced together.  A host-side plan cuts every patch into strip tasks.
// A patch with tref > 1 substeps forms one item: a fixed grid of workgroups
// pulls items from a device queue ordered longest first, and an item's
// workgroup runs the substeps back to back, with a workgroup barrier between
// them (the patch's writes of one substep are the next substep's reads, and
// all of them stay on one compute unit).  The tasks of single-substep
// patches run one wave each in a second launch, which the hardware
// dispatcher balances as it does the single-patch step.  Ghost cells of
// physical boundaries are synthesised on load, so each substep refreshes
// them without a separate pass.  The arithmetic per cell is the same device
// code as the single-patch step, so a patch's result does not depend on the
// batch it runs in.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

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

template __global__ void k_batched<false, 64, false>(BatchArgs);
template __global__ void k_batched<false, 32, false>(BatchArgs);
template __global__ void k_batched<true, 64, false>(BatchArgs);
template __global__ void k_batched<true, 32, false>(BatchArgs);
template __global__ void k_batched<false, 64, true>(BatchArgs);
template __global__ void k_batched<false, 32, true>(BatchArgs);
template __global__ void k_batched<true, 64, true>(BatchArgs);
template __global__ void k_batched<true, 32, true>(BatchArgs);
template __global__ void k_plain<false, 64, false>(BatchArgs);
template __global__ void k_plain<false, 32, false>(BatchArgs);
template __global__ void k_plain<true, 64, false>(BatchArgs);
template __global__ void k_plain<true, 32, false>(BatchArgs);
template __global__ void k_plain<false, 64, true>(BatchArgs);
template __global__ void k_plain<false, 32, true>(BatchArgs);
template __global__ void k_plain<true, 64, true>(BatchArgs);
template __global__ void k_plain<true, 32, true>(BatchArgs);
template __global__ void k_pack<false, false>(BatchArgs);
template __global__ void k_pack<true, false>(BatchArgs);
template __global__ void k_pack<false, true>(BatchArgs);
template __global__ void k_pack<true, true>(BatchArgs);

}  // namespace swe

// ===========================================================================
// C ABI

namespace {

// Compute units of the current device and the occupancy (workgroups per
// compute unit) of `kern` at `threads` threads, queried once per device and
// kernel shape.
bool launch_limits(const void* kern, int threads, int* ncu, int* occ) {
    struct Key {
        int dev;
        const void* kern;
        int threads;
        int ncu, occ;
    };
    static std::mutex mu;
    static std::vector<Key> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    std::lock_guard<std::mutex> lock(mu);
    for (const Key& k : cache)
        if (k.dev == dev && k.kern == kern && k.threads == threads) {
            *ncu = k.ncu;
            *occ = k.occ;
            return true;
        }
    int n = 0, o = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
        return false;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, kern, threads, 0) != hipSuccess || o < 1)
        o = 1;
    cache.push_back(Key{dev, kern, threads, n, o});
    *ncu = n;
    *occ = o;
    return true;
}

int bfail(int code, const std::string& msg);

int check_sched(const swe_schedule* s) {
    if (!s) return bfail(SWE_EINVAL, "schedule is NULL");
    if (s->seg != 64 && s->seg != 32 && s->seg != 0)
        return bfail(SWE_EINVAL, "schedule: seg must be 64, 32 or 0");
    if (s->waves_per_group != 1 && s->waves_per_group != 2 && s->waves_per_group != 4 &&
        s->waves_per_group != 8)
        return bfail(SWE_EINVAL, "schedule: waves_per_group must be 1, 2, 4 or 8");
    if (s->rows_per_task < 0 || s->per_substep < 0 || s->per_substep > 1 ||
        s->groups_per_cu < 0 ||
        (s->order != 0 && s->order != 1))
        return bfail(SWE_EINVAL, "schedule: bad rows_per_task, per_substep, groups_per_cu or order");
    return SWE_OK;
}

}  // namespace

// error slot and the CFL rule with pending conditions, shared with
// swe_step.hip (not part of the ABI)
extern "C" __attribute__((visibility("hidden"))) int swe_internal_set_error(int code,
                                                                           const char* msg);
extern "C" __attribute__((visibility("hidden"))) int swe_internal_check_params(
    const swe_params* p);
extern "C" __attribute__((visibility("hidden"))) int swe_internal_cfl_reduce_pending(
    const swe_params* p, const swe_patch* patches, int32_t n, int32_t ngroups,
    double* smax_patch, double* dt_group, uint32_t* status, uint32_t* group_flags,
    uint32_t* retake, uint32_t* pending, uint32_t* group_status, void* stream);

namespace {
int bfail(int code, const std::string& msg) { return swe_internal_set_error(code, msg.c_str()); }
}  // namespace

extern "C" {

int swe_batched_plan(const swe_patch* patches, int32_t n, const swe_schedule* sched,
                     swe_item* items, int32_t* nitems, swe_task* tasks, int32_t* ntasks,
                     int32_t* nplain, int32_t* nsub) {
    int rc = check_sched(sched);
    if (rc) return rc;
    if (!patches || n < 0 || !nitems || !ntasks || !nplain || !nsub)
        return bfail(SWE_EINVAL, "swe_batched_plan: bad arguments");
    const bool packed = sched->seg == 0;
    const bool per_sub = sched->per_substep != 0 || packed;
    int max_tref = 0;
    const int seg = packed ? 64 : sched->seg;
    const int out_cols = seg - 4;
    const int segs_per_group = sched->waves_per_group * (64 / seg);
    struct PItem {
        swe_item it;
        double cost;
    };
    std::vector<PItem> its;
    std::vector<swe_task> tks;    // tasks of the substep items
    std::vector<swe_task> plain;  // tasks of single-substep patches
    struct Run {
        int patch, row0, rows, tref;
    };
    std::vector<Run> runs;  // seg = 0: row runs of every patch
    for (int k = 0; k < n; ++k) {
        const swe_patch& p = patches[k];
        if (p.mx < 1 || p.my < 1 || p.pitch < p.mx + 4 || p.tref < 1 || !(p.dx > 0) ||
            !(p.dy > 0) || p.off < 0 || p.plane_stride < (int64_t)p.pitch * (p.my + 4))
            return bfail(SWE_EINVAL, "swe_batched_plan: patch " + std::to_string(k) + " has a bad shape");
        for (int s = 0; s < 4; ++s) {
            if (p.bc[s] != SWE_BC_WALL && p.bc[s] != SWE_BC_EXTRAP && p.bc[s] != SWE_BC_USER)
                return bfail(SWE_EINVAL, "swe_batched_plan: unknown boundary code");
            if (p.bc[s] == SWE_BC_USER && p.tref > 1)
                return bfail(SWE_EINVAL, "swe_batched_plan: a user boundary needs tref == 1");
        }
        if ((p.bc[0] == SWE_BC_WALL || p.bc[1] == SWE_BC_WALL) && p.mx < 2)
            return bfail(SWE_EINVAL, "swe_batched_plan: a wall in x needs mx >= 2");
        if ((p.bc[2] == SWE_BC_WALL || p.bc[3] == SWE_BC_WALL) && p.my < 2)
            return bfail(SWE_EINVAL, "swe_batched_plan: a wall in y needs my >= 2");
        if (packed) {
            // equal runs of at most H rows; laid into packs below
            const int H = sched->rows_per_task > 0 ? sched->rows_per_task : 48;
            const int nch = (p.my + H - 1) / H;
            int row = 2;
            for (int cidx = 0; cidx < nch; ++cidx) {
                const int r = p.my / nch + (cidx < p.my % nch ? 1 : 0);
                runs.push_back(Run{k, row, r, p.tref});
                row += r;
            }
            if (p.tref > max_tref) max_tref = p.tref;
            continue;
        }
        const int nstrips = (p.mx + out_cols - 1) / out_cols;
        const bool item = p.tref > 1 && !per_sub;
        int H = sched->rows_per_task;
        if (H == 0) {
            if (!item) {
                // short tasks balance best (waves over water at rest finish early)
                H = 32;
            } else {
                // enough tasks to keep every segment of the workgroup busy, rows >= 8
                const int want = (segs_per_group + nstrips - 1) / nstrips;
                H = (p.my + want - 1) / want;
                if (H < 8) H = 8;
            }
        }
        if (H > p.my) H = p.my;
        const int nchunks = (p.my + H - 1) / H;
        std::vector<swe_task>& dst = item ? tks : plain;
        const int first = (int)dst.size();
        if (!item && p.tref > max_tref) max_tref = p.tref;
        for (int cidx = 0; cidx < nchunks; ++cidx)
            for (int st = 0; st < nstrips; ++st) {
                swe_task t;
                t.patch = k;
                t.strip = st;
                t.row0 = 2 + cidx * H;
                t.rows = std::min(H, p.my - cidx * H);
                t.col0 = st * out_cols;
                t.lanes = seg;
                dst.push_back(t);
            }
        if (item) {
            const int last = (int)tks.size();
            PItem pi;
            pi.it = swe_item{first, last, k, p.tref};
            pi.cost = (double)seg * (H + 4) * (last - first) * p.tref / segs_per_group;
            its.push_back(pi);
        }
    }
    if (packed) {
        // runs by tref, then height, largest first; each laid left to right
        // into 64 lanes, its columns cut where a pack fills up (a segment of
        // c columns takes c + 4 lanes; no cut leaves fewer than kMinCols
        // columns to a segment unless the patch is narrower)
        constexpr int kMinCols = 4;
        std::stable_sort(runs.begin(), runs.end(), [](const Run& x, const Run& y) {
            if (x.tref != y.tref) return x.tref > y.tref;
            return x.rows > y.rows;
        });
        int free = 0;  // lanes left in the open pack
        for (const Run& r : runs) {
            if (!its.empty() && its.back().it.substeps != r.tref) free = 0;  // one tref per pack
            const int mx = patches[r.patch].mx;
            int col = 0, piece = 0;
            while (col < mx) {
                const int rem = mx - col;
                if (free < 4 + std::min(rem, kMinCols)) {
                    PItem pi;
                    pi.it = swe_item{(int)plain.size(), (int)plain.size(), -1, r.tref};
                    pi.cost = 0.0;
                    its.push_back(pi);
                    free = 64;
                }
                int take = std::min(rem, free - 4);
                if (take < rem && rem - take < kMinCols) take = rem - kMinCols;
                if (take < 1) {
                    free = 0;
                    continue;
                }
                swe_task t;
                t.patch = r.patch;
                t.strip = piece++;
                t.row0 = r.row0;
                t.rows = r.rows;
                t.col0 = col;
                t.lanes = take + 4;
                plain.push_back(t);
                its.back().it.task_end = (int)plain.size();
                free -= take + 4;
                col += take;
            }
        }
    } else if (sched->order == 0)
        std::stable_sort(its.begin(), its.end(),
                         [](const PItem& x, const PItem& y) { return x.cost > y.cost; });
    // plain tasks by tref, largest first (a patch's tasks stay together)
    if (!packed)
        std::stable_sort(plain.begin(), plain.end(), [&](const swe_task& x, const swe_task& y) {
            return patches[x.patch].tref > patches[y.patch].tref;
        });
    const int32_t nt = (int32_t)(tks.size() + plain.size());
    *nsub = plain.empty() ? 0 : max_tref;
    if (!items || !tasks) {
        *nitems = (int32_t)its.size();
        *ntasks = nt;
        *nplain = (int32_t)plain.size();
        return SWE_OK;
    }
    if (*nitems < (int32_t)its.size() || *ntasks < nt)
        return bfail(SWE_EINVAL, "swe_batched_plan: output arrays too small");
    for (size_t i = 0; i < its.size(); ++i) items[i] = its[i].it;
    std::copy(tks.begin(), tks.end(), tasks);
    std::copy(plain.begin(), plain.end(), tasks + tks.size());
    *nitems = (int32_t)its.size();
    *ntasks = nt;
    *nplain = (int32_t)plain.size();
    return SWE_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// swe_batched_step_static: the same step with its item queue and its
// intermediate substep pool in the library's own device memory, for callers
// that cannot allocate.  Layout of the array: the queue's two counters in the
// first 256 bytes, the substep pool (at most SWE_STATIC_WORK_BYTES) after
// them.  Each device holds its own copy; host code reaches it only through
// the address hipGetSymbolAddress returns for the current device.
namespace {

constexpr size_t kStaticQueueBytes = 256;
__device__ __align__(256) unsigned char scratch[kStaticQueueBytes + SWE_STATIC_WORK_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per
// device, with that device current).
int static_scratch(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return bfail(SWE_EHIP, "swe_batched_step_static: cannot query the current device");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return bfail(SWE_EHIP, std::string("swe_batched_step_static: hipGetSymbolAddress: ") +
                                       hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SWE_OK;
}

// Zero the queue's two counters (a kernel rather than a memset node, so the
// call stays safe to capture).
__global__ void k_zero_queue(uint32_t* q) {
    if (threadIdx.x < 2) q[threadIdx.x] = 0u;
}

}  // namespace

extern "C" {

static int batched_step(const swe_params* p, const swe_patch* patches, const swe_item* items,
                        int32_t nitems, const swe_task* tasks, const swe_task* plain,
                        int32_t nplain, int32_t nsub, const void* pool_in, void* pool_out,
                        void* pool_work, int64_t pool_elems,
                        const void* pool_b, const double* dt_group, double* smax_patch,
                        uint32_t* status, uint32_t* queue, const swe_schedule* sched,
                        const uint32_t* retake, int32_t ngroups, uint32_t* group_status,
                        void* stream, bool zero_queue = false, bool pending = false,
                        const swe::CflTail* tail = nullptr) {
    if (!p) return bfail(SWE_EINVAL, "params is NULL");
    int rc = check_sched(sched);
    if (rc) return rc;
    if (p->method != SWE_SPLIT) return bfail(SWE_EINVAL, "swe_batched_step: only the split step");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return bfail(SWE_EINVAL, "swe_batched_step: precision must be SWE_F64 or SWE_F32_DEV");
    if (p->order != 1 && p->order != 2) return bfail(SWE_EINVAL, "params: order must be 1 or 2");
    if (nitems < 0 || nplain < 0 || nsub < 0 || (nplain > 0 && nsub < 1))
        return bfail(SWE_EINVAL, "swe_batched_step: bad counts");
    // items (patches with tref > 1) and per-substep launches alternate
    // between pool_out and pool_work
    const bool packed = sched->seg == 0;
    if (((nitems > 0 && !packed) || nsub > 1) && !pool_work)
        return bfail(SWE_EINVAL, "swe_batched_step: substeps need pool_work");
    if (packed && nitems > 0 && nsub < 1)
        return bfail(SWE_EINVAL, "swe_batched_step: packs need nsub >= 1");
    // pending: the steps report into group_status alone (the caller's pending
    // pairs, which the CFL rule settles)
    if (pending && !group_status) return bfail(SWE_EINVAL, "swe_batched_step: null pending pairs");
    if (!patches || !pool_in || !pool_out || !pool_b || !dt_group || !smax_patch ||
        (!status && !pending) ||
        (nitems > 0 && !items) || (nitems > 0 && !packed && (!tasks || !queue)) ||
        ((nplain > 0 || (packed && nitems > 0)) && !plain))
        return bfail(SWE_EINVAL, "swe_batched_step: null pointer");
    if (pool_elems < 1) return bfail(SWE_EINVAL, "swe_batched_step: pool_elems must be >= 1");
    {
        const size_t esz = p->precision == SWE_F64 ? sizeof(double) : sizeof(float);
        const size_t nb = (size_t)pool_elems * esz;
        auto lap = [nb](const void* x, const void* y) {
            const char* a = static_cast<const char*>(x);
            const char* b = static_cast<const char*>(y);
            return x && y && a < b + nb && b < a + nb;
        };
        if (lap(pool_in, pool_out) || lap(pool_work, pool_in) || lap(pool_work, pool_out))
            return bfail(SWE_EINVAL, "swe_batched_step: pools overlap");
    }
    if (nitems == 0 && nplain == 0) return SWE_OK;
    swe::BatchArgs a;
    a.patches = patches;
    a.items = items;
    a.tasks = tasks;
    a.pin = pool_in;
    a.pout = pool_out;
    a.pwork = pool_work ? pool_work : pool_out;  // unused without substeps
    a.pb = pool_b;
    a.dt_group = dt_group;
    a.smax = smax_patch;
    a.status = pending ? nullptr : status;
    a.group_status = group_status;
    a.queue = queue;
    a.nitems = nitems;
    a.P.g = p->g;
    a.P.drytol = p->drytol;
    a.P.h_corr = p->h_corr;
    a.P.manning_n = p->manning_n;
    a.P.sea_level = p->sea_level;
    a.P.h_fp64 = p->h_fp64;
    a.P.order = p->order;
    a.retake = retake;
    a.ngroups = ngroups;
    a.sub = 0;
    a.t = tail ? *tail : swe::CflTail{};

    const bool dev = p->precision == SWE_F32_DEV;
    const bool fric = p->manning_n > 0.0;
    const int si = sched->seg == 64 ? 0 : 1;
    hipStream_t st = static_cast<hipStream_t>(stream);
    using Kern = void (*)(swe::BatchArgs);
    if (sched->seg == 0) {
        // packs: one wave each, one launch per substep
        const Kern table[2][2] = {{swe::k_pack<false, false>, swe::k_pack<false, true>},
                                  {swe::k_pack<true, false>, swe::k_pack<true, true>}};
        swe::BatchArgs b = a;
        b.tasks = plain;
        for (int sub = 0; sub < nsub && nitems > 0; ++sub) {
            b.sub = sub;
            hipLaunchKernelGGL(table[dev ? 1 : 0][fric ? 1 : 0], dim3(nitems), dim3(64), 0, st,
                               b);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return bfail(SWE_EHIP, std::string("swe_batched_step: ") + hipGetErrorString(e));
        return SWE_OK;
    }
    if (nitems > 0) {
        // substep items: persistent workgroups on the item queue
        // [precision][segment 64 / 32][friction]
        const Kern table[2][2][2] = {
            {{swe::k_batched<false, 64, false>, swe::k_batched<false, 64, true>},
             {swe::k_batched<false, 32, false>, swe::k_batched<false, 32, true>}},
            {{swe::k_batched<true, 64, false>, swe::k_batched<true, 64, true>},
             {swe::k_batched<true, 32, false>, swe::k_batched<true, 32, true>}}};
        const Kern kern = table[dev ? 1 : 0][si][fric ? 1 : 0];
        const int threads = 64 * sched->waves_per_group;
        int ncu = 0, occ = 0;
        if (!launch_limits(reinterpret_cast<const void*>(kern), threads, &ncu, &occ))
            return bfail(SWE_EHIP, "swe_batched_step: cannot query the device");
        const int per_cu = sched->groups_per_cu ? sched->groups_per_cu : occ;
        int grid = ncu * per_cu;
        if (grid > nitems) grid = nitems;
        if (grid < 1) grid = 1;
        if (zero_queue) hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, queue);
        hipLaunchKernelGGL(kern, dim3(grid), dim3(threads), 0, st, a);
    }
    if (nplain > 0) {
        // single-substep tasks: one wave each, balanced by the dispatcher
        const Kern table[2][2][2] = {
            {{swe::k_plain<false, 64, false>, swe::k_plain<false, 64, true>},
             {swe::k_plain<false, 32, false>, swe::k_plain<false, 32, true>}},
            {{swe::k_plain<true, 64, false>, swe::k_plain<true, 64, true>},
             {swe::k_plain<true, 32, false>, swe::k_plain<true, 32, true>}}};
        swe::BatchArgs b = a;
        b.tasks = plain;
        b.nitems = nplain;
        const int per_wave = sched->seg == 64 ? 1 : 2;
        const int grid = (nplain + per_wave - 1) / per_wave;
        for (int sub = 0; sub < nsub; ++sub) {
            b.sub = sub;
            hipLaunchKernelGGL(table[dev ? 1 : 0][si][fric ? 1 : 0], dim3(grid), dim3(64), 0,
                               st, b);
        }
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return bfail(SWE_EHIP, std::string("swe_batched_step: ") + hipGetErrorString(e));
    return SWE_OK;
}

int swe_batched_step(const swe_params* p, const swe_patch* patches, const swe_item* items,
                     int32_t nitems, const swe_task* tasks, const swe_task* plain,
                     int32_t nplain, int32_t nsub, const void* pool_in, void* pool_out,
                     void* pool_work, int64_t pool_elems, const void* pool_b,
                     const double* dt_group, double* smax_patch, uint32_t* status,
                     uint32_t* group_status, uint32_t* queue, const swe_schedule* sched,
                     void* stream) {
    return batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool_in,
                        pool_out, pool_work, pool_elems, pool_b, dt_group, smax_patch, status,
                        queue, sched, nullptr, 0, group_status, stream);
}

int swe_batched_step_static(const swe_params* p, const swe_patch* patches,
                            const swe_item* items, int32_t nitems, const swe_task* tasks,
                            const swe_task* plain, int32_t nplain, int32_t nsub,
                            const void* pool_in, void* pool_out, int64_t pool_elems,
                            const void* pool_b, const double* dt_group, double* smax_patch,
                            uint32_t* status, uint32_t* group_status,
                            const swe_schedule* sched, void* stream) {
    if (!p) return bfail(SWE_EINVAL, "params is NULL");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return bfail(SWE_EINVAL, "swe_batched_step_static: precision must be SWE_F64 or SWE_F32_DEV");
    if (pool_elems < 1) return bfail(SWE_EINVAL, "swe_batched_step_static: pool_elems must be >= 1");
    const size_t esz = p->precision == SWE_F64 ? sizeof(double) : sizeof(float);
    const bool work = (nitems > 0 && sched && sched->seg != 0) || nsub > 1;
    if (work && (uint64_t)pool_elems > SWE_STATIC_WORK_BYTES / esz)
        return bfail(SWE_EINVAL,
                     "swe_batched_step_static: the pool (" + std::to_string(pool_elems) +
                         " elements) exceeds the static substep pool of " +
                         std::to_string(SWE_STATIC_WORK_BYTES) +
                         " bytes; use swe_batched_step with a caller-provided pool_work");
    void* base = nullptr;
    int rc = static_scratch(&base);
    if (rc) return rc;
    uint32_t* queue = static_cast<uint32_t*>(base);
    void* pwork = static_cast<unsigned char*>(base) + kStaticQueueBytes;
    return batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool_in, pool_out,
                        work ? pwork : nullptr, pool_elems, pool_b, dt_group, smax_patch, status,
                        queue, sched, nullptr, 0, group_status, stream, true);
}

int swe_batched_advance(const swe_params* p, const swe_patch* patches, int32_t npatches,
                        int32_t ngroups, const swe_item* items, int32_t nitems,
                        const swe_task* tasks, const swe_task* plain, int32_t nplain,
                        int32_t nsub, void* pool_0, void* pool_1, int32_t first,
                        void* pool_work, int64_t pool_elems, const void* pool_b,
                        double* dt_group, double* smax_patch, uint32_t* status,
                        uint32_t* group_status, uint32_t* group_flags, uint32_t* retake,
                        uint32_t* pending, uint32_t* queue, const swe_schedule* sched,
                        int32_t nsteps, void* stream) {
    if (first != 0 && first != 1) return bfail(SWE_EINVAL, "swe_batched_advance: first must be 0 or 1");
    if (nsteps < 0 || npatches < 0 || ngroups < 1)
        return bfail(SWE_EINVAL, "swe_batched_advance: bad nsteps, npatches or ngroups");
    if (!retake || !pending || !status || !pool_0 || !pool_1)
        return bfail(SWE_EINVAL, "swe_batched_advance: null retake flags, pending pairs, status or pool");
    void* pool[2] = {pool_0, pool_1};
    int cur = first;
    // a step that is one launch (single-substep plain tasks, or packs with
    // one substep) carries the CFL rule in its last workgroup, with the
    // queue's two words as its counters
    const bool fused = queue && sched && nsub == 1 && ngroups <= swe::kTailGroups &&
                       (sched->seg == 0 ? nitems > 0 : (nitems == 0 && nplain > 0));
    if (fused) {
        int rc = swe_internal_check_params(p);
        if (rc) return rc;
        swe::CflTail t{};
        t.ctr = queue;
        t.npatches = npatches;
        t.ngroups = ngroups;
        t.dt_next = dt_group;
        t.retake_out = retake;
        t.status_out = status;
        t.gstatus_out = group_status;
        t.group_flags = group_flags;
        t.cfl_desired = p->cfl_desired;
        t.cfl_max = p->cfl_max;
        swe::CflTail last = t;
        last.retake_out = nullptr;
        for (int k = 0; k < nsteps; ++k) {
            // the step, then up to two gated redos, each launch ending with the
            // rule (the last one flags a step still above the limit)
            rc = batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool[cur],
                              pool[1 - cur], pool_work, pool_elems, pool_b, dt_group, smax_patch,
                              nullptr, queue, sched, nullptr, 0, pending, stream, false, true, &t);
            if (rc) return rc;
            for (int redo = 0; redo < 2; ++redo) {
                rc = batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub,
                                  pool[cur], pool[1 - cur], pool_work, pool_elems, pool_b,
                                  dt_group, smax_patch, nullptr, queue, sched, retake, ngroups,
                                  pending, stream, false, true, redo == 0 ? &t : &last);
                if (rc) return rc;
            }
            cur ^= 1;
        }
        return SWE_OK;
    }
    for (int k = 0; k < nsteps; ++k) {
        // the step, the CFL rule with the retake flags, the gated redo of the
        // flagged groups, and the CFL rule of the redone steps
        // the steps report their conditions as pending per group; the CFL
        // rule settles them (a step it redoes reports nothing)
        int rc = batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool[cur],
                              pool[1 - cur], pool_work, pool_elems, pool_b, dt_group, smax_patch,
                              nullptr, queue, sched, nullptr, 0, pending, stream, false, true);
        if (rc) return rc;
        rc = swe_internal_cfl_reduce_pending(p, patches, npatches, ngroups, smax_patch, dt_group,
                                             status, group_flags, retake, pending, group_status,
                                             stream);
        if (rc) return rc;
        // up to two redos: a redone step still above the limit is redone once
        // more, and only a second redo still above it stands, flagged
        for (int redo = 0; redo < 2; ++redo) {
            rc = batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool[cur],
                              pool[1 - cur], pool_work, pool_elems, pool_b, dt_group, smax_patch,
                              nullptr, queue, sched, retake, ngroups, pending, stream, false,
                              true);
            if (rc) return rc;
            rc = swe_internal_cfl_reduce_pending(p, patches, npatches, ngroups, smax_patch,
                                                 dt_group, status, group_flags,
                                                 redo == 0 ? retake : nullptr, pending,
                                                 group_status, stream);
            if (rc) return rc;
        }
        cur ^= 1;
    }
    return SWE_OK;
}

int swe_batched_retake(const swe_params* p, const swe_patch* patches, const swe_item* items,
                       int32_t nitems, const swe_task* tasks, const swe_task* plain,
                       int32_t nplain, int32_t nsub, const void* pool_in, void* pool_out,
                       void* pool_work, int64_t pool_elems, const void* pool_b,
                       const double* dt_group, double* smax_patch, uint32_t* status,
                       uint32_t* group_status, uint32_t* queue, const swe_schedule* sched,
                       const uint32_t* retake, int32_t ngroups, void* stream) {
    if (!retake || ngroups < 1)
        return bfail(SWE_EINVAL, "swe_batched_retake: null retake flags or ngroups < 1");
    return batched_step(p, patches, items, nitems, tasks, plain, nplain, nsub, pool_in,
                        pool_out, pool_work, pool_elems, pool_b, dt_group, smax_patch, status,
                        queue, sched, retake, ngroups, group_status, stream);
}

}  // extern "C"
