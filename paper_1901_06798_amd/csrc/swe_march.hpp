// swe_march.hpp -- the split step of one strip of a patch, marched down its
// rows by a segment of SEG lanes (SEG = 64: a whole wave64; SEG = 32: two
// strips, possibly of different patches, share a wave; SEG = 0: the task
// states its own width, so strips of any width, each with its own halo
// lanes, lie side by side in one wave).
//
// Qin, LeVeque & Motley, Sec. 2, dimensionally split x/y forms.  A segment
// owns SEG adjacent columns and updates the SEG - 4 inner ones over a chunk of
// rows.  For every row it loads (h or eta', hu, hv, b) once (coalesced along
// x), solves the x-edges of the row one lane per edge, exchanges neighbour
// data across lanes for the limiter and the update, and so obtains Q* of the
// row in registers.  The y-sweep is a per-lane pipeline over the rows of Q*:
// each lane keeps the waves of the last y-edge, so every y-edge of its column
// is solved once, and the cell two rows behind is finished and written.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "swe.h"
#include "swe_common.hpp"
#include "swe_math.hpp"

namespace swe {

template <bool DEV>
struct Prec;
template <>
struct Prec<false> {
    using S = double;
};
template <>
struct Prec<true> {
    using S = float;
};

// Side of a cell from its stored values (q0 = h, or eta' on the deviation
// path, where h = eta' + sea_level - b).
template <bool DEV, typename T, typename S>
__device__ __forceinline__ Side<T> side_base_from(S q0, S m, S t, S b, const DevParams& P) {
    if (!DEV) return side_base<T>(T(q0), T(m), T(t), T(b), P);
    const T h = T(q0) + T(P.sea_level) - T(b);
    Side<T> s = side_base<T>(h, T(m), T(t), T(b), P);
    s.eta = T(q0);
    return s;
}

template <bool DEV, typename T, typename S>
__device__ __forceinline__ Side<T> side_from(S q0, S m, S t, S b, const DevParams& P) {
    Side<T> s = side_base_from<DEV, T, S>(q0, m, t, b, P);
    side_finish(s);
    return s;
}

// Riemann solve of one edge.  On the deviation path an edge with a cell at
// or below h_fp64 deep (dry cells included) is solved in FP64 from the exact
// FP64 values of the stored floats; its waves are rounded to FP32.
template <bool DEV, typename S>
__device__ __forceinline__ void solve_edge(const Side<S>& L, const Side<S>& R, S mL, S tL, S mR,
                                           S tR, const DevParams& P, Waves<S>& w) {
    if (!DEV) {
        riemann<S, false>(L, R, P, w);
        return;
    }
    if (sizeof(S) == sizeof(double)) {  // FP64 arithmetic over FP32 storage
        riemann<S, true>(L, R, P, w);
        return;
    }
    const bool wide = L.h <= S(P.h_fp64) || R.h <= S(P.h_fp64);
    if (wide) {
        const Side<double> L64 = side_from<true, double, double>(L.eta, mL, tL, L.b, P);
        const Side<double> R64 = side_from<true, double, double>(R.eta, mR, tR, R.b, P);
        Waves<double> w64;
        riemann<double, true>(L64, R64, P, w64);
        w.kind = w64.kind;
        w.shallow = w64.shallow;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            w.s[p] = S(w64.s[p]);
            w.z[p][0] = S(w64.z[p][0]);
            w.z[p][1] = S(w64.z[p][1]);
            w.z[p][2] = S(w64.z[p][2]);
        }
    } else {
        riemann<S, true>(L, R, P, w);
    }
}

// Dry cleanup after a sweep: no momentum at or below the dry tolerance; a
// negative depth is reset to 0 and counted.  `valid` marks lanes whose value
// belongs to the patch (only those report).
template <bool DEV, typename S>
__device__ __forceinline__ void cleanup(S q[3], S b, const DevParams& P, bool valid, bool count,
                                        uint32_t& clamps, uint32_t& flags) {
    if (valid && !(isfinite(q[0]) && isfinite(q[1]) && isfinite(q[2])))
        flags |= SWE_STATUS_NONFINITE;
    const S h = DEV ? q[0] + S(P.sea_level) - b : q[0];
    if (h < S(0)) {
        q[0] = DEV ? b - S(P.sea_level) : S(0);
        q[1] = q[2] = S(0);
        if (count) {
            ++clamps;
            flags |= SWE_STATUS_NEG_DEPTH;
        }
    } else if (h <= S(P.drytol)) {
        q[1] = q[2] = S(0);
    }
}

#ifndef SWE_QUIET
#define SWE_QUIET 1
#endif

// Edges whose waves are known without a solve:
// - both cells dry: no waves, all speeds 0 (the solver's first exit);
// - both cells wet, no momentum, bitwise equal surfaces: the decomposition of
//   a zero jump, so all f-waves are exactly 0, and the largest speed is
//   max(c_L, c_R): with u = 0 the speed bounds are -max(c_L, c_hat) and
//   max(c_R, c_hat), and c_hat = sqrt(g (h_L + h_R) / 2) never exceeds
//   max(c_L, c_R), also after rounding.
// When every lane of the wave whose edge feeds a result has such an edge the
// solve is skipped (the halo lanes then carry waves that are not their
// solver's, which reach no result).  With
// zero f-waves the fluctuations and corrections are 0 whatever the speeds, so
// the step's results, including the speed maximum, are the solver's.
template <bool DEV, typename S>
__device__ __forceinline__ bool quiet_edge(const Side<S>& L, const Side<S>& R) {
    const S deta = DEV ? (R.eta - L.eta) : (R.h - L.h) + (R.b - L.b);
    const bool rest = !L.dry && !R.dry && L.m == S(0) && L.t == S(0) && R.m == S(0) &&
                      R.t == S(0) && deta == S(0);
    return rest || (L.dry && R.dry);
}

template <typename S>
__device__ __forceinline__ void quiet_waves(const Side<S>& L, const Side<S>& R,
                                            const DevParams& P, Waves<S>& w) {
    const bool dry = L.dry && R.dry;
    const S c = L.c > R.c ? L.c : R.c;
    const S m = dry ? S(0) : c;
    w.kind = dry ? kEdgeDry : kEdgeWet;
    w.shallow = L.h <= S(P.h_corr) || R.h <= S(P.h_corr);
#pragma unroll
    for (int p = 0; p < 3; ++p) w.z[p][0] = w.z[p][1] = w.z[p][2] = S(0);
    w.s[0] = -m;
    w.s[1] = S(0);
    w.s[2] = m;
}

// One strip task as seen by one lane.
struct Task {
    const void* qin;
    void* qout;
    const void* b;
    int64_t off, ps;
    double dt, dx, dy;
    int pitch, mx, my;
    int c0;       // column (ghosts included) of the segment's first lane
    int segw;     // lanes of the segment (read when SEG = 0; 5 .. kWave)
    int U0, U1;   // first and last row updated (ghost rows are 0, 1, my + 2, my + 3)
    int8_t bc[4];
    bool active;  // false: the lane only takes part in the cross-lane moves
    // latitude-longitude patches: capacities of rows 0 .. my + 3, then the
    // length ratios of the edges between rows e - 1 and e, e = 0 .. my + 4
    const double* metric;
};

// Per-lane results of a march.
struct MarchOut {
    double smx, smy;
    uint32_t clamps, flags;
    uint32_t work;  // row sweeps (x or y) that needed Riemann solves
};

// ---- LDS row ring: rows of the strip loaded RING rows ahead of their use by
// direct global-to-LDS loads, which occupy no vector registers while in
// flight.  Each wave owns RING slots of 4 planes x kWave elements (h or eta',
// hu, hv, b).  A dword load writes lane i's dword to LDS at M0 + 4 i; an FP64
// plane row (kWave doubles) therefore takes two loads, each lane fetching one
// half of a double.  Every element's address comes from map_cell, so ghost
// cells of physical boundaries are synthesised as in the register path
// (mirrored momenta change sign when read).  The loads are issued as inline
// assembly, so the compiler does not track them: the march waits for them
// itself (vector-memory loads complete in issue order, so "at most N
// outstanding" with N = the loads issued after a row's guarantees that row).

template <int N>
__device__ __forceinline__ void wait_vmem_at_most() {
    asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
}

__device__ __forceinline__ void lds_dword_load(const void* src, uint32_t lds_addr) {
    asm volatile("global_load_lds_dword %0, off" ::"v"(src), "{m0}"(lds_addr) : "memory");
}

template <typename S>
struct RingRow;
template <>
struct RingRow<double> {
    static constexpr int kLoads = 8;  // dword loads per row: 4 planes x 2 halves
};
template <>
struct RingRow<float> {
    static constexpr int kLoads = 4;
};

// Issue the loads of strip row `row` into ring slot `slot`.  The slot's
// previous contents must have been read: wait for outstanding LDS reads first.
template <typename S>
__device__ __forceinline__ void ring_issue(const Task& tk, int row, int lane, uint32_t slot_lds,
                                           bool cols_in) {
    const S* qin = static_cast<const S*>(tk.qin);
    const S* bpl = static_cast<const S*>(tk.b);
    const bool inside = __all(cols_in && row >= 2 && row <= tk.my + 1);
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    constexpr uint32_t kPlane = kWave * sizeof(S);
    if constexpr (sizeof(S) == 8) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            int ce = tk.c0 + k * (kWave / 2) + (lane >> 1);
            ce = ce < tk.mx + 3 ? ce : tk.mx + 3;
            const Src sr = map_cell_voted(inside, row, ce, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
            const int half = 4 * (lane & 1);
            const uint32_t m = slot_lds + k * (kWave * 4);
            lds_dword_load(reinterpret_cast<const char*>(qin + sr.idx) + half, m);
            lds_dword_load(reinterpret_cast<const char*>(qin + sr.idx + tk.ps) + half, m + kPlane);
            lds_dword_load(reinterpret_cast<const char*>(qin + sr.idx + 2 * tk.ps) + half,
                           m + 2 * kPlane);
            lds_dword_load(reinterpret_cast<const char*>(bpl + sr.idx) + half, m + 3 * kPlane);
        }
    } else {
        int ce = tk.c0 + lane;
        ce = ce < tk.mx + 3 ? ce : tk.mx + 3;
        const Src sr = map_cell_voted(inside, row, ce, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
        lds_dword_load(qin + sr.idx, slot_lds);
        lds_dword_load(qin + sr.idx + tk.ps, slot_lds + kPlane);
        lds_dword_load(qin + sr.idx + 2 * tk.ps, slot_lds + 2 * kPlane);
        lds_dword_load(bpl + sr.idx, slot_lds + 3 * kPlane);
    }
}

// March one strip task.  `steps` is the number of row iterations every lane
// of the wave executes (the largest over the wave's segments); a lane whose
// own strip is shorter repeats its last row with writes and reports masked.
// FRIC: the Manning friction step is compiled in (the caller picks it when
// the friction coefficient is positive), so the step without friction
// carries none of its registers.
// RING > 0: rows come through an LDS ring of RING slots at `ring` (this
// wave's RING x 4 x kWave elements; SEG must be kWave); RING = 0: each row is
// loaded into registers one iteration ahead.
// SPH: a latitude-longitude patch (FP64): a row's cells have capacity kappa
// (area over the area at the equator) and a parallel edge's length is its
// ratio len times dx; the updates divide by kappa and weight the y-edge
// amounts by len, the corrections and the speed maxima use the mean inverse
// capacity of the edge's cells, and the mass update takes out the term
// f(Q) (len_lower - len_upper) that edge-weighted fluctuations add (the
// continuity equation has no metric source).
template <bool DEV, int SEG, bool FRIC, int RING = 0, bool SPH = false, bool WIDE = false>
__device__ __forceinline__ MarchOut march(const Task& tk, const DevParams& P, int lane_in_seg,
                                          int steps, typename Prec<DEV>::S* ring = nullptr) {
    static_assert(!SPH || !DEV, "latitude-longitude patches: FP64 only");
    static_assert(!SPH || SEG == kWave, "per-row tables are held one row per lane");
    static_assert(RING == 0 || SEG == kWave, "the row ring serves whole-wave strips");
    static_assert((RING & (RING - 1)) == 0, "ring depth is a power of two");
    using S = typename Prec<DEV>::S;
    // lane moves run over the whole wave unless segments have a fixed width
    constexpr int LS = SEG ? SEG : kWave;
    const int segw = SEG ? SEG : tk.segw;
    // arithmetic type: the storage type, or FP64 over FP32 storage (WIDE)
    using A = typename std::conditional<WIDE, double, S>::type;
    const S* __restrict__ qin = static_cast<const S*>(tk.qin);
    S* __restrict__ qout = static_cast<S*>(tk.qout);
    const S* __restrict__ bpl = static_cast<const S*>(tk.b);
    const int lane = lane_in_seg;
    const int c = tk.c0 + lane;  // column of this lane (ghosts included)
    const int cc = c < tk.mx + 3 ? c : tk.mx + 3;
    const bool upd_col = tk.active && lane >= 2 && lane <= segw - 3 && c <= tk.mx + 1;
    const bool xedge_own = tk.active && lane >= 2 && lane <= segw - 2 && c >= 2 && c <= tk.mx + 2;
    const int U0 = tk.U0, U1 = tk.U1;
    const A lamx = A(tk.dt / tk.dx), lamy = A(tk.dt / tk.dy);
    // rows U0 - 2 .. U1 + 2 of the task, one per lane (at most kWave of
    // them): lane l holds 1 / kappa of row U0 - 2 + l; a row's value is read
    // from its lane, so no division is left in the march
    const int rbase = U0 - 2;
    double ik_l = 0.0;
    if (SPH) ik_l = 1.0 / tk.metric[min(rbase + lane, tk.my + 3)];
    const double* lenv = SPH ? tk.metric + (tk.my + 4) : nullptr;
    const bool second = P.order >= 2;
    const int tlast = U1 - U0 + 4;
    // the segment's columns all lie inside the patch (no ghost column)
    const bool cols_in = tk.c0 >= 2 && tk.c0 + segw - 1 <= tk.mx + 1;

    A smx = A(0), smy = A(0);
    uint32_t clamps = 0, flags = 0;
    uint32_t work = 0;

    // rolling state of the y-pipeline (row R - 1, R - 2 of Q*, edge E - 1)
    Side<A> prev;
    prev.h = prev.m = prev.t = prev.b = prev.u = prev.v = prev.sq = prev.c = prev.eta = A(0);
    prev.dry = true;
    A qm2[3] = {0, 0, 0};
    A qm2_b = A(0);
    Waves<A> wprev;
    bool wprev_quiet = false;  // wprev came from the quiet-edge path (zero f-waves)
    bool prev_full = false;    // prev carries its velocities and sqrt(h)
    A dprev[3] = {0, 0, 0};
    A ap_prev[3] = {0, 0, 0}, F_prev[3] = {0, 0, 0};
    // finished row held for one iteration: its stores are issued before the
    // next row's loads, so waiting for those loads never waits for stores
    A po[3] = {0, 0, 0};
    int po_row = 0;
    bool po_wr = false;

    // Row t of the march is patch row U0 - 2 + min(t, tlast): every row index
    // stays within 0 .. my + 3, also one past the last iteration, so the
    // next row's loads are issued unconditionally one iteration ahead and
    // their latency hides behind the current row's arithmetic.  Signs of
    // mirrored ghost momenta are applied at use, so no arithmetic waits on
    // the loads before then.
    S nq0, nhu, nhv, nbb;
    bool nfx, nfy;
    uint32_t ring_lds = 0;
    if constexpr (RING > 0) {
        ring_lds = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(
            reinterpret_cast<uintptr_t>((__attribute__((address_space(3))) S*)ring)));
#pragma unroll
        for (int k = 0; k < RING; ++k)
            ring_issue<S>(tk, U0 - 2 + (k <= tlast ? k : tlast), lane,
                          ring_lds + k * (4 * kWave * sizeof(S)), cols_in);
    } else {
        const Src s0 = map_cell(U0 - 2, cc, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
        nq0 = qin[s0.idx];
        nhu = qin[s0.idx + tk.ps];
        nhv = qin[s0.idx + 2 * tk.ps];
        nbb = bpl[s0.idx];
        nfx = s0.sx < 0.0;
        nfy = s0.sy < 0.0;
    }

    for (int t = 0; t < steps; ++t) {
        const bool live = t <= tlast;
        const int R = U0 - 2 + (live ? t : tlast);
        const bool interior_row = live && R >= U0 && R <= U1;

        // ---- row R (ghosts synthesised for physical boundaries), loaded one
        // iteration ago; then issue the loads of the next row
        A q0, hu, hv, bb;
        if constexpr (RING > 0) {
            // row t is complete once at most the loads of rows t + 1 ..
            // t + RING - 1 are outstanding
            wait_vmem_at_most<(RING - 1) * RingRow<S>::kLoads>();
            const S* rs = ring + (t & (RING - 1)) * (4 * kWave);
            const Src sg = map_cell_voted(__all(cols_in && R >= 2 && R <= tk.my + 1), R, cc,
                                          tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
            q0 = rs[lane];
            const S rhu = rs[kWave + lane];
            const S rhv = rs[2 * kWave + lane];
            bb = rs[3 * kWave + lane];
            hu = sg.sx < 0.0 ? -rhu : rhu;
            hv = sg.sy < 0.0 ? -rhv : rhv;
        } else {
            q0 = nq0;
            hu = nfx ? -nhu : nhu;
            hv = nfy ? -nhv : nhv;
            bb = nbb;
        }
        if (po_wr) {
            const int64_t o = tk.off + (int64_t)po_row * tk.pitch + c;
            qout[o] = po[0];
            qout[o + tk.ps] = po[1];
            qout[o + 2 * tk.ps] = po[2];
        }
        po_wr = false;
        if constexpr (RING > 0) {
            // row t + RING into the slot just read
            const int ta = t + RING;
            ring_issue<S>(tk, U0 - 2 + (ta <= tlast ? ta : tlast), lane,
                          ring_lds + (t & (RING - 1)) * (4 * kWave * sizeof(S)), cols_in);
        } else {
            const int Rn = U0 - 2 + (t + 1 <= tlast ? t + 1 : tlast);
            const Src sn = map_cell(Rn, cc, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
            nq0 = qin[sn.idx];
            nhu = qin[sn.idx + tk.ps];
            nhv = qin[sn.idx + 2 * tk.ps];
            nbb = bpl[sn.idx];
            nfx = sn.sx < 0.0;
            nfy = sn.sy < 0.0;
        }

        // ---- x-sweep of row R: lane k solves the edge between columns k-1, k
        Side<A> me = side_base_from<DEV, A, A>(q0, hu, hv, bb, P);
        Side<A> lf = side_up<A, DEV, LS>(me, P);
        Waves<A> w;
        A qs[3];
        // lane 0's edge (its left cell lies outside the segment) feeds nothing,
        // nor does a lane outside every task
        if (SWE_QUIET && __all(lane == 0 || !tk.active || quiet_edge<DEV, A>(lf, me))) {
            // zero f-waves: the fluctuations and corrections are +0 and the
            // update returns Q itself, as the arithmetic below would
            quiet_waves(lf, me, P, w);
            qs[0] = q0;
            qs[1] = hu;
            qs[2] = hv;
        } else {
            ++work;
            side_finish(me);
            lf.u = lane_up<LS>(me.u);
            lf.v = lane_up<LS>(me.v);
            lf.sq = lane_up<LS>(me.sq);
            const A lf_m = DEV ? lane_up<LS>(hu) : A(0);
            const A lf_t = DEV ? lane_up<LS>(hv) : A(0);
            solve_edge<DEV, A>(lf, me, lf_m, lf_t, hu, hv, P, w);
            A am[3], ap[3];
            fluctuations(w, am, ap);
            A F[3] = {A(0), A(0), A(0)};
            if (second) {
                A dr[3], dl[3];
#pragma unroll
                for (int p = 0; p < 3; ++p) {
                    const A zr0 = lane_down<LS>(w.z[p][0]);
                    const A zr1 = lane_down<LS>(w.z[p][1]);
                    const A zr2 = lane_down<LS>(w.z[p][2]);
                    dr[p] = w.z[p][0] * zr0 + w.z[p][1] * zr1 + w.z[p][2] * zr2;
                }
#pragma unroll
                for (int p = 0; p < 3; ++p) dl[p] = lane_up<LS>(dr[p]);
                if (SPH) {
                    correction(w, dl, dr, A(lamx * lane_read(ik_l, R - rbase)), F);
                } else {
                    correction(w, dl, dr, lamx, F);
                }
            }
            const A qc[3] = {q0, hu, hv};
            const A lx = SPH ? A(lamx * lane_read(ik_l, R - rbase)) : lamx;
            if (second) {
                // positivity limit: the donor of this lane's edge is the left
                // cell (lane k - 1) for a positive mass correction, else this
                // lane's cell; h1 = depth after the first-order part of the update
                const A h1 = me.h - lx * (ap[0] + lane_down<LS>(am[0]));
                const A h1l = lane_up<LS>(h1);
                drain_limit(F, F[0] > A(0) ? h1l : h1, lx, A(1));
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const A amr = lane_down<LS>(am[k]);
                const A Fr = lane_down<LS>(F[k]);
                qs[k] = qc[k] - lx * (ap[k] + amr) - lx * (Fr - F[k]);
            }
        }
        cleanup<DEV, A>(qs, bb, P, upd_col && live, interior_row && upd_col, clamps, flags);
        if (interior_row && xedge_own) {
            A s = max_speed(w);
            if (SPH) s = A(s * lane_read(ik_l, R - rbase));
            smx = s > smx ? s : smx;
        }

        // ---- y-sweep pipeline on the column of Q* (normal momentum hv)
        Side<A> cur = side_base_from<DEV, A, A>(qs[0], qs[2], qs[1], bb, P);
        bool cur_full = false;
        if (t >= 1) {
            Waves<A> wy;
            // the y-sweep of a lane feeds only its own column's update
            const bool yq = SWE_QUIET && __all(!upd_col || quiet_edge<DEV, A>(prev, cur));
            if (yq) {
                quiet_waves(prev, cur, P, wy);
            } else {
                ++work;
                // velocities and sqrt(h) only for a solve (same values whenever
                // they are computed)
                if (!prev_full) side_finish(prev);
                side_finish(cur);
                cur_full = true;
                // Q* is cleaned up, so a dry side's stored momenta are 0 and
                // the Sides carry the stored values for the FP64 islands too
                solve_edge<DEV, A>(prev, cur, prev.m, prev.t, cur.m, cur.t, P, wy);
            }
            const int E = R;  // edge between rows R - 1 and R
            const double a_e =
                SPH ? 0.5 * (lane_read(ik_l, E - 1 - rbase) + lane_read(ik_l, E - rbase)) : 1.0;
            if (live && E >= U0 && E <= U1 + 1 && upd_col) {
                A s = max_speed(wy);
                if (SPH) s = A(s * a_e);
                smy = s > smy ? s : smy;
            }
            // with either edge quiet the dot product is a zero, and a zero
            // numerator gives theta = +-0, whose limiter value is +0 either way
            A dcur[3] = {A(0), A(0), A(0)};
            if (second && t >= 2 && !yq && !wprev_quiet) {
#pragma unroll
                for (int p = 0; p < 3; ++p) dcur[p] = dot3(wprev.z[p], wy.z[p]);
            }
            if (t >= 2) {
                // edge E - 1: fluctuations (from t = 2, so that the edge below
                // a task's first updated row has its A+dQ for the positivity
                // limit) and, from t = 3, the correction (+0 for a quiet edge)
                A am1[3] = {A(0), A(0), A(0)}, ap1[3] = {A(0), A(0), A(0)};
                A F1[3] = {A(0), A(0), A(0)};
                if (!wprev_quiet) {
                    fluctuations(wprev, am1, ap1);
                    if (second && t >= 3) correction(wprev, dprev, dcur,
                                   SPH ? A(lamy * (0.5 * (lane_read(ik_l, E - 2 - rbase) +
                                                          lane_read(ik_l, E - 1 - rbase))))
                                       : lamy,
                                   F1);
                }
                if (second && t >= 3) {
                    // positivity limit of edge E - 1's correction: its donor is
                    // row R - 2 (below) for a positive mass correction, else row
                    // R - 1; h1 = depth after the first-order part of the update
                    // (between edges E - 2, E - 1, and E - 1, E)
                    const bool up = !(F1[0] > A(0));
                    const A hlo = DEV ? qm2[0] + A(P.sea_level) - qm2_b : qm2[0];
                    const A hd = up ? prev.h : hlo;
                    const A apd = up ? ap1[0] : ap_prev[0];
                    const A amd = up ? minus_mass(wy) : am1[0];
                    if (SPH) {
                        const int rd = up ? R - 1 : R - 2;  // donor row
                        const A lc = lamy * lane_read(ik_l, rd - rbase);
                        const A ll = lenv[rd], lu = lenv[rd + 1];
                        const A md = up ? prev.m : qm2[1];
                        const A h1 = (hd - lc * (ll * apd + lu * amd)) + lc * (md * (ll - lu));
                        drain_limit(F1, h1, lc, A(lenv[E - 1]));
                    } else {
                        const A h1 = hd - lamy * (apd + amd);
                        drain_limit(F1, h1, lamy, A(1));
                    }
                }
                if (t >= 4) {
                    // finish row R - 2 between edges E - 2 and E - 1
                    A qn[3];
                    if (SPH) {
                        // cell c = R - 2 between edges c (below) and c + 1 (above)
                        const int cr = R - 2;
                        const A lc = lamy * lane_read(ik_l, cr - rbase);
                        const A ll = lenv[cr], lu = lenv[cr + 1];
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            qn[k] = qm2[k] - lc * (ll * ap_prev[k] + lu * am1[k])
                                           - lc * (lu * F1[k] - ll * F_prev[k]);
                        qn[0] += lc * (qm2[1] * (ll - lu));
                    } else {
#pragma unroll
                        for (int k = 0; k < 3; ++k)
                            qn[k] = qm2[k] - lamy * (ap_prev[k] + am1[k]) -
                                    lamy * (F1[k] - F_prev[k]);
                    }
                    // the y-sweep works in (h, hv, hu)
                    A out[3] = {qn[0], qn[2], qn[1]};
                    const A bo = qm2_b;
                    const bool wr = upd_col && live;
                    cleanup<DEV, A>(out, bo, P, wr, wr, clamps, flags);
                    if (FRIC) {
                        const A hd = DEV ? out[0] + A(P.sea_level) - bo : out[0];
                        if (hd > A(P.drytol)) {
                            const A n2g = A(P.manning_n) * A(P.manning_n) * A(P.g);
                            const A speed = sqrt(out[1] * out[1] + out[2] * out[2]) / hd;
                            const A D = n2g * A(pow(double(hd), -7.0 / 3.0)) * speed;
                            const A f = A(1) / (A(1) + A(tk.dt) * D);
                            out[1] *= f;
                            out[2] *= f;
                        }
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) po[k] = out[k];
                    po_row = R - 2;
                    po_wr = wr;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    ap_prev[k] = ap1[k];
                    F_prev[k] = F1[k];
                }
            }
#pragma unroll
            for (int p = 0; p < 3; ++p) dprev[p] = dcur[p];
            wprev = wy;
            wprev_quiet = yq;
        }
        // Q* of row R - 1 in y order (h or eta', hv, hu) is what `prev` was
        // made from: after the cleanup a dry cell carries no momentum, so
        // prev.m and prev.t are the stored hv and hu also there
        qm2[0] = DEV ? prev.eta : prev.h;
        qm2[1] = prev.m;
        qm2[2] = prev.t;
        qm2_b = prev.b;
        prev = cur;
        prev_full = cur_full;
    }
    if (po_wr) {
        const int64_t o = tk.off + (int64_t)po_row * tk.pitch + c;
        qout[o] = po[0];
        qout[o + tk.ps] = po[1];
        qout[o + 2 * tk.ps] = po[2];
    }
    // no ring load may still be writing LDS when the wave moves on
    if constexpr (RING > 0) wait_vmem_at_most<0>();
    MarchOut o;
    o.smx = double(smx);
    o.smy = double(smy);
    o.clamps = clamps;
    o.flags = flags;
    o.work = work;
    return o;
}

}  // namespace swe
