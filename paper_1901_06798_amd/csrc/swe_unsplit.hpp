// swe_unsplit.hpp -- the unsplit step with transverse waves (FP64), marched
// down the rows of a strip like the split step.
//
// Every edge is solved from Q^n (Sec. 2, wave-propagation form and its
// second-order corrections).  The amount entering a cell through an x-edge
// (A+dQ - F~ through its left edge, A-dQ + F~ through its right edge) is split
// by a Roe solver in y into an up-going and a down-going part, which move part
// of the cell's change into its upper/lower neighbour through the y-correction
// fluxes G~; the amounts entering through y-edges are split in x into F~.
//
// Pipeline per lane (column c), with R the row loaded in this iteration:
//   x-edges of row R (across lanes)           -> A+-dQ, F~, entering amounts
//   y-edge between rows R-1 and R              -> waves, B+-dQ
//   transverse parts for G~ at that y-edge     (pair (R-1, R), both directions)
//   limited G~ of the y-edge one row behind    -> G~ total, entering amounts
//   transverse parts for F~ of row R-2         (pair (c-1, c) on row R-2)
//   update of row R-2.
// Every correction is accumulated in the same order as in the plain
// all-x-edges-then-all-y-edges formulation, so the result does not depend on
// the strip or chunk that computed it.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "swe.h"
#include "swe_common.hpp"
#include "swe_march.hpp"
#include "swe_math.hpp"

namespace swe {

template <int SEG>
__device__ __forceinline__ TCell<double> tcell_up(const TCell<double>& x) {
    TCell<double> r;
    r.h = lane_up<SEG>(x.h);
    r.b = lane_up<SEG>(x.b);
    r.un = lane_up<SEG>(x.un);
    r.ut = lane_up<SEG>(x.ut);
    r.sq = lane_up<SEG>(x.sq);
    return r;
}

// The cell as seen by the transverse solvers: (un, ut) = (u, v) for the split
// in y of x-edge amounts, (v, u) for the split in x of y-edge amounts.
__device__ __forceinline__ TCell<double> tcell(double h, double hu, double hv, double b,
                                               bool swap, const DevParams& P) {
    TCell<double> t;
    t.h = h;
    t.b = b;
    const bool dry = h <= P.drytol;
    const double u = dry ? 0.0 : hu / h;
    const double v = dry ? 0.0 : hv / h;
    t.un = swap ? v : u;
    t.ut = swap ? u : v;
    t.sq = sqrt(h);
    return t;
}

__device__ __forceinline__ bool zero3(const double a[3]) {
    return a[0] == 0.0 && a[1] == 0.0 && a[2] == 0.0;
}

// A zero amount splits into zero transverse parts (its coefficients are 0, or
// the pair is dry and the part is 0 by rule), so when nothing enters the
// cells of a wave the Roe averages and the splits are skipped; the parts are
// then +0 where the split could give -0, which changes no value.
template <int SEG, bool FRIC>
__device__ __forceinline__ MarchOut march_unsplit(const Task& tk, const DevParams& P,
                                                  int lane_in_seg, int steps,
                                                  int transverse_order) {
    using S = double;
    const S* __restrict__ qin = static_cast<const S*>(tk.qin);
    S* __restrict__ qout = static_cast<S*>(tk.qout);
    const S* __restrict__ bpl = static_cast<const S*>(tk.b);
    const int lane = lane_in_seg;
    const int c = tk.c0 + lane;
    const int cc = c < tk.mx + 3 ? c : tk.mx + 3;
    const bool upd_col = tk.active && lane >= 2 && lane <= SEG - 3 && c <= tk.mx + 1;
    const bool xedge_own = tk.active && lane >= 2 && lane <= SEG - 2 && c >= 2 && c <= tk.mx + 2;
    const int U0 = tk.U0, U1 = tk.U1;
    const S lamx = tk.dt / tk.dx, lamy = tk.dt / tk.dy;
    const bool second = P.order >= 2;
    const bool tr2 = transverse_order >= 2;
    const int tlast = U1 - U0 + 4;

    S smx = 0.0, smy = 0.0;
    uint32_t clamps = 0, flags = 0;
    uint32_t work = 0;

    // state carried between rows (suffix 1: row R - 1, suffix 2: row R - 2)
    TCell<S> tv1{}, th1{}, th2{};    // vertical-split view of row R-1; horizontal view of R-1, R-2
    Side<S> sy1;                     // y-normal side of row R-1
    S q1[3] = {0, 0, 0}, q2[3] = {0, 0, 0};
    S xap1[3] = {0, 0, 0}, xap2[3] = {0, 0, 0};
    S xamr1[3] = {0, 0, 0}, xamr2[3] = {0, 0, 0};
    S xF1[3] = {0, 0, 0}, xF2[3] = {0, 0, 0};
    S aP1[3] = {0, 0, 0}, aM1[3] = {0, 0, 0};
    S T1[4][3] = {};                 // transverse parts for G~ of the y-edge one row behind
    Waves<S> wy1;
    S dprev[3] = {0, 0, 0};
    S yap2[3] = {0, 0, 0};           // B+dQ of y-edge R-2 (h, hu, hv)
    S bP2[3] = {0, 0, 0};            // amount entering (c, R-2) through y-edge R-2
    S Gt2[3] = {0, 0, 0};            // G~ total of y-edge R-2

    // finished row held for one iteration (its stores go out before the next
    // row's loads) and the next row's values, loaded one iteration ahead
    S po[3] = {0, 0, 0};
    int po_row = 0;
    bool po_wr = false;
    S nh, nhu, nhv, nbb;
    bool nfx, nfy;
    {
        const Src s0 = map_cell(U0 - 2, cc, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
        nh = qin[s0.idx];
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

        // ---- row R of Q^n (loaded one iteration ago); flush the finished
        // row, then issue the loads of the next one (every row index of the
        // march stays inside the patch, one past the last iteration too)
        const S h = nh;
        const S hu = nfx ? -nhu : nhu;
        const S hv = nfy ? -nhv : nhv;
        const S bb = nbb;
        if (po_wr) {
            const int64_t o = tk.off + (int64_t)po_row * tk.pitch + c;
            qout[o] = po[0];
            qout[o + tk.ps] = po[1];
            qout[o + 2 * tk.ps] = po[2];
        }
        po_wr = false;
        {
            const int Rn = U0 - 2 + (t + 1 <= tlast ? t + 1 : tlast);
            const Src sn = map_cell(Rn, cc, tk.mx, tk.my, tk.pitch, tk.off, tk.bc);
            nh = qin[sn.idx];
            nhu = qin[sn.idx + tk.ps];
            nhv = qin[sn.idx + 2 * tk.ps];
            nbb = bpl[sn.idx];
            nfx = sn.sx < 0.0;
            nfy = sn.sy < 0.0;
        }
        const TCell<S> tv0 = tcell(h, hu, hv, bb, false, P);
        const TCell<S> th0 = tcell(h, hu, hv, bb, true, P);

        // ---- x-edges of row R
        const Side<S> me = make_side<S>(h, hu, hv, bb, P);
        Side<S> lf = side_up<S, false, SEG>(me, P);
        Waves<S> w;
        // lane 0's edge feeds no result; see quiet_edge
        if (SWE_QUIET && __all(lane == 0 || quiet_edge<false, S>(lf, me))) {
            quiet_waves(lf, me, P, w);
        } else {
            ++work;
            lf.u = lane_up<SEG>(me.u);
            lf.v = lane_up<SEG>(me.v);
            lf.sq = lane_up<SEG>(me.sq);
            riemann<S, false>(lf, me, P, w);
        }
        S xam0[3], xap0[3];
        fluctuations(w, xam0, xap0);
        S xF0[3] = {0.0, 0.0, 0.0};
        if (second) {
            S dr[3], dl[3];
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const S zr0 = lane_down<SEG>(w.z[p][0]);
                const S zr1 = lane_down<SEG>(w.z[p][1]);
                const S zr2 = lane_down<SEG>(w.z[p][2]);
                dr[p] = w.z[p][0] * zr0 + w.z[p][1] * zr1 + w.z[p][2] * zr2;
            }
#pragma unroll
            for (int p = 0; p < 3; ++p) dl[p] = lane_up<SEG>(dr[p]);
            correction(w, dl, dr, lamx, xF0);
        }
        if (interior_row && xedge_own) {
            const S s = max_speed(w);
            smx = s > smx ? s : smx;
        }
        // amounts entering cell (c, R): through its left edge (this lane) and
        // its right edge (the next lane)
        S aP0[3], aM0[3], xamr0[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const S corr = tr2 ? xF0[k] : S(0);
            aP0[k] = xap0[k] - corr;
            aM0[k] = lane_down<SEG>(xam0[k] + corr);
            xamr0[k] = lane_down<SEG>(xam0[k]);
        }

        // ---- y-edge between rows R - 1 and R
        const Side<S> sy0 = make_side<S>(h, hv, hu, bb, P);
        if (t >= 1) {
            Waves<S> wy;
            // lane 0's y-edge feeds only lane 1, whose cell is not updated
            if (SWE_QUIET && __all(lane == 0 || quiet_edge<false, S>(sy1, sy0)))
                quiet_waves(sy1, sy0, P, wy);
            else {
                ++work;
                riemann<S, false>(sy1, sy0, P, wy);
            }
            const int E = R;
            if (live && E >= U0 && E <= U1 + 1 && upd_col) {
                const S s = max_speed(wy);
                smy = s > smy ? s : smy;
            }
            // transverse parts of the x-edge amounts of rows R - 1 (up) and R
            // (down), all through the pair (R - 1, R) of this column
            S T0[4][3];
            if (__all(lane == 0 || (zero3(aP1) && zero3(aM1) && zero3(aP0) && zero3(aM0)))) {
                // nothing enters: every transverse part is a zero
#pragma unroll
                for (int i = 0; i < 4; ++i) T0[i][0] = T0[i][1] = T0[i][2] = S(0);
            } else {
                const TPair<S> pv = tpair(tv1, tv0, P);
                transverse(tv1, tv0, pv, true, aP1, +1, P, T0[0]);
                transverse(tv1, tv0, pv, true, aM1, +1, P, T0[1]);
                transverse(tv1, tv0, pv, false, aP0, -1, P, T0[2]);
                transverse(tv1, tv0, pv, false, aM0, -1, P, T0[3]);
            }
            S dcur[3] = {0.0, 0.0, 0.0};
            if (second && t >= 2) {
#pragma unroll
                for (int p = 0; p < 3; ++p) dcur[p] = dot3(wy1.z[p], wy.z[p]);
            }
            if (t >= 3) {
                // y-edge R - 1: fluctuations, limited correction, G~ total
                S am[3], ap[3], G[3] = {0.0, 0.0, 0.0};
                fluctuations(wy1, am, ap);
                if (second) correction(wy1, dprev, dcur, lamy, G);
                // (h, hv, hu) -> (h, hu, hv)
                const S yam1[3] = {am[0], am[2], am[1]};
                const S yap1[3] = {ap[0], ap[2], ap[1]};
                const S yG1[3] = {G[0], G[2], G[1]};
                const S sx = 0.5 * lamx;
                S Gt1[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    S g = yG1[k];
                    g -= sx * T1[0][k];
                    g -= sx * T1[1][k];
                    g -= sx * T1[2][k];
                    g -= sx * T1[3][k];
                    Gt1[k] = g;
                }
                // amounts entering (c, R-1) from below and (c, R-2) from above
                S bP1[3], bM1[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const S corr = tr2 ? yG1[k] : S(0);
                    bP1[k] = yap1[k] - corr;
                    bM1[k] = yam1[k] + corr;
                }
                if (t >= 4) {
                    // F~ of the x-edge between columns c - 1 and c on row R - 2
                    const TCell<S> thl = tcell_up<SEG>(th2);
                    S bPl[3], bMl[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        bPl[k] = lane_up<SEG>(bP2[k]);
                        bMl[k] = lane_up<SEG>(bM1[k]);
                    }
                    // (h, hu, hv) -> (h, normal = hv, transverse = hu)
                    const S a1[3] = {bPl[0], bPl[2], bPl[1]};
                    const S a2[3] = {bMl[0], bMl[2], bMl[1]};
                    const S a3[3] = {bP2[0], bP2[2], bP2[1]};
                    const S a4[3] = {bM1[0], bM1[2], bM1[1]};
                    S r1[3], r2[3], l1[3], l2[3];
                    if (__all(lane == 0 ||
                              (zero3(a1) && zero3(a2) && zero3(a3) && zero3(a4)))) {
#pragma unroll
                        for (int k = 0; k < 3; ++k) r1[k] = r2[k] = l1[k] = l2[k] = S(0);
                    } else {
                        const TPair<S> ph = tpair(thl, th2, P);
                        transverse(thl, th2, ph, true, a1, +1, P, r1);
                        transverse(thl, th2, ph, true, a2, +1, P, r2);
                        transverse(thl, th2, ph, false, a3, -1, P, l1);
                        transverse(thl, th2, ph, false, a4, -1, P, l2);
                    }
                    const S sy = 0.5 * lamy;
                    // back to (h, hu, hv): local (h, hv, hu)
                    const int perm[3] = {0, 2, 1};
                    S Ft[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        S f = xF2[k];
                        f -= sy * r1[perm[k]];
                        f -= sy * r2[perm[k]];
                        f -= sy * l1[perm[k]];
                        f -= sy * l2[perm[k]];
                        Ft[k] = f;
                    }
                    // ---- update row R - 2
                    S out[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        const S Ftr = lane_down<SEG>(Ft[k]);
                        out[k] = q2[k] - lamx * (xap2[k] + xamr2[k] + Ftr - Ft[k]) -
                                 lamy * (yap2[k] + yam1[k] + Gt1[k] - Gt2[k]);
                    }
                    const bool wr = upd_col && live;
                    cleanup<false, S>(out, bb, P, wr, wr, clamps, flags);
                    if (FRIC && out[0] > P.drytol) {
                        const S n2g = P.manning_n * P.manning_n * P.g;
                        const S speed = sqrt(out[1] * out[1] + out[2] * out[2]) / out[0];
                        const S D = n2g * pow(out[0], -7.0 / 3.0) * speed;
                        const S f = 1.0 / (1.0 + tk.dt * D);
                        out[1] *= f;
                        out[2] *= f;
                    }
#pragma unroll
                    for (int k = 0; k < 3; ++k) po[k] = out[k];
                    po_row = R - 2;
                    po_wr = wr;
                }
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    yap2[k] = yap1[k];
                    bP2[k] = bP1[k];
                    Gt2[k] = Gt1[k];
                }
            }
#pragma unroll
            for (int p = 0; p < 3; ++p) dprev[p] = dcur[p];
            wy1 = wy;
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int k = 0; k < 3; ++k) T1[i][k] = T0[i][k];
        }
        // shift the row state
        th2 = th1;
        th1 = th0;
        tv1 = tv0;
        sy1 = sy0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            q2[k] = q1[k];
            xap2[k] = xap1[k];
            xamr2[k] = xamr1[k];
            xF2[k] = xF1[k];
            aP1[k] = aP0[k];
            aM1[k] = aM0[k];
            xap1[k] = xap0[k];
            xamr1[k] = xamr0[k];
            xF1[k] = xF0[k];
        }
        q1[0] = h;
        q1[1] = hu;
        q1[2] = hv;
    }
    if (po_wr) {
        const int64_t o = tk.off + (int64_t)po_row * tk.pitch + c;
        qout[o] = po[0];
        qout[o + tk.ps] = po[1];
        qout[o + 2 * tk.ps] = po[2];
    }
    MarchOut o;
    o.smx = smx;
    o.smy = smy;
    o.clamps = clamps;
    o.flags = flags;
    o.work = work;
    return o;
}

}  // namespace swe
