// swe_math.hpp -- per-edge arithmetic of the shallow water step on gfx950.
//
// Augmented Riemann solve with wet/dry handling, fluctuations and the limited
// second-order correction of the wave-propagation method (Qin, LeVeque &
// Motley, Sec. 2: wave-propagation form, second-order form with theta and the
// MC limiter; the Riemann solver is the augmented solver the paper cites,
// read as: Einfeldt speed bounds, a wall test against dry banks, a
// positivity-bounded stationary bed jump and a corrector wave).
//
// All functions are templated on the real type so the FP64 path and the
// FP32 surface-deviation path share one instruction sequence per type; the
// library is built with -ffp-contract=off, so a cell's result does not depend
// on which lane, tile or launch computed it.  In FP64 every quotient and root
// is a correctly rounded IEEE division or square root, and products and sums
// are grouped as the method's formulas are written: in deep water the momentum is
// a small signal over a large depth, and two groupings of the same formula
// already differ there by about 1e-11 of the momentum after 100 steps, so
// the FP64 path keeps one fixed, plain grouping.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace swe {

enum : int { kEdgeWet = 0, kEdgeWallR = 1, kEdgeWallL = 2, kEdgeDry = 3 };

struct DevParams {
    double g, drytol, h_corr, manning_n, sea_level, h_fp64;
    int order;
};

// Quotients and roots.  In FP64 they are the correctly rounded IEEE
// operations (the FP64 path reproduces the reference arithmetic).  In FP32
// (the surface-deviation path, whose bar is an error in metres against FP64)
// they are the hardware reciprocal and square root (about 1 ulp).
__device__ __forceinline__ double qdiv(double a, double b) { return a / b; }
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
__device__ __forceinline__ double qsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float qsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }

// One side of an edge, seen along the edge normal: depth, normal and
// transverse momentum, bed, and the derived velocities and celerity.
template <typename T>
struct Side {
    T h, m, t, b;
    T u, v;   // m / h, t / h; 0 on a dry side
    T sq, c;  // sqrt(h), sqrt(g h); 0 on a dry side
    T eta;    // surface deviation h + b - sea level (deviation path only)
    bool dry;
};

// The fields a quiet-edge test and the wave speeds need: depth, momenta, bed,
// dry flag and celerity.  side_finish adds the velocities and sqrt(h) that
// the Riemann solve needs; make_side is both.
template <typename T>
__device__ __forceinline__ Side<T> side_base(T h, T m, T t, T b, const DevParams& P) {
    Side<T> s;
    s.h = h;
    s.b = b;
    s.eta = T(0);
    s.u = T(0);
    s.v = T(0);
    s.sq = T(0);
    s.dry = h <= T(P.drytol);
    s.m = s.dry ? T(0) : m;
    s.t = s.dry ? T(0) : t;
    s.c = s.dry ? T(0) : qsqrt(T(P.g) * h);
    return s;
}

template <typename T>
__device__ __forceinline__ void side_finish(Side<T>& s) {
    if (!s.dry) {
        s.u = qdiv(s.m, s.h);
        s.v = qdiv(s.t, s.h);
        s.sq = qsqrt(s.h);
    }
}

template <typename T>
__device__ __forceinline__ Side<T> make_side(T h, T m, T t, T b, const DevParams& P) {
    Side<T> s = side_base(h, m, t, b, P);
    side_finish(s);
    return s;
}

template <typename T>
struct Waves {
    T z[3][3];  // z[p][k]: f-wave p, component (mass, normal mom., transverse mom.)
    T s[3];
    int kind;
    bool shallow;  // a cell of the edge is at or below h_corr deep
};

// Augmented Riemann solve at the edge between L and R.  DEV = true takes the
// surface jump from the stored deviations (eta'_R - eta'_L) instead of
// (h_R - h_L) + (b_R - b_L), so that in FP32 a 1 m wave over 4000 m does not
// cancel.
template <typename T, bool DEV = false>
__device__ __forceinline__ void riemann(const Side<T>& L, const Side<T>& R, const DevParams& P,
                                        Waves<T>& w) {
    w.shallow = L.h <= T(P.h_corr) || R.h <= T(P.h_corr);
    w.kind = kEdgeWet;
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        w.s[p] = T(0);
        w.z[p][0] = w.z[p][1] = w.z[p][2] = T(0);
    }
    if (L.dry && R.dry) {
        w.kind = kEdgeDry;
        return;
    }
    T hL = L.h, mL = L.m, tL = L.t, bL = L.b, uL = L.u, vL = L.v, sqL = L.sq, cL = L.c;
    T hR = R.h, mR = R.m, tR = R.t, bR = R.b, uR = R.u, vR = R.v, sqR = R.sq, cR = R.c;
    T eL = L.eta, eR = R.eta;
    bool dryL = L.dry, dryR = R.dry;
    const T g = T(P.g);

    // wall test: can the water of the wet side reach over the dry side's bed?
    if (dryR) {
        T a = cL + T(0.5) * uL;
        a = a < T(0) ? T(0) : a;
        T hstar = qdiv(a * a, g);
        hstar = hstar < hL ? hL : hstar;
        if (hstar + bL < bR) {
            w.kind = kEdgeWallR;
            hR = hL; mR = -mL; tR = tL; bR = bL; uR = -uL; vR = vL; sqR = sqL; cR = cL;
            eR = eL;
            dryR = false;
        }
    } else if (dryL) {
        T a = cR - T(0.5) * uR;
        a = a < T(0) ? T(0) : a;
        T hstar = qdiv(a * a, g);
        hstar = hstar < hR ? hR : hstar;
        if (hstar + bR < bL) {
            w.kind = kEdgeWallL;
            hL = hR; mL = -mR; tL = tR; bL = bR; uL = -uR; vL = vR; sqL = sqR; cL = cR;
            eL = eR;
            dryL = false;
        }
    }

    // speeds
    T s1, s3;
    if (dryR) {
        s1 = uL - cL;
        s3 = uL + T(2) * cL;
    } else if (dryL) {
        s1 = uR - T(2) * cR;
        s3 = uR + cR;
    } else {
        T uhat = qdiv(sqL * uL + sqR * uR, sqL + sqR);
        T chat = qsqrt(g * (T(0.5) * (hL + hR)));
        T a = uL - cL, c = uhat - chat;
        s1 = a < c ? a : c;
        a = uR + cR;
        c = uhat + chat;
        s3 = a > c ? a : c;
    }
    const T s2 = T(0.5) * (s1 + s3);

    // Stationary bed jump -(b_R - b_L), bounded so that both middle depths of
    // the HLL state stay >= 0.  The middle depths of the unclamped
    // decomposition are h_L + beta1 and h_R - beta3; when no bound is hit
    // those quotients are the decomposition itself.  The HLL middle depth is
    // needed only to place a bound.
    const T dm = mR - mL;
    const T db = bR - bL;
    const T deta = DEV ? (eR - eL) : (hR - hL) + db;
    T beta1, beta3;
    bool clamped = false;
    int bound = 0;  // 1: the left middle depth is at its bound, 3: the right one
    T hm = T(0);
    T delta = -db;
    if (s1 < T(0) && s3 > T(0)) {
        beta1 = qdiv(s3 * deta - dm, s3 - s1);
        beta3 = qdiv(dm - s1 * deta, s3 - s1);
        if (hL + beta1 < T(0)) {
            hm = qdiv(s3 * hR - s1 * hL - dm, s3 - s1);
            hm = hm < T(0) ? T(0) : hm;
            delta = qdiv(hm * (s3 - s1), s3);
            clamped = true;
            bound = 1;
        } else if (hR - beta3 < T(0)) {
            hm = qdiv(s3 * hR - s1 * hL - dm, s3 - s1);
            hm = hm < T(0) ? T(0) : hm;
            delta = qdiv(hm * (s3 - s1), s1);
            clamped = true;
            bound = 3;
        }
    } else {
        if (s1 >= T(0)) {
            if (delta < -hL) { delta = -hL; clamped = true; }
        } else {
            if (delta > hR) { delta = hR; clamped = true; }
        }
        if (!clamped) {
            beta1 = qdiv(s3 * deta - dm, s3 - s1);
            beta3 = qdiv(dm - s1 * deta, s3 - s1);
        }
    }
    if (clamped) {
        // at a bound (with a positive HLL middle depth) that side's middle
        // depth is zero in exact arithmetic: its coefficient takes that exact
        // value (computed, it can land a rounding error past it and drain an
        // empty cell below zero) and the other follows from the mass flux
        // s1 beta1 + s3 beta3 = dm
        if (bound == 1 && hm > T(0)) {
            beta1 = -hL;
            beta3 = qdiv(dm + s1 * hL, s3);
        } else if (bound == 3 && hm > T(0)) {
            beta3 = hR;
            beta1 = qdiv(dm - s3 * hR, s1);
        } else {
            const T dh = (hR - hL) - delta;
            beta1 = qdiv(s3 * dh - dm, s3 - s1);
            beta3 = qdiv(dm - s1 * dh, s3 - s1);
        }
    }

    const T hbar = T(0.5) * (hL + hR);
    const T dphi = (mR * uR - mL * uL) + g * hbar * deta;
    const T dtr = mR * vR - mL * vL;

    const T beta2 = dphi - (s1 * s1 * beta1 + s3 * s3 * beta3);

    const T f1 = s1 * beta1, f3 = s3 * beta3;
    w.z[0][0] = f1;
    w.z[0][1] = s1 * s1 * beta1;
    w.z[0][2] = f1 * vL;
    w.z[2][0] = f3;
    w.z[2][1] = s3 * s3 * beta3;
    w.z[2][2] = f3 * vR;
    w.z[1][0] = T(0);
    w.z[1][1] = beta2;
    w.z[1][2] = dtr - (f1 * vL + f3 * vR);
    w.s[0] = s1;
    w.s[1] = s2;
    w.s[2] = s3;

    // a wall reflects: waves running into the dry bank are removed (a branch,
    // so that a wave with no wall edge skips the selects)
    const bool wallR = w.kind == kEdgeWallR, wallL = w.kind == kEdgeWallL;
    if (wallR || wallL) {
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            const bool drop = (wallR && w.s[p] > T(0)) || (wallL && w.s[p] < T(0));
            w.s[p] = drop ? T(0) : w.s[p];
            w.z[p][0] = drop ? T(0) : w.z[p][0];
            w.z[p][1] = drop ? T(0) : w.z[p][1];
            w.z[p][2] = drop ? T(0) : w.z[p][2];
        }
    }
}

// A-dQ (left-going) and A+dQ (right-going); a zero-speed wave is shared half
// and half; at a wall the side facing the dry bank receives nothing.
//
// Branch-free: each wave enters each sum with a weight 1, 1/2 or 0 chosen
// from its speed (and the wall kind).  For finite waves this is exactly the
// sum of the waves on their sides: 1 * z and 0.5 * z are the values added
// there, and 0 * z is a zero, which leaves a sum as it is (the sums start at
// +0 and never become -0 by adding).
template <typename T>
__device__ __forceinline__ void fluctuations(const Waves<T>& w, T am[3], T ap[3]) {
    const bool zap = w.kind == kEdgeWallR, zam = w.kind == kEdgeWallL;
    T wm[3], wp[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const T s = w.s[p];
        const T m = s < T(0) ? T(1) : (s > T(0) ? T(0) : T(0.5));
        const T q = s > T(0) ? T(1) : (s < T(0) ? T(0) : T(0.5));
        wm[p] = zam ? T(0) : m;
        wp[p] = zap ? T(0) : q;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        am[k] = T(0);
        ap[k] = T(0);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            am[k] += wm[p] * w.z[p][k];
            ap[k] += wp[p] * w.z[p][k];
        }
    }
}

template <typename T>
__device__ __forceinline__ T dot3(const T* a, const T* b) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

template <typename T>
__device__ __forceinline__ T mc_limiter(T theta) {
    T a = T(0.5) * (T(1) + theta);
    T c = T(2) * theta;
    T m = a < T(2) ? a : T(2);
    m = m < c ? m : c;
    return m > T(0) ? m : T(0);
}

// Limited correction at an edge from its waves and the dot products of its
// f-waves with those of the left (dl) and right (dr) neighbour edges.
template <typename T>
__device__ __forceinline__ void correction(const Waves<T>& w, const T dl[3], const T dr[3], T lam,
                                           T F[3]) {
    F[0] = F[1] = F[2] = T(0);
    if (w.shallow) return;
    // Branch-free over the waves: a wave of zero speed or zero size enters
    // with coefficient 0 (its quotient is computed and discarded), so for
    // finite waves it adds a zero, which leaves the sums as they are (they
    // start at +0 and never become -0 by adding).
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const T s = w.s[p];
        const T zz = dot3(w.z[p], w.z[p]);
        const bool use = s != T(0) && zz != T(0);
        const T theta = qdiv(s > T(0) ? dl[p] : dr[p], zz);
        const T phi = mc_limiter(theta);
        const T sg = s > T(0) ? T(1) : T(-1);
        const T as = s > T(0) ? s : -s;
        const T coef = T(0.5) * sg * (T(1) - lam * as) * phi;
        const T cu = use ? coef : T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) F[k] += cu * w.z[p][k];
    }
}

// Mass component of A-dQ, computed exactly as fluctuations() computes am[0].
template <typename T>
__device__ __forceinline__ T minus_mass(const Waves<T>& w) {
    const bool zam = w.kind == kEdgeWallL;
    T am = T(0);
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const T s = w.s[p];
        const T m = s < T(0) ? T(1) : (s > T(0) ? T(0) : T(0.5));
        am += (zam ? T(0) : m) * w.z[p][0];
    }
    return am;
}

// Share of its donor's water that one edge's correction may carry out (per
// sweep a cell has two edges, so at most half of its depth after the
// first-order part of its update; the FP64 share sits 5e-13 below a half so
// that the rounding of the update cannot take a drained cell below zero, the
// FP32 share 1e-5 below).
template <typename T>
struct DrainShare;
template <>
struct DrainShare<double> {
    static constexpr double v = 0.4999999999995;
};
template <>
struct DrainShare<float> {
    static constexpr float v = 0.49999f;
};

// Positivity limit of a correction F (Sec. 2: depths stay non-negative): h1
// is the depth of the donor cell, the one F's mass flux leaves, after the
// first-order part of its update; coef * (len * |F[0]|) is what F takes out
// of it.  If that exceeds the donor's share of h1 (0 for h1 <= 0), all of F
// is scaled down to it.
template <typename T>
__device__ __forceinline__ void drain_limit(T F[3], T h1, T coef, T len) {
    const T out = coef * (len * fabs(F[0]));
    const T cap = h1 > T(0) ? T(DrainShare<T>::v) * h1 : T(0);
    if (out > cap) {
        const T r = qdiv(cap, out);
        F[0] = r * F[0];
        F[1] = r * F[1];
        F[2] = r * F[2];
    }
}

// A cell as seen by the transverse solver: depth, bed, velocities along the
// edge normal (un) and along the split direction (ut; 0 when dry), sqrt(h).
template <typename T>
struct TCell {
    T h, b, un, ut, sq;
};

// Roe averages of a pair of cells along the split direction.
template <typename T>
struct TPair {
    T un, ut, c;
    bool all_dry;
};

template <typename T>
__device__ __forceinline__ TPair<T> tpair(const TCell<T>& l, const TCell<T>& r,
                                          const DevParams& P) {
    TPair<T> q;
    const bool dl = l.h <= T(P.drytol), dr = r.h <= T(P.drytol);
    q.all_dry = dl && dr;
    q.un = qdiv(l.sq * l.un + r.sq * r.un, l.sq + r.sq);
    q.ut = qdiv(l.sq * l.ut + r.sq * r.ut, l.sq + r.sq);
    q.c = qsqrt(T(P.g) * (T(0.5) * (l.h + r.h)));
    return q;
}

// Transverse split of the amount a = (mass, normal, transverse) entering cell
// C, with the Roe eigenstructure along the split direction of the pair (l, r):
// eigenvalues ut - c, ut, ut + c; eigenvectors (1, un, ut - c), (0, 1, 0),
// (1, un, ut + c).  sgn > 0 keeps the positive-speed part (moving toward r),
// sgn < 0 the negative-speed part.  c_is_left tells which of the pair is C.
// The part is 0 if the pair is dry, or if the neighbour is dry with its bed at
// or above C's surface.
template <typename T>
__device__ __forceinline__ void transverse(const TCell<T>& l, const TCell<T>& r,
                                           const TPair<T>& q, bool c_is_left, const T a[3],
                                           int sgn, const DevParams& P, T out[3]) {
    out[0] = out[1] = out[2] = T(0);
    const TCell<T>& C = c_is_left ? l : r;
    const TCell<T>& N = c_is_left ? r : l;
    if (q.all_dry) return;
    if (N.h <= T(P.drytol) && N.b >= C.h + C.b) return;
    const T lam[3] = {q.ut - q.c, q.ut, q.ut + q.c};
    T gam[3];
    gam[0] = qdiv((q.ut + q.c) * a[0] - a[2], T(2) * q.c);
    gam[1] = a[1] - q.un * a[0];
    gam[2] = qdiv(a[2] - (q.ut - q.c) * a[0], T(2) * q.c);
    const T rv[3][3] = {{T(1), q.un, q.ut - q.c}, {T(0), T(1), T(0)}, {T(1), q.un, q.ut + q.c}};
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        const T l2 = sgn > 0 ? (lam[p] > T(0) ? lam[p] : T(0)) : (lam[p] < T(0) ? lam[p] : T(0));
#pragma unroll
        for (int k = 0; k < 3; ++k) out[k] += l2 * gam[p] * rv[p][k];
    }
}

template <typename T>
__device__ __forceinline__ T max_speed(const Waves<T>& w) {
    T a = fabs(w.s[0]), b = fabs(w.s[1]), c = fabs(w.s[2]);
    T m = a > b ? a : b;
    return m > c ? m : c;
}

}  // namespace swe
