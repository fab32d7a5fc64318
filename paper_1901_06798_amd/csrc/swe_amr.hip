// swe_amr.hip -- coupling of AMR levels on the device (gfx950; FP64 planes,
// or FP32 surface-deviation planes combined in FP64).
//
// Qin, LeVeque & Motley, Sec. 3: a finer level's ghost cells come from an
// adjacent patch of the same level or, where none exists, from the level
// below, interpolated in space and time; after the finer level has taken its
// r substeps, the cells of the level below that lie under it are replaced by
// averages of the fine cells (the updating process; refluxing is left out, as
// in the paper's GPU code).  Both strategies must keep a sea at rest at rest,
// so they work on the surface elevation h + b and recover the depth from the
// bed of the cell written.  A host plan lists every ghost cell and every
// covered coarse cell once (swe_amr_fill_op, swe_amr_avg_op); one thread
// handles one entry, so writes never collide, and reads touch only interior
// cells, which no entry writes.  The cells of patches made by regridding are
// found on the device from the patch rectangles alone, one thread per cell.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstdlib>
#include <string>
#include <vector>

#include "swe.h"

namespace swe {

struct FillArgs {
    const swe_amr_fill_op* ops;
    int64_t nops;
    void* qf;
    int64_t psf;
    const void* qcopy;  // planes SWE_AMR_COPY entries read (qf for ghost fills)
    int64_t pscopy;
    const void* bf;
    const void* qco;
    const void* qcn;
    int64_t psc;
    const void* bc;
    double alpha, drytol, sea;
};

// Depth of a stored cell: h itself (FP64 planes), or eta' + sea level - b
// formed in FP64 (FP32 surface-deviation planes).
template <typename S>
__device__ __forceinline__ double depth(const S* q, const S* b, int64_t k, double sea) {
    if (sizeof(S) == sizeof(double)) return double(q[k]);
    return (double(q[k]) + sea) - double(b[k]);
}

// First stored value of a cell of depth h, surface eta and bed b: h (FP64) or
// eta' = eta - sea level, which is b - sea level on a dry cell (FP32).
template <typename S>
__device__ __forceinline__ S first_value(double h, double eta, double b, double sea) {
    if (sizeof(S) == sizeof(double)) return S(h);
    return S(h > 0.0 ? eta - sea : b - sea);
}

// Values of coarse cell k at time alpha between its states before (qco) and
// after (qcn) its step: the surface (depth + bed) and the momenta, each
// linear in time.
template <typename S>
__device__ __forceinline__ void coarse_at(const FillArgs& a, const S* qco, const S* qcn,
                                          const S* bc, int64_t k, double ho, double hn,
                                          double w0, double w1, double v[3]) {
    const double b = double(bc[k]);
    v[0] = w0 * (ho + b) + w1 * (hn + b);
    v[1] = w0 * double(qco[k + a.psc]) + w1 * double(qcn[k + a.psc]);
    v[2] = w0 * double(qco[k + 2 * a.psc]) + w1 * double(qcn[k + 2 * a.psc]);
}

// One cell of the finer level from the level below (the rule stated for
// swe_amr_fill): linear in time between the coarse states before (qco) and
// after (qcn) their step, bilinear in space from the stencil cells st[0..3]
// of weights wx, wy when every stencil cell of non-zero weight lies in a
// coarse interior (st >= 0) and is wet in both states, else the cell under
// it (src) alone.  FP32 planes are read into FP64, combined there and
// rounded once.
template <typename S>
__device__ __forceinline__ void fill_from_coarse(const FillArgs& a, S* qf, int64_t dst,
                                                 int64_t src, const int64_t st_in[4], double wx,
                                                 double wy) {
    const S* bf = static_cast<const S*>(a.bf);
    const S* qco = static_cast<const S*>(a.qco);
    const S* qcn = static_cast<const S*>(a.qcn);
    const S* bc = static_cast<const S*>(a.bc);
    S* q = qf + dst;
    const double b_f = double(bf[dst]);
    const double w0 = 1.0 - a.alpha, w1 = a.alpha;
    // stencil cells of non-zero weight: c0 always, c1 with wx > 0, c2 with
    // wy > 0, c3 with both
    const bool two_x = wx > 0.0, two_y = wy > 0.0;
    int64_t st[4];
    double ho[4], hn[4];
    bool linear = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const bool used = (k & 1 ? two_x : true) && (k & 2 ? two_y : true);
        st[k] = st_in[k];
        ho[k] = hn[k] = 0.0;
        if (!used) continue;
        if (st[k] < 0) {
            linear = false;
            continue;
        }
        ho[k] = depth(qco, bc, st[k], a.sea);
        hn[k] = depth(qcn, bc, st[k], a.sea);
        linear = linear && ho[k] > a.drytol && hn[k] > a.drytol;
    }
    double v[3];
    if (linear) {
        double c[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const bool used = (k & 1 ? two_x : true) && (k & 2 ? two_y : true);
            if (used) coarse_at(a, qco, qcn, bc, st[k], ho[k], hn[k], w0, w1, c[k]);
        }
        const double ux = 1.0 - wx, uy = 1.0 - wy;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            double line0 = ux * c[0][m];
            if (two_x) line0 = line0 + wx * c[1][m];
            double val = uy * line0;
            if (two_y) {
                double line1 = ux * c[2][m];
                if (two_x) line1 = line1 + wx * c[3][m];
                val = val + wy * line1;
            }
            v[m] = val;
        }
    } else {
        const double h0 = depth(qco, bc, src, a.sea), h1 = depth(qcn, bc, src, a.sea);
        if (h0 <= a.drytol && h1 <= a.drytol) {
            q[0] = first_value<S>(0.0, b_f, b_f, a.sea);
            q[a.psf] = S(0);
            q[2 * a.psf] = S(0);
            return;
        }
        coarse_at(a, qco, qcn, bc, src, h0, h1, w0, w1, v);
    }
    const double d = v[0] - b_f;
    const double h = d > 0.0 ? d : 0.0;
    q[0] = first_value<S>(h, v[0], b_f, a.sea);
    if (h <= a.drytol) {
        q[a.psf] = S(0);
        q[2 * a.psf] = S(0);
    } else {
        q[a.psf] = S(v[1]);
        q[2 * a.psf] = S(v[2]);
    }
}

// Ghost cells of the finer level, as listed in the plan: a copy takes the
// same level's cell, a coarse entry fill_from_coarse.
template <typename S>
__global__ void __launch_bounds__(256) k_amr_fill(FillArgs a) {
    S* qf = static_cast<S*>(a.qf);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nops; i += stride) {
        const swe_amr_fill_op& op = a.ops[i];
        if (op.kind == SWE_AMR_COPY) {
            S* q = qf + op.dst;
            const S* src = static_cast<const S*>(a.qcopy) + op.src;
            q[0] = src[0];
            q[a.psf] = src[a.pscopy];
            q[2 * a.psf] = src[2 * a.pscopy];
            continue;
        }
        const int64_t st[4] = {op.st[0], op.st[1], op.st[2], op.st[3]};
        fill_from_coarse<S>(a, qf, op.dst, op.src, st, op.wx, op.wy);
    }
}

// First rectangle of `rects` whose interior holds global cell (I, J), or -1.
__device__ __forceinline__ int covering(const swe_amr_rect* rects, int n, int I, int J) {
    for (int k = 0; k < n; ++k) {
        const swe_amr_rect r = rects[k];
        if (I >= r.i0 && I < r.i0 + r.mx && J >= r.j0 && J < r.j0 + r.my) return k;
    }
    return -1;
}

__device__ __forceinline__ int floor_div(int a, int r) {
    return a >= 0 ? a / r : -((-a + r - 1) / r);
}

__device__ __forceinline__ int64_t rect_elem(const swe_amr_rect& r, int I, int J) {
    return r.off + (int64_t)(J - r.j0 + 2) * r.pitch + (I - r.i0 + 2);
}

struct InitArgs {
    const swe_amr_rect* nw;
    const swe_amr_rect* old;
    int nold;
    const swe_amr_rect* crs;
    int ncrs;
    int ratio;
};

// Interior cells of new patches (one block row per new patch): the first
// old patch of the level whose interior holds the cell gives a copy; else
// the level below gives fill_from_coarse with alpha = 1 and one state, the
// cell under it and the bilinear stencil of its centre X = (I + 1/2) / r -
// 1/2, Y = (J + 1/2) / r - 1/2 each looked up in the first coarse patch that
// holds it (the host plan of swe_amr_fill computes the same).
template <typename S>
__global__ void __launch_bounds__(256) k_amr_init_rects(FillArgs a, InitArgs g) {
    S* qn = static_cast<S*>(a.qf);
    const swe_amr_rect pn = g.nw[blockIdx.y];
    const int64_t ncell = (int64_t)pn.mx * pn.my;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int ii = (int)(c % pn.mx), jj = (int)(c / pn.mx);
        const int I = pn.i0 + ii, J = pn.j0 + jj;
        const int64_t dst = rect_elem(pn, I, J);
        const int ko = covering(g.old, g.nold, I, J);
        if (ko >= 0) {
            const S* src = static_cast<const S*>(a.qcopy) + rect_elem(g.old[ko], I, J);
            qn[dst] = src[0];
            qn[dst + a.psf] = src[a.pscopy];
            qn[dst + 2 * a.psf] = src[2 * a.pscopy];
            continue;
        }
        const int Ic = floor_div(I, g.ratio), Jc = floor_div(J, g.ratio);
        const int kc = covering(g.crs, g.ncrs, Ic, Jc);
        if (kc < 0) continue;  // over no coarse patch: not written
        const double r = (double)g.ratio;
        const double X = ((double)I + 0.5) / r - 0.5, Y = ((double)J + 0.5) / r - 0.5;
        const double fx = floor(X), fy = floor(Y);
        const int i0 = (int)fx, j0 = (int)fy;
        const double wx = X - fx, wy = Y - fy;
        int64_t st[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const int Is = i0 + (k & 1), Js = j0 + (k >> 1);
            const int ks = covering(g.crs, g.ncrs, Is, Js);
            st[k] = ks >= 0 ? rect_elem(g.crs[ks], Is, Js) : -1;
        }
        fill_from_coarse<S>(a, qn, dst, rect_elem(g.crs[kc], Ic, Jc), st, wx, wy);
    }
}

struct PlanArgs {
    const swe_amr_rect* fine;
    int nfine;
    const swe_amr_rect* crs;
    int ncrs;
    int ratio;
    swe_amr_fill_op* fill;
    const int64_t* fill_first;  // per fine patch: index of its first ghost entry
    swe_amr_avg_op* avg;
    const int64_t* avg_first;   // per fine patch: index of its first averaging entry
    uint32_t* err;              // bit 0: a ghost over no cell; bit 1: a patch not over level l
};

// The ghost-fill and averaging plans of a level (one block row per fine
// patch), in the order swe_amr_fill and swe_amr_average document and the
// host plans use: a patch's ghost cells row by row of its frame, then its
// coarse cells row by row.  A ghost cell over another patch of its level
// (the first in order) copies it; else it takes the cell under it and the
// bilinear stencil of its centre in the level below, each looked up in the
// first coarse patch that holds it.
__global__ void __launch_bounds__(256) k_amr_plans(PlanArgs g) {
    const int k = blockIdx.y;
    const swe_amr_rect f = g.fine[k];
    const int r = g.ratio;
    const int64_t W = f.mx + 4;
    const int64_t nghost = W * (f.my + 4) - (int64_t)f.mx * f.my;
    const int ic0 = floor_div(f.i0, r), jc0 = floor_div(f.j0, r);
    const int ncx = floor_div(f.i0 + f.mx, r) - ic0;
    const int ncy = floor_div(f.j0 + f.my, r) - jc0;
    const int64_t navg = (int64_t)ncx * ncy;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nghost + navg;
         t += (int64_t)gridDim.x * blockDim.x) {
        if (t < nghost) {
            int row, col;
            if (t < 2 * W) {
                row = (int)(t / W);
                col = (int)(t % W);
            } else if (t < 2 * W + 4 * (int64_t)f.my) {
                const int64_t u = t - 2 * W;
                row = 2 + (int)(u / 4);
                const int m = (int)(u % 4);
                col = m < 2 ? m : f.mx + m;
            } else {
                const int64_t u = t - 2 * W - 4 * (int64_t)f.my;
                row = f.my + 2 + (int)(u / W);
                col = (int)(u % W);
            }
            const int I = f.i0 + col - 2, J = f.j0 + row - 2;
            swe_amr_fill_op op;
            op.dst = f.off + (int64_t)row * f.pitch + col;
            op.st[0] = op.st[1] = op.st[2] = op.st[3] = -1;
            op.wx = 0.0;
            op.wy = 0.0;
            op.reserved = 0;
            int same = -1;
            for (int n = 0; n < g.nfine && same < 0; ++n) {
                const swe_amr_rect o = g.fine[n];
                if (n != k && I >= o.i0 && I < o.i0 + o.mx && J >= o.j0 && J < o.j0 + o.my)
                    same = n;
            }
            if (same >= 0) {
                op.kind = SWE_AMR_COPY;
                op.src = rect_elem(g.fine[same], I, J);
            } else {
                op.kind = SWE_AMR_COARSE;
                const int Ic = floor_div(I, r), Jc = floor_div(J, r);
                const int kc = covering(g.crs, g.ncrs, Ic, Jc);
                if (kc < 0) {
                    atomicOr(g.err, 1u);
                    op.src = 0;
                } else {
                    op.src = rect_elem(g.crs[kc], Ic, Jc);
                }
                const double X = ((double)I + 0.5) / (double)r - 0.5;
                const double Y = ((double)J + 0.5) / (double)r - 0.5;
                const double fx = floor(X), fy = floor(Y);
                const int i0 = (int)fx, j0 = (int)fy;
                op.wx = X - fx;
                op.wy = Y - fy;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int Is = i0 + (m & 1), Js = j0 + (m >> 1);
                    const int ks = covering(g.crs, g.ncrs, Is, Js);
                    op.st[m] = ks >= 0 ? rect_elem(g.crs[ks], Is, Js) : -1;
                }
            }
            g.fill[g.fill_first[k] + t] = op;
        } else {
            const int64_t a = t - nghost;
            const int Ic = ic0 + (int)(a % ncx), Jc = jc0 + (int)(a / ncx);
            swe_amr_avg_op op;
            const int kc = covering(g.crs, g.ncrs, Ic, Jc);
            if (kc < 0) {
                atomicOr(g.err, 2u);
                op.dst = 0;
            } else {
                op.dst = rect_elem(g.crs[kc], Ic, Jc);
            }
            op.src = rect_elem(f, Ic * r, Jc * r);
            op.pitch = f.pitch;
            op.reserved = 0;
            g.avg[g.avg_first[k] + a] = op;
        }
    }
}

struct AvgArgs {
    const swe_amr_avg_op* ops;
    int64_t nops;
    int r;
    const void* qf;
    int64_t psf;
    const void* bf;
    void* qc;
    int64_t psc;
    const void* bc;
    double drytol, sea;
};

// Coarse cells under the finer level: the surface averaged over the wet fine
// cells above, the momenta over all r x r of them; rows, then columns, in
// increasing order (FP32 planes in FP64, rounded once).
template <typename S>
__global__ void __launch_bounds__(256) k_amr_average(AvgArgs a) {
    const S* qf = static_cast<const S*>(a.qf);
    const S* bf = static_cast<const S*>(a.bf);
    S* qc = static_cast<S*>(a.qc);
    const S* bc = static_cast<const S*>(a.bc);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nops; i += stride) {
        const swe_amr_avg_op op = a.ops[i];
        double seta = 0.0, shu = 0.0, shv = 0.0;
        int nwet = 0;
        for (int dj = 0; dj < a.r; ++dj)
            for (int di = 0; di < a.r; ++di) {
                const int64_t k = op.src + (int64_t)dj * op.pitch + di;
                const double h = depth(qf, bf, k, a.sea);
                if (h > a.drytol) {
                    seta += h + double(bf[k]);
                    ++nwet;
                }
                shu += double(qf[k + a.psf]);
                shv += double(qf[k + 2 * a.psf]);
            }
        S* q = qc + op.dst;
        const double b_c = double(bc[op.dst]);
        if (nwet == 0) {
            q[0] = first_value<S>(0.0, b_c, b_c, a.sea);
            q[a.psc] = S(0);
            q[2 * a.psc] = S(0);
            continue;
        }
        const double eta = seta / (double)nwet;
        const double d = eta - b_c;
        const double h = d > 0.0 ? d : 0.0;
        q[0] = first_value<S>(h, eta, b_c, a.sea);
        if (h <= a.drytol) {
            q[a.psc] = S(0);
            q[2 * a.psc] = S(0);
        } else {
            const double n = (double)(a.r * a.r);
            q[a.psc] = S(shu / n);
            q[2 * a.psc] = S(shv / n);
        }
    }
}

// Refinement flags of the interior cells of level-l patches (one block row
// per patch): a wet cell whose surface departs from rest by more than tol
// flags itself and every cell within `buffer` cells (max norm) of the same
// patch; cells within `margin` cells of the patch's edge are never flagged.
// A cell gathers its window rather than flagged cells scattering theirs, so
// every flag is written once.
template <typename S>
__global__ void __launch_bounds__(256) k_amr_flag(const swe_patch* __restrict__ patches,
                                                  const S* __restrict__ q,
                                                  const S* __restrict__ b,
                                                  uint8_t* __restrict__ flags, double tol,
                                                  double drytol, double sea, int buffer,
                                                  int margin) {
    const swe_patch p = patches[blockIdx.y];
    const int64_t ncell = (int64_t)p.mx * p.my;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(c % p.mx), j = (int)(c / p.mx);
        const int64_t at = p.off + (int64_t)(j + 2) * p.pitch + (i + 2);
        bool f = false;
        if (i >= margin && i < p.mx - margin && j >= margin && j < p.my - margin) {
            const int j0 = j - buffer > 0 ? j - buffer : 0;
            const int j1 = j + buffer < p.my - 1 ? j + buffer : p.my - 1;
            const int i0 = i - buffer > 0 ? i - buffer : 0;
            const int i1 = i + buffer < p.mx - 1 ? i + buffer : p.mx - 1;
            for (int jj = j0; jj <= j1 && !f; ++jj)
                for (int ii = i0; ii <= i1 && !f; ++ii) {
                    const int64_t k = p.off + (int64_t)(jj + 2) * p.pitch + (ii + 2);
                    const double h = depth(q, b, k, sea);
                    const double dev = h + double(b[k]) - sea;
                    f = h > drytol && (dev > tol || -dev > tol);
                }
        }
        flags[at] = f ? 1 : 0;
    }
}

}  // namespace swe

extern "C" __attribute__((visibility("hidden"))) int swe_internal_set_error(int code,
                                                                           const char* msg);

namespace {

int afail(int code, const std::string& msg) { return swe_internal_set_error(code, msg.c_str()); }

int check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return afail(SWE_EHIP, std::string(what) + ": " + hipGetErrorString(e));
    return SWE_OK;
}

// Flag clustering on the host (the recursive reading stated in swe.h).
struct Box {
    int i0, j0, i1, j1;
};

class Clusterer {
  public:
    Clusterer(const uint8_t* f, int64_t pitch, double eff, int min_side)
        : f_(f), pitch_(pitch), eff_(eff), min_side_(min_side) {}
    std::vector<Box> boxes;

    void run(Box bx) {
        int i0 = INT_MAX, j0 = INT_MAX, i1 = -1, j1 = -1;
        long n = 0;
        for (int j = bx.j0; j <= bx.j1; ++j)
            for (int i = bx.i0; i <= bx.i1; ++i)
                if (on(i, j)) {
                    ++n;
                    i0 = i < i0 ? i : i0;
                    i1 = i > i1 ? i : i1;
                    j0 = j < j0 ? j : j0;
                    j1 = j > j1 ? j : j1;
                }
        if (n == 0) return;
        const int w = i1 - i0 + 1, h = j1 - j0 + 1;
        const bool can[2] = {w >= 2 * min_side_, h >= 2 * min_side_};
        if ((double)n / ((double)w * (double)h) >= eff_ || !(can[0] || can[1])) {
            boxes.push_back(Box{i0, j0, i1, j1});
            return;
        }
        // signatures: flags per column (dimension 0) and per row (dimension 1)
        std::vector<long> sig[2] = {std::vector<long>(w, 0), std::vector<long>(h, 0)};
        for (int j = j0; j <= j1; ++j)
            for (int i = i0; i <= i1; ++i)
                if (on(i, j)) {
                    ++sig[0][i - i0];
                    ++sig[1][j - j0];
                }
        const int lo[2] = {i0, j0}, hi[2] = {i1, j1};
        int order[2], nd = 0;  // splittable dimensions, longer side first (x on ties)
        const int first = w >= h ? 0 : 1;
        if (can[first]) order[nd++] = first;
        if (can[1 - first]) order[nd++] = 1 - first;
        int dim = -1, cut = 0;
        // a hole nearest the centre, in the first dimension that has one
        for (int r = 0; r < nd && dim < 0; ++r) {
            const int d = order[r];
            long best = -1;
            for (int s = lo[d]; s <= hi[d]; ++s) {
                if (sig[d][s - lo[d]] != 0 || !allowed(lo[d], hi[d], s)) continue;
                const long dist = std::labs(2L * s - (lo[d] + hi[d]));
                if (best < 0 || dist < best) {
                    best = dist;
                    dim = d;
                    cut = s;
                }
            }
        }
        // the strongest inflection over the dimensions
        if (dim < 0) {
            long bs = -1, bdist = 0;
            int brank = 0;
            for (int r = 0; r < nd; ++r) {
                const int d = order[r];
                const std::vector<long>& g = sig[d];
                auto lap = [&](int k) { return g[k - 1 - lo[d]] - 2 * g[k - lo[d]] + g[k + 1 - lo[d]]; };
                for (int s = lo[d] + 1; s <= hi[d] - 2; ++s) {
                    const long a = lap(s), c = lap(s + 1);
                    if (!((a < 0 && c > 0) || (a > 0 && c < 0)) || !allowed(lo[d], hi[d], s))
                        continue;
                    const long strength = std::labs(c - a);
                    const long dist = std::labs(2L * s - (lo[d] + hi[d]));
                    const bool better =
                        bs < 0 || strength > bs ||
                        (strength == bs &&
                         (r < brank || (r == brank && (dist < bdist || (dist == bdist && s < cut)))));
                    if (better) {
                        bs = strength;
                        brank = r;
                        bdist = dist;
                        dim = d;
                        cut = s;
                    }
                }
            }
        }
        if (dim < 0) {  // bisect the first dimension
            dim = order[0];
            cut = (lo[dim] + hi[dim]) / 2;
        }
        if (dim == 0) {
            run(Box{i0, j0, cut, j1});
            run(Box{cut + 1, j0, i1, j1});
        } else {
            run(Box{i0, j0, i1, cut});
            run(Box{i0, cut + 1, i1, j1});
        }
    }

  private:
    bool on(int i, int j) const { return f_[(int64_t)j * pitch_ + i] != 0; }
    bool allowed(int lo, int hi, int s) const { return lo + min_side_ - 1 <= s && s <= hi - min_side_; }
    const uint8_t* f_;
    int64_t pitch_;
    double eff_;
    int min_side_;
};

int grid_for(int64_t n) {
    const int64_t blocks = (n + 255) / 256;
    return (int)(blocks < 4096 ? blocks : 4096);
}

}  // namespace

extern "C" {

int swe_amr_fill(const swe_params* p, const swe_amr_fill_op* ops, int64_t nops, void* q_fine,
                 int64_t fine_plane_stride, const void* b_fine, const void* q_coarse_old,
                 const void* q_coarse_new, int64_t coarse_plane_stride, const void* b_coarse,
                 double alpha, void* stream) {
    if (!p) return afail(SWE_EINVAL, "params is NULL");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return afail(SWE_EINVAL, "swe_amr_fill: unknown precision");
    if (nops < 0 || fine_plane_stride < 1 || coarse_plane_stride < 1 || !(alpha >= 0.0) ||
        !(alpha <= 1.0))
        return afail(SWE_EINVAL, "swe_amr_fill: bad count, plane stride or alpha");
    if (nops == 0) return SWE_OK;
    if (!ops || !q_fine || !b_fine || !q_coarse_old || !q_coarse_new || !b_coarse)
        return afail(SWE_EINVAL, "swe_amr_fill: null pointer");
    if (q_fine == q_coarse_old || q_fine == q_coarse_new)
        return afail(SWE_EINVAL, "swe_amr_fill: fine and coarse planes must differ");
    swe::FillArgs a;
    a.ops = ops;
    a.nops = nops;
    a.qf = q_fine;
    a.psf = fine_plane_stride;
    a.qcopy = q_fine;
    a.pscopy = fine_plane_stride;
    a.bf = b_fine;
    a.qco = q_coarse_old;
    a.qcn = q_coarse_new;
    a.psc = coarse_plane_stride;
    a.bc = b_coarse;
    a.alpha = alpha;
    a.drytol = p->drytol;
    a.sea = p->sea_level;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_amr_fill<double>, dim3(grid_for(nops)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(swe::k_amr_fill<float>, dim3(grid_for(nops)), dim3(256), 0, st, a);
    return check_launch("swe_amr_fill");
}

int swe_amr_average(const swe_params* p, const swe_amr_avg_op* ops, int64_t nops, int32_t ratio,
                    const void* q_fine, int64_t fine_plane_stride, const void* b_fine,
                    void* q_coarse, int64_t coarse_plane_stride, const void* b_coarse,
                    void* stream) {
    if (!p) return afail(SWE_EINVAL, "params is NULL");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return afail(SWE_EINVAL, "swe_amr_average: unknown precision");
    if (nops < 0 || ratio < 1 || fine_plane_stride < 1 || coarse_plane_stride < 1)
        return afail(SWE_EINVAL, "swe_amr_average: bad count, ratio or plane stride");
    if (nops == 0) return SWE_OK;
    if (!ops || !q_fine || !b_fine || !q_coarse || !b_coarse)
        return afail(SWE_EINVAL, "swe_amr_average: null pointer");
    if (q_fine == q_coarse)
        return afail(SWE_EINVAL, "swe_amr_average: fine and coarse planes must differ");
    swe::AvgArgs a;
    a.ops = ops;
    a.nops = nops;
    a.r = ratio;
    a.qf = q_fine;
    a.psf = fine_plane_stride;
    a.bf = b_fine;
    a.qc = q_coarse;
    a.psc = coarse_plane_stride;
    a.bc = b_coarse;
    a.drytol = p->drytol;
    a.sea = p->sea_level;
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_amr_average<double>, dim3(grid_for(nops)), dim3(256), 0, st, a);
    else
        hipLaunchKernelGGL(swe::k_amr_average<float>, dim3(grid_for(nops)), dim3(256), 0, st, a);
    return check_launch("swe_amr_average");
}

int swe_amr_cluster(const uint8_t* flags, int32_t mx, int32_t my, int32_t pitch,
                    double efficiency, int32_t min_side, int32_t* boxes, int32_t max_boxes,
                    int32_t* nboxes) {
    if (!flags || !nboxes || mx < 1 || my < 1 || pitch < mx || min_side < 1 ||
        !(efficiency > 0.0) || !(efficiency <= 1.0) || max_boxes < 0 || (max_boxes > 0 && !boxes))
        return afail(SWE_EINVAL, "swe_amr_cluster: bad arguments");
    Clusterer c(flags, pitch, efficiency, min_side);
    c.run(Box{0, 0, mx - 1, my - 1});
    *nboxes = (int32_t)c.boxes.size();
    if ((int32_t)c.boxes.size() > max_boxes)
        return afail(SWE_EINVAL, "swe_amr_cluster: more boxes than max_boxes (count in *nboxes)");
    for (size_t k = 0; k < c.boxes.size(); ++k) {
        boxes[4 * k] = c.boxes[k].i0;
        boxes[4 * k + 1] = c.boxes[k].j0;
        boxes[4 * k + 2] = c.boxes[k].i1;
        boxes[4 * k + 3] = c.boxes[k].j1;
    }
    return SWE_OK;
}

int swe_amr_init(const swe_params* p, int32_t ratio, const swe_amr_rect* new_rects, int32_t n_new,
                 int64_t max_cells, void* q_new, int64_t new_plane_stride, const void* b_new,
                 const swe_amr_rect* old_rects, int32_t n_old, const void* q_old,
                 int64_t old_plane_stride, const swe_amr_rect* coarse_rects, int32_t n_coarse,
                 const void* q_coarse, int64_t coarse_plane_stride, const void* b_coarse,
                 void* stream) {
    if (!p) return afail(SWE_EINVAL, "params is NULL");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return afail(SWE_EINVAL, "swe_amr_init: unknown precision");
    if (ratio < 1 || n_new < 0 || n_old < 0 || n_coarse < 0 || max_cells < 0 ||
        new_plane_stride < 1 || coarse_plane_stride < 1 || (n_old > 0 && old_plane_stride < 1))
        return afail(SWE_EINVAL, "swe_amr_init: bad ratio, count, size or plane stride");
    if (n_new == 0 || max_cells == 0) return SWE_OK;
    if (!new_rects || !q_new || !b_new || !coarse_rects || !q_coarse || !b_coarse ||
        (n_old > 0 && (!old_rects || !q_old)))
        return afail(SWE_EINVAL, "swe_amr_init: null pointer");
    if (q_new == q_coarse || (n_old > 0 && q_new == q_old))
        return afail(SWE_EINVAL, "swe_amr_init: the new planes must differ from the sources");
    if (n_new > 65535) return afail(SWE_EINVAL, "swe_amr_init: more than 65535 new patches");
    swe::FillArgs a{};
    a.qf = q_new;
    a.psf = new_plane_stride;
    a.qcopy = n_old > 0 ? q_old : q_new;
    a.pscopy = n_old > 0 ? old_plane_stride : new_plane_stride;
    a.bf = b_new;
    a.qco = q_coarse;
    a.qcn = q_coarse;
    a.psc = coarse_plane_stride;
    a.bc = b_coarse;
    a.alpha = 1.0;
    a.drytol = p->drytol;
    a.sea = p->sea_level;
    swe::InitArgs g;
    g.nw = new_rects;
    g.old = n_old > 0 ? old_rects : nullptr;
    g.nold = n_old;
    g.crs = coarse_rects;
    g.ncrs = n_coarse;
    g.ratio = ratio;
    const int64_t bx64 = (max_cells + 255) / 256;
    const dim3 grid((unsigned)(bx64 < 1024 ? bx64 : 1024), (unsigned)n_new);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_amr_init_rects<double>, grid, dim3(256), 0, st, a, g);
    else
        hipLaunchKernelGGL(swe::k_amr_init_rects<float>, grid, dim3(256), 0, st, a, g);
    return check_launch("swe_amr_init");
}

int swe_amr_plans(const swe_amr_rect* fine, int32_t n_fine, const swe_amr_rect* coarse,
                  int32_t n_coarse, int32_t ratio, int64_t max_entries, swe_amr_fill_op* fill_ops,
                  const int64_t* fill_first, swe_amr_avg_op* avg_ops, const int64_t* avg_first,
                  uint32_t* err, void* stream) {
    if (ratio < 1 || n_fine < 0 || n_coarse < 0 || max_entries < 0)
        return afail(SWE_EINVAL, "swe_amr_plans: bad ratio, count or size");
    if (n_fine == 0 || max_entries == 0) return SWE_OK;
    if (!fine || !coarse || !fill_ops || !fill_first || !avg_ops || !avg_first || !err)
        return afail(SWE_EINVAL, "swe_amr_plans: null pointer");
    if (n_fine > 65535) return afail(SWE_EINVAL, "swe_amr_plans: more than 65535 fine patches");
    swe::PlanArgs g;
    g.fine = fine;
    g.nfine = n_fine;
    g.crs = coarse;
    g.ncrs = n_coarse;
    g.ratio = ratio;
    g.fill = fill_ops;
    g.fill_first = fill_first;
    g.avg = avg_ops;
    g.avg_first = avg_first;
    g.err = err;
    const int64_t bx64 = (max_entries + 255) / 256;
    const dim3 grid((unsigned)(bx64 < 1024 ? bx64 : 1024), (unsigned)n_fine);
    hipLaunchKernelGGL(swe::k_amr_plans, grid, dim3(256), 0, static_cast<hipStream_t>(stream), g);
    return check_launch("swe_amr_plans");
}

int swe_amr_flag(const swe_params* p, const swe_patch* patches, int32_t n, int32_t max_mx,
                 int32_t max_my, const void* q, const void* b, double tol, int32_t buffer,
                 int32_t margin, uint8_t* flags, void* stream) {
    if (!p) return afail(SWE_EINVAL, "params is NULL");
    if (p->precision != SWE_F64 && p->precision != SWE_F32_DEV)
        return afail(SWE_EINVAL, "swe_amr_flag: unknown precision");
    if (n < 0 || max_mx < 1 || max_my < 1 || buffer < 0 || margin < 0 || !(tol >= 0.0))
        return afail(SWE_EINVAL, "swe_amr_flag: bad count, size, buffer, margin or tol");
    if (n == 0) return SWE_OK;
    if (!patches || !q || !b || !flags) return afail(SWE_EINVAL, "swe_amr_flag: null pointer");
    const int64_t ncell = (int64_t)max_mx * max_my;
    const int64_t bx64 = (ncell + 255) / 256;
    const dim3 grid((unsigned)(bx64 < 1024 ? bx64 : 1024), (unsigned)n);
    const hipStream_t st = static_cast<hipStream_t>(stream);
    if (p->precision == SWE_F64)
        hipLaunchKernelGGL(swe::k_amr_flag<double>, grid, dim3(256), 0, st, patches,
                           static_cast<const double*>(q), static_cast<const double*>(b), flags,
                           tol, p->drytol, p->sea_level, buffer, margin);
    else
        hipLaunchKernelGGL(swe::k_amr_flag<float>, grid, dim3(256), 0, st, patches,
                           static_cast<const float*>(q), static_cast<const float*>(b), flags,
                           tol, p->drytol, p->sea_level, buffer, margin);
    return check_launch("swe_amr_flag");
}

}  // extern "C"
