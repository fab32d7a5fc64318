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
// cells, which no entry writes.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "swe.h"

namespace swe {

struct FillArgs {
    const swe_amr_fill_op* ops;
    int64_t nops;
    void* qf;
    int64_t psf;
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

// Ghost cells of the finer level.  A copy takes the same level's cell; a
// coarse entry takes the cell below (constant in space), linear in time
// between its states before (qco) and after (qcn) its step.  FP32 planes are
// read into FP64, combined there and rounded once.
template <typename S>
__global__ void __launch_bounds__(256) k_amr_fill(FillArgs a) {
    S* qf = static_cast<S*>(a.qf);
    const S* bf = static_cast<const S*>(a.bf);
    const S* qco = static_cast<const S*>(a.qco);
    const S* qcn = static_cast<const S*>(a.qcn);
    const S* bc = static_cast<const S*>(a.bc);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < a.nops; i += stride) {
        const swe_amr_fill_op op = a.ops[i];
        S* q = qf + op.dst;
        if (op.kind == SWE_AMR_COPY) {
            const S* src = qf + op.src;
            q[0] = src[0];
            q[a.psf] = src[a.psf];
            q[2 * a.psf] = src[2 * a.psf];
            continue;
        }
        const double ho = depth(qco, bc, op.src, a.sea), hn = depth(qcn, bc, op.src, a.sea);
        const double b_f = double(bf[op.dst]);
        if (ho <= a.drytol && hn <= a.drytol) {
            q[0] = first_value<S>(0.0, b_f, b_f, a.sea);
            q[a.psf] = S(0);
            q[2 * a.psf] = S(0);
            continue;
        }
        const double b = double(bc[op.src]);
        const double w0 = 1.0 - a.alpha, w1 = a.alpha;
        const double eta = w0 * (ho + b) + w1 * (hn + b);
        const double d = eta - b_f;
        const double h = d > 0.0 ? d : 0.0;
        q[0] = first_value<S>(h, eta, b_f, a.sea);
        if (h <= a.drytol) {
            q[a.psf] = S(0);
            q[2 * a.psf] = S(0);
        } else {
            q[a.psf] = S(w0 * double(qco[op.src + a.psc]) + w1 * double(qcn[op.src + a.psc]));
            q[2 * a.psf] =
                S(w0 * double(qco[op.src + 2 * a.psc]) + w1 * double(qcn[op.src + 2 * a.psc]));
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

}  // extern "C"
