// swe_common.hpp -- layout helpers shared by the gfx950 kernels: ghost-cell
// synthesis on load, wave64 cross-lane moves and reductions, status words.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "swe.h"
#include "swe_math.hpp"

namespace swe {

constexpr int kWave = 64;
constexpr int kStripOut = kWave - 4;  // columns updated per wave64 strip

// Where cell (R, c) of a patch (row R, column c, ghosts included) comes from.
// Sides with a physical boundary code are synthesised from the interior:
// x-ghosts of interior rows from the x-sides, then y-ghosts of all columns
// from the y-sides; a side with SWE_BC_USER is read from memory as stored.
struct Src {
    int64_t idx;   // element index in the planes
    double sx;     // sign applied to hu (x-wall)
    double sy;     // sign applied to hv (y-wall)
};

__device__ __forceinline__ Src map_cell(int R, int c, int mx, int my, int pitch, int64_t off,
                                        const int8_t* bc) {
    double sx = 1.0, sy = 1.0;
    int rr = R, ci = c;
    bool user_row = false;
    if (R < 2) {
        if (bc[2] == SWE_BC_USER) user_row = true;
        else if (bc[2] == SWE_BC_WALL) { rr = 3 - R; sy = -1.0; }
        else rr = 2;
    } else if (R > my + 1) {
        if (bc[3] == SWE_BC_USER) user_row = true;
        else if (bc[3] == SWE_BC_WALL) { rr = 2 * my + 3 - R; sy = -1.0; }
        else rr = my + 1;
    }
    if (!user_row) {
        if (c < 2) {
            if (bc[0] == SWE_BC_WALL) { ci = 3 - c; sx = -1.0; }
            else if (bc[0] == SWE_BC_EXTRAP) ci = 2;
        } else if (c > mx + 1) {
            if (bc[1] == SWE_BC_WALL) { ci = 2 * mx + 3 - c; sx = -1.0; }
            else if (bc[1] == SWE_BC_EXTRAP) ci = mx + 1;
        }
    }
    Src s;
    s.idx = off + (int64_t)rr * pitch + ci;
    s.sx = sx;
    s.sy = sy;
    return s;
}

// map_cell when the caller's wave-wide vote found every lane's cell inside
// its patch: such a cell is stored where it lies (the vote keeps the branch
// uniform, so interior rows skip the boundary cases).
__device__ __forceinline__ Src map_cell_voted(bool all_inside, int R, int c, int mx, int my,
                                              int pitch, int64_t off, const int8_t* bc) {
    if (all_inside) {
        Src s;
        s.idx = off + (int64_t)R * pitch + c;
        s.sx = 1.0;
        s.sy = 1.0;
        return s;
    }
    return map_cell(R, c, mx, my, pitch, off, bc);
}

// Lane moves within a segment of SEG lanes (SEG = 64: the whole wave):
// up(x) gives lane k the value of lane k - 1, down(x) the value of lane k + 1.
// What the first lane of a segment receives from up(), and the last from
// down(), is unspecified: those are halo lanes, whose edges and cells feed
// no result (callers also leave them out of wave-wide votes).
#ifndef SWE_LANE_DPP
#define SWE_LANE_DPP 1
#endif
#if SWE_LANE_DPP
// Whole-wave DPP rotations (wave_ror:1 / wave_rol:1), one VALU move per
// dword.  Lane 0 receives lane 63's value and lane 63 lane 0's: real cells of
// the strip, so a halo lane's edge takes the same code path as its
// neighbours' (no divergence at the strip ends).  The rotations cross segment
// boundaries, which only feeds the halo lanes of a segment.
constexpr int kDppWaveRor1 = 0x13C;
constexpr int kDppWaveRol1 = 0x134;
__device__ __forceinline__ int dpp_up(int v) {
    return __builtin_amdgcn_mov_dpp(v, kDppWaveRor1, 0xf, 0xf, false);
}
__device__ __forceinline__ int dpp_down(int v) {
    return __builtin_amdgcn_mov_dpp(v, kDppWaveRol1, 0xf, 0xf, false);
}
template <int SEG = kWave>
__device__ __forceinline__ double lane_up(double x) {
    return __hiloint2double(dpp_up(__double2hiint(x)), dpp_up(__double2loint(x)));
}
template <int SEG = kWave>
__device__ __forceinline__ double lane_down(double x) {
    return __hiloint2double(dpp_down(__double2hiint(x)), dpp_down(__double2loint(x)));
}
template <int SEG = kWave>
__device__ __forceinline__ float lane_up(float x) {
    return __int_as_float(dpp_up(__float_as_int(x)));
}
template <int SEG = kWave>
__device__ __forceinline__ float lane_down(float x) {
    return __int_as_float(dpp_down(__float_as_int(x)));
}
#else
template <int SEG = kWave>
__device__ __forceinline__ double lane_up(double x) { return __shfl_up(x, 1, SEG); }
template <int SEG = kWave>
__device__ __forceinline__ double lane_down(double x) { return __shfl_down(x, 1, SEG); }
template <int SEG = kWave>
__device__ __forceinline__ float lane_up(float x) { return __shfl_up(x, 1, SEG); }
template <int SEG = kWave>
__device__ __forceinline__ float lane_down(float x) { return __shfl_down(x, 1, SEG); }
#endif

// Lane l's value, for a wave-uniform l (two scalar reads of the dwords).
__device__ __forceinline__ double lane_read(double x, int l) {
    const int hi = __builtin_amdgcn_readlane(__double2hiint(x), l);
    const int lo = __builtin_amdgcn_readlane(__double2loint(x), l);
    return __hiloint2double(hi, lo);
}

// The left neighbour's side: the fields side_base makes (velocities and
// sqrt(h) are moved separately, once the neighbour has computed them).
template <typename T, bool DEV = false, int SEG = kWave>
__device__ __forceinline__ Side<T> side_up(const Side<T>& s, const DevParams& P) {
    Side<T> r;
    r.h = lane_up<SEG>(s.h);
    r.m = lane_up<SEG>(s.m);
    r.t = lane_up<SEG>(s.t);
    r.b = lane_up<SEG>(s.b);
    r.u = T(0);
    r.v = T(0);
    r.sq = T(0);
    r.c = lane_up<SEG>(s.c);
    r.eta = DEV ? lane_up<SEG>(s.eta) : T(0);
    r.dry = r.h <= T(P.drytol);
    return r;
}

// Largest of the lanes' non-negative doubles.  Such doubles order like their
// bit patterns read as unsigned integers, and a NaN sorts above every number,
// so the comparison is done on the bits: NaN propagates.
template <int SEG = kWave>
__device__ __forceinline__ double wave_max_nonneg(double v) {
    unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(v));
#pragma unroll
    for (int o = SEG / 2; o >= 1; o >>= 1) {
        unsigned long long w = static_cast<unsigned long long>(
            __shfl_xor(static_cast<long long>(b), o, SEG));
        b = b > w ? b : w;
    }
    return __longlong_as_double(static_cast<long long>(b));
}

__device__ __forceinline__ void atomic_max_nonneg(double* addr, double v) {
    atomicMax(reinterpret_cast<unsigned long long*>(addr),
              static_cast<unsigned long long>(__double_as_longlong(v)));
}

}  // namespace swe
