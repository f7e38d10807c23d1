// Device-side building blocks shared by the xkp kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "xkp.h"

#ifndef XKP_NT
#define XKP_NT 512
#endif
#ifndef XKP_VARIANT
#define XKP_VARIANT v512
#endif

namespace xkp {
namespace XKP_VARIANT {

constexpr int kNT = XKP_NT;         // threads per workgroup
constexpr int kNW = kNT / 64;       // wavefronts per workgroup
constexpr int kMMax = 64;           // largest restart length / basis dimension
constexpr int kRedSlots = 8;        // values reduced together by block_sum_multi

typedef double double4_t __attribute__((ext_vector_type(4)));

// Barrier that orders LDS traffic only: outstanding global loads (the prefetched next basis
// column) stay in flight across it.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS accesses between the lanes of one wavefront.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

// Lane permutation of a double by a DPP control; every control used here reads a valid source
// lane for every lane, so the destination needs no initial value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    int lo = __double2loint(v), hi = __double2hiint(v);
    lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int lane) {
    int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
    int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
    return __hiloint2double(hi, lo);
}

// Sum over the 64 lanes, same fixed order on every call (deterministic); every lane gets it.
// quad_perm [1,0,3,2] and [2,3,0,1] give quad sums, row_ror 4 and 8 give 16-lane row sums,
// then the four row sums are read out and added.
// Sum over each 16-lane row, every lane of the row getting it: the first four steps below.
__device__ __forceinline__ double row_sum16(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x124>(v);
    v += dpp_d<0x128>(v);
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    v = row_sum16(v);
    return (readlane_d(v, 0) + readlane_d(v, 16)) + (readlane_d(v, 32) + readlane_d(v, 48));
}

__device__ __forceinline__ double wave_max(double v) {
    v = fmax(v, dpp_d<0xB1>(v));
    v = fmax(v, dpp_d<0x4E>(v));
    v = fmax(v, dpp_d<0x124>(v));
    v = fmax(v, dpp_d<0x128>(v));
    return fmax(fmax(readlane_d(v, 0), readlane_d(v, 16)), fmax(readlane_d(v, 32), readlane_d(v, 48)));
}

// Workgroup reductions.  `red` is LDS of 2 * kRedSlots * kNW doubles; `par` alternates the half
// used so that one barrier per reduction suffices.
// Sum of p[0..N) as a balanced tree (fixed order, short dependency chain), N a power of two.
template <int N>
__device__ __forceinline__ double tree_sum(const double *p) {
    if constexpr (N == 1) {
        return p[0];
    } else {
        return tree_sum<N / 2>(p) + tree_sum<N / 2>(p + N / 2);
    }
}

struct BlockRed {
    double *red;
    int par;
    __device__ __forceinline__ double sum(double v) {
        const double s = wave_sum(v);
        double *slot = red + par * (kRedSlots * kNW);
        if ((threadIdx.x & 63) == 0) slot[threadIdx.x >> 6] = s;
        lds_barrier();
        const double t = tree_sum<kNW>(slot);
        par ^= 1;
        return t;
    }
    template <int NV>
    __device__ __forceinline__ void sum_multi(double (&v)[NV]) {
        static_assert(NV <= kRedSlots, "too many values");
        double *slot = red + par * (kRedSlots * kNW);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double s = wave_sum(v[q]);
            if ((threadIdx.x & 63) == 0) slot[q * kNW + (threadIdx.x >> 6)] = s;
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = tree_sum<kNW>(slot + q * kNW);
        par ^= 1;
    }
};

// Per-system constants of the operator (Section 2.3): C_diag and the symmetric part -a of the
// four neighbour coefficients; the antisymmetric parts are the per-row ex, ey.
struct OpConst {
    int n, H;
    double cd, a, c8, inv2h;
};

__device__ __forceinline__ OpConst op_const(const xkp_system &s) {
    OpConst o;
    o.H = s.H;
    o.n = s.H * s.H;
    const double h = 1.0 / (double)s.H;
    const double g2 = s.g * s.g;
    o.cd = 1.0 / s.dt + 2.0 * g2 / (h * h);
    o.a = g2 / (2.0 * h * h);
    o.c8 = g2 / (8.0 * h * h);
    o.inv2h = 1.0 / (2.0 * h);
    return o;
}


}  // namespace XKP_VARIANT
}  // namespace xkp
