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

// A double from lane src_lane (ds_bpermute: a lane permute, no LDS memory is touched).
__device__ __forceinline__ double bperm_d(double v, int src_lane) {
    const int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2loint(v));
    const int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of 16 values at once (d[i] per lane, overwritten): a butterfly inside
// each 16-lane row halves the values per level (partners 1, 2, 4 and 8 apart: a lane keeps the
// half of its values picked by its own lane bit and adds the partner's copy of that half), then
// the four rows are added.  Lane r < 16 returns the wave's sum of value bfly_index(r) (the
// bit-reversed r); every value is formed in a fixed order, so results do not depend on
// scheduling.
__device__ __forceinline__ int bfly_index(int lane) {
    return (lane & 1) << 3 | (lane & 2) << 1 | (lane & 4) >> 1 | (lane & 8) >> 3;
}

__device__ __forceinline__ double wave_bfly16(double (&d)[16]) {
    const int lane = threadIdx.x & 63;
    const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const double keep = b0 ? d[i + 8] : d[i], send = b0 ? d[i] : d[i + 8];
        d[i] = keep + dpp_d<0xB1>(send);   // quad_perm [1,0,3,2]: partner lane ^ 1
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double keep = b1 ? d[i + 4] : d[i], send = b1 ? d[i] : d[i + 4];
        d[i] = keep + dpp_d<0x4E>(send);   // quad_perm [2,3,0,1]: partner lane ^ 2
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        const double keep = b2 ? d[i + 2] : d[i], send = b2 ? d[i] : d[i + 2];
        d[i] = keep + dpp_d<0x124>(send);  // row_ror 4: a partner whose lane bit 2 differs
    }
    const double keep = b3 ? d[1] : d[0], send = b3 ? d[0] : d[1];
    double s = keep + dpp_d<0x128>(send);  // row_ror 8: partner lane ^ 8
    s += bperm_d(s, lane ^ 16);
    s += bperm_d(s, lane ^ 32);
    return s;
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
    float invH;   // 1/H rounded to FP32: grid row of p as (int)((p + 0.5) invH), exact here
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
    o.invH = 1.0f / (float)s.H;
    return o;
}

// A descriptor a launch can solve: a grid of at most nmax unknowns with its arrays and dt > 0.
__device__ __forceinline__ bool desc_ok(const xkp_system &s, int nmax) {
    return s.H > 0 && (long)s.H * s.H <= nmax && s.mt != nullptr && s.b != nullptr &&
           s.x != nullptr && s.dt > 0.0;
}

// The antisymmetric parts ex, ey of row p < n's neighbour coefficients (Section 2.3: the
// lagged-density drift terms and the drift field f; m~ and f zero outside the grid).
__device__ __forceinline__ void row_drift(const xkp_system &s, const OpConst &o, int p,
                                          double &ex, double &ey) {
    const int H = o.H;
    const double *__restrict__ mt = s.mt;
    const int i = p / H, j = p - (p / H) * H;
    const double mE = (i + 1 < H) ? mt[p + H] : 0.0;
    const double mW = (i > 0) ? mt[p - H] : 0.0;
    const double mN = (j + 1 < H) ? mt[p + 1] : 0.0;
    const double mS = (j > 0) ? mt[p - 1] : 0.0;
    const double fxp = s.fx ? s.fx[p] : 0.0;
    const double fyp = s.fy ? s.fy[p] : 0.0;
    ex = fxp * o.inv2h - o.c8 * (mE - mW);
    ey = fyp * o.inv2h - o.c8 * (mN - mS);
}

// The four neighbour coefficients of row p from its ex, ey: -a +- ex (east, west) and -a +- ey
// (north, south), zero where the neighbour lies outside the grid and for rows p >= n.
__device__ __forceinline__ void coeffs_of(const OpConst &o, int p, double ex, double ey,
                                          double &cE, double &cW, double &cN, double &cS) {
    const int H = o.H;
    const int i = (int)(((float)p + 0.5f) * o.invH), j = p - i * H;
    const bool in = p < o.n;
    cE = (in && i + 1 < H) ? -o.a + ex : 0.0;
    cW = (in && i > 0) ? -o.a - ex : 0.0;
    cN = (in && j + 1 < H) ? -o.a + ey : 0.0;
    cS = (in && j > 0) ? -o.a - ey : 0.0;
}

// The same in FP32 from FP32 parts (the mixed-precision operator): -a +- ex, -a +- ey formed in
// FP32, zero where the neighbour lies outside the grid and for rows p >= n.
__device__ __forceinline__ void coeffs_of_f32(const OpConst &o, int p, float ex, float ey,
                                              float &cE, float &cW, float &cN, float &cS) {
    const int H = o.H;
    const int i = (int)(((float)p + 0.5f) * o.invH), j = p - i * H;
    const bool in = p < o.n;
    const float a = (float)o.a;
    cE = (in && i + 1 < H) ? -a + ex : 0.0f;
    cW = (in && i > 0) ? -a - ex : 0.0f;
    cN = (in && j + 1 < H) ? -a + ey : 0.0f;
    cS = (in && j > 0) ? -a - ey : 0.0f;
}

// The four neighbour coefficients of row p < n.
__device__ __forceinline__ void row_coeffs(const xkp_system &s, const OpConst &o, int p,
                                           double &cE, double &cW, double &cN, double &cS) {
    double ex, ey;
    row_drift(s, o, p, ex, ey);
    coeffs_of(o, p, ex, ey, cE, cW, cN, cS);
}

// BF16 bits of a double: rounded to FP32, then to the nearest BF16 (ties to even); finite
// values only.
__device__ __forceinline__ unsigned short to_bf16(double d) {
    const unsigned u = __builtin_bit_cast(unsigned, (float)d);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// ----------------------------------------------------------------------------------------
// Small dense solves of the projection (Section 3, Phase 2), one wavefront.

// Least squares min ||z - Hbar alpha|| for the (kk+1) x kk upper Hessenberg matrix in LDS (row
// major) by Givens rotations, wavefront 0, lane q owning column q.  z is in LDS (kk+1 values).
__device__ inline bool lsq_hessenberg_wave(double *A, int lda, int kk, double *z, double *out) {
    const int q = threadIdx.x;
    double cmax = 0.0;
    if (q < kk)
        for (int r = 0; r <= kk; ++r) cmax = fmax(cmax, fabs(A[r * lda + q]));
    const double amax = wave_max(cmax);
    if (!(amax > 0.0)) return true;
    for (int c = 0; c < kk; ++c) {
        const double a0 = A[c * lda + c], a1 = A[(c + 1) * lda + c];
        const double den = sqrt(a0 * a0 + a1 * a1);
        if (!(den > 1e-13 * amax)) return true;
        const double cs = a0 / den, sn = a1 / den;
        wave_lds_sync();
        if (q >= c && q < kk) {
            const double u = A[c * lda + q], v = A[(c + 1) * lda + q];
            A[c * lda + q] = cs * u + sn * v;
            A[(c + 1) * lda + q] = -sn * u + cs * v;
        }
        if (q == 0) {
            const double u = z[c], v = z[c + 1];
            z[c] = cs * u + sn * v;
            z[c + 1] = -sn * u + cs * v;
        }
        wave_lds_sync();
    }
    // back substitution on the triangle, lane r holding z_r
    double zl = (q < kk) ? z[q] : 0.0;
    for (int c = kk - 1; c >= 0; --c) {
        const double xc = readlane_d(zl, c) / A[c * lda + c];
        if (q < c) zl -= A[q * lda + c] * xc;
        if (q == 0) out[c] = xc;
    }
    wave_lds_sync();
    return false;
}

// LU with partial pivoting of the kk x kk row-major LDS matrix A (leading dimension lda >= KM,
// even; A 16-byte aligned; kk <= KM, KM a multiple of 8) by one wavefront, lane r holding row r
// in registers.  Per column the pivot is the largest remaining |A[r][c]| (lowest lane on ties);
// rows are not moved.  The registers hold the columns from the current one on: after each
// elimination step every row shifts down by one register, so the column loop is a plain loop
// and the code stays small (one wave runs this once per system, from a cold instruction cache;
// a fully unrolled column loop spent much of its time fetching instructions).  The pivot lane of
// column c stores its row (columns c, c+1, ...) over row c of A and its right-hand side entry
// in zbuf[c] (LDS, kk doubles); every lane reads them back as broadcasts.  Stores, reads and
// updates go in chunks of 8 registers, and chunks wholly past the last column are skipped
// (they hold zeros and stay so).  Back substitution then runs on the stored rows.  zr is lane
// r's right-hand side entry; the solution goes to out[0..kk) in LDS.  A pivot <= 1e-13 max|A|
// reports singular (true).  A is overwritten.
template <int KM>
__device__ __forceinline__ bool lu_regs(double *A, int lda, int kk, double zr, double *out,
                                        double *zbuf) {
    typedef double d2_t __attribute__((ext_vector_type(2)));
    constexpr int CH = 8;
    static_assert(KM % CH == 0, "whole chunks");
    const int r = threadIdx.x & 63;
    kk = __builtin_amdgcn_readfirstlane(kk);
    double a[KM];
    double rowmax = 0.0;
#pragma unroll
    for (int q = 0; q < KM; ++q) {
        a[q] = (r < kk && q < kk) ? A[r * lda + q] : 0.0;
        rowmax = fmax(rowmax, fabs(a[q]));
    }
    const double amax = wave_max(rowmax);
    if (!(amax > 0.0)) return true;
    wave_lds_sync();   // every row read before pivot rows are stored over A
    bool active = r < kk;
#pragma unroll 1
    for (int c = 0; c < kk; ++c) {
        const double v = active ? fabs(a[0]) : -1.0;
        const double vmax = wave_max(v);
        if (!(vmax > 1e-13 * amax)) return true;
        const int pl = __ffsll((unsigned long long)__ballot(active && v == vmax)) - 1;
        // registers [0, live) hold columns c..kk-1; a chunk starting at q0 <= live still sets
        // register q0 - 1, so it runs (its stored entries past the last column are zeros)
        const int live = kk - c;
        double *U = A + c * lda;
        if (r == pl) {
#pragma unroll
            for (int q0 = 0; q0 < KM; q0 += CH)
                if (q0 <= live) {
#pragma unroll
                    for (int q = q0; q < q0 + CH; q += 2) *(d2_t *)(U + q) = d2_t{a[q], a[q + 1]};
                }
            zbuf[c] = zr;
            active = false;
        }
        wave_lds_sync();
        const double l = active ? a[0] / U[0] : 0.0;
        // column c + q of the row minus l times the pivot row's, into register q - 1
#pragma unroll
        for (int q0 = 0; q0 < KM; q0 += CH)
            if (q0 <= live) {
#pragma unroll
                for (int q = q0; q < q0 + CH; q += 2) {
                    const d2_t u = *(const d2_t *)(U + q);
                    if (q > 0) a[q - 1] = a[q] - l * u[0];
                    a[q] = a[q + 1] - l * u[1];
                }
            }
        a[KM - 1] = 0.0;
        zr -= l * zbuf[c];
    }
    // back substitution on the stored pivot rows, last column first: lane r holds pivot row
    // r's right-hand side entry and the reciprocal of its pivot; row r's entry of column c is
    // A[r * lda + c - r]
    const double rp = r < kk ? 1.0 / A[r * lda] : 0.0;
    double zb = r < kk ? zbuf[r] : 0.0;
    double unext = r < kk - 1 ? A[r * lda + (kk - 1 - r)] : 0.0;
#pragma unroll 1
    for (int c = kk - 1; c >= 0; --c) {
        const double u = unext;
        unext = r < c - 1 ? A[r * lda + (c - 1 - r)] : 0.0;
        const double xc = readlane_d(zb, c) * readlane_d(rp, c);
        if (r < c) zb -= u * xc;
    }
    if (r < kk) out[r] = zb * rp;
    wave_lds_sync();
    return false;
}



}  // namespace XKP_VARIANT
}  // namespace xkp
