// HIP kernels (gfx950) of the cross-matrix Krylov projection path.
//
// One workgroup of kNT threads owns one linear system at a time (persistent loop over the
// batch).  Thread t owns the row pairs p = 2t + 2k*kNT + e (e = 0, 1; k < rmax/2) of every grid
// vector, so that a basis column moves through 16-byte loads and stores: basis columns are read
// and written only by the thread owning the row, so global memory needs no cross-thread
// ordering; the stencil's neighbour values come from an LDS copy of the vector.
//
//   solve_kernel    one persistent launch per batch, systems taken from a work queue:
//     gmres_one     restarted GMRES(m): stencil operator (Section 2.3), Arnoldi with modified
//                   Gram-Schmidt (two passes while a basis is kept), Givens rotations, restart
//                   on the FP64 true residual; optionally keeps the first cycle as the seed
//                   basis (Section 3, Phase 1) or starts from the projected guess (Phase 2).
//     project_one   Phase 2 projection of a target onto its seed basis: the k x k system
//                   V^T A' V (FP64 matrix cores), H_k, or the least-squares Hessenberg problem,
//                   solved by one wavefront; x0 = x_base + V alpha.
//   residual_kernel ||b - A x|| / ||b|| in FP64;  apply_kernel y = A u.
#include <mutex>
#include <vector>

#include "xkp_device.h"
#include "xkp_internal.h"

#ifndef XKP_DEPTH4
#define XKP_DEPTH4 4
#endif
#ifndef XKP_DEPTH8
#define XKP_DEPTH8 2
#endif
#ifndef XKP_STENCIL_GROUP
#define XKP_STENCIL_GROUP 2
#endif
#ifndef XKP_DEPTH16
#define XKP_DEPTH16 1
#endif
#ifndef XKP_DEPTH32
#define XKP_DEPTH32 2
#endif


namespace xkp {
namespace XKP_VARIANT {

constexpr int kLdA = 81;   // leading dimension of the projected matrix in LDS (<= 80 columns)
// Column tiles of V^T W per matrix-core pass: two at 8 waves, one at 16 waves (128 registers per
// lane leave no room for a second set of accumulators).
constexpr int kNtcMax = kNT >= 1024 ? 1 : 2;
// Mixed precision: a GMRES cycle with the FP32 operator stops once its residual estimate has
// dropped by this factor (about 170 FP32 unit roundoffs, the attainable reduction for operators
// of condition number up to a few hundred); the FP64 true residual then restarts it.
constexpr double kMixedCycleDrop = 1e-5;

// ----------------------------------------------------------------------------------------
// Vector helpers over the rows a thread owns.

// Row accessors on buffer resources: a vector is addressed through a scalar descriptor (base and
// size in bytes) plus a 32-bit byte offset per row, the same offset register for every vector
// and basis column.  The hardware range check makes rows past the end read as zero and drops
// stores past the end, so no access needs a mask or a branch.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
constexpr int kRsrcWord3 = 0x00020000;   // raw (untyped) buffer, gfx9-family descriptor

__device__ __forceinline__ rsrc_t mkbuf(const double *base, int count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<double *>(base), (short)0, count * 8,
                                             kRsrcWord3);
}
__device__ __forceinline__ double bld(rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, soff, 0));
}
__device__ __forceinline__ void bst(rsrc_t r, unsigned byte_off, double v, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, byte_off, soff, 0);
}
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef double double2_t __attribute__((ext_vector_type(2)));
// Two consecutive doubles (one 16-byte access); the pair lies wholly inside or wholly outside
// every range it is used with (even element counts).
__device__ __forceinline__ double2_t bld2(rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    return __builtin_bit_cast(double2_t, __builtin_amdgcn_raw_buffer_load_b128(r, byte_off, soff, 0));
}
__device__ __forceinline__ void bst2(rsrc_t r, unsigned byte_off, double a, double b,
                                     unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4_t, double2_t{a, b}), r,
                                           byte_off, soff, 0);
}

// FP32 / BF16 views: the same resources with 4- and 2-byte elements.
__device__ __forceinline__ rsrc_t mkbuf32(const float *base, int count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<float *>(base), (short)0, count * 4,
                                             kRsrcWord3);
}
__device__ __forceinline__ rsrc_t mkbuf16(const unsigned short *base, int count) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<unsigned short *>(base), (short)0,
                                             count * 2, kRsrcWord3);
}
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ f32x2_t bldf2(rsrc_t r, unsigned byte_off, unsigned soff = 0) {
    return __builtin_bit_cast(f32x2_t, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, soff, 0));
}
__device__ __forceinline__ void bstf(rsrc_t r, unsigned byte_off, float v, unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, byte_off, soff, 0);
}
__device__ __forceinline__ void bst16(rsrc_t r, unsigned byte_off, unsigned short v,
                                      unsigned soff = 0) {
    __builtin_amdgcn_raw_buffer_store_b16(v, r, byte_off, soff, 0);
}

// Row k of this thread: p = 2t + (k & 1) + (k >> 1) * 2 kNT, addressed as the lane offset of the
// pair (one register) + a scalar offset.  Every per-row array a thread holds is indexed by k.
__device__ __forceinline__ int row_of(int k) {
    return 2 * (int)threadIdx.x + (k & 1) + (k >> 1) * 2 * kNT;
}
__device__ __forceinline__ unsigned lane_off() { return threadIdx.x * 16u; }
__device__ __forceinline__ unsigned row_soff(int k) {
    return (unsigned)(((k >> 1) * 2 * kNT + (k & 1)) * 8);
}
__device__ __forceinline__ unsigned row_off(int k) { return (unsigned)row_of(k) * 8u; }

// Plain global accessors (global address space) for the few non-row accesses.
typedef __attribute__((address_space(1))) const double gcdouble;
__device__ __forceinline__ double ld(const double *__restrict__ base, unsigned idx) {
    return *(gcdouble *)((__attribute__((address_space(1))) const char *)base + (idx << 3));
}

// load_rows / store_rows / load_col / store_col / mkbuf take GLOBAL-memory vectors only; LDS
// vectors go through store_rows_lds and plain indexing.
template <int RMAX>
__device__ __forceinline__ void load_rows(const double *__restrict__ v, int n, double (&r)[RMAX]) {
    const rsrc_t b = mkbuf(v, n);
    const unsigned lo = lane_off();
#pragma unroll
    for (int k = 0; k < RMAX; ++k) r[k] = bld(b, lo, row_soff(k));
}

template <int RMAX>
__device__ __forceinline__ void store_rows(double *__restrict__ v, int n, const double (&r)[RMAX]) {
    const rsrc_t b = mkbuf(v, n);
    const unsigned lo = lane_off();
#pragma unroll
    for (int k = 0; k < RMAX; ++k) bst(b, lo, r[k], row_soff(k));
}

template <int RMAX>
__device__ __forceinline__ double dot_rows(const double (&a)[RMAX], const double (&b)[RMAX]) {
    // two interleaved partial sums halve the dependent FMA chain
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        s0 += a[k] * b[k];
        if (k + 1 < RMAX) s1 += a[k + 1] * b[k + 1];
    }
    return s0 + s1;
}

// Basis columns have leading dimension ldv = roundup(n + 1, 8) and zeros in rows n..ldv-1, so a
// column is read and written in row pairs over its ldv rows (a pair never straddles ldv).
__device__ __forceinline__ int ldv_for(int n) { return (n + 8) & ~7; }

template <int RMAX>
__device__ __forceinline__ void load_buf(rsrc_t b, double (&r)[RMAX]) {
    const unsigned lo = lane_off();
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        const double2_t v = bld2(b, lo, row_soff(k));
        r[k] = v[0];
        r[k + 1] = v[1];
    }
}

// FP32 columns (the discarded Krylov basis of mixed-precision solves): a row pair is one 8-byte
// access; values are widened to FP64 on load and rounded to FP32 on store.
template <int RMAX>
__device__ __forceinline__ void load_buf_f32(rsrc_t b, double (&r)[RMAX]) {
    const unsigned lo = threadIdx.x * 8u;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        const f32x2_t v = bldf2(b, lo, (unsigned)(k * kNT * 4));
        r[k] = (double)v[0];
        r[k + 1] = (double)v[1];
    }
}

template <int RMAX>
__device__ __forceinline__ void store_col_f32(float *__restrict__ v, int ldv,
                                              const double (&r)[RMAX]) {
    const rsrc_t b = mkbuf32(v, ldv);
    const unsigned lo = threadIdx.x * 8u;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2)
        __builtin_amdgcn_raw_buffer_store_b64(
            __builtin_bit_cast(u32x2, f32x2_t{(float)r[k], (float)r[k + 1]}), b, lo,
            (unsigned)(k * kNT * 4), 0);
}

template <int RMAX>
__device__ __forceinline__ void load_col(const double *__restrict__ v, int ldv, double (&r)[RMAX]) {
    load_buf<RMAX>(mkbuf(v, ldv), r);
}

// Stores rows p < ldv (the rows past n carry zeros), keeping the column's zero padding.
template <int RMAX>
__device__ __forceinline__ void store_col(double *__restrict__ v, int ldv, const double (&r)[RMAX]) {
    const rsrc_t b = mkbuf(v, ldv);
    const unsigned lo = lane_off();
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) bst2(b, lo, r[k], r[k + 1], row_soff(k));
}

// Visits basis columns col(q), q = 0..nvisit-1 (col(q) = q mod ncols), with a ring of D columns
// in flight: the loads for visit q+D are issued as soon as visit q has consumed its buffer, so
// memory latency overlaps the per-column work (the reductions of modified Gram-Schmidt are
// sequential in q).  The refill is issued unconditionally -- past the last visit it goes through
// a zero-size descriptor, which returns zeros without touching memory -- so every path through
// the loop has the same loads outstanding and the waits stay partial.  f(q, column) must not
// access global memory.
template <int RMAX, bool F32>
__device__ __forceinline__ void load_col_any(const void *V, int c, int ldv, bool live,
                                             double (&r)[RMAX]) {
    if constexpr (F32)
        load_buf_f32<RMAX>(mkbuf32((const float *)V + (size_t)c * ldv, live ? ldv : 0), r);
    else
        load_buf<RMAX>(mkbuf((const double *)V + (size_t)c * ldv, live ? ldv : 0), r);
}

// F32: the columns are stored in FP32 (mixed-precision Krylov basis).
template <int RMAX, int D, bool F32 = false, typename F>
__device__ __forceinline__ void sweep_cols(const void *__restrict__ V, int ldv, int ncols,
                                           int nvisit, F &&f) {
    double buf[D][RMAX];
#pragma unroll
    for (int d = 0; d < D; ++d) {
        const int c = d < ncols ? d : d % ncols;
        load_col_any<RMAX, F32>(V, c, ldv, d < nvisit, buf[d]);
    }
    for (int q0 = 0; q0 < nvisit; q0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int q = q0 + d;
            if (q < nvisit) f(q, buf[d]);
            const int qn = q + D;
            const int c = qn < ncols ? qn : (qn < 2 * ncols ? qn - ncols : 0);
            load_col_any<RMAX, F32>(V, c, ldv, qn < nvisit, buf[d]);
        }
    }
}

// Prefetch depth per rows-per-thread, bounded by the register budget of the variant.
template <int R> struct Depth { static constexpr int value = 2; };
template <> struct Depth<2> { static constexpr int value = 8; };
template <> struct Depth<4> { static constexpr int value = XKP_DEPTH4; };
template <> struct Depth<8> { static constexpr int value = XKP_DEPTH8; };
template <> struct Depth<16> { static constexpr int value = XKP_DEPTH16; };
template <> struct Depth<32> { static constexpr int value = XKP_DEPTH32; };

// Per-row off-diagonal coefficients of the operator (Section 2.3), in the workspace:
//   C_east  = -g^2/(2h^2) + f_x/(2h) - g^2/(8h^2) (m~_{i+1,j} - m~_{i-1,j})
//   C_west  = -g^2/(2h^2) - f_x/(2h) + g^2/(8h^2) (m~_{i+1,j} - m~_{i-1,j})
//   C_north = -g^2/(2h^2) + f_y/(2h) - g^2/(8h^2) (m~_{i,j+1} - m~_{i,j-1})
//   C_south = -g^2/(2h^2) - f_y/(2h) + g^2/(8h^2) (m~_{i,j+1} - m~_{i,j-1})
// (m~ and f zero outside the grid).  Systems of up to 4096 unknowns (whose workspace stays in the
// caches) keep the four coefficients: a coefficient whose neighbour lies outside the grid is
// stored as zero, and rows n <= p < npad are zero, so the stencil needs no boundary branches.
// Larger systems, whose launches stream from HBM, keep only the antisymmetric parts ex, ey (in
// the E and W arrays, zero for rows p >= n) and the stencil forms the four coefficients from
// them (coeffs_of): 16 bytes of coefficients per row and operator application instead of 32.
// Mixed precision keeps FP32 copies the same way: the four coefficients rounded to FP32, or the
// two parts rounded to FP32 with the coefficients formed in FP32 (coeffs_of_f32; 8 bytes per
// row instead of 16).  C_diag is the same for every row and stays a scalar.
struct Coef {
    double *E, *W, *N, *S;
    float *E32, *W32, *N32, *S32;   // FP32 copies (mixed precision)
};

// Whether systems of the row class RMAX keep ex, ey instead of the four coefficients.
template <int RMAX>
constexpr bool kDriftCoef = RMAX * kNT > 4096;

template <int RMAX>
__device__ void build_coeffs(const xkp_system &s, const OpConst &o, const Coef &C, bool mixed) {
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = row_of(k);
        double ex = 0.0, ey = 0.0;
        if (p < o.n) row_drift(s, o, p, ex, ey);
        double cE, cW, cN, cS;
        coeffs_of(o, p, ex, ey, cE, cW, cN, cS);
        const unsigned off = (unsigned)p * 8u;
        if constexpr (kDriftCoef<RMAX>) {
            bst(mkbuf(C.E, kNT * RMAX), off, ex);
            bst(mkbuf(C.W, kNT * RMAX), off, ey);
        } else {
            bst(mkbuf(C.E, kNT * RMAX), off, cE);
            bst(mkbuf(C.W, kNT * RMAX), off, cW);
            bst(mkbuf(C.N, kNT * RMAX), off, cN);
            bst(mkbuf(C.S, kNT * RMAX), off, cS);
        }
        if (mixed) {
            const unsigned o4 = (unsigned)p * 4u;
            if constexpr (kDriftCoef<RMAX>) {
                bstf(mkbuf32(C.E32, kNT * RMAX), o4, (float)ex);
                bstf(mkbuf32(C.W32, kNT * RMAX), o4, (float)ey);
            } else {
                bstf(mkbuf32(C.E32, kNT * RMAX), o4, (float)cE);
                bstf(mkbuf32(C.W32, kNT * RMAX), o4, (float)cW);
                bstf(mkbuf32(C.N32, kNT * RMAX), o4, (float)cN);
                bstf(mkbuf32(C.S32, kNT * RMAX), o4, (float)cS);
            }
        }
    }
}

// w = A u with u in LDS, zero-padded by at least one grid column (+1) on both sides: every
// neighbour read is in bounds and unconditional (the coefficient is 0 where the neighbour lies
// outside the grid), so each neighbour needs one address register, rows differing by an
// immediate offset.
template <int RMAX>
__device__ __forceinline__ void stencil_lds(const double *u, const Coef &C, const OpConst &o,
                                            double (&w)[RMAX]) {
    const int H = o.H;
    const double *uc = u + 2 * threadIdx.x;
    const rsrc_t bE = mkbuf(C.E, kNT * RMAX), bW = mkbuf(C.W, kNT * RMAX);
    const rsrc_t bN = mkbuf(C.N, kNT * RMAX), bS = mkbuf(C.S, kNT * RMAX);
    const unsigned lo = lane_off();
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        // rows q[0], q[1] of the pair; q[-1] and q[2] are their south and north neighbours
        const unsigned so = row_soff(k);
        const double *q = uc + k * kNT;
        double2_t cE, cW, cN, cS;
        if constexpr (kDriftCoef<RMAX>) {
            const double2_t ex = bld2(bE, lo, so), ey = bld2(bW, lo, so);
            const int p = row_of(k);
            double e0, w0, n0, s0, e1, w1, n1, s1;
            coeffs_of(o, p, ex[0], ey[0], e0, w0, n0, s0);
            coeffs_of(o, p + 1, ex[1], ey[1], e1, w1, n1, s1);
            cE = double2_t{e0, e1};
            cW = double2_t{w0, w1};
            cN = double2_t{n0, n1};
            cS = double2_t{s0, s1};
        } else {
            cE = bld2(bE, lo, so);
            cW = bld2(bW, lo, so);
            cN = bld2(bN, lo, so);
            cS = bld2(bS, lo, so);
        }
        const double2_t u0 = *(const double2_t *)q;
        w[k] = o.cd * u0[0] + cE[0] * q[H] + cW[0] * q[-H] + cN[0] * u0[1] + cS[0] * q[-1];
        w[k + 1] = o.cd * u0[1] + cE[1] * q[H + 1] + cW[1] * q[1 - H] + cN[1] * q[2] + cS[1] * u0[0];
        // bound the scheduling region: issuing every row's loads at once needs more registers
        // than the kernel has while the basis prefetch is in flight
        if (XKP_STENCIL_GROUP > 0 && (k / 2) % XKP_STENCIL_GROUP == XKP_STENCIL_GROUP - 1)
            __builtin_amdgcn_sched_barrier(0);
    }
}

// The same operator in FP32 (mixed precision): coefficients and the five values of u rounded to
// FP32, the row's sum formed in FP32, the result widened to FP64.
template <int RMAX>
__device__ __forceinline__ void stencil_lds_f32(const double *u, const Coef &C, const OpConst &o,
                                                double (&w)[RMAX]) {
    const int H = o.H;
    const float cd = (float)o.cd;
    const double *uc = u + 2 * threadIdx.x;
    const rsrc_t bE = mkbuf32(C.E32, kNT * RMAX), bW = mkbuf32(C.W32, kNT * RMAX);
    const rsrc_t bN = mkbuf32(C.N32, kNT * RMAX), bS = mkbuf32(C.S32, kNT * RMAX);
    const unsigned lo = threadIdx.x * 8u;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        const unsigned so = (unsigned)(k * kNT * 4);
        const double *q = uc + k * kNT;
        f32x2_t cE, cW, cN, cS;
        if constexpr (kDriftCoef<RMAX>) {
            const f32x2_t ex = bldf2(bE, lo, so), ey = bldf2(bW, lo, so);
            const int p = row_of(k);
            float e0, w0, n0, s0, e1, w1, n1, s1;
            coeffs_of_f32(o, p, ex[0], ey[0], e0, w0, n0, s0);
            coeffs_of_f32(o, p + 1, ex[1], ey[1], e1, w1, n1, s1);
            cE = f32x2_t{e0, e1};
            cW = f32x2_t{w0, w1};
            cN = f32x2_t{n0, n1};
            cS = f32x2_t{s0, s1};
        } else {
            cE = bldf2(bE, lo, so);
            cW = bldf2(bW, lo, so);
            cN = bldf2(bN, lo, so);
            cS = bldf2(bS, lo, so);
        }
        const double2_t u0 = *(const double2_t *)q;
        const float y0 = cd * (float)u0[0] + cE[0] * (float)q[H] + cW[0] * (float)q[-H]
                         + cN[0] * (float)u0[1] + cS[0] * (float)q[-1];
        const float y1 = cd * (float)u0[1] + cE[1] * (float)q[H + 1] + cW[1] * (float)q[1 - H]
                         + cN[1] * (float)q[2] + cS[1] * (float)u0[0];
        w[k] = (double)y0;
        w[k + 1] = (double)y1;
        if (XKP_STENCIL_GROUP > 0 && (k / 2) % XKP_STENCIL_GROUP == XKP_STENCIL_GROUP - 1)
            __builtin_amdgcn_sched_barrier(0);
    }
}

// BF16 copy of a column (rows p < ldv), 2-byte elements, one 4-byte store per row pair.
template <int RMAX>
__device__ __forceinline__ void store_col_bf16(unsigned short *v, int ldv, const double (&r)[RMAX]) {
    const rsrc_t b = mkbuf16(v, ldv);
    const unsigned lo = threadIdx.x * 4u;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) {
        const unsigned pair = (unsigned)to_bf16(r[k]) | ((unsigned)to_bf16(r[k + 1]) << 16);
        __builtin_amdgcn_raw_buffer_store_b32(pair, b, lo, (unsigned)(k * kNT * 2), 0);
    }
}

// The operator with coefficients formed on the fly from m~ (no workspace; residual and apply).
template <int RMAX>
__device__ __forceinline__ void stencil_direct(const double *u, const xkp_system &s,
                                               const OpConst &o, double (&w)[RMAX]) {
    const int H = o.H;
    const double *__restrict__ mt = s.mt;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = row_of(k);
        double r = 0.0;
        if (p < o.n) {
            const int i = p / H, j = p - (p / H) * H;
            const bool e = i + 1 < H, wv = i > 0, nn = j + 1 < H, ss = j > 0;
            const double ex = (s.fx ? ld(s.fx, p) : 0.0) * o.inv2h
                              - o.c8 * ((e ? ld(mt, p + H) : 0.0) - (wv ? ld(mt, p - H) : 0.0));
            const double ey = (s.fy ? ld(s.fy, p) : 0.0) * o.inv2h
                              - o.c8 * ((nn ? ld(mt, p + 1) : 0.0) - (ss ? ld(mt, p - 1) : 0.0));
            const double uE = e ? u[p + H] : 0.0;
            const double uW = wv ? u[p - H] : 0.0;
            const double uN = nn ? u[p + 1] : 0.0;
            const double uS = ss ? u[p - 1] : 0.0;
            r = o.cd * u[p] + (-o.a + ex) * uE + (-o.a - ex) * uW + (-o.a + ey) * uN
                + (-o.a - ey) * uS;
        }
        w[k] = r;
    }
}

// All rows (including the zero rows past n) into the padded LDS vector.
template <int RMAX>
__device__ __forceinline__ void store_rows_lds(double *v, const double (&r)[RMAX]) {
    double *vc = v + 2 * threadIdx.x;
#pragma unroll
    for (int k = 0; k < RMAX; k += 2) *(double2_t *)(vc + k * kNT) = double2_t{r[k], r[k + 1]};
}


// ----------------------------------------------------------------------------------------
// LDS layout of the GMRES kernel: vbuf[nlds] | Rp[kMMax*(kMMax+1)/2] | cs | sn | gv | h1 | yv | red
struct GmresLds {
    double *vbuf, *Rp, *cs, *sn, *gv, *h1, *h2, *yv, *red, *ext;
    __device__ GmresLds(double *base, int nlds, int npad) {
        vbuf = base + (nlds - npad) / 2;   // front pad
        Rp = base + nlds;
        cs = Rp + kMMax * (kMMax + 1) / 2;
        sn = cs + kMMax;
        gv = sn + kMMax;
        h1 = gv + kMMax + 1;
        h2 = h1 + kMMax + 1;
        yv = h2 + kMMax + 1;
        red = yv + kMMax;
        ext = red + 2 * kRedSlots * kNW;
    }
};

__device__ __forceinline__ int tri(int c) { return c * (c + 1) / 2; }

// LDS of the delayed-reorthogonalisation cycle (arnoldi_dcgs2), after the GMRES layout:
//   hbar  unrotated Hessenberg matrix of the cycle, column-major, leading dimension kLdH
//   part  per-row partial sums of one step's 2j + 2 inner products (value-major, 4 kNW each:
//         the 16-lane rows of every wave)
//   tot   their workgroup sums: tot[2i] = v_i.u, tot[2i+1] = v_i.z (i < j), then u.u, u.z
//   f     coefficients of the next pending vector; sc: broadcast scalars and flags
constexpr int kLdH = kMMax + 1;
constexpr int kDcgsParts = 4 * kNW;   // partial sums per value
constexpr int kDcgsDoubles =
    kLdH * kMMax + (2 * kMMax + 2) * kDcgsParts + (2 * kMMax + 2) + kLdH + 4;
struct DcgsLds {
    double *hbar, *part, *tot, *f, *sc;
    __device__ explicit DcgsLds(double *ext) {
        hbar = ext;
        part = hbar + kLdH * kMMax;
        tot = part + (2 * kMMax + 2) * kDcgsParts;
        f = tot + 2 * kMMax + 2;
        sc = f + kLdH;
    }
};

// The kept first cycle of a seed by Arnoldi with delayed classical Gram-Schmidt and
// re-orthogonalisation (DCGS2: A. Bielich, J. Langou, S. Thomas, K. Swirydowicz, I. Yamazaki and
// E. G. Boman, Parallel Computing 112, 2022), which gives the orthonormal basis and Hessenberg
// matrix of two Gram-Schmidt passes with ONE workgroup reduction per step instead of one per
// basis column.  Step j holds the pending vector u = A v_{j-1} - V_j g (orthogonalised once,
// unnormalised; g = its first-pass coefficients) and forms z = A u; one sweep over v_0..v_{j-1}
// and one reduction give c = V_j^T u, b = V_j^T z, u.u and u.z.  Then
//   beta = sqrt(u.u - c.c),  v_j = (u - V_j c) / beta,  H[0..j-1][j-1] = g + c,  H[j][j-1] = beta
// (the second pass of column j-1), and since A V_j = V_{j+1} Hbar_j, with e = Hbar_j c:
//   A v_j = (z - V_{j+1} e) / beta,   g'_i = (b_i - e_i) / beta (i < j),
//   g'_j = ((u.z - c.b) / beta - e_j) / beta,   next u = z / beta - V_{j+1} (e / beta + g')
// (the first pass of column j, without a reduction of its own).  One more sweep updates both
// vectors.  Step 0 starts from the normalised v_0 (beta = 1, no correction).  Column j-1 gets its
// Givens rotation as soon as it is final (wave 1, while wave 0 forms e and the coefficients);
// the cycle stops at the tolerance, a breakdown or mc columns.  u holds v_0 on entry (also in L.vbuf); returns the column count k, with v_0..v_k,
// Hbar (also in Hb and, for the mixed-precision seed, the BF16 copy) written as gmres_one's own
// cycle writes them.
template <int RMAX>
__device__ __forceinline__ int arnoldi_dcgs2(const Coef &C, const OpConst &o, double *V, int ldv,
                                             int mc, int m, double *Hb, unsigned short *Vb,
                                             double tol_abs, GmresLds &L, double (&u)[RMAX],
                                             double (&z)[RMAX], double &gcur, int &iters) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const DcgsLds D(L.ext);
    int *flg = (int *)(D.sc + 2);
    // wave 1, lane i: the rotation of row i (set when column i is final)
    double cs_r = 1.0, sn_r = 0.0;
    const int slot = wave * 4 + (lane >> 4);   // this lane's row partial, written by row lane 0
    const bool row_lead = (lane & 15) == 0;
    for (int j = 0;; ++j) {
        const bool have_z = j < mc;
        if (have_z) stencil_lds<RMAX>(L.vbuf, C, o, z);
        // sweep A: the step's inner products, summed per 16-lane row (no barrier per column)
        if (j > 0) {
            sweep_cols<RMAX, Depth<RMAX>::value>(V, ldv, j, j,
                [&](int i, const double(&col)[RMAX]) {
                const double pa = row_sum16(dot_rows<RMAX>(col, u));
                const double pb = have_z ? row_sum16(dot_rows<RMAX>(col, z)) : 0.0;
                if (row_lead) {
                    D.part[(2 * i) * kDcgsParts + slot] = pa;
                    D.part[(2 * i + 1) * kDcgsParts + slot] = pb;
                }
            });
        }
        {
            const double puu = row_sum16(dot_rows<RMAX>(u, u));
            const double puz = have_z ? row_sum16(dot_rows<RMAX>(u, z)) : 0.0;
            if (row_lead) {
                D.part[(2 * j) * kDcgsParts + slot] = puu;
                D.part[(2 * j + 1) * kDcgsParts + slot] = puz;
            }
        }
        lds_barrier();
        for (int t = tid; t < 2 * j + 2; t += kNT)
            D.tot[t] = tree_sum<kDcgsParts>(D.part + t * kDcgsParts);
        lds_barrier();
        if (wave < 2) {
            // waves 0 and 1 both form beta and the breakdown test from the same sums (the
            // same values); wave 0 then builds e, g' and f, wave 1 the rotations
            const double uu = D.tot[2 * j], uz = D.tot[2 * j + 1];
            double beta = 1.0;
            int brk = 0;
            // lane l < j holds c_l, b_l and the first-pass g_l of column j-1 (j <= 64); the
            // first-pass coefficients alternate between h1 and h2 by step, so that wave 0's
            // new ones never overwrite those wave 1 still reads
            double *g_in = (j & 1) ? L.h2 : L.h1, *g_out = (j & 1) ? L.h1 : L.h2;
            const double cl = lane < j ? D.tot[2 * lane] : 0.0;
            const double bl = lane < j ? D.tot[2 * lane + 1] : 0.0;
            const double gl = lane < j ? g_in[lane] : 0.0;
            const double hl = gl + cl;
            if (j > 0) {
                const double cc = wave_sum(cl * cl), gg = wave_sum(gl * gl);
                const double gc = wave_sum(gl * cl);
                beta = sqrt(fmax(uu - cc, 0.0));
                const double wn0 = sqrt(fmax(uu + gg + 2.0 * gc, 0.0));   // ||A v_{j-1}||
                brk = !(beta > 1e-14 * wn0);
            }
            if (wave == 0) {
                if (j > 0) {
                    // column j-1 of Hbar: rows < j from both passes, row j the new norm
                    if (lane < j) D.hbar[(j - 1) * kLdH + lane] = hl;
                    if (lane == 0) D.hbar[(j - 1) * kLdH + j] = beta;
                }
                wave_lds_sync();   // the column above before the reads below
                // e = Hbar_j c in four independent partial sums (lane i holds row i: j < 64
                // unless the cycle stops at this step, when e is not used; entries of column
                // l below row l + 1 are not read), then g' and f
                const double cb = wave_sum(cl * bl);
                const int i = lane;
                double e4[4] = {0.0, 0.0, 0.0, 0.0};
                for (int l0 = 0; l0 < j; l0 += 4) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int l = l0 + q;
                        if (l < j && l + 1 >= i) e4[q] += D.hbar[l * kLdH + i] * D.tot[2 * l];
                    }
                }
                const double e = (e4[0] + e4[1]) + (e4[2] + e4[3]);
                if (i <= j) {
                    const double rb = 1.0 / beta;
                    const double gp = i < j ? (bl - e) * rb : ((uz - cb) * rb - e) * rb;
                    g_out[i] = gp;
                    D.f[i] = e * rb + gp;
                }
                if (lane == 0) {
                    D.sc[0] = beta;
                    flg[1] = brk;
                }
            } else {
                int stop = 0;
                if (j > 0) {
                    for (int r = lane; r <= m; r += 64)
                        Hb[(size_t)(j - 1) * (m + 1) + r] = r < j ? hl : (r == j ? beta : 0.0);
                    // Givens rotations of the earlier columns (lane-held), then the new one;
                    // lane i - 1 writes the rotated entry of row i - 1
                    double t = readlane_d(hl, 0);
                    for (int i = 1; i < j; ++i) {
                        const double c = readlane_d(cs_r, i - 1), sn = readlane_d(sn_r, i - 1);
                        const double hi = readlane_d(hl, i);
                        const double rr = c * t + sn * hi;
                        t = -sn * t + c * hi;
                        if (lane == i - 1) L.Rp[tri(j - 1) + i - 1] = rr;
                    }
                    const double den = sqrt(t * t + beta * beta), rden = 1.0 / den;
                    const double cj = t * rden, sj = beta * rden;
                    if (lane == j - 1) {
                        cs_r = cj;
                        sn_r = sj;
                    }
                    if (lane == 0) {
                        L.Rp[tri(j - 1) + j - 1] = den;
                        L.gv[j - 1] = cj * gcur;
                    }
                    gcur = -sj * gcur;
                    stop = (fabs(gcur) <= tol_abs || brk || j == mc) ? 1 : 0;
                }
                if (lane == 0) {
                    D.sc[1] = gcur;
                    flg[0] = stop;
                }
            }
        }
        lds_barrier();
        const double beta = D.sc[0];
        gcur = D.sc[1];
        const bool stop = __builtin_amdgcn_readfirstlane(flg[0]) != 0;
        const bool brk = __builtin_amdgcn_readfirstlane(flg[1]) != 0;
        const double rbeta = 1.0 / beta;   // one division, then products per row
        if (j > 0) ++iters;
        // sweep B: u - V_j c (-> v_j) and z / beta - V_j f (-> the next pending vector)
        if (!stop) {
#pragma unroll
            for (int k = 0; k < RMAX; ++k) z[k] = z[k] * rbeta;
        }
        if (j > 0) {
            // each column's two coefficients are read one column ahead
            double cn = D.tot[0], fn = stop ? 0.0 : D.f[0];
            sweep_cols<RMAX, Depth<RMAX>::value>(V, ldv, j, j,
                [&](int i, const double(&col)[RMAX]) {
                const double ci = cn, fi = fn;
                if (i + 1 < j) {
                    cn = D.tot[2 * (i + 1)];
                    if (!stop) fn = D.f[i + 1];
                }
#pragma unroll
                for (int k = 0; k < RMAX; ++k) u[k] -= ci * col[k];
                if (!stop) {
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) z[k] -= fi * col[k];
                }
            });
#pragma unroll
            for (int k = 0; k < RMAX; ++k) u[k] = brk ? 0.0 : u[k] * rbeta;
            store_col<RMAX>(V + (size_t)j * ldv, ldv, u);
            if (Vb) store_col_bf16<RMAX>(Vb + (size_t)j * ldv, ldv, u);
        }
        if (stop) return j;
        const double fj = D.f[j];
#pragma unroll
        for (int k = 0; k < RMAX; ++k) u[k] = z[k] - fj * u[k];
        store_rows_lds<RMAX>(L.vbuf, u);
        lds_barrier();
    }
}

// ----------------------------------------------------------------------------------------
// GMRES with the Krylov basis in registers (cycles whose basis is discarded: target polish and
// plain GMRES, systems of up to 8 rows per thread).  Each thread keeps its rows of the cycle's
// basis vectors, so the Gram-Schmidt sweeps read no memory at all; the two Gram-Schmidt passes
// are classical (CGS2: all inner products of a pass in one workgroup reduction, two reductions
// per Arnoldi step instead of one per basis column), and the norm of the twice-orthogonalised
// vector follows from the second pass's reduction, ||w2||^2 = ||w1||^2 - ||V^T w1||^2 (the
// second correction is of the order of the unit roundoff, so there is no cancellation).  Two
// classical passes give an orthonormal basis to working precision, as two modified passes do.

// Columns the register path holds at R rows per thread (2 R registers each), by workgroup
// size: what fits the per-lane register budget (256 at two waves per SIMD, 512 with the
// accumulation registers at one) next to the rest of the cycle without spilling to memory.
// Sixteen-wave workgroups (128 registers per lane) have no register path.
template <int R> struct RegCols { static constexpr int value = 0; };
#if XKP_NT == 512
template <> struct RegCols<2> { static constexpr int value = 9; };
template <> struct RegCols<8> { static constexpr int value = 7; };
#elif XKP_NT == 256
template <> struct RegCols<4> { static constexpr int value = 16; };
template <> struct RegCols<16> { static constexpr int value = 10; };
#endif
constexpr int kWideMax = 26;   // values reduced together by WideRed (>= every RegCols + 2)

// Workgroup sum of up to kWideMax values at once, one barrier: `red` is LDS of
// 2 * kWideMax * kNW doubles, halves alternating between calls.  Only the first nv values are
// summed (nv a compile-time constant after unrolling in the callers).
struct WideRed {
    double *red;
    int par;
    template <int NV>
    __device__ __forceinline__ void sum(double (&v)[NV], int nv) {
        double *slot = red + par * (kWideMax * kNW);
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            if (q < nv) {
                const double t = wave_sum(v[q]);
                if ((threadIdx.x & 63) == 0) slot[q * kNW + (threadIdx.x >> 6)] = t;
            }
        }
        lds_barrier();
#pragma unroll
        for (int q = 0; q < NV; ++q)
            if (q < nv) v[q] = tree_sum<kNW>(slot + q * kNW);
        par ^= 1;
    }
};

// One cycle's Arnoldi steps with the basis in registers.  The steps are instantiated one by one
// (step<J> calls step<J + 1>), so every basis column is addressed by a compile-time index and
// the array stays in registers.
template <int RMAX, bool MIXED, int MC>
struct RegCycle {
    typedef double vt;   // mixed precision stores FP32-rounded values (the FP32 basis)
    vt (&V)[MC][RMAX];
    double (&w)[RMAX];
    const Coef &C;
    const OpConst &o;
    GmresLds &L;
    WideRed &wr;
    int mc;            // steps allowed in this cycle
    double tol_abs;    // stop when the residual estimate reaches max(tol_abs, gfloor)
    double gfloor;
    double gcur;
    int kk, iters;

    template <int J>
    __device__ __forceinline__ void step() {
        if constexpr (J < MC - 1) {
            if (J >= mc) return;
            const int tid = threadIdx.x;
            if constexpr (MIXED)
                stencil_lds_f32<RMAX>(L.vbuf, C, o, w);
            else
                stencil_lds<RMAX>(L.vbuf, C, o, w);
            ++iters;
            // pass 1: h1 = V_{J+1}^T w and ||w||^2 in one reduction
            double d[J + 2];
#pragma unroll
            for (int i = 0; i <= J; ++i) {
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int k = 0; k < RMAX; k += 2) {
                    a0 += (double)V[i][k] * w[k];
                    a1 += (double)V[i][k + 1] * w[k + 1];
                }
                d[i] = a0 + a1;
            }
            d[J + 1] = dot_rows<RMAX>(w, w);
            wr.template sum<J + 2>(d, J + 2);
            const double wn0 = sqrt(d[J + 1]);
            double h[J + 1];
#pragma unroll
            for (int i = 0; i <= J; ++i) {
                h[i] = d[i];
#pragma unroll
                for (int k = 0; k < RMAX; ++k) w[k] -= d[i] * (double)V[i][k];
            }
            // pass 2: h2 = V_{J+1}^T w1 and ||w1||^2 in one reduction
#pragma unroll
            for (int i = 0; i <= J; ++i) {
                double a0 = 0.0, a1 = 0.0;
#pragma unroll
                for (int k = 0; k < RMAX; k += 2) {
                    a0 += (double)V[i][k] * w[k];
                    a1 += (double)V[i][k + 1] * w[k + 1];
                }
                d[i] = a0 + a1;
            }
            d[J + 1] = dot_rows<RMAX>(w, w);
            wr.template sum<J + 2>(d, J + 2);
            double c2 = 0.0;
#pragma unroll
            for (int i = 0; i <= J; ++i) {
                h[i] += d[i];
                c2 += d[i] * d[i];
#pragma unroll
                for (int k = 0; k < RMAX; ++k) w[k] -= d[i] * (double)V[i][k];
            }
            const double hn = sqrt(fmax(d[J + 1] - c2, 0.0));
            const bool brk = !(hn > 1e-14 * wn0);
            const double rhn = brk ? 0.0 : 1.0 / hn;
#pragma unroll
            for (int k = 0; k < RMAX; ++k) {
                w[k] = MIXED ? (double)(float)(w[k] * rhn) : w[k] * rhn;
                V[J + 1][k] = w[k];
            }
            // Givens rotations of column J (every thread holds the same values)
            double t = h[0];
#pragma unroll
            for (int i = 1; i <= J; ++i) {
                const double c = L.cs[i - 1], sn = L.sn[i - 1];
                const double rr = c * t + sn * h[i];
                t = -sn * t + c * h[i];
                if (tid == 0) L.Rp[tri(J) + i - 1] = rr;
            }
            const double den = sqrt(t * t + hn * hn);
            const double rden = 1.0 / den;
            const double cj = t * rden, sj = hn * rden;
            if (tid == 0) {
                L.Rp[tri(J) + J] = den;
                L.cs[J] = cj;
                L.sn[J] = sj;
                L.gv[J] = cj * gcur;
            }
            gcur = -sj * gcur;
            kk = J + 1;
            // the next operator application reads the new vector's neighbours
            store_rows_lds<RMAX>(L.vbuf, w);
            lds_barrier();
            if (fabs(gcur) <= fmax(tol_abs, gfloor) || brk) return;
            step<J + 1>();
        }
    }

    // x += V_k y (y in LDS)
    template <int J>
    __device__ __forceinline__ void add_to(double (&x)[RMAX]) {
        if constexpr (J < MC - 1) {
            if (J >= kk) return;
            const double yc = L.yv[J];
#pragma unroll
            for (int k = 0; k < RMAX; ++k) x[k] += yc * (double)V[J][k];
            add_to<J + 1>(x);
        }
    }
};

template <int RMAX, bool MIXED, int MC>
__device__ __forceinline__ void gmres_reg(const xkp_system &s, const xkp_params &P, int flags,
                                          int prestatus, int gsrc, const Coef &C, xkp_info *info,
                                          GmresLds &L) {
    typedef double vt;
    const OpConst o = op_const(s);
    const int n = o.n, mpol = P.polish_m > 0 ? P.polish_m : P.m;
    const int tid = threadIdx.x;
    BlockRed br{L.red, 0};
    WideRed wr{L.ext, 0};
    constexpr bool mixed = MIXED;

    build_coeffs<RMAX>(s, o, C, mixed);
    vt V[MC][RMAX];   // this thread's rows of the cycle's basis vectors
    double w[RMAX], cur[RMAX];

    load_rows<RMAX>(s.b, n, cur);
    const double bnorm = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
    int iters = 0, restarts = 0, status = XKP_OK;
    double res_est = 0.0, res_true = 0.0, guess = 0.0;

    if (bnorm == 0.0) {
#pragma unroll
        for (int k = 0; k < RMAX; ++k) w[k] = 0.0;
        store_rows<RMAX>(s.x, n, w);
    } else {
        const double *xs = (flags & kStartFromX) ? s.x : s.x0;
        if (xs) {
            load_rows<RMAX>(xs, n, w);
            store_rows_lds<RMAX>(L.vbuf, w);
            if (xs != s.x) store_rows<RMAX>(s.x, n, w);
            lds_barrier();
            stencil_lds<RMAX>(L.vbuf, C, o, w);
#pragma unroll
            for (int k = 0; k < RMAX; ++k) cur[k] -= w[k];
        } else {
#pragma unroll
            for (int k = 0; k < RMAX; ++k) w[k] = 0.0;
            store_rows<RMAX>(s.x, n, w);
        }
        double beta = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
        guess = res_true = res_est = beta / bnorm;
        // data that are not finite (NaN or Inf in m~, f, b or x0) cannot be solved
        if (!isfinite(beta) || !isfinite(bnorm)) status = XKP_EINVAL;
        if (status == XKP_OK && beta > P.tol * bnorm) {
            for (;;) {
                // v_0 = r / beta (rounded to FP32 in mixed precision: the stored basis)
                const double rbeta = 1.0 / beta;
#pragma unroll
                for (int k = 0; k < RMAX; ++k) {
                    w[k] = mixed ? (double)(float)(cur[k] * rbeta) : cur[k] * rbeta;
                    V[0][k] = w[k];
                }
                store_rows_lds<RMAX>(L.vbuf, w);
                lds_barrier();
                RegCycle<RMAX, MIXED, MC> cy{V, w, C, o, L, wr, mpol, P.tol * bnorm,
                                             mixed ? kMixedCycleDrop * beta : 0.0, beta, 0,
                                             iters};
                cy.template step<0>();
                iters = cy.iters;
                const int kk = cy.kk;
                res_est = fabs(cy.gcur) / bnorm;
                // y = R^{-1} g by one wavefront (lane c holds g_c and 1 / R_cc)
                if (tid < 64) {
                    double gl = (tid < kk) ? L.gv[tid] : 0.0;
                    const double rdiag = (tid < kk) ? 1.0 / L.Rp[tri(tid) + tid] : 0.0;
                    for (int c = kk - 1; c >= 0; --c) {
                        const double yc = readlane_d(gl, c) * readlane_d(rdiag, c);
                        if (tid < c) gl -= L.Rp[tri(c) + tid] * yc;
                        if (tid == 0) L.yv[c] = yc;
                    }
                }
                lds_barrier();
                // x += V_k y
                load_rows<RMAX>(s.x, n, w);
                cy.template add_to<0>(w);
                store_rows<RMAX>(s.x, n, w);
                store_rows_lds<RMAX>(L.vbuf, w);
                lds_barrier();
                // true residual in FP64
                stencil_lds<RMAX>(L.vbuf, C, o, w);
                load_rows<RMAX>(s.b, n, cur);
#pragma unroll
                for (int k = 0; k < RMAX; ++k) cur[k] -= w[k];
                beta = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
                res_true = beta / bnorm;
                if (beta <= P.tol * bnorm) break;
                if (!isfinite(beta)) {
                    status = XKP_EINVAL;   // the operator produced a non-finite value
                    break;
                }
                if (restarts >= P.max_restarts) {
                    status = XKP_ENOCONV;
                    break;
                }
                ++restarts;
            }
        }
    }
    if (tid == 0) {
        int st = status;
        if (st == XKP_OK && (flags & kTarget) && prestatus == XKP_ESINGULAR) st = XKP_ESINGULAR;
        info->status = st;
        info->iters = iters;
        info->restarts = restarts;
        if (!(flags & kTarget)) info->basis_dim = 0;
        info->res_est = res_est;
        info->res_true = res_true;
        info->guess_res = guess;
        info->guess_source = gsrc;
        info->pad = 0;
    }
    __syncthreads();
}

template <int RMAX, bool MIXED>
__device__ __forceinline__ void gmres_one(const xkp_system &s, const xkp_params &P, int flags,
                                          int prestatus, int gsrc,
                          xkp_basis_header *hdr, double *Vfirst, double *Hb, double *Vws,
                          const Coef &C, xkp_info *info, GmresLds &L) {
    const OpConst o = op_const(s);
    const bool keep = hdr != nullptr;
    // restart lengths: the kept first cycle of a seed has m = P.m steps (the basis dimension);
    // every other cycle (targets, plain GMRES, a seed's later cycles) has polish_m (0: m)
    const int n = o.n, m = P.m, mpol = P.polish_m > 0 ? P.polish_m : P.m;
    const int tid = threadIdx.x, ldv = ldv_for(o.n);
    BlockRed br{L.red, 0};
    // mixed precision: FP32 operator inside the Krylov cycles and the (discarded) Krylov basis
    // stored in FP32; Gram-Schmidt, rotations, updates and the restart residual in FP64
    constexpr bool mixed = MIXED;
    constexpr bool vf32 = MIXED;   // mixed-precision solves never keep their basis
    // a mixed-precision seed (solved with the FP64 operator) also writes the BF16 basis copy
    unsigned short *Vb = (keep && P.precision == XKP_MIXED)
                             ? (unsigned short *)((char *)hdr + basis_off_vb(n, m))
                             : nullptr;

    build_coeffs<RMAX>(s, o, C, mixed);
    if (keep) {
        for (int t = tid; t < (m + 1) * m; t += kNT) Hb[t] = 0.0;
        __syncthreads();   // thread 0 overwrites some of these entries later
    }
    double w[RMAX], cur[RMAX], nxt[RMAX];

    load_rows<RMAX>(s.b, n, cur);
    const double bnorm = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));

    int iters = 0, restarts = 0, kfirst = 0, status = XKP_OK;
    double res_est = 0.0, res_true = 0.0, guess = 0.0, beta_first = 0.0;

    if (bnorm == 0.0) {
#pragma unroll
        for (int k = 0; k < RMAX; ++k) w[k] = 0.0;
        store_rows<RMAX>(s.x, n, w);
    } else {
        // r0 = b - A x0
        const double *xs = (flags & kStartFromX) ? s.x : s.x0;
        if (xs) {
            load_rows<RMAX>(xs, n, nxt);
            store_rows_lds<RMAX>(L.vbuf, nxt);
            if (xs != s.x) store_rows<RMAX>(s.x, n, nxt);
            lds_barrier();
            stencil_lds<RMAX>(L.vbuf, C, o, w);
#pragma unroll
            for (int k = 0; k < RMAX; ++k) cur[k] -= w[k];
        } else {
#pragma unroll
            for (int k = 0; k < RMAX; ++k) nxt[k] = 0.0;
            store_rows<RMAX>(s.x, n, nxt);
        }
        double beta = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
        guess = res_true = res_est = beta / bnorm;
        bool first = true;
        // data that are not finite (NaN or Inf in m~, f, b or x0) cannot be solved
        if (!isfinite(beta) || !isfinite(bnorm)) status = XKP_EINVAL;
        if (status == XKP_OK && beta > P.tol * bnorm) {
            for (;;) {
                double *V = first ? Vfirst : Vws;
                // v_0 = r / beta (as stored); the LDS copy feeds the stencil
#pragma unroll
                for (int k = 0; k < RMAX; ++k)
                    cur[k] = vf32 ? (double)(float)(cur[k] / beta) : cur[k] / beta;
                if constexpr (vf32)
                    store_col_f32<RMAX>((float *)V, ldv, cur);
                else
                    store_col<RMAX>(V, ldv, cur);
                if (Vb && first) store_col_bf16<RMAX>(Vb, ldv, cur);
                store_rows_lds<RMAX>(L.vbuf, cur);
                if (first) beta_first = beta;
                lds_barrier();
                double gcur = beta;
                // With the FP32 operator a cycle cannot lower the true residual much below
                // kMixedCycleDrop times its start; the cycle ends there and the FP64 restart
                // takes over (the kept first cycle of a seed runs to m or the tolerance).
                const double gfloor =
                    (mixed && !(keep && first)) ? kMixedCycleDrop * beta : 0.0;
                const bool two_pass = (keep && first) || P.reorth == XKP_REORTH_ALWAYS;
                int kk = 0;
                const int mc = (keep && first) ? m : mpol;
                // the kept cycle of a launch flagged for it (systems of up to 4096 unknowns,
                // whose LDS has room for the Hessenberg copy) runs by DCGS2
                bool dcgs = false;
                if constexpr (!MIXED && RMAX * kNT <= 4096) {
                    if (keep && first && (flags & kDcgs)) {
                        kk = arnoldi_dcgs2<RMAX>(C, o, V, ldv, mc, m, Hb, Vb, P.tol * bnorm, L,
                                                 cur, w, gcur, iters);
                        res_est = fabs(gcur) / bnorm;
                        dcgs = true;
                    }
                }
                for (int j = 0; !dcgs && j < mc; ++j) {
                    if constexpr (mixed)
                        stencil_lds_f32<RMAX>(L.vbuf, C, o, w);
                    else
                        stencil_lds<RMAX>(L.vbuf, C, o, w);
                    ++iters;
                    const double wsq = dot_rows<RMAX>(w, w);
                    double wn0 = 0.0, t = 0.0;
                    // modified Gram-Schmidt over v_0..v_j: two passes as one sweep of 2(j+1)
                    // column visits while the basis is kept (the second pass re-orthogonalises
                    // and completes h_{i,j}), else one pass
                    const int nc = j + 1, nvis = two_pass ? 2 * nc : nc;
                    sweep_cols<RMAX, Depth<RMAX>::value, vf32>(V, ldv, nc, nvis,
                        [&](int q, const double(&col)[RMAX]) {
                        const int i = q < nc ? q : q - nc;
                        const double part = dot_rows<RMAX>(w, col);
                        double d;
                        if (q == 0) {
                            double two[2] = {part, wsq};
                            br.sum_multi<2>(two);
                            d = two[0];
                            wn0 = sqrt(two[1]);
                        } else {
                            d = br.sum(part);
                        }
#pragma unroll
                        for (int k = 0; k < RMAX; ++k) w[k] -= d * col[k];
                        if (q < nvis - nc) {
                            if (tid == 0) L.h1[i] = d;
                        } else {
                            // final h_{i,j}; fold the Givens rotations in as entries arrive
                            const double hf = two_pass ? L.h1[i] + d : d;
                            if (tid == 0) L.h2[i] = hf;
                            if (i == 0) {
                                t = hf;
                            } else {
                                const double c = L.cs[i - 1], sn = L.sn[i - 1];
                                const double rr = c * t + sn * hf;
                                t = -sn * t + c * hf;
                                if (tid == 0) L.Rp[tri(j) + i - 1] = rr;
                            }
                        }
                    });
                    const double hn = sqrt(br.sum(dot_rows<RMAX>(w, w)));
                    const bool brk = !(hn > 1e-14 * wn0);
                    const double rhn = 1.0 / hn;   // one division, then products per row
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) {
                        w[k] = brk ? 0.0 : w[k] * rhn;
                        if constexpr (vf32) w[k] = (double)(float)w[k];
                    }
                    if constexpr (vf32)
                        store_col_f32<RMAX>((float *)V + (size_t)(j + 1) * ldv, ldv, w);
                    else
                        store_col<RMAX>(V + (size_t)(j + 1) * ldv, ldv, w);
                    if (Vb && first) store_col_bf16<RMAX>(Vb + (size_t)(j + 1) * ldv, ldv, w);
                    store_rows_lds<RMAX>(L.vbuf, w);
                    if (keep && first) {
                        // unrotated Hessenberg column j of the kept basis
                        for (int r = tid; r <= m; r += kNT)
                            Hb[(size_t)j * (m + 1) + r] = r <= j ? L.h2[r] : (r == j + 1 ? hn : 0.0);
                    }
                    const double den = sqrt(t * t + hn * hn);
                    const double rden = 1.0 / den;
                    const double cj = t * rden, sj = hn * rden;
                    if (tid == 0) {
                        L.Rp[tri(j) + j] = den;
                        L.cs[j] = cj;
                        L.sn[j] = sj;
                        L.gv[j] = cj * gcur;
                    }
                    gcur = -sj * gcur;
                    kk = j + 1;
                    lds_barrier();
                    if (fabs(gcur) <= fmax(P.tol * bnorm, gfloor) || brk) break;
                }
                if (!dcgs) res_est = fabs(gcur) / bnorm;
                // y = R^{-1} g by one wavefront (lane c holds g_c and 1 / R_cc), column-oriented
                if (tid < 64) {
                    double gl = (tid < kk) ? L.gv[tid] : 0.0;
                    const double rdiag = (tid < kk) ? 1.0 / L.Rp[tri(tid) + tid] : 0.0;
                    for (int c = kk - 1; c >= 0; --c) {
                        const double yc = readlane_d(gl, c) * readlane_d(rdiag, c);
                        if (tid < c) gl -= L.Rp[tri(c) + tid] * yc;
                        if (tid == 0) L.yv[c] = yc;
                    }
                }
                lds_barrier();
                // x += V_k y
                load_rows<RMAX>(s.x, n, w);
                sweep_cols<RMAX, Depth<RMAX>::value, vf32>(V, ldv, kk, kk,
                    [&](int c, const double(&col)[RMAX]) {
                    const double yc = L.yv[c];
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) w[k] += yc * col[k];
                });
                store_rows<RMAX>(s.x, n, w);
                store_rows_lds<RMAX>(L.vbuf, w);
                if (first) {
                    kfirst = kk;
                    first = false;
                }
                lds_barrier();
                // true residual in FP64
                stencil_lds<RMAX>(L.vbuf, C, o, w);
                load_rows<RMAX>(s.b, n, cur);
#pragma unroll
                for (int k = 0; k < RMAX; ++k) cur[k] -= w[k];
                beta = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
                res_true = beta / bnorm;
                if (beta <= P.tol * bnorm) break;
                if (!isfinite(beta)) {
                    status = XKP_EINVAL;   // the operator produced a non-finite value
                    break;
                }
                if (restarts >= P.max_restarts) {
                    status = XKP_ENOCONV;
                    break;
                }
                ++restarts;
            }
        }
    }
    if (tid == 0) {
        if (keep) {
            hdr->n = n;
            hdr->m = m;
            hdr->k = kfirst;
            hdr->status = status;
            hdr->beta = beta_first;
            hdr->ldv = ldv;
            hdr->bf16 = Vb ? 1 : 0;
            hdr->kind = XKP_BASIS_ARNOLDI;
        }
        int st = status;
        if (st == XKP_OK && (flags & kTarget) && prestatus == XKP_ESINGULAR) st = XKP_ESINGULAR;
        info->status = st;
        info->iters = iters;
        info->restarts = restarts;
        if (keep) info->basis_dim = kfirst;
        else if (!(flags & kTarget)) info->basis_dim = 0;
        info->res_est = res_est;
        info->res_true = res_true;
        if (!(flags & kKeepBasis)) info->guess_res = guess;
        else info->guess_res = 1.0;
        info->guess_source = gsrc;
        info->pad = 0;
    }
    // no wave may start the next system (and overwrite LDS / workspace) while others still
    // read this one's values
    __syncthreads();
}

// ----------------------------------------------------------------------------------------
// Projection (Section 3, Phase 2)

// LU with partial pivoting of the kk x kk row-major LDS matrix A (leading dimension lda) by
// wavefront 0, lane r owning row r; zr is lane r's right-hand side entry.  Rows are not moved:
// the pivot of column c is the largest remaining |A[r][c]| (lowest lane on ties).  A pivot
// <= 1e-13 max|A| reports singular.  The solution goes to out[0..kk).
__device__ bool lu_solve_wave(double *A, int lda, int kk, double zr, double *out, int *pivl) {
    const int r = threadIdx.x;
    kk = __builtin_amdgcn_readfirstlane(kk);
    double rowmax = 0.0;
    if (r < kk)
        for (int q = 0; q < kk; ++q) rowmax = fmax(rowmax, fabs(A[r * lda + q]));
    const double amax = wave_max(rowmax);
    if (!(amax > 0.0)) return true;
    bool active = r < kk;
    int pc = 1 << 20;
    for (int c = 0; c < kk; ++c) {
        const double v = active ? fabs(A[r * lda + c]) : -1.0;
        const double vmax = wave_max(v);
        if (!(vmax > 1e-13 * amax)) return true;
        const unsigned long long bal = __ballot(active && v == vmax);
        const int pl = __ffsll(bal) - 1;
        if (r == pl) {
            active = false;
            pc = c;
        }
        if (r == 0) pivl[c] = pl;
        const double piv = A[pl * lda + c];
        const double zp = readlane_d(zr, pl);
        if (active) {
            const double l = A[r * lda + c] / piv;
            A[r * lda + c] = 0.0;
            // eight entries per round trip: all reads of a chunk before its writes, so the
            // reads do not wait for the previous entry's write
            for (int q0 = c + 1; q0 < kk; q0 += 8) {
                double pr[8], own[8];
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    const int q = q0 + t < kk ? q0 + t : kk - 1;
                    pr[t] = A[pl * lda + q];
                    own[t] = A[r * lda + q];
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (q0 + t < kk) A[r * lda + q0 + t] = own[t] - l * pr[t];
            }
            zr -= l * zp;
        }
        wave_lds_sync();
    }
    // the reciprocal of each pivot, in its row's lane (rows that were no pivot hold 0)
    const double rpiv = pc < kk ? 1.0 / A[r * lda + pc] : 0.0;
    for (int c = kk - 1; c >= 0; --c) {
        const int pl = __builtin_amdgcn_readfirstlane(pivl[c]);
        const double xc = readlane_d(zr, pl) * readlane_d(rpiv, pl);
        if (pc < c) zr -= A[r * lda + c] * xc;
        if (r == 0) out[c] = xc;
    }
    wave_lds_sync();
    return false;
}

// Partial [V_k^T W] over the 8-row groups g = wave, wave + kNW, ... for KTR row tiles and NTC
// column tiles starting at column tile tc0, FP64 matrix cores (v_mfma_f64_16x16x4: A 16x4 from
// lane i + 16 kk, B 4x16 from lane j + 16 kk).  Lane l loads rows 8g + 2(l/16) and the next one
// of its column in one 16-byte access; the group's first product takes the first of each pair
// (rows 8g, 8g+2, 8g+4, 8g+6 as kk = 0..3), the second the other rows: the same row for A and
// B in every product, 8 rows per load.  Each wave keeps all KTR x NTC accumulators; the
// operands of the next group are loaded before the current group's products.
template <int KTR, int NTC>
__device__ __forceinline__ void vtw_chunk(rsrc_t rV, rsrc_t rW, int n, int ldv, int k, int tc0,
                                          double *Ap, double *tred) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double4_t acc[KTR][NTC];
    unsigned offA[KTR], offB[NTC];
    bool okA[KTR], okB[NTC];
#pragma unroll
    for (int t = 0; t < KTR; ++t) {
        const int a = t * 16 + (lane & 15);
        okA[t] = a < k;
        offA[t] = (unsigned)(okA[t] ? a : 0) * (unsigned)ldv * 8u;
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
        const int c = (tc0 + t) * 16 + (lane & 15);
        okB[t] = c <= k;
        offB[t] = (unsigned)(okB[t] ? c : 0) * (unsigned)ldv * 8u;
    }
#pragma unroll
    for (int a = 0; a < KTR; ++a)
#pragma unroll
        for (int b = 0; b < NTC; ++b) acc[a][b] = double4_t{0.0, 0.0, 0.0, 0.0};
    // rows p, p + 1 lie inside the column (ldv is a multiple of 8 above n); rows at or past n
    // are zeroed
    const int ngroups = (n + 7) / 8;
    double2_t an[KTR], bn[NTC];
    int g = wave;
    {
        const unsigned po = (8u * g + 2u * (lane >> 4)) * 8u;
#pragma unroll
        for (int t = 0; t < KTR; ++t) an[t] = bld2(rV, offA[t] + po);
#pragma unroll
        for (int t = 0; t < NTC; ++t) bn[t] = bld2(rW, offB[t] + po);
    }
    for (; g < ngroups; g += kNW) {
        const unsigned p = 8u * g + 2u * (lane >> 4);
        const bool pin0 = p < (unsigned)n, pin1 = p + 1u < (unsigned)n;
        double2_t av[KTR], bv[NTC];
#pragma unroll
        for (int t = 0; t < KTR; ++t) {
            av[t][0] = (okA[t] && pin0) ? an[t][0] : 0.0;
            av[t][1] = (okA[t] && pin1) ? an[t][1] : 0.0;
        }
#pragma unroll
        for (int t = 0; t < NTC; ++t) {
            bv[t][0] = (okB[t] && pin0) ? bn[t][0] : 0.0;
            bv[t][1] = (okB[t] && pin1) ? bn[t][1] : 0.0;
        }
        // next group's operands (past the end: clamped to the last group, never used)
        const int gn = g + kNW < ngroups ? g + kNW : g;
        const unsigned pon = (8u * gn + 2u * (lane >> 4)) * 8u;
#pragma unroll
        for (int t = 0; t < KTR; ++t) an[t] = bld2(rV, offA[t] + pon);
#pragma unroll
        for (int t = 0; t < NTC; ++t) bn[t] = bld2(rW, offB[t] + pon);
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int a = 0; a < KTR; ++a)
#pragma unroll
                for (int b = 0; b < NTC; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a][h], bv[b][h],
                                                                      acc[a][b], 0, 0, 0);
    }
    // reduce each tile over the waves in a fixed order; lane l, register r holds
    // D[4r + l/16][l%16] of the 16x16 tile
#pragma unroll
    for (int ta = 0; ta < KTR; ++ta) {
#pragma unroll
        for (int tb = 0; tb < NTC; ++tb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tred[wave * 256 + lane * 4 + r] = acc[ta][tb][r];
            lds_barrier();
            // the 256 entries of the tile, strided over the workgroup
            for (int e = threadIdx.x; e < 256; e += kNT) {
                double sum = 0.0;
#pragma unroll
                for (int w2 = 0; w2 < kNW; ++w2) sum += tred[w2 * 256 + e];
                const int l = e >> 2, r = e & 3;
                const int a = ta * 16 + 4 * r + (l >> 4);
                const int c = (tc0 + tb) * 16 + (l & 15);
                if (a < k && c <= k) Ap[a * kLdA + c] = sum;
            }
            lds_barrier();
        }
    }
}

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

// Mixed-precision counterpart of vtw_chunk: partial Vb^T Wb of the BF16 copies of V_k and
// A'V_k (k columns each, leading dimension ldv elements), over 32-row chunks
// g = wave, wave + kNW, ..., on BF16 matrix cores with FP32 accumulation
// (v_mfma_f32_16x16x32_bf16: lane l holds A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16] as eight
// consecutive rows of one column, one 16-byte load; output register r of lane l is
// D[4(l/16) + r][l%16]).  Chunks are zero past row n; the tiles are summed over the waves in a
// fixed order in FP64.
template <int KTR, int NTC>
__device__ __forceinline__ void vtw_bf16(rsrc_t rV, rsrc_t rW, int n, int ldv, int k, int tc0,
                                         double *Ap, double *tred) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    f32x4_t acc[KTR][NTC];
    unsigned offA[KTR], offB[NTC];
    bool okA[KTR], okB[NTC];
#pragma unroll
    for (int t = 0; t < KTR; ++t) {
        const int a = t * 16 + (lane & 15);
        okA[t] = a < k;
        offA[t] = (unsigned)(okA[t] ? a : 0) * (unsigned)ldv * 2u;
    }
#pragma unroll
    for (int t = 0; t < NTC; ++t) {
        const int c = (tc0 + t) * 16 + (lane & 15);
        okB[t] = c < k;
        offB[t] = (unsigned)(okB[t] ? c : 0) * (unsigned)ldv * 2u;
    }
#pragma unroll
    for (int a = 0; a < KTR; ++a)
#pragma unroll
        for (int b = 0; b < NTC; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
    const int nchunks = (n + 31) / 32;
    u32x4_t an[KTR], bn[NTC];
    int g = wave;
    {
        const unsigned po = (32u * g + 8u * (lane >> 4)) * 2u;
#pragma unroll
        for (int t = 0; t < KTR; ++t) an[t] = __builtin_amdgcn_raw_buffer_load_b128(rV, offA[t] + po, 0, 0);
#pragma unroll
        for (int t = 0; t < NTC; ++t) bn[t] = __builtin_amdgcn_raw_buffer_load_b128(rW, offB[t] + po, 0, 0);
    }
    const u32x4_t zero4 = {0u, 0u, 0u, 0u};
    for (; g < nchunks; g += kNW) {
        // rows p..p+7 of a column lie inside it (ldv is a multiple of 8 above n); groups at or
        // past n are zeroed
        const unsigned p = 32u * g + 8u * (lane >> 4);
        const bool pin = p < (unsigned)n;
        bf16x8_t av[KTR], bv[NTC];
#pragma unroll
        for (int t = 0; t < KTR; ++t)
            av[t] = __builtin_bit_cast(bf16x8_t, (okA[t] && pin) ? an[t] : zero4);
#pragma unroll
        for (int t = 0; t < NTC; ++t)
            bv[t] = __builtin_bit_cast(bf16x8_t, (okB[t] && pin) ? bn[t] : zero4);
        const int gn = g + kNW < nchunks ? g + kNW : g;
        const unsigned pon = (32u * gn + 8u * (lane >> 4)) * 2u;
#pragma unroll
        for (int t = 0; t < KTR; ++t) an[t] = __builtin_amdgcn_raw_buffer_load_b128(rV, offA[t] + pon, 0, 0);
#pragma unroll
        for (int t = 0; t < NTC; ++t) bn[t] = __builtin_amdgcn_raw_buffer_load_b128(rW, offB[t] + pon, 0, 0);
#pragma unroll
        for (int a = 0; a < KTR; ++a)
#pragma unroll
            for (int b = 0; b < NTC; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
#pragma unroll
    for (int ta = 0; ta < KTR; ++ta) {
#pragma unroll
        for (int tb = 0; tb < NTC; ++tb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) tred[wave * 256 + lane * 4 + r] = (double)acc[ta][tb][r];
            lds_barrier();
            for (int e = threadIdx.x; e < 256; e += kNT) {
                double sum = 0.0;
#pragma unroll
                for (int w2 = 0; w2 < kNW; ++w2) sum += tred[w2 * 256 + e];
                const int l = e >> 2, r = e & 3;
                const int a = ta * 16 + 4 * (l >> 4) + r;
                const int c = (tc0 + tb) * 16 + (l & 15);
                if (a < k && c < k) Ap[a * kLdA + c] = sum;
            }
            lds_barrier();
        }
    }
}

// Projection of one target onto its seed basis (Section 3, Phase 2): writes x0 = x_base + V alpha
// into s.x and returns XKP_OK, XKP_ESINGULAR (the projected system was singular: x0 = x_base)
// or XKP_EINVAL (no usable basis: s.x untouched, info->status set).  The LDS holds nbuf
// zero-padded vector copies (each nlds long) during the operator applications, then the
// projected matrix and the tile-reduction scratch: never live together.
template <int RMAX, bool MIXED>
__device__ __forceinline__ int project_one(const xkp_system &s, xkp_info *info, int n_bases,
                           const void *const *bases, const xkp_params &P, const Coef &C,
                           double *W, double *lds, int nlds, int nbuf, int nregion) {
    double *vbuf = lds + (nlds - kNT * RMAX) / 2;   // after the front pad
    double *vbuf1 = vbuf + nlds;
    double *Ap = lds;
    double *zv = lds + nregion;        // kMMax + 1
    double *alpha = zv + kMMax + 1;    // kMMax
    int *pivl = (int *)(alpha + kMMax);
    double *red = alpha + kMMax + kMMax / 2;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        const int n = s.H * s.H;
        const xkp_basis_header *hdr = nullptr;
        int k = 0;
        bool ok = s.basis_id >= 0 && s.basis_id < n_bases;
        if (ok) {
            hdr = (const xkp_basis_header *)bases[s.basis_id];
            ok = hdr != nullptr && hdr->n == n && hdr->m == P.m && hdr->k >= 0 && hdr->k <= P.m;
            // the seed modes use the Hessenberg matrix: an accumulated basis has none
            if (ok && P.mode != XKP_PROJ_TARGET_GALERKIN) ok = hdr->kind == XKP_BASIS_ARNOLDI;
            // the mixed target-Galerkin contraction needs the seed's BF16 basis copy
            if (ok && P.precision == XKP_MIXED && P.mode == XKP_PROJ_TARGET_GALERKIN)
                ok = hdr->bf16 == 1;
            // the same header for the whole workgroup: a scalar basis dimension keeps every
            // loop over the columns on scalar branches
            if (ok) k = __builtin_amdgcn_readfirstlane(hdr->k);
        }
        if (!ok) {
            if (tid == 0) {
                info->status = XKP_EINVAL;
                info->basis_dim = 0;
            }
            return XKP_EINVAL;
        }
        const int m = P.m;
        const double *V = (const double *)((const char *)hdr + 256);
        const int ldv = ldv_for(n);
        const double *Hb = (const double *)((const char *)hdr + basis_off_h(n, m));
        const OpConst o = op_const(s);
        BlockRed br{red, 0};
        constexpr bool mixed = MIXED;
        build_coeffs<RMAX>(s, o, C, mixed);
        // the LDS vector shares space with the projected matrix of the previous system: clear it
        for (int t = tid; t < nregion; t += kNT) lds[t] = 0.0;
        lds_barrier();   // the cleared words belong to other threads' rows

        // r_base = b - A' x_base
        double rb[RMAX], cur[RMAX];
        load_rows<RMAX>(s.b, n, rb);
        if (s.x0) {
            load_rows<RMAX>(s.x0, n, cur);
            store_rows_lds<RMAX>(vbuf, cur);
            lds_barrier();
            stencil_lds<RMAX>(vbuf, C, o, cur);
#pragma unroll
            for (int q = 0; q < RMAX; ++q) rb[q] -= cur[q];
        }
        bool singular = false;
        // zv = V_{nz}^T r_base in FP64, eight columns per reduction
        auto vt_rbase = [&](int nz) {
            for (int c0 = 0; c0 < nz; c0 += kRedSlots) {
                double part[kRedSlots];
#pragma unroll
                for (int q = 0; q < kRedSlots; ++q) {
                    part[q] = 0.0;
                    if (c0 + q < nz) {
                        load_col<RMAX>(V + (size_t)(c0 + q) * ldv, ldv, cur);
                        part[q] = dot_rows<RMAX>(cur, rb);
                    }
                }
                br.sum_multi<kRedSlots>(part);
                if (tid == 0)
                    for (int q = 0; q < kRedSlots && c0 + q < nz; ++q) zv[c0 + q] = part[q];
            }
        };
        if (k > 0) {
            if (mixed && P.mode == XKP_PROJ_TARGET_GALERKIN) {
                // A' V_k with the FP32 operator, rounded to BF16 into the workspace;
                // V_k^T (A' V_k) on BF16 matrix cores with FP32 accumulation; V_k^T r_base and
                // the k x k solve in FP64
                unsigned short *Wb = (unsigned short *)W;
                const unsigned short *Vb =
                    (const unsigned short *)((const char *)hdr + basis_off_vb(n, m));
                sweep_cols<RMAX, Depth<RMAX>::value>(V, ldv, k, k,
                    [&](int c, const double(&col)[RMAX]) {
                    double *vb = (nbuf == 2 && (c & 1)) ? vbuf1 : vbuf;
                    if (nbuf == 1 && c > 0) lds_barrier();   // readers of the previous column
                    store_rows_lds<RMAX>(vb, col);
                    lds_barrier();
                    double y[RMAX];
                    stencil_lds_f32<RMAX>(vb, C, o, y);
                    store_col_bf16<RMAX>(Wb + (size_t)c * ldv, ldv, y);
                });
                vt_rbase(k);
                __syncthreads();   // Wb rows written by other threads are read below
                const int ktr = (k + 15) / 16;
                const rsrc_t rV = mkbuf16(Vb, ldv * k), rW = mkbuf16(Wb, ldv * k);
                double *tred = Ap + (kMMax + 1) * kLdA;
                for (int tc0 = 0; tc0 < ktr; tc0 += kNtcMax) {
                    const int ntc = ktr - tc0 < kNtcMax ? ktr - tc0 : kNtcMax;
#define XKP_VTWB(R_, C_) vtw_bf16<R_, C_>(rV, rW, n, ldv, k, tc0, Ap, tred)
                    switch (ktr * 2 + ntc - 1) {
                    case 2: XKP_VTWB(1, 1); break;
                    case 4: XKP_VTWB(2, 1); break;
                    case 6: XKP_VTWB(3, 1); break;
                    case 8: XKP_VTWB(4, 1); break;
                    default:
                        if constexpr (kNtcMax > 1) {
                            if (ntc == 2) {
                                if (ktr == 2) XKP_VTWB(2, 2);
                                else if (ktr == 3) XKP_VTWB(3, 2);
                                else XKP_VTWB(4, 2);
                            }
                        }
                        break;
                    }
#undef XKP_VTWB
                }
                lds_barrier();
                if (wave == 0) {
                    const double zr = (lane < k) ? zv[lane] : 0.0;
                    singular = lu_solve_wave(Ap, kLdA, k, zr, alpha, pivl);
                }
            } else if (P.mode == XKP_PROJ_TARGET_GALERKIN) {
                // W = [A' V_k | r_base] in the workspace.  Each thread keeps its rows'
                // coefficients in registers; the basis columns stream through the prefetch ring
                // and, for the neighbours, through one of two zero-padded LDS copies.
                // (with 32 rows per thread the coefficients are re-read from the workspace
                // instead: four register arrays of 32 would not fit)
                // (so do 16-wave variants: 128 registers per lane)
                constexpr bool kRegC = RMAX < 32 && kNT < 1024;
                constexpr int RC = kRegC ? RMAX : 1;
                double cEr[RC], cWr[RC], cNr[RC], cSr[RC];
                if constexpr (kRegC) {
                    const rsrc_t bE = mkbuf(C.E, kNT * RMAX), bW = mkbuf(C.W, kNT * RMAX);
                    const rsrc_t bN = mkbuf(C.N, kNT * RMAX), bS = mkbuf(C.S, kNT * RMAX);
#pragma unroll
                    for (int q = 0; q < RMAX; ++q) {
                        if constexpr (kDriftCoef<RMAX>) {
                            coeffs_of(o, row_of(q), bld(bE, row_off(q)), bld(bW, row_off(q)),
                                      cEr[q], cWr[q], cNr[q], cSr[q]);
                        } else {
                            cEr[q] = bld(bE, row_off(q));
                            cWr[q] = bld(bW, row_off(q));
                            cNr[q] = bld(bN, row_off(q));
                            cSr[q] = bld(bS, row_off(q));
                        }
                    }
                }
                const int H = o.H;
                store_col<RMAX>(W + (size_t)k * ldv, ldv, rb);
                sweep_cols<RMAX, Depth<RMAX>::value>(V, ldv, k, k,
                    [&](int c, const double(&col)[RMAX]) {
                    double *vb = (nbuf == 2 && (c & 1)) ? vbuf1 : vbuf;
                    if (nbuf == 1 && c > 0) lds_barrier();   // readers of the previous column
                    store_rows_lds<RMAX>(vb, col);
                    lds_barrier();
                    double y[RMAX];
                    if constexpr (kRegC) {
#pragma unroll
                        for (int q = 0; q < RMAX; ++q) {
                            const double *u = vb + row_of(q);
                            y[q] = o.cd * u[0] + cEr[q] * u[H] + cWr[q] * u[-H] + cNr[q] * u[1]
                                   + cSr[q] * u[-1];
                        }
                    } else {
                        stencil_lds<RMAX>(vb, C, o, y);
                    }
                    store_col<RMAX>(W + (size_t)c * ldv, ldv, y);
                });
                __syncthreads();   // W rows written by other threads are read below
                // [V_k^T A' V_k | V_k^T r_base]: rows split over the waves, all tiles per wave,
                // column tiles two at a time; partial tiles reduced across waves in a fixed order.
                const int ktr = (k + 15) / 16, ktc = (k + 16) / 16;
                const rsrc_t rV = mkbuf(V, ldv * (k + 1)), rW = mkbuf(W, ldv * (k + 1));
                double *tred = Ap + (kMMax + 1) * kLdA;   // kNW x 256 partial tile
                for (int tc0 = 0; tc0 < ktc; tc0 += kNtcMax) {
                    const int ntc = ktc - tc0 < kNtcMax ? ktc - tc0 : kNtcMax;
#define XKP_VTW(R_, C_) vtw_chunk<R_, C_>(rV, rW, n, ldv, k, tc0, Ap, tred)
                    switch (ktr * 2 + ntc - 1) {
                    case 2: XKP_VTW(1, 1); break;
                    case 4: XKP_VTW(2, 1); break;
                    case 6: XKP_VTW(3, 1); break;
                    case 8: XKP_VTW(4, 1); break;
                    default:
                        if constexpr (kNtcMax > 1) {
                            if (ntc == 2) {
                                if (ktr == 1) XKP_VTW(1, 2);
                                else if (ktr == 2) XKP_VTW(2, 2);
                                else if (ktr == 3) XKP_VTW(3, 2);
                                else XKP_VTW(4, 2);
                            }
                        }
                        break;
                    }
#undef XKP_VTW
                }
                lds_barrier();
                if (wave == 0) {
                    const double zr = (lane < k) ? Ap[lane * kLdA + k] : 0.0;
                    singular = lu_solve_wave(Ap, kLdA, k, zr, alpha, pivl);
                }
            } else {
                // z = V_{k(+1)}^T r_base
                vt_rbase((P.mode == XKP_PROJ_SEED_LSQ) ? k + 1 : k);
                // Hbar (k+1 rows) or H_k into LDS, row-major
                for (int t = tid; t < (k + 1) * k; t += kNT) {
                    const int a = t / k, c = t % k;
                    Ap[a * kLdA + c] = Hb[(size_t)c * (m + 1) + a];
                }
                lds_barrier();
                if (wave == 0) {
                    if (P.mode == XKP_PROJ_SEED_GALERKIN) {
                        const double zr = (lane < k) ? zv[lane] : 0.0;
                        singular = lu_solve_wave(Ap, kLdA, k, zr, alpha, pivl);
                    } else {
                        singular = lsq_hessenberg_wave(Ap, kLdA, k, zv, alpha);
                    }
                }
            }
            // broadcast the (wave 0) singular flag
            if (tid == 0) pivl[kMMax - 1] = singular ? 1 : 0;
            lds_barrier();
            singular = pivl[kMMax - 1] != 0;
        }
        // x0 = x_base + V_k alpha (x_base reloaded: not kept live through the projection)
        double xr[RMAX];
        if (s.x0) {
            load_rows<RMAX>(s.x0, n, xr);
        } else {
#pragma unroll
            for (int q = 0; q < RMAX; ++q) xr[q] = 0.0;
        }
        if (k > 0 && !singular) {
            sweep_cols<RMAX, Depth<RMAX>::value>(V, ldv, k, k,
                [&](int c, const double(&col)[RMAX]) {
                const double al = alpha[c];
#pragma unroll
                for (int q = 0; q < RMAX; ++q) xr[q] += al * col[q];
            });
        }
        store_rows<RMAX>(s.x, n, xr);
        if (tid == 0) info->basis_dim = k;
        // the polish reads x0 rows written by other threads, and reuses the LDS
        __syncthreads();
        return singular ? XKP_ESINGULAR : XKP_OK;
    }
}

// ----------------------------------------------------------------------------------------
// The batched solve: one persistent launch over a batch of systems of possibly different sizes.
// Workgroups take systems from a work queue (an atomic counter) in descriptor order, so a batch
// ordered largest first is balanced as in longest-processing-time-first scheduling.  Each system
// runs the code path compiled for the smallest rows-per-thread count that covers it.
//   seeds   (kKeepBasis): restarted GMRES from x0 = 0, first cycle kept (Section 3, Phase 1)
//   targets (kTarget):    projection onto the seed basis, then GMRES polish from the projected
//                         guess (Phase 2)
//   plain   (no flag):    restarted GMRES from x_base
// queue[0] counts the systems handed out and queue[1] the workgroups that have finished; the last
// workgroup to finish sets both back to zero, so consecutive launches on the stream, and replays
// of a captured graph, need no reset.

#if XKP_NT == 512
constexpr int kRClass0 = 2, kRClass1 = 8;
#else
constexpr int kRClass0 = 4, kRClass1 = 16;
#endif

// Each size class's projection and GMRES are compiled as functions of their own, so that the
// register allocation of one (MFMA accumulators, prefetch rings of other row counts) cannot make
// another spill inside its loops.  Their arguments arrive in vector registers; every one is
// the same across the workgroup, and readfirstlane says so to the compiler (buffer descriptors
// and loop bounds must be scalar).  The LDS is addressed through the dynamic-LDS symbol itself.
// (16-byte aligned: row pairs are read and written as 16-byte LDS accesses)
extern __shared__ __attribute__((aligned(16))) double xkp_dyn_lds[];

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ double uni(double v) {
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
template <typename T>
__device__ __forceinline__ T *uni(T *p) {
    const unsigned long long u = (unsigned long long)p;
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)u);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(u >> 32));
    return (T *)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ xkp_system uni(xkp_system s) {
    s.H = uni(s.H);
    s.basis_id = uni(s.basis_id);
    s.dt = uni(s.dt);
    s.g = uni(s.g);
    s.mt = uni(s.mt);
    s.fx = uni(s.fx);
    s.fy = uni(s.fy);
    s.b = uni(s.b);
    s.x0 = uni(s.x0);
    s.x = uni(s.x);
    return s;
}
__device__ __forceinline__ xkp_params uni(xkp_params P) {
    P.m = uni(P.m);
    P.max_restarts = uni(P.max_restarts);
    P.tol = uni(P.tol);
    P.precision = uni(P.precision);
    P.mode = uni(P.mode);
    P.batch_max_n = uni(P.batch_max_n);
    P.polish_m = uni(P.polish_m);
    P.reorth = uni(P.reorth);
    return P;
}
__device__ __forceinline__ Coef uni(Coef C) {
    return Coef{uni(C.E),   uni(C.W),   uni(C.N),   uni(C.S),
                uni(C.E32), uni(C.W32), uni(C.N32), uni(C.S32)};
}

template <int R, bool MIXED>
__device__ __noinline__ int project_call(xkp_system s, xkp_info *info, int n_bases,
                                         const void *const *bases, xkp_params P, Coef C,
                                         double *W, int nlds, int nbuf, int nregion) {
    return project_one<R, MIXED>(uni(s), uni(info), uni(n_bases), uni(bases), uni(P), uni(C), uni(W),
                          xkp_dyn_lds, uni(nlds), uni(nbuf), uni(nregion));
}

template <int R, bool MIXED, int MC>
__device__ __noinline__ void gmres_reg_call(xkp_system s, xkp_params P, int flags, int pre,
                                            int gsrc, Coef C, xkp_info *info, int nlds) {
    GmresLds L(xkp_dyn_lds, uni(nlds), kNT * R);
    gmres_reg<R, MIXED, MC>(uni(s), uni(P), uni(flags), uni(pre), uni(gsrc), uni(C), uni(info),
                            L);
}

template <int R, bool MIXED>
__device__ __noinline__ void gmres_call(xkp_system s, xkp_params P, int flags, int pre, int gsrc,
                                        xkp_basis_header *hdr, double *Vfirst, double *Hb,
                                        double *Vws, Coef C, xkp_info *info, int nlds) {
    GmresLds L(xkp_dyn_lds, uni(nlds), kNT * R);
    gmres_one<R, MIXED>(uni(s), uni(P), uni(flags), uni(pre), uni(gsrc), uni(hdr), uni(Vfirst),
                        uni(Hb), uni(Vws), uni(C), uni(info), L);
}

// Learned starting guess of one target.  The network predicts the target's residual
// coordinates in the seed's Arnoldi basis, zeta ~ Hbar_k alpha* / beta_seed (k+1 values, FP32);
// alpha = argmin || beta_seed * scale * zeta - Hbar_k alpha || (Givens least squares on the seed's
// Hessenberg matrix, as the least-squares projection mode), x0 = x_base + V_k alpha, written to
// s.x.  Returns ||b - A x0|| / ||b|| in FP64 (0 when b = 0), or -1 when the target has no usable
// basis or the least-squares problem is singular (s.x may then hold a partial guess; the caller
// falls back).  LDS: the projection layout (matrix at the base, vectors after nregion).
// ||b - A' x|| / ||b|| (FP64 operator; 0 when b = 0) of the iterate x whose rows the threads
// hold in xr; vbuf is the zero-padded LDS vector copy (cleared pads).
template <int R>
__device__ __forceinline__ double guess_rel_residual(const xkp_system &s, const Coef &C,
                                                    const OpConst &o, const double (&xr)[R],
                                                    double *vbuf, BlockRed &br) {
    const int n = s.H * s.H;
    double w[R], b[R];
    store_rows_lds<R>(vbuf, xr);
    lds_barrier();
    stencil_lds<R>(vbuf, C, o, w);
    load_rows<R>(s.b, n, b);
#pragma unroll
    for (int q = 0; q < R; ++q) w[q] = b[q] - w[q];
    double two[2] = {dot_rows<R>(w, w), dot_rows<R>(b, b)};
    br.sum_multi<2>(two);
    return two[1] > 0.0 ? sqrt(two[0]) / sqrt(two[1]) : 0.0;
}

template <int R>
__device__ __noinline__ double learned_call(xkp_system s0, int n_bases, const void *const *bases,
                                            xkp_params P0, const float *a, int ka, double scale,
                                            Coef C0, int nlds, int nregion) {
    const xkp_system s = uni(s0);
    const xkp_params P = uni(P0);
    const Coef C = uni(C0);
    a = uni(a);
    ka = uni(ka);
    scale = uni(scale);
    nlds = uni(nlds);
    nregion = uni(nregion);
    bases = uni(bases);
    n_bases = uni(n_bases);
    const int n = s.H * s.H, tid = threadIdx.x;
    if (!(s.basis_id >= 0 && s.basis_id < n_bases)) return -1.0;
    const xkp_basis_header *hdr = (const xkp_basis_header *)bases[s.basis_id];
    if (!(hdr != nullptr && hdr->n == n && hdr->m == P.m && hdr->k >= 0 && hdr->k <= P.m &&
          hdr->kind == XKP_BASIS_ARNOLDI))
        return -1.0;
    const int m = P.m, k = hdr->k;
    if (ka < k + 1) return -1.0;
    const double *V = (const double *)((const char *)hdr + 256);
    const double *Hb = (const double *)((const char *)hdr + basis_off_h(n, m));
    const int ldv = ldv_for(n);
    double *lds = xkp_dyn_lds;
    double *Ap = lds;
    double *zv = lds + nregion;
    double *alpha = zv + kMMax + 1;
    int *pivl = (int *)(alpha + kMMax);
    double *red = alpha + kMMax + kMMax / 2;
    double *vbuf = lds + (nlds - kNT * R) / 2;
    BlockRed br{red, 0};
    const OpConst o = op_const(s);
    build_coeffs<R>(s, o, C, false);
    bool singular = false;
    if (k > 0) {
        const double zs = hdr->beta * scale;
        for (int r = tid; r <= k; r += kNT) zv[r] = zs * (double)a[r];
        for (int t = tid; t < (k + 1) * k; t += kNT) {
            const int r = t / k, c = t % k;
            Ap[r * kLdA + c] = Hb[(size_t)c * (m + 1) + r];
        }
        lds_barrier();
        if ((tid >> 6) == 0) singular = lsq_hessenberg_wave(Ap, kLdA, k, zv, alpha);
        if (tid == 0) pivl[kMMax - 1] = singular ? 1 : 0;
        lds_barrier();
        singular = pivl[kMMax - 1] != 0;
    }
    double xr[R];
    if (s.x0) {
        load_rows<R>(s.x0, n, xr);
    } else {
#pragma unroll
        for (int q = 0; q < R; ++q) xr[q] = 0.0;
    }
    if (k > 0 && !singular) {
        sweep_cols<R, Depth<R>::value>(V, ldv, k, k, [&](int c, const double(&col)[R]) {
            const double al = alpha[c];
#pragma unroll
            for (int q = 0; q < R; ++q) xr[q] += al * col[q];
        });
    }
    // the matrix area holds the zero-padded vector copy from here on
    lds_barrier();
    for (int t = tid; t < nlds; t += kNT) lds[t] = 0.0;
    lds_barrier();
    store_rows<R>(s.x, n, xr);
    const double rel = guess_rel_residual<R>(s, C, o, xr, vbuf, br);
    __syncthreads();   // the polish reads rows of x0 written by other threads, and reuses LDS
    if (singular) return -1.0;
    return rel;
}



// The projected guess in s.x: its rows copied to `stash` (device workspace) and its FP64
// relative residual returned (the coefficients were built by the projection).
template <int R>
__device__ __noinline__ double stash_guess_call(xkp_system s0, Coef C0, double *stash, int nlds) {
    const xkp_system s = uni(s0);
    const Coef C = uni(C0);
    stash = uni(stash);
    nlds = uni(nlds);
    const int n = s.H * s.H;
    double *lds = xkp_dyn_lds;
    double *vbuf = lds + (nlds - kNT * R) / 2;
    BlockRed br{lds + nlds, 0};
    for (int t = threadIdx.x; t < nlds + 2 * kRedSlots * kNW; t += kNT) lds[t] = 0.0;
    lds_barrier();
    double xr[R];
    load_rows<R>(s.x, n, xr);
    store_rows<R>(stash, n, xr);
    const double rel = guess_rel_residual<R>(s, C, op_const(s), xr, vbuf, br);
    __syncthreads();
    return rel;
}

// s.x = the stashed rows (a rejected correction of the projected guess is undone).
template <int R>
__device__ __noinline__ void unstash_guess_call(xkp_system s0, const double *stash) {
    const xkp_system s = uni(s0);
    stash = uni(stash);
    double xr[R];
    load_rows<R>(stash, s.H * s.H, xr);
    store_rows<R>(s.x, s.H * s.H, xr);
    __syncthreads();   // the polish reads rows written by other threads
}

template <int R, bool PROJ>
__device__ __forceinline__ void solve_one(const xkp_system &s, xkp_info *info,
                                          const xkp_params &P, int flags, int n_bases,
                                          const void *const *bases, void *keep_base,
                                          const Coef &C, double *slot, const WsLayout &Lw,
                                          double *lds, int nlds, int nbuf, int nregion,
                                          const Learned &lg, const float *al, int pre0) {
    int pre = XKP_OK;
    // guess source: 1 targets, 4 a seed solved again after its spread-out solve gave up
    int gsrc = (flags & kTarget) ? 1 : ((flags & kRedo) ? 4 : 0);
    bool project = PROJ;
    if (flags & kPreProjected) {
        // projected by the projection launches: x holds x0; no basis (XKP_EINVAL) was reported
        // there
        if (pre0 != XKP_OK && pre0 != XKP_ESINGULAR) return;
        pre = pre0;
        flags |= kStartFromX;
    } else if ((flags & kLearned) && (flags & kCorrection)) {
        if constexpr (PROJ) {
            // the projection first; then the network's correction of the projected coordinates,
            // kept when its FP64 residual passes the gate and is below the projected guess's
            pre = P.precision == XKP_MIXED
                      ? project_call<R, true>(s, info, n_bases, bases, P, C, slot + Lw.w, nlds,
                                              nbuf, nregion)
                      : project_call<R, false>(s, info, n_bases, bases, P, C, slot + Lw.w, nlds,
                                               nbuf, nregion);
            if (pre == XKP_EINVAL) return;
            project = false;
            flags |= kStartFromX;
            if (pre == XKP_OK) {
                double *stash = slot + Lw.w;
                const double rel_p = stash_guess_call<R>(s, C, stash, nlds);
                for (int t = threadIdx.x; t < nlds; t += kNT) lds[t] = 0.0;
                lds_barrier();
                xkp_system sc = s;
                sc.x0 = s.x;   // the correction starts from the projected guess
                const double rel =
                    learned_call<R>(sc, n_bases, bases, P, al, lg.ld, lg.scale, C, nlds, nregion);
                if (rel >= 0.0 && rel <= lg.gate && rel < rel_p)
                    gsrc = 3;
                else
                    unstash_guess_call<R>(s, stash);
            }
        }
    } else if (flags & kLearned) {
        // the network's guess, kept when its FP64 residual passes the gate
        for (int t = threadIdx.x; t < nlds; t += kNT) lds[t] = 0.0;
        lds_barrier();
        const double rel =
            learned_call<R>(s, n_bases, bases, P, al, lg.ld, lg.scale, C, nlds, nregion);
        if (rel >= 0.0 && rel <= lg.gate) {
            project = false;
            gsrc = 2;
            flags |= kStartFromX;
            // the guess used the seed basis: report its dimension as the projection does
            if (threadIdx.x == 0)
                info->basis_dim = ((const xkp_basis_header *)bases[s.basis_id])->k;
        }
    }
    if (PROJ && project) {
        pre = P.precision == XKP_MIXED
                  ? project_call<R, true>(s, info, n_bases, bases, P, C, slot + Lw.w, nlds, nbuf,
                                          nregion)
                  : project_call<R, false>(s, info, n_bases, bases, P, C, slot + Lw.w, nlds, nbuf,
                                           nregion);
        if (pre == XKP_EINVAL) return;
        flags |= kStartFromX;
    }
    // the GMRES vector copy needs zero pads: clear what the previous system or the projection
    // left in the LDS
    for (int t = threadIdx.x; t < nlds; t += kNT) lds[t] = 0.0;
    lds_barrier();
    xkp_basis_header *hdr = nullptr;
    double *Vfirst = slot + Lw.v, *Hb = nullptr;
    if (keep_base) {
        hdr = (xkp_basis_header *)keep_base;
        Vfirst = (double *)((char *)keep_base + 256);
        Hb = (double *)((char *)keep_base + basis_off_h(s.H * s.H, P.m));
    }
    // discarded cycles that fit the register budget keep their basis in registers
    constexpr int MC = RegCols<R>::value;
    if constexpr (MC > 0) {
        const int mpol = P.polish_m > 0 ? P.polish_m : P.m;
        if (!keep_base && (flags & kRegBasis) && mpol + 1 <= MC &&
            P.reorth == XKP_REORTH_AUTO) {
            if (P.precision == XKP_MIXED)
                gmres_reg_call<R, true, MC>(s, P, flags, pre, gsrc, C, info, nlds);
            else
                gmres_reg_call<R, false, MC>(s, P, flags, pre, gsrc, C, info, nlds);
            return;
        }
    }
    // seeds keep the FP64 operator in mixed precision: one system per timestep on the chain's
    // critical path, where the FP32 operator's cycle limit would cost restarts
    if (P.precision == XKP_MIXED && !keep_base)
        gmres_call<R, true>(s, P, flags, pre, gsrc, hdr, Vfirst, Hb, slot + Lw.v, C, info, nlds);
    else
        gmres_call<R, false>(s, P, flags, pre, gsrc, hdr, Vfirst, Hb, slot + Lw.v, C, info, nlds);
}

template <int RMAX, bool PROJ>
__global__ __launch_bounds__(kNT) void solve_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                    xkp_params P, int flags, int n_bases,
                                                    const void *const *bases,
                                                    void *const *keep_bases, xkp_info *infos,
                                                    double *ws, WsLayout Lw, int nmax, int nlds,
                                                    int nbuf, int nregion, unsigned *queue,
                                                    Learned lg, const int *pre) {
    double *lds = xkp_dyn_lds;
    __shared__ int next[2];
    double *slot = ws + (size_t)blockIdx.x * Lw.stride;
    float *c32 = (float *)(slot + Lw.c32);
    const Coef C{slot + Lw.cE, slot + Lw.cW, slot + Lw.cN, slot + Lw.cS,
                 c32, c32 + Lw.npad, c32 + 2 * Lw.npad, c32 + 3 * Lw.npad};
    for (int it = 0;; ++it) {
        // alternating broadcast slots: a fast thread 0 can fetch the next index before slow
        // waves have read this one without overwriting it
        if (threadIdx.x == 0) next[it & 1] = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int si = next[it & 1];
        if (si >= nsys) break;
        const xkp_system s = sys[si];
        xkp_info *info = infos + si;
        if ((flags & kRedo) && __builtin_amdgcn_readfirstlane(info->status) != XKP_EDEVICE)
            continue;
        if (!desc_ok(s, nmax) || P.m < 1 || P.m > kMMax || P.polish_m < 0 || P.polish_m > kMMax) {
            if (threadIdx.x == 0) info->status = XKP_EINVAL;
            continue;
        }
        void *kb = (flags & kKeepBasis) ? keep_bases[si] : nullptr;
        const int n = s.H * s.H;
        const float *al = (flags & kLearned) ? lg.alpha + (size_t)si * lg.ld : nullptr;
        const int pre0 = (flags & kPreProjected) ? pre[si] : XKP_OK;
#define XKP_SOLVE(R_)                                                                            \
    solve_one<R_, PROJ>(s, info, P, flags, n_bases, bases, kb, C, slot, Lw, lds, nlds, nbuf, nregion, \
                        lg, al, pre0)
        if constexpr (RMAX > kRClass0) {
            if (n <= kNT * kRClass0) {
                XKP_SOLVE(kRClass0);
                continue;
            }
        }
        if constexpr (RMAX > kRClass1) {
            if (n <= kNT * kRClass1) {
                XKP_SOLVE(kRClass1);
                continue;
            }
        }
        XKP_SOLVE(RMAX);
#undef XKP_SOLVE
    }
    if (threadIdx.x == 0) {
        // every workgroup's last fetch precedes its increment here (the fetched value decided
        // the exit), so the last one to arrive may reset the queue
        if (atomicAdd(queue + 1, 1u) == gridDim.x - 1) {
            atomicExch(queue, 0u);
            atomicExch(queue + 1, 0u);
        }
    }
}

// ----------------------------------------------------------------------------------------

// alpha[i][c] = v_c . x_i for c < k (the kept basis of system i's seed), 0 for k <= c < m_out:
// the coordinates of x_i in the seed subspace (the regression targets of the learned guess).
// kind 1: the residual coordinates zeta = Hbar_k (V_k^T x_i) / beta_seed (k+1 values, 0 past),
// the regression targets of the learned guess.
template <int RMAX>
__global__ __launch_bounds__(kNT) void coeffs_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                     int n_bases, const void *const *bases,
                                                     int m_out, int kind, double *alpha,
                                                     int nmax) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    BlockRed br{lds, 0};
    double *av = lds + 2 * kRedSlots * kNW;   // kMMax coordinates
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        double *out = alpha + (size_t)si * m_out;
        const int n = s.H * s.H;
        bool ok = s.H > 0 && n <= nmax && s.x != nullptr && s.basis_id >= 0 &&
                  s.basis_id < n_bases;
        const xkp_basis_header *hdr = nullptr;
        if (ok) {
            hdr = (const xkp_basis_header *)bases[s.basis_id];
            ok = hdr != nullptr && hdr->n == n && hdr->k >= 0 && hdr->k <= hdr->m &&
                 (kind == 0 || hdr->kind == XKP_BASIS_ARNOLDI);
        }
        if (!ok) {
            for (int c = threadIdx.x; c < m_out; c += kNT) out[c] = __builtin_nan("");
            continue;
        }
        const int k = hdr->k, ldv = ldv_for(n);
        const double *V = (const double *)((const char *)hdr + 256);
        double xr[RMAX], col[RMAX];
        load_rows<RMAX>(s.x, n, xr);
        for (int c0 = 0; c0 < m_out; c0 += kRedSlots) {
            double part[kRedSlots];
#pragma unroll
            for (int q = 0; q < kRedSlots; ++q) {
                part[q] = 0.0;
                if (c0 + q < k) {
                    load_col<RMAX>(V + (size_t)(c0 + q) * ldv, ldv, col);
                    part[q] = dot_rows<RMAX>(col, xr);
                }
            }
            br.sum_multi<kRedSlots>(part);
            if (threadIdx.x == 0)
                for (int q = 0; q < kRedSlots && c0 + q < m_out; ++q) {
                    if (kind == 0) out[c0 + q] = part[q];
                    else if (c0 + q < kMMax) av[c0 + q] = part[q];
                }
        }
        if (kind == 1) {
            __syncthreads();
            const double *Hb = (const double *)((const char *)hdr + basis_off_h(n, hdr->m));
            const int m = hdr->m;
            for (int r = threadIdx.x; r < m_out; r += kNT) {
                double z = 0.0;
                if (r <= k)
                    for (int c = (r > 0 ? r - 1 : 0); c < k; ++c) z += Hb[(size_t)c * (m + 1) + r] * av[c];
                out[r] = hdr->beta > 0.0 ? z / hdr->beta : 0.0;
            }
        }
        __syncthreads();
    }
}

// Krylov subspace accumulation over an image cycle: workgroup j gathers out_bases[j] from the
// first-cycle bases of sources 0..j in order; every column is orthogonalised by two modified
// Gram-Schmidt passes against the columns gathered before it and appended, normalised, when the
// norm left exceeds 1e-8; at most per_source columns per source and cap in total.  Source
// columns go in blocks of AccB: the two passes over the columns gathered before the block (read
// once per pass through the prefetch ring, AccB products per multi-value reduction), then the
// two passes over the block's own accepted columns, held in registers.  Rows are owned as in
// the solve, so the columns a thread writes are the ones it reads back.
template <int R> struct AccB { static constexpr int value = R <= 8 ? 4 : (R <= 16 ? 2 : 1); };

template <int RMAX>
__global__ __launch_bounds__(kNT) void accum_kernel(int n, int nsrc, const void *const *srcs,
                                                     void *const *outs, int per_source, int cap,
                                                     int *out_k) {
    constexpr int B = AccB<RMAX>::value;
    extern __shared__ __attribute__((aligned(16))) double lds[];
    const int j = blockIdx.x;
    if (j >= nsrc) return;
    const int ldv = ldv_for(n);
    bool ok = outs[j] != nullptr;
    for (int s = 0; s <= j && ok; ++s) {
        const xkp_basis_header *h = (const xkp_basis_header *)srcs[s];
        ok = h != nullptr && h->n == n && h->ldv == ldv && h->kind == XKP_BASIS_ARNOLDI &&
             h->k >= 0 && h->k <= h->m;
    }
    if (!ok) {
        if (threadIdx.x == 0 && out_k) out_k[j] = -1;
        return;
    }
    BlockRed br{lds, 0};
    xkp_basis_header *oh = (xkp_basis_header *)outs[j];
    double *Vo = (double *)((char *)oh + 256);
    unsigned short *Vob = (unsigned short *)((char *)oh + basis_off_vb(n, cap));
    int kd = 0;
    double w[B][RMAX];
    for (int s = 0; s <= j && kd < cap; ++s) {
        const xkp_basis_header *h = (const xkp_basis_header *)srcs[s];
        const double *Vs = (const double *)((const char *)h + 256);
        const int ks = h->k;
        int taken = 0, c = 0;
        while (c < ks && taken < per_source && kd < cap) {
            // the block: as many columns as the caps can still take, at most B
            int nb = ks - c;
            if (nb > per_source - taken) nb = per_source - taken;
            if (nb > cap - kd) nb = cap - kd;
            if (nb > B) nb = B;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b < nb) {
                    load_col<RMAX>(Vs + (size_t)(c + b) * ldv, ldv, w[b]);
                } else {
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) w[b][k] = 0.0;
                }
            }
            c += nb;
            const int k0 = kd;
            if (k0 > 0)
                sweep_cols<RMAX, Depth<RMAX>::value>(Vo, ldv, k0, 2 * k0,
                    [&](int, const double(&col)[RMAX]) {
                    double d[B];
#pragma unroll
                    for (int b = 0; b < B; ++b) d[b] = dot_rows<RMAX>(w[b], col);
                    br.sum_multi<B>(d);
#pragma unroll
                    for (int b = 0; b < B; ++b)
#pragma unroll
                        for (int k = 0; k < RMAX; ++k) w[b][k] -= d[b] * col[k];
                });
            // within the block: against the block's columns accepted before, in order
            int acc[B];
            int na = 0;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (b >= nb) break;
                for (int pass = 0; pass < 2; ++pass)
#pragma unroll
                    for (int q = 0; q < B; ++q) {
                        if (q >= na) break;
#pragma unroll
                        for (int qq = 0; qq < B; ++qq) {
                            if (qq != acc[q]) continue;
                            const double d = br.sum(dot_rows<RMAX>(w[b], w[qq]));
#pragma unroll
                            for (int k = 0; k < RMAX; ++k) w[b][k] -= d * w[qq][k];
                        }
                    }
                const double nw = sqrt(br.sum(dot_rows<RMAX>(w[b], w[b])));
                if (nw > 1e-8) {
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) w[b][k] = w[b][k] / nw;
                    store_col<RMAX>(Vo + (size_t)kd * ldv, ldv, w[b]);
                    store_col_bf16<RMAX>(Vob + (size_t)kd * ldv, ldv, w[b]);
                    acc[na++] = b;
                    ++kd;
                    ++taken;
                }
            }
        }
    }
    if (threadIdx.x == 0) {
        oh->n = n;
        oh->m = cap;
        oh->k = kd;
        oh->status = XKP_OK;
        oh->beta = 0.0;
        oh->ldv = ldv;
        oh->bf16 = 1;
        oh->kind = XKP_BASIS_ACCUMULATED;
        if (out_k) out_k[j] = kd;
    }
}

template <int RMAX>
__global__ __launch_bounds__(kNT) void residual_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                       double *rel, int nmax, int nlds) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    double *vbuf = lds;
    double *red = lds + nlds;
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        if (!desc_ok(s, nmax)) {
            if (threadIdx.x == 0) rel[si] = __builtin_nan("");
            continue;
        }
        const OpConst o = op_const(s);
        BlockRed br{red, 0};
        double x[RMAX], w[RMAX], b[RMAX];
        load_rows<RMAX>(s.x, o.n, x);
        load_rows<RMAX>(s.b, o.n, b);
        store_rows_lds<RMAX>(vbuf, x);
        lds_barrier();
        stencil_direct<RMAX>(vbuf, s, o, w);
#pragma unroll
        for (int k = 0; k < RMAX; ++k) w[k] = b[k] - w[k];
        double two[2] = {dot_rows<RMAX>(w, w), dot_rows<RMAX>(b, b)};
        br.sum_multi<2>(two);
        if (threadIdx.x == 0) rel[si] = two[1] > 0.0 ? sqrt(two[0]) / sqrt(two[1]) : sqrt(two[0]);
        __syncthreads();
    }
}

template <int RMAX>
__global__ __launch_bounds__(kNT) void apply_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                    int nmax, int nlds) {
    extern __shared__ __attribute__((aligned(16))) double lds[];
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        if (!desc_ok(s, nmax) || s.x0 == nullptr) continue;
        const OpConst o = op_const(s);
        double u[RMAX], w[RMAX];
        load_rows<RMAX>(s.x0, o.n, u);
        store_rows_lds<RMAX>(lds, u);
        lds_barrier();
        stencil_direct<RMAX>(lds, s, o, w);
        store_rows<RMAX>(s.x, o.n, w);
        __syncthreads();
    }
}

// b = m^{n-1}/dt - div_h f (Section 2.3), m^{n-1} = mt.
template <int RMAX>
__global__ __launch_bounds__(kNT) void rhs_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                  int nmax) {
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        if (!(s.H > 0 && (long)s.H * s.H <= nmax && s.mt && s.b && s.dt > 0.0)) continue;
        const OpConst o = op_const(s);
        double *b = const_cast<double *>(s.b);
        const int H = o.H;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
            const int p = row_of(k);
            const int i = p / H, j = p - i * H;
            if (p < o.n) {
                double div = 0.0;
                if (s.fx) div += ((i + 1 < H) ? ld(s.fx, p + H) : 0.0) - ((i > 0) ? ld(s.fx, p - H) : 0.0);
                if (s.fy) div += ((j + 1 < H) ? ld(s.fy, p + 1) : 0.0) - ((j > 0) ? ld(s.fy, p - 1) : 0.0);
                b[p] = ld(s.mt, p) / s.dt - div * o.inv2h;
            }
        }
    }
}

// ----------------------------------------------------------------------------------------
// Host launchers

int threads() { return kNT; }

#if XKP_NT == 512
int rmax_for(int n) {
    if (n <= kNT * 2) return 2;
    if (n <= kNT * 8) return 8;
    if (n <= kNT * 32) return 32;
    return 0;
}
#define XKP_DISPATCH(RM, CALL)                       \
    switch (RM) {                                    \
    case 2: { constexpr int R = 2; CALL; } break;    \
    case 8: { constexpr int R = 8; CALL; } break;    \
    case 32: { constexpr int R = 32; CALL; } break;  \
    default: return hipErrorInvalidValue;            \
    }
#else
int rmax_for(int n) {
    if (n <= kNT * 4) return 4;
    if (n <= kNT * 16) return 16;
    return 0;
}
#define XKP_DISPATCH(RM, CALL)                       \
    switch (RM) {                                    \
    case 4: { constexpr int R = 4; CALL; } break;    \
    case 16: { constexpr int R = 16; CALL; } break;  \
    default: return hipErrorInvalidValue;            \
    }
#endif

int lds_vec_len(int nmax) {
    int h = 1;
    while (h * h < nmax) ++h;
    const int pad = (h + 2) & ~1;            // >= one grid column + 1, on each side
    return kNT * rmax_for(nmax) + 2 * pad;
}

static size_t gmres_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + kMMax * (kMMax + 1) / 2 + 6 * kMMax + 3 +
                             2 * kRedSlots * kNW + 2 * kWideMax * kNW);
}
static size_t project_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + (kMMax + 1) + kMMax + kMMax / 2 + 2 * kRedSlots * kNW);
}
static size_t small_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + 2 * kRedSlots * kNW);
}

// Raises a kernel's dynamic-LDS limit once per kernel and device (to the largest size asked
// for): a launch enqueued later, for instance inside a graph capture, makes no attribute call.
static hipError_t set_lds_ptr(const void *kern, size_t bytes) {
    struct Entry {
        const void *kern;
        int dev;
        size_t bytes;
    };
    static std::mutex mu;
    static std::vector<Entry> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    for (Entry &d : done)
        if (d.kern == kern && d.dev == dev) {
            if (d.bytes >= bytes) return hipSuccess;
            e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e == hipSuccess) d.bytes = bytes;
            return e;
        }
    e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.push_back({kern, dev, bytes});
    return e;
}
template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
    return set_lds_ptr((const void *)kern, bytes);
}


// LDS plan of a solve launch: the GMRES layout, and for projected targets the projection's
// vector copies (two when they fit next to the rest, else one: two barriers per column).
struct SolvePlan {
    int nbuf, nregion;
    size_t lds;
};
static SolvePlan solve_plan(int nlds, bool proj) {
    SolvePlan sp{1, nlds, gmres_lds_bytes(nlds)};
    if (proj) {
        const int small = (kMMax + 1) * kLdA + kNW * 256;
        sp.nbuf = 2;
        if (project_lds_bytes(2 * nlds > small ? 2 * nlds : small) > 150 * 1024) sp.nbuf = 1;
        sp.nregion = sp.nbuf * nlds > small ? sp.nbuf * nlds : small;
        const size_t pl = project_lds_bytes(sp.nregion);
        if (pl > sp.lds) sp.lds = pl;
    }
    return sp;
}

hipError_t launch_solve(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys,
                        int nsys, xkp_params P, int flags, int n_bases, const void *const *bases,
                        void *const *keep_bases, xkp_info *infos, double *ws, WsLayout L,
                        int nmax, unsigned *queue, Learned lg, const int *pre) {
    // targets projected by the projection launches need no projection code or LDS here
    const bool proj = (flags & kTarget) != 0 && (flags & kPreProjected) == 0;
    SolvePlan sp = solve_plan(nlds, proj || (flags & kLearned) != 0);
    // seeds of up to 4096 unknowns: the kept cycle by DCGS2, its LDS after the GMRES layout
    if ((flags & kKeepBasis) && !proj && rmax * kNT <= 4096) {
        const size_t need = gmres_lds_bytes(nlds) + sizeof(double) * kDcgsDoubles;
        if (need > sp.lds) sp.lds = need;
        flags |= kDcgs;
    }
#define XKP_LAUNCH_SOLVE(PJ)                                                                   \
    {                                                                                          \
        hipError_t e = set_lds(solve_kernel<R, PJ>, sp.lds);                                   \
        if (e != hipSuccess) return e;                                                         \
        hipLaunchKernelGGL((solve_kernel<R, PJ>), dim3(grid), dim3(kNT), sp.lds, st, sys, nsys, \
                           P, flags, n_bases, bases, keep_bases, infos, ws, L, nmax, nlds,     \
                           sp.nbuf, sp.nregion, queue, lg, pre);                               \
    }
    XKP_DISPATCH(rmax, {
        if (proj) XKP_LAUNCH_SOLVE(true) else XKP_LAUNCH_SOLVE(false)
    });
#undef XKP_LAUNCH_SOLVE
    return hipGetLastError();
}

// Workgroups of the solve kernels for systems of up to nmax unknowns that can be resident on one
// compute unit at once (the larger of the projected and plain kernels), 0 on error.
int solve_per_cu(int nmax) {
    const int rmax = rmax_for(nmax), nlds = lds_vec_len(nmax);
    int best = 0;
    for (int pj = 0; pj < 2; ++pj) {
        const SolvePlan sp = solve_plan(nlds, pj != 0);
        int nb = 0;
        hipError_t e = hipSuccess;
        auto occ = [&](const void *k) {
            e = set_lds_ptr(k, sp.lds);
            if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, kNT, sp.lds);
        };
        switch (rmax) {
#if XKP_NT == 512
        case 2: occ(pj ? (const void *)solve_kernel<2, true> : (const void *)solve_kernel<2, false>); break;
        case 8: occ(pj ? (const void *)solve_kernel<8, true> : (const void *)solve_kernel<8, false>); break;
        case 32: occ(pj ? (const void *)solve_kernel<32, true> : (const void *)solve_kernel<32, false>); break;
#else
        case 4: occ(pj ? (const void *)solve_kernel<4, true> : (const void *)solve_kernel<4, false>); break;
        case 16: occ(pj ? (const void *)solve_kernel<16, true> : (const void *)solve_kernel<16, false>); break;
#endif
        default: return 0;
        }
        if (e != hipSuccess) return 0;
        if (nb > best) best = nb;
    }
    return best;
}

hipError_t launch_coeffs(hipStream_t st, int grid, int rmax, const xkp_system *sys, int nsys,
                         int n_bases, const void *const *bases, int m_out, int kind,
                         double *alpha, int nmax) {
    const size_t lds = sizeof(double) * (2 * kRedSlots * kNW + kMMax);
    XKP_DISPATCH(rmax, {
        hipLaunchKernelGGL(coeffs_kernel<R>, dim3(grid), dim3(kNT), lds, st, sys, nsys, n_bases,
                           bases, m_out, kind, alpha, nmax);
    });
    return hipGetLastError();
}

hipError_t launch_residual(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys,
                           int nsys, double *rel, int nmax) {
    const size_t lds = small_lds_bytes(nlds);
    XKP_DISPATCH(rmax, {
        hipError_t e = set_lds(residual_kernel<R>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(residual_kernel<R>, dim3(grid), dim3(kNT), lds, st, sys, nsys, rel,
                           nmax, nlds);
    });
    return hipGetLastError();
}

hipError_t launch_rhs(hipStream_t st, int grid, int rmax, const xkp_system *sys, int nsys,
                      int nmax) {
    XKP_DISPATCH(rmax, {
        hipLaunchKernelGGL(rhs_kernel<R>, dim3(grid), dim3(kNT), 0, st, sys, nsys, nmax);
    });
    return hipGetLastError();
}

hipError_t launch_accum(hipStream_t st, int rmax, int n, int nsrc, const void *const *srcs,
                        void *const *outs, int per_source, int cap, int *out_k) {
    const size_t lds = sizeof(double) * 2 * kRedSlots * kNW;
    XKP_DISPATCH(rmax, {
        hipLaunchKernelGGL(accum_kernel<R>, dim3(nsrc), dim3(kNT), lds, st, n, nsrc, srcs, outs,
                           per_source, cap, out_k);
    });
    return hipGetLastError();
}

hipError_t launch_apply(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys,
                        int nsys, int nmax) {
    const size_t lds = small_lds_bytes(nlds);
    XKP_DISPATCH(rmax, {
        hipError_t e = set_lds(apply_kernel<R>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(apply_kernel<R>, dim3(grid), dim3(kNT), lds, st, sys, nsys, nmax, nlds);
    });
    return hipGetLastError();
}

}  // namespace XKP_VARIANT
}  // namespace xkp
