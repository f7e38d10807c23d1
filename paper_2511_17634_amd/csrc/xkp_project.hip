// Target projection (Section 3, Phase 2) in launches of its own, spread over the chip (gfx950).
//
// Inside the solve launch each target is projected by the one workgroup that then polishes it,
// so a batch of fewer targets than compute units leaves most of the chip idle during the
// projection.  Here every target's projection is split into row tiles (at most tpt per target),
// one workgroup of 256 threads per (target, tile):
//   gram  the workgroup forms its rows of W = A' V_k (the target operator of Section 2.3 applied
//         to the seed basis) in LDS, 64 rows per wavefront, and accumulates its rows' share of
//         V_k^T W on the matrix cores, FP64 (v_mfma_f64_16x16x4) or, in mixed precision, the
//         FP32 operator rounded to BF16 against the seed's BF16 copy (v_mfma_f32_16x16x32_bf16);
//         and its share of z = V^T r_base (r_base = b - A' x_base) in FP64.  The shares go to a
//         partial slot with device-coherent stores; the last tile of a target to arrive (an
//         arrival counter per target) adds the target's slots in tile order, so the sums do not
//         depend on arrival order, and solves the small system on one wavefront: LU with
//         partial pivoting of V^T A' V or of H_k (the Galerkin modes), Givens rotations on Hbar
//         (the seed least-squares mode)
//   x0    x0 = x_base + V_k alpha by row tiles (x_base where the small system was singular)
// and the solve launch then polishes from x0.  The arithmetic is the in-launch projection's
// (the same operator rows, FP64 z and small solve); only the order of the row sums differs.
#define XKP_NT 256
#define XKP_VARIANT pdev
#include "xkp_device.h"
#include "xkp_internal.h"

#include <mutex>
#include <type_traits>
#include <vector>

namespace xkp {
namespace proj {

using namespace xkp::pdev;

constexpr int NT = 256, NW = NT / 64;
constexpr int KMX = 64;          // largest basis dimension
constexpr int CT = 2;            // column tiles (16 columns each) of W per pass
constexpr int LDW = 66;          // FP64 W chunk in LDS: doubles per column (64 rows + pad)
constexpr int LDB = 72;          // BF16 W chunk: elements per column
constexpr int LDA = KMX + 2;     // the reduced matrix in LDS, row-major
constexpr int kAux = 16;         // cache policy sc1: device-coherent store / load
// LDS (doubles): the four wavefronts' W chunks; after the passes the same space holds the
// reduced matrix, the LU's pivot row, the least-squares right-hand side and alpha
constexpr int kLdsDoubles = NW * 16 * CT * LDW;
static_assert((KMX + 1) * LDA % 2 == 0 && (KMX + 1) * LDA + 3 * KMX + 1 <= kLdsDoubles,
              "LDS too small");

typedef __amdgpu_buffer_rsrc_t rsrc_t;
typedef double double2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

extern __shared__ __attribute__((aligned(16))) double proj_lds[];

__device__ __forceinline__ rsrc_t rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                             0x00020000);
}
__device__ __forceinline__ double ldd(rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ __forceinline__ double2_t ld2_coherent(rsrc_t r, unsigned off) {
    return __builtin_bit_cast(double2_t, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kAux));
}
__device__ __forceinline__ void st_coherent(rsrc_t r, unsigned off, double v) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2_t, v), r, off, 0, kAux);
}

// A value every lane loads from the same address, made uniform word by word: through a generic
// pointer the compiler must assume per-lane private memory, and every buffer descriptor built
// from such a value would be taken as varying across lanes (a loop over lanes per access).
template <typename T>
__device__ __forceinline__ T gload(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "whole words only");
    T v = *p;
    int w[sizeof(T) / 4];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (unsigned q = 0; q < sizeof(T) / 4; ++q) w[q] = __builtin_amdgcn_readfirstlane(w[q]);
    __builtin_memcpy(&v, w, sizeof(T));
    return v;
}

// Row tiles of a system of n unknowns: T tiles of RT rows (a multiple of 256), T <= tpt.
struct Tile {
    int T, RT;
};
__host__ __device__ inline Tile tile_of(int n, int tpt) {
    int t0 = (n + NT - 1) / NT;
    if (t0 > tpt) t0 = tpt;
    const int per = (n + t0 - 1) / t0;
    const int rt = (per + NT - 1) / NT * NT;
    return Tile{(n + rt - 1) / rt, rt};
}

// Arguments of both launches.
struct Args {
    const xkp_system *sys;
    int nsys, n_bases;
    const void *const *bases;
    xkp_params P;
    int tpt, nmax;
    double *part;      // partial slots of sstride doubles: (k+1) x (k+1), row-major
    int sstride;
    unsigned *ctr;     // per target: tiles arrived (zero between launches)
    double *alpha;     // per target: KMX coefficients
    int *stat;         // per target: XKP_OK, XKP_ESINGULAR, XKP_EINVAL, or -1 (bad descriptor)
    xkp_info *infos;
};

// The target's seed basis and its dimension k, or -1 when there is no usable basis (the checks
// of the in-launch projection).
__device__ __forceinline__ int basis_k(const xkp_system &s, int n, const Args &A,
                                        const xkp_basis_header *&hdr) {
    if (s.basis_id < 0 || s.basis_id >= A.n_bases) return -1;
    hdr = (const xkp_basis_header *)gload(A.bases + s.basis_id);
    if (!hdr) return -1;
    const xkp_basis_header h = gload(hdr);
    if (h.n != n || h.m != A.P.m || h.k < 0 || h.k > A.P.m) return -1;
    if (A.P.mode != XKP_PROJ_TARGET_GALERKIN && h.kind != XKP_BASIS_ARNOLDI) return -1;
    if (A.P.precision == XKP_MIXED && A.P.mode == XKP_PROJ_TARGET_GALERKIN && h.bf16 != 1)
        return -1;
    return h.k;
}

// One (target, tile) work item of the Gram launch.
struct Job {
    xkp_system s;
    OpConst o;
    int k, ldv, row0, row1;
    rsrc_t rV, rVb, rP;   // FP64 basis, BF16 basis copy, the item's partial slot
    __device__ __forceinline__ void put(int a, int c, double v) const {
        st_coherent(rP, (unsigned)(a * (k + 1) + c) * 8u, v);
    }
};

// Columns [16 ct0, 16 (ct0 + NTC)) of V_k^T A' V_k over the item's rows: per 256-row sub-tile,
// lane l of wavefront w forms row sub + 64 w + l of those columns of W into the wavefront's LDS
// chunk (column-major), then the wavefront's 64 rows of V_k^T W go through the matrix cores:
//   FP64  v_mfma_f64_16x16x4: A[i][kk] = V[row][16 ta + i] from lane i + 16 kk, B[kk][j] =
//         W[row][col j] likewise, rows 8g + 2(l/16) and the next one of each 8-row group g
//         loaded as one 16-byte pair (the first of the pair in the first product, the other in
//         the second); D[4r + l/16][l%16] in register r of lane l
//   BF16  v_mfma_f32_16x16x32_bf16: lane l holds eight consecutive rows 32q + 8(l/16) of one
//         column (of the BF16 basis copy, and of the BF16-rounded W); D[4(l/16) + r][l%16]
// The per-wavefront tiles are then added over the wavefronts in a fixed order and stored.
template <int KTR, int NTC, bool BF>
__device__ __forceinline__ void gram_pass(const Job &J, int ct0) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int H = J.o.H, k = J.k;
    // FP64: W = [A' V_k | r_base], z = V_k^T r_base its last column; BF16: W = A' V_k
    const int kc = BF ? k : k + 1;
    const int c0 = 16 * ct0;
    const int ncol = kc - c0 < 16 * NTC ? kc - c0 : 16 * NTC;
    typedef typename std::conditional<BF, f32x4_t, double4_t>::type acc_t;
    acc_t acc[KTR][NTC];
#pragma unroll
    for (int a = 0; a < KTR; ++a)
#pragma unroll
        for (int b = 0; b < NTC; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    unsigned offA[KTR];
    bool okA[KTR];
#pragma unroll
    for (int t = 0; t < KTR; ++t) {
        const int a = 16 * t + (lane & 15);
        okA[t] = a < k;
        offA[t] = (unsigned)(okA[t] ? a : 0) * (unsigned)J.ldv * (BF ? 2u : 8u);
    }
    double *Wl = proj_lds + wave * (16 * CT * LDW);
    unsigned short *Wb = (unsigned short *)proj_lds + wave * (16 * CT * LDB);
    const float cdf = (float)J.o.cd;
    for (int sub = J.row0; sub < J.row1; sub += NT) {
        const int p = sub + 64 * wave + lane;
        const bool own = p < J.row1;
        double cE = 0.0, cW = 0.0, cN = 0.0, cS = 0.0;
        int i = 0, j = 0;
        if (own) {
            row_coeffs(J.s, J.o, p, cE, cW, cN, cS);
            i = p / H;
            j = p - i * H;
        }
        const bool hE = own && i + 1 < H, hW = own && i > 0, hN = own && j + 1 < H,
                   hS = own && j > 0;
        const unsigned po = (unsigned)p * 8u;
        const unsigned dH = (unsigned)H * 8u;
        int nst = ncol;   // operator columns of this pass
        if (!BF && c0 + ncol == k + 1) {
            // the last pass ends with r_base = b - A' x_base (FP64 operator)
            nst = ncol - 1;
            double r = 0.0;
            if (own) {
                r = J.s.b[p];
                if (J.s.x0) {
                    const double *x = J.s.x0;
                    const double xE = hE ? x[p + H] : 0.0, xW = hW ? x[p - H] : 0.0;
                    const double xN = hN ? x[p + 1] : 0.0, xS = hS ? x[p - 1] : 0.0;
                    r -= J.o.cd * x[p] + cE * xE + cW * xW + cN * xN + cS * xS;
                }
            }
            Wl[nst * LDW + lane] = r;
        }
#pragma unroll 4
        for (int t = 0; t < nst; ++t) {
            // neighbours outside the grid (and rows past the tile) read as zero, as in the
            // zero-padded copies of the in-launch operator
            const unsigned cb = (unsigned)((c0 + t) * J.ldv) * 8u + po;
            const double vC = own ? ldd(J.rV, cb) : 0.0;
            const double vE = hE ? ldd(J.rV, cb + dH) : 0.0;
            const double vW = hW ? ldd(J.rV, cb - dH) : 0.0;
            const double vN = hN ? ldd(J.rV, cb + 8u) : 0.0;
            const double vS = hS ? ldd(J.rV, cb - 8u) : 0.0;
            if constexpr (!BF) {
                Wl[t * LDW + lane] = J.o.cd * vC + cE * vE + cW * vW + cN * vN + cS * vS;
            } else {
                const float y = cdf * (float)vC + (float)cE * (float)vE + (float)cW * (float)vW +
                                (float)cN * (float)vN + (float)cS * (float)vS;
                Wb[t * LDB + lane] = to_bf16((double)y);
            }
        }
        wave_lds_sync();
        const int wb = sub + 64 * wave;
        if constexpr (!BF) {
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                const int rr = 8 * g + 2 * (lane >> 4);
                const int pr = wb + rr;
                const bool in0 = pr < J.row1, in1 = pr + 1 < J.row1;
                double2_t av[KTR], bv[NTC];
#pragma unroll
                for (int ta = 0; ta < KTR; ++ta) {
                    const double2_t v = __builtin_bit_cast(
                        double2_t,
                        __builtin_amdgcn_raw_buffer_load_b128(J.rV, offA[ta] + (unsigned)pr * 8u, 0, 0));
                    av[ta][0] = (okA[ta] && in0) ? v[0] : 0.0;
                    av[ta][1] = (okA[ta] && in1) ? v[1] : 0.0;
                }
#pragma unroll
                for (int tb = 0; tb < NTC; ++tb)
                    bv[tb] = *(const double2_t *)(Wl + (16 * tb + (lane & 15)) * LDW + rr);
#pragma unroll
                for (int h = 0; h < 2; ++h)
#pragma unroll
                    for (int ta = 0; ta < KTR; ++ta)
#pragma unroll
                        for (int tb = 0; tb < NTC; ++tb)
                            acc[ta][tb] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                av[ta][h], bv[tb][h], acc[ta][tb], 0, 0, 0);
            }
        } else {
            const u32x4_t zero4 = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                // rows pr..pr+7 lie inside their basis column (its length is a multiple of 8
                // above n); groups at or past the tile end are zeroed
                const int rr = 32 * q + 8 * (lane >> 4);
                const int pr = wb + rr;
                const bool in = pr < J.row1;
                bf16x8_t av[KTR], bv[NTC];
#pragma unroll
                for (int ta = 0; ta < KTR; ++ta) {
                    const u32x4_t u = __builtin_amdgcn_raw_buffer_load_b128(
                        J.rVb, offA[ta] + (unsigned)pr * 2u, 0, 0);
                    av[ta] = __builtin_bit_cast(bf16x8_t, (okA[ta] && in) ? u : zero4);
                }
#pragma unroll
                for (int tb = 0; tb < NTC; ++tb)
                    bv[tb] = *(const bf16x8_t *)(Wb + (16 * tb + (lane & 15)) * LDB + rr);
#pragma unroll
                for (int ta = 0; ta < KTR; ++ta)
#pragma unroll
                    for (int tb = 0; tb < NTC; ++tb)
                        acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                            av[ta], bv[tb], acc[ta][tb], 0, 0, 0);
            }
        }
        wave_lds_sync();   // the next sub-tile rewrites this wavefront's chunk
    }
    // every wavefront is done with its chunk: the space serves the cross-wavefront sums
    __syncthreads();
    double *red = proj_lds;
#pragma unroll
    for (int ta = 0; ta < KTR; ++ta) {
#pragma unroll
        for (int tb = 0; tb < NTC; ++tb) {
#pragma unroll
            for (int r = 0; r < 4; ++r) red[wave * 256 + lane * 4 + r] = (double)acc[ta][tb][r];
            __syncthreads();
            {
                const int e = threadIdx.x;   // 256 entries, one per thread
                double sum = 0.0;
#pragma unroll
                for (int w2 = 0; w2 < NW; ++w2) sum += red[w2 * 256 + e];
                const int l = e >> 2, r = e & 3;
                const int a = 16 * ta + (BF ? 4 * (l >> 4) + r : 4 * r + (l >> 4));
                const int c = c0 + 16 * tb + (l & 15);
                if (a < k && c < kc) J.put(a, c, sum);
            }
            __syncthreads();
        }
    }
}

// Entries [q0c, min(q0c + ZC, ka)) of z = V_{ka}^T r_base over the item's rows (column k of the
// slot), FP64, thread t owning row sub + t of each 256-row sub-tile; per-thread sums, then
// wavefront and workgroup sums in a fixed order.  r_base = b - A' x_base with the FP64 operator.
template <int ZC>
__device__ __forceinline__ void z_sweep(const Job &J, int q0c, int ka) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int H = J.o.H;
    double z[ZC];
#pragma unroll
    for (int q = 0; q < ZC; ++q) z[q] = 0.0;
    for (int sub = J.row0; sub < J.row1; sub += NT) {
        const int p = sub + threadIdx.x;
        if (p < J.row1) {
            double r = J.s.b[p];
            if (J.s.x0) {
                double cE, cW, cN, cS;
                row_coeffs(J.s, J.o, p, cE, cW, cN, cS);
                const int i = p / H, j = p - (p / H) * H;
                const double *x = J.s.x0;
                const double xE = (i + 1 < H) ? x[p + H] : 0.0;
                const double xW = (i > 0) ? x[p - H] : 0.0;
                const double xN = (j + 1 < H) ? x[p + 1] : 0.0;
                const double xS = (j > 0) ? x[p - 1] : 0.0;
                r -= J.o.cd * x[p] + cE * xE + cW * xW + cN * xN + cS * xS;
            }
            const unsigned po = (unsigned)p * 8u;
            // sixteen columns at a time, so that the loads in flight stay within the registers
#pragma unroll
            for (int q0 = 0; q0 < ZC; q0 += 16) {
                if (q0c + q0 < ka) {
                    double v[16];
#pragma unroll
                    for (int u = 0; u < 16; ++u) {
                        const int c = q0c + q0 + u;
                        v[u] = c < ka ? ldd(J.rV, (unsigned)(c * J.ldv) * 8u + po) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 16; ++u) z[q0 + u] += v[u] * r;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    double *red = proj_lds;
#pragma unroll
    for (int q = 0; q < ZC; ++q) {
        if (q0c + q < ka) {
            const double s = wave_sum(z[q]);
            if (lane == 0) red[q * NW + wave] = s;
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q0c + q < ka && q < ZC; q += NT)
        J.put(q0c + q, J.k, tree_sum<NW>(red + q * NW));
    __syncthreads();
}

template <bool BF>
__device__ __forceinline__ void gram_all(const Job &J) {
    const int ktr = (J.k + 15) / 16;
    const int ktc = (J.k + (BF ? 15 : 16)) / 16;   // FP64: the r_base column too
    for (int ct0 = 0; ct0 < ktc; ct0 += CT) {
        const int ntc = ktc - ct0 < CT ? ktc - ct0 : CT;
#define XKP_PASS(R_, C_) gram_pass<R_, C_, BF>(J, ct0)
        switch (ktr * 2 + ntc - 1) {
        case 2: XKP_PASS(1, 1); break;
        case 3: XKP_PASS(1, 2); break;
        case 4: XKP_PASS(2, 1); break;
        case 5: XKP_PASS(2, 2); break;
        case 6: XKP_PASS(3, 1); break;
        case 7: XKP_PASS(3, 2); break;
        case 8: XKP_PASS(4, 1); break;
        case 9: XKP_PASS(4, 2); break;
        default: break;
        }
#undef XKP_PASS
    }
}

__global__ __launch_bounds__(NT, 2) void gram_kernel(Args A) {
    __shared__ int last;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int items = A.nsys * A.tpt;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int t = item / A.tpt, j = item - (item / A.tpt) * A.tpt;
        const xkp_system s = gload(A.sys + t);
        xkp_info *info = A.infos + t;
        if (!desc_ok(s, A.nmax)) {
            if (j == 0 && tid == 0) A.stat[t] = -1;   // the solve launch reports it
            continue;
        }
        const int n = s.H * s.H;
        const xkp_basis_header *hdr = nullptr;
        const int k = basis_k(s, n, A, hdr);
        if (k < 0) {
            if (j == 0 && tid == 0) {
                info->status = XKP_EINVAL;
                info->basis_dim = 0;
                A.stat[t] = XKP_EINVAL;
            }
            continue;
        }
        const Tile tl = tile_of(n, A.tpt);
        if (j >= tl.T) continue;
        if (k == 0) {   // an empty basis: x0 = x_base
            if (j == 0 && tid == 0) {
                info->basis_dim = 0;
                A.stat[t] = XKP_OK;
            }
            continue;
        }
        const int m = A.P.m;
        const int ldv = (n + 8) & ~7;
        const double *V = (const double *)((const char *)hdr + 256);
        const unsigned short *Vb =
            (const unsigned short *)((const char *)hdr + basis_off_vb(n, m));
        // one slot per item when targets are split, else the workgroup's own slot
        const int slot = A.tpt > 1 ? item : (int)blockIdx.x;
        Job J;
        J.s = s;
        J.o = op_const(s);
        J.k = k;
        J.ldv = ldv;
        J.row0 = j * tl.RT;
        J.row1 = J.row0 + tl.RT < n ? J.row0 + tl.RT : n;
        J.rV = rsrc(V, (unsigned)ldv * (unsigned)(k + 1) * 8u);
        J.rVb = rsrc(Vb, (unsigned)ldv * (unsigned)k * 2u);
        J.rP = rsrc(A.part + (size_t)slot * A.sstride, (unsigned)A.sstride * 8u);
        const int mode = A.P.mode;
        const bool tg = mode == XKP_PROJ_TARGET_GALERKIN;
        const int ka = mode == XKP_PROJ_SEED_LSQ ? k + 1 : k;
        if (tg) {
            if (A.P.precision == XKP_MIXED)
                gram_all<true>(J);
            else
                gram_all<false>(J);
        }
        // z separately where the FP64 Gram pass does not carry it (mixed precision, the seed
        // modes); at most 48 entries per sweep: the per-thread sums stay in registers
        if (!tg || A.P.precision == XKP_MIXED) {
            if (ka <= 16) {
                z_sweep<16>(J, 0, ka);
            } else if (ka <= 32) {
                z_sweep<32>(J, 0, ka);
            } else {
                z_sweep<48>(J, 0, ka);
                if (ka > 48) z_sweep<32>(J, 48, ka);
            }
        }
        // the slot's device-coherent stores (uncached memory: they reach the memory side, not
        // this XCD's L2) have completed once every thread's store counter is zero; then the
        // target's last tile to arrive goes on and reads the slots with device-coherent loads
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (tl.T > 1) {
            if (tid == 0) last = atomicAdd(A.ctr + t, 1u) == (unsigned)(tl.T - 1);
            __syncthreads();
            // the same for every thread (read from LDS): say so, or the compiler takes the
            // item loop's exit, and every descriptor after it, as varying across lanes
            const bool go = __builtin_amdgcn_readfirstlane(last) != 0;
            __syncthreads();   // read before the next item may set it again
            if (!go) continue;
            if (tid == 0) atomicExch(A.ctr + t, 0u);   // ready for the next launch
        }
        // the target's slots summed in tile order into the LDS matrix (row-major, LDA)
        double *Ap = proj_lds;
        double *zbuf = Ap + (KMX + 1) * LDA;   // the LU's stored right-hand side entries
        double *zl = zbuf + KMX;
        double *al = zl + KMX + 1;
        const int nc = k + 1;
        const int first = A.tpt > 1 ? t * A.tpt : slot;
        const rsrc_t rAll = rsrc(A.part + (size_t)first * A.sstride,
                                 (unsigned)(A.sstride * tl.T) * 8u);
        const int npair = (ka * nc + 1) / 2;
        for (int e2 = tid; e2 < npair; e2 += NT) {
            double2_t sum = {0.0, 0.0};
            for (int j0 = 0; j0 < tl.T; j0 += 8) {
                double2_t v[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    v[u] = j0 + u < tl.T
                               ? ld2_coherent(rAll, (unsigned)((j0 + u) * A.sstride + 2 * e2) * 8u)
                               : double2_t{0.0, 0.0};
#pragma unroll
                for (int u = 0; u < 8; ++u)
                    if (j0 + u < tl.T) sum += v[u];
            }
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int e = 2 * e2 + h;
                if (e < ka * nc) {
                    const int a = e / nc, c = e - (e / nc) * nc;
                    if (tg || c == k) Ap[a * LDA + c] = sum[h];
                }
            }
        }
        if (!tg) {
            // the seed modes: H_k (Galerkin) or Hbar (least squares) from the basis buffer
            const double *Hb = (const double *)((const char *)hdr + basis_off_h(n, m));
            for (int e = tid; e < ka * k; e += NT) {
                const int a = e / k, c = e - (e / k) * k;
                Ap[a * LDA + c] = Hb[(size_t)c * (m + 1) + a];
            }
        }
        __syncthreads();
        bool singular = false;
        if (mode == XKP_PROJ_SEED_LSQ) {
            if (wave == 0) {
                if (lane <= k) zl[lane] = Ap[lane * LDA + k];
                wave_lds_sync();
                singular = lsq_hessenberg_wave(Ap, LDA, k, zl, al);
            }
        } else if (wave == 0) {
            // the Galerkin modes: the right-hand side z is column k
            const double zr = lane < k ? Ap[lane * LDA + k] : 0.0;
            if (k <= 16) singular = lu_regs<16>(Ap, LDA, k, zr, al, zbuf);
            else if (k <= 32) singular = lu_regs<32>(Ap, LDA, k, zr, al, zbuf);
            else if (k <= 48) singular = lu_regs<48>(Ap, LDA, k, zr, al, zbuf);
            else singular = lu_regs<64>(Ap, LDA, k, zr, al, zbuf);
        }
        if (wave == 0) {
            if (!singular && lane < k) A.alpha[(size_t)t * KMX + lane] = al[lane];
            if (lane == 0) {
                info->basis_dim = k;
                A.stat[t] = singular ? XKP_ESINGULAR : XKP_OK;
            }
        }
        __syncthreads();   // the LDS is the next item's
    }
}

// x0 = x_base + V_k alpha on the item's rows (x_base, or zero, where the system was singular);
// the FP64 sum in column order, as the in-launch projection forms it.
__global__ __launch_bounds__(NT) void x0_kernel(Args A) {
    const int items = A.nsys * A.tpt;
    for (int item = blockIdx.x; item < items; item += gridDim.x) {
        const int t = item / A.tpt, j = item - (item / A.tpt) * A.tpt;
        const xkp_system s = gload(A.sys + t);
        if (!desc_ok(s, A.nmax)) continue;
        const int st = gload(A.stat + t);
        if (st != XKP_OK && st != XKP_ESINGULAR) continue;
        const int n = s.H * s.H;
        const Tile tl = tile_of(n, A.tpt);
        if (j >= tl.T) continue;
        const xkp_basis_header *hdr = (const xkp_basis_header *)gload(A.bases + s.basis_id);
        const int k = st == XKP_OK ? gload(&hdr->k) : 0;
        const int ldv = (n + 8) & ~7;
        const double *V = (const double *)((const char *)hdr + 256);
        const double *al = A.alpha + (size_t)t * KMX;
        const int row0 = j * tl.RT;
        const int row1 = row0 + tl.RT < n ? row0 + tl.RT : n;
        // four rows per thread and four columns at a time: sixteen loads in flight, each row's
        // sum still taken column by column
        for (int p0 = row0 + threadIdx.x; p0 < row1; p0 += 4 * NT) {
            double x[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + r * NT;
                x[r] = (p < row1 && s.x0) ? s.x0[p] : 0.0;
            }
            for (int c = 0; c < k; c += 4) {
                double a[4], v[4][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    a[q] = c + q < k ? al[c + q] : 0.0;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int p = p0 + r * NT;
                        v[q][r] = (c + q < k && p < row1) ? V[(size_t)(c + q) * ldv + p] : 0.0;
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (c + q < k) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) x[r] += a[q] * v[q][r];
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int p = p0 + r * NT;
                if (p < row1) s.x[p] = x[r];
            }
        }
    }
}

// Raises the Gram kernel's dynamic-LDS limit once per device.
hipError_t set_lds() {
    static std::mutex mu;
    static std::vector<int> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> g(mu);
    for (int d : done)
        if (d == dev) return hipSuccess;
    e = hipFuncSetAttribute((const void *)gram_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(double) * kLdsDoubles));
    if (e == hipSuccess) done.push_back(dev);
    return e;
}

// doubles per partial slot (even, so that entry pairs stay 16-byte aligned)
int slot_doubles(int mmax) { return ((mmax + 1) * (mmax + 1) + 1) & ~1; }

// Tiles per target: at most one per 256 rows of the largest system, at most tiles_cap (when
// > 0), else about as many items as the chip holds Gram workgroups at once (two per compute
// unit, so that the items run in one round), and never more than the partial slots hold.
int tiles_per_target(int nsys, int nmax, int slots, int tiles_cap, int cus) {
    int tpt = (nmax + NT - 1) / NT;
    if (tiles_cap > 0 && tpt > tiles_cap) tpt = tiles_cap;
    if (tiles_cap == 0 && nsys > 0 && tpt > 2 * cus / nsys) tpt = 2 * cus / nsys;
    if (nsys > 0 && tpt > slots / nsys) tpt = slots / nsys;
    return tpt < 1 ? 1 : tpt;
}

hipError_t launch_project(hipStream_t st, const xkp_system *sys, int nsys, int n_bases,
                          const void *const *bases, xkp_params P, int nmax, double *part,
                          int slots, int sstride, unsigned *ctr, double *alpha, int *stat,
                          xkp_info *infos, int tiles_cap, int cus) {
    if (nsys < 1) return hipSuccess;
    hipError_t e = set_lds();
    if (e != hipSuccess) return e;
    Args A;
    A.sys = sys;
    A.nsys = nsys;
    A.n_bases = n_bases;
    A.bases = bases;
    A.P = P;
    A.tpt = tiles_per_target(nsys, nmax, slots, tiles_cap, cus);
    A.nmax = nmax;
    A.part = part;
    A.sstride = sstride;
    A.ctr = ctr;
    A.alpha = alpha;
    A.stat = stat;
    A.infos = infos;
    const int items = nsys * A.tpt;
    // split targets: one workgroup (and slot) per item; whole targets: at most one workgroup
    // per slot, each reusing its slot
    const int grid = A.tpt > 1 ? items : (nsys < slots ? nsys : slots);
    hipLaunchKernelGGL(gram_kernel, dim3(grid), dim3(NT), sizeof(double) * kLdsDoubles, st, A);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int grid2 = items < 4096 ? items : 4096;
    hipLaunchKernelGGL(x0_kernel, dim3(grid2), dim3(NT), 0, st, A);
    return hipGetLastError();
}

}  // namespace proj
}  // namespace xkp
