// Seed solve spread over several workgroups (gfx950).
//
// A seed is one system per timestep on the projected chain's critical path (Section 3, Phase 1:
// every target of the timestep waits for its basis), so one workgroup per seed leaves the chip
// idle while it runs.  Here each seed is split into G = ceil(n / 256) contiguous row blocks,
// one workgroup of 256 threads per block, thread t owning row p = 256 g + t; the block keeps its
// rows of every basis vector of the current cycle in LDS, so the Gram-Schmidt passes read no
// device memory.  Per Arnoldi step:
//   operator   w = A v_j on the owned rows; the neighbours H rows away come from the adjacent
//              blocks' boundary rows (exchanged), the rest from the block's own LDS vector
//   Gram-Schmidt  two classical passes (CGS2): pass k forms the block's share of V^T w (and of
//              ||w||^2), the G shares are exchanged and summed in a fixed order (the same in
//              every workgroup, so every workgroup holds bitwise the same sums and takes the
//              same decisions), w -= V h; ||w2||^2 = ||w1||^2 - ||h2||^2
//   then       v_{j+1} = w2 / ||w2|| on the owned rows, its boundary rows exchanged for the next
//              operator application; the Givens rotations by the first wavefront of every
//              workgroup, identically
// i.e. three exchanges per step.  The basis, Hessenberg matrix, header, solution and info are
// those of the single-workgroup seed solve (restarted GMRES from x0, first cycle kept); the two
// classical passes give an orthonormal basis to working precision as two modified passes do.
//
// An exchange round: each workgroup publishes its values as tagged units (below) in the seed's
// exchange area (uncached device memory, so that workgroups on different XCDs see each other's
// stores) and polls the units it needs until they carry the round's tag.  Every wait is bounded
// in time: a workgroup whose partners do not arrive (they must all be resident at once) gives
// up, the seed gets XKP_EDEVICE, and the caller solves it again on one workgroup.  A seed's
// workgroups share one XCD (ids congruent mod 8) when G <= 32; larger seeds spread over the
// XCDs.
#define XKP_NT 256
#define XKP_VARIANT wdev
#include "xkp_device.h"
#include "xkp_internal.h"

#include <mutex>
#include <vector>

namespace xkp {
namespace wide {

using namespace xkp::wdev;

constexpr int NT = 256, NW = NT / 64;
constexpr int HM = 128;                    // largest grid side (halo rows on each side)
constexpr int kMM = 64;                    // largest restart length
constexpr int kWV = kMM + 4;               // values of one exchange (j + 2 <= kMM + 1)
constexpr int kSeg = 4;                    // threads (block segments) per reduced value

// Per-seed exchange area: four rounds of per-workgroup value slots, then two rounds of
// per-workgroup boundary rows (low H rows, high H rows).  Every published double is a 16-byte
// unit {low word, tag, high word, tag} written with one store: a reader that sees both tags
// equal to the round it waits for has the value (no separate flag, no counter), and a launch
// starts by setting every tag to 0xFFFFFFFF, a round no solve reaches.
// Reuse of a slot: a round that exchanges only boundary rows ties a workgroup to its two
// neighbours, not to all, and up to two such rounds follow each other (the last step's row
// exchange, then the new x's), so a workgroup may publish values up to three rounds after a
// round whose values a distant workgroup is still reading: value slots rotate over four rounds.
// Boundary rows are read by the neighbours only, which have finished the previous round before
// a workgroup can start the next one, so two rounds suffice there.
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));
constexpr int kAux = 16;   // cache policy sc1: device-coherent store / load
__host__ __device__ inline size_t xch_units(int gmax) {
    return 4 * (size_t)gmax * kWV + 2 * (size_t)gmax * 2 * HM;
}
size_t xch_bytes(int gmax) { return (16 * xch_units(gmax) + 255) & ~(size_t)255; }
int rows_per_block() { return NT; }

struct Wide {
    __amdgpu_buffer_rsrc_t rs;   // the seed's exchange area
    int gmax, G, g;
    unsigned round;
    long long limit;
    int *abort_lds;
    double *red, *tot, *seg;   // LDS

    __device__ __forceinline__ unsigned part_unit(unsigned rnd, int gg, int v) const {
        return (unsigned)(((size_t)(rnd & 3) * gmax + gg) * kWV + v);
    }
    __device__ __forceinline__ unsigned bnd_unit(unsigned rnd, int gg, int side, int t) const {
        return (unsigned)(4 * (size_t)gmax * kWV + (((size_t)(rnd & 1) * gmax + gg) * 2 + side) * HM + t);
    }
    __device__ __forceinline__ void put(unsigned unit, double v) const {
        const unsigned lo = __double2loint(v), hi = __double2hiint(v);
        __builtin_amdgcn_raw_buffer_store_b128(u32x4_t{lo, round, hi, round}, rs, unit * 16u, 0,
                                               kAux);
    }
    __device__ __forceinline__ u32x4_t load(unsigned unit) const {
        return __builtin_amdgcn_raw_buffer_load_b128(rs, unit * 16u, 0, kAux);
    }
    static __device__ __forceinline__ bool ready(u32x4_t u, unsigned rnd) {
        return u[1] == rnd && u[3] == rnd;
    }
    static __device__ __forceinline__ double value(u32x4_t u) {
        return __hiloint2double((int)u[2], (int)u[0]);
    }
    // the unit's value once it carries round rnd; false (and the workgroup told) on time-out.
    // The pause between polls doubles up to about 2 us, so that workgroups waiting long (for
    // partners not yet resident) do not flood the memory system with polls.
    __device__ __forceinline__ bool wait(unsigned unit, unsigned rnd, u32x4_t &u) const {
        if (ready(u, rnd)) return true;
        const long long t0 = __builtin_amdgcn_s_memrealtime();
        int pause = 1;
        for (;;) {
            if (*(volatile int *)abort_lds) return false;   // another wait already gave up
            u = load(unit);
            if (ready(u, rnd)) return true;
            if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                *(volatile int *)abort_lds = 1;
                return false;
            }
            for (int i = 0; i < pause; ++i) __builtin_amdgcn_s_sleep(1);
            if (pause < 64) pause *= 2;
        }
    }
    // ends a round: every thread has its data; false if a wait timed out anywhere
    __device__ __forceinline__ bool end_round() {
        __syncthreads();
        ++round;
        return *abort_lds == 0;
    }
    // The workgroup's share of nv values, already summed per wave in red[v * NW + wave], is
    // published; then tot[v] = the sums over the G blocks: kSeg threads per value each load one
    // segment of ceil(G / kSeg) consecutive blocks' shares at once (up to 16) and add them in
    // block order, and the segment sums are added as a fixed tree, the same in every workgroup.
    // Callers may publish other units of this round before calling.
    __device__ __forceinline__ bool reduce(int nv) {
        __syncthreads();
        const unsigned rnd = round;
        for (int v = threadIdx.x; v < nv; v += NT) put(part_unit(rnd, g, v), tree_sum<NW>(red + v * NW));
        const int L = (G + kSeg - 1) / kSeg;
        for (int idx = threadIdx.x; idx < nv * kSeg; idx += NT) {
            const int v = idx / kSeg, g0 = (idx - v * kSeg) * L;
            const int g1 = g0 + L < G ? g0 + L : G;
            double t = 0.0;
            for (int gb = g0; gb < g1; gb += 16) {
                u32x4_t sh[16];
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    sh[e] = gb + e < g1 ? load(part_unit(rnd, gb + e, v)) : u32x4_t{0, 0, 0, 0};
#pragma unroll
                for (int e = 0; e < 16; ++e)
                    if (gb + e < g1 && wait(part_unit(rnd, gb + e, v), rnd, sh[e]))
                        t += value(sh[e]);
            }
            seg[idx] = t;
        }
        __syncthreads();
        for (int v = threadIdx.x; v < nv; v += NT) tot[v] = tree_sum<kSeg>(seg + v * kSeg);
        return end_round();
    }
};

// Wave sums of four values at once (independent chains interleave), lane 0 storing them.
__device__ __forceinline__ void wave_put4(double a, double b, double c, double d, double *red,
                                          int v0, int nv) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    d = wave_sum(d);
    if (lane == 0) {
        red[v0 * NW + wave] = a;
        if (v0 + 1 < nv) red[(v0 + 1) * NW + wave] = b;
        if (v0 + 2 < nv) red[(v0 + 2) * NW + wave] = c;
        if (v0 + 3 < nv) red[(v0 + 3) * NW + wave] = d;
    }
}

// The wave's sums of 16 values d[0..16) at once (values v0 + i, those < nv kept;
// wave_bfly16), lanes 0..15 writing them to red[v * NW + wave].
__device__ __forceinline__ void wave_put16(double (&d)[16], double *red, int v0, int nv) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const double s = wave_bfly16(d);
    const int v = v0 + bfly_index(lane);
    if (lane < 16 && v < nv) red[v * NW + wave] = s;
}

// w - sum_{c <= j} h[c] V[c NT] (this thread's row of columns 0..j, LDS), subtracted in column
// order, four columns' loads at a time; with SQ also c2 += h[c]^2 in the same order.
template <bool SQ>
__device__ __forceinline__ double sub_cols(double w, int j, const double *h, const double *V,
                                           double &c2) {
    int c = 0;
    for (; c + 3 <= j; c += 4) {
        const double v0 = V[c * NT], v1 = V[(c + 1) * NT], v2 = V[(c + 2) * NT];
        const double v3 = V[(c + 3) * NT];
        const double h0 = h[c], h1 = h[c + 1], h2 = h[c + 2], h3 = h[c + 3];
        if (SQ) {
            c2 += h0 * h0;
            c2 += h1 * h1;
            c2 += h2 * h2;
            c2 += h3 * h3;
        }
        w -= h0 * v0;
        w -= h1 * v1;
        w -= h2 * v2;
        w -= h3 * v3;
    }
    for (; c <= j; ++c) {
        const double hc = h[c];
        if (SQ) c2 += hc * hc;
        w -= hc * V[c * NT];
    }
    return w;
}

// LDS layout (doubles), mmax = the largest cycle length of the call:
//   Vl    (mmax + 1) x NT: the block's rows of the cycle's basis vectors, column-major
//   vbuf  NT + 2 HM: the operator's input, owned rows at HM + t, halos around them
//   red   kWV x NW, tot kWV, seg kWV x kSeg, Rp mmax (mmax + 1) / 2, cs, sn, yv mmax,
//   gv mmax + 1, flags
__host__ __device__ inline size_t lds_doubles(int mmax) {
    return (size_t)(mmax + 1) * NT + NT + 2 * HM + kWV * NW + kWV + kWV * kSeg +
           (size_t)mmax * (mmax + 1) / 2 + 4 * (size_t)mmax + 1 + 2;
}

__global__ __launch_bounds__(NT) void wide_seed_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                       xkp_params P, void *const *keep_bases,
                                                       xkp_info *infos, unsigned char *xch,
                                                       size_t xch_stride, int gmax, int packed,
                                                       int nmax, long long limit) {
    const int tid = threadIdx.x;
    // seed si, block g: packed, a seed's blocks share an XCD (ids congruent mod 8)
    int si, g;
    if (packed) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        si = xcd + 8 * (slot / gmax);
        g = slot % gmax;
    } else {
        si = blockIdx.x / gmax;
        g = blockIdx.x % gmax;
    }
    if (si >= nsys) return;
    const xkp_system s = sys[si];
    xkp_info *info = infos + si;
    const int H = s.H;
    const int m = P.m, mpol = P.polish_m > 0 ? P.polish_m : P.m;
    const int mmax = m > mpol ? m : mpol;
    const bool ok = H > 0 && H <= HM && (long)H * H <= nmax && s.mt && s.b && s.x &&
                    s.dt > 0.0 && keep_bases[si] != nullptr && P.m >= 1 && P.m <= kMM &&
                    P.polish_m >= 0 && P.polish_m <= kMM;
    if (!ok) {
        if (g == 0 && tid == 0) info->status = XKP_EINVAL;
        return;
    }
    const int n = H * H, G = (n + NT - 1) / NT;
    if (g >= G) return;

    extern __shared__ __attribute__((aligned(16))) double lds[];
    double *Vl = lds;
    double *vbuf = Vl + (size_t)(mmax + 1) * NT;
    double *red = vbuf + NT + 2 * HM;
    double *tot = red + kWV * NW;
    double *seg = tot + kWV;
    double *Rp = seg + kWV * kSeg;
    double *cs = Rp + (size_t)mmax * (mmax + 1) / 2, *sn = cs + mmax, *yv = sn + mmax;
    double *gv = yv + mmax;
    int *flags = (int *)(gv + mmax + 1);

    if (tid == 0) flags[0] = 0;
    for (int t = tid; t < NT + 2 * HM; t += NT) vbuf[t] = 0.0;
    __syncthreads();
    unsigned char *xs = xch + (size_t)si * xch_stride;
    Wide X{__builtin_amdgcn_make_buffer_rsrc(xs, (short)0, (int)xch_stride, 0x00020000), gmax,
           G, g, 0u, limit, flags, red, tot, seg};

    // this thread's row p = g NT + tid; rows at or past n (last block) are zero throughout
    const int base = g * NT, p = base + tid;
    const bool own = p < n;
    const OpConst o = op_const(s);
    double cE = 0.0, cW = 0.0, cN = 0.0, cS = 0.0;
    if (own) {
        const int i = p / H, j = p - (p / H) * H;
        const double mE = (i + 1 < H) ? s.mt[p + H] : 0.0;
        const double mW = (i > 0) ? s.mt[p - H] : 0.0;
        const double mN = (j + 1 < H) ? s.mt[p + 1] : 0.0;
        const double mS = (j > 0) ? s.mt[p - 1] : 0.0;
        const double fxp = s.fx ? s.fx[p] : 0.0;
        const double fyp = s.fy ? s.fy[p] : 0.0;
        const double ex = fxp * o.inv2h - o.c8 * (mE - mW);
        const double ey = fyp * o.inv2h - o.c8 * (mN - mS);
        cE = (i + 1 < H) ? -o.a + ex : 0.0;
        cW = (i > 0) ? -o.a - ex : 0.0;
        cN = (j + 1 < H) ? -o.a + ey : 0.0;
        cS = (j > 0) ? -o.a - ey : 0.0;
    }
    // y = A u for this row, u in vbuf
    auto apply = [&]() {
        const double *u = vbuf + HM + tid;
        return o.cd * u[0] + cE * u[H] + cW * u[-H] + cN * u[1] + cS * u[-1];
    };
    // this row's value, if it is a boundary row, to the neighbours (this round)
    auto publish_bnd = [&](double v) {
        if (tid < H) X.put(X.bnd_unit(X.round, g, 0, tid), v);
        if (tid >= NT - H) X.put(X.bnd_unit(X.round, g, 1, tid - (NT - H)), v);
    };
    // the halos from the neighbours' boundary rows of this round (before end_round)
    auto get_halo = [&]() {
        const unsigned rnd = X.round;
        for (int t = tid; t < H; t += NT) {
            double lo = 0.0, hi = 0.0;
            u32x4_t u0 = g > 0 ? X.load(X.bnd_unit(rnd, g - 1, 1, t)) : u32x4_t{0, 0, 0, 0};
            u32x4_t u1 = g + 1 < G ? X.load(X.bnd_unit(rnd, g + 1, 0, t)) : u32x4_t{0, 0, 0, 0};
            if (g > 0 && X.wait(X.bnd_unit(rnd, g - 1, 1, t), rnd, u0)) lo = Wide::value(u0);
            if (g + 1 < G && X.wait(X.bnd_unit(rnd, g + 1, 0, t), rnd, u1)) hi = Wide::value(u1);
            vbuf[HM - H + t] = lo;
            vbuf[HM + NT + t] = hi;
        }
    };
    // this row into the LDS vector and the neighbours' halos, theirs into ours: one round
    auto exchange_row = [&](double v) -> bool {
        vbuf[HM + tid] = v;
        publish_bnd(v);
        get_halo();
        return X.end_round();
    };
    // one classical pass over columns 0..j: the block's shares of V^T w and ||w||^2, summed
    // over the blocks into tot[0..j+1]
    auto pass = [&](int j, double w) -> bool {
        for (int c0 = 0; c0 <= j + 1; c0 += 16) {
            double d[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int c = c0 + e;
                d[e] = c <= j ? Vl[c * NT + tid] * w : (c == j + 1 ? w * w : 0.0);
            }
            wave_put16(d, red, c0, j + 2);
        }
        return X.reduce(j + 2);
    };

    xkp_basis_header *hdr = (xkp_basis_header *)keep_bases[si];
    const int ldv = (n + 8) & ~7;
    double *Vk = (double *)((char *)hdr + 256);
    double *Hb = (double *)((char *)hdr + basis_off_h(n, m));
    unsigned short *Vb = P.precision == XKP_MIXED
                             ? (unsigned short *)((char *)hdr + basis_off_vb(n, m))
                             : nullptr;
    if (g == 0)
        for (int t = tid; t < (m + 1) * m; t += NT) Hb[t] = 0.0;

    const double b = own ? s.b[p] : 0.0;
    double x = (own && s.x0) ? s.x0[p] : 0.0;
    // x halo for the first residual: straight from the input x0 (or zero)
    for (int t = tid; t < H; t += NT) {
        const int pl = base - H + t, ph = base + NT + t;
        vbuf[HM - H + t] = (s.x0 && pl >= 0 && pl < n) ? s.x0[pl] : 0.0;
        vbuf[HM + NT + t] = (s.x0 && ph < n) ? s.x0[ph] : 0.0;
    }
    vbuf[HM + tid] = x;
    __syncthreads();

    int iters = 0, restarts = 0, kfirst = 0, status = XKP_OK;
    double res_est = 0.0, res_true = 0.0, beta_first = 0.0, bnorm = 0.0, beta = 0.0, r = 0.0;
    bool alive = true, first = true;
    // r = b - A x (x in the LDS vector with its halos), ||r|| (and ||b|| on the first call),
    // r's boundary rows exchanged into the halos: one exchange
    auto residual = [&](bool with_b) -> bool {
        r = own ? b - apply() : 0.0;
        wave_put4(r * r, b * b, 0.0, 0.0, red, 0, 2);
        // r's boundary rows in the same round as the norms
        __syncthreads();   // every thread has read the LDS vector (x) before the halos change
        publish_bnd(r);
        get_halo();
        if (!X.reduce(2)) return false;
        beta = sqrt(tot[0]);
        if (with_b) bnorm = sqrt(tot[1]);
        return true;
    };
    alive = residual(true);
    if (own) s.x[p] = x;
    // data that are not finite (NaN or Inf in m~, f, b or x0) cannot be solved
    if (alive && (!isfinite(beta) || !isfinite(bnorm))) status = XKP_EINVAL;
    if (alive && status == XKP_OK && bnorm > 0.0) {
        res_true = res_est = beta / bnorm;
        while (alive && beta > P.tol * bnorm) {
            const bool keep = first;
            const int mc = keep ? m : mpol;
            // v_0 = r / beta (this row and the halos)
            const double rb0 = 1.0 / beta;
            double w = own ? r * rb0 : 0.0;
            vbuf[HM + tid] = w;
            for (int t = tid; t < H; t += NT) {
                vbuf[HM - H + t] *= rb0;
                vbuf[HM + NT + t] *= rb0;
            }
            Vl[tid] = w;
            if (keep) {
                if (own) {
                    Vk[p] = w;
                    if (Vb) Vb[p] = to_bf16(w);
                }
                if (g + 1 == G)
                    for (int q = n + tid; q < ldv; q += NT) Vk[q] = 0.0;
                beta_first = beta;
            }
            __syncthreads();
            double gcur = beta;
            int kk = 0;
            for (int j = 0; j < mc; ++j) {
                w = apply();
                ++iters;
                if (!(alive = pass(j, w))) break;
                const double wn0 = sqrt(tot[j + 1]);
                double c2 = 0.0;
                w = sub_cols<false>(w, j, tot, Vl + tid, c2);
                // pass 1's coefficients wait in yv while pass 2 reuses tot
                for (int c = tid; c <= j; c += NT) yv[c] = tot[c];
                if (!(alive = pass(j, w))) break;
                w = sub_cols<true>(w, j, tot, Vl + tid, c2);
                const double hn = sqrt(fmax(tot[j + 1] - c2, 0.0));
                const bool brk = !(hn > 1e-14 * wn0);
                const double rhn = brk ? 0.0 : 1.0 / hn;
                w = own ? w * rhn : 0.0;
                Vl[(j + 1) * NT + tid] = w;
                if (keep) {
                    if (own) {
                        Vk[(size_t)(j + 1) * ldv + p] = w;
                        if (Vb) Vb[(size_t)(j + 1) * ldv + p] = to_bf16(w);
                    }
                    if (g + 1 == G)
                        for (int q = n + tid; q < ldv; q += NT)
                            Vk[(size_t)(j + 1) * ldv + q] = 0.0;
                    // unrotated Hessenberg column j (its other entries are zero), by block 0
                    if (g == 0)
                        for (int rr = tid; rr <= j + 1; rr += NT)
                            Hb[(size_t)j * (m + 1) + rr] = rr <= j ? yv[rr] + tot[rr] : hn;
                }
                // v_{j+1}'s boundary rows to the neighbours first (every thread has read the
                // LDS vector in this step's operator application, before the reductions), then
                // the Givens rotations of column j by the first wavefront while those rows travel:
                // lane i holds entry i of the column and rotation i, the chain reads them with
                // readlane, and lane i keeps rotated entry i; the others take the new rotation
                // from the LDS after the round
                vbuf[HM + tid] = w;
                publish_bnd(w);
                if (tid < 64) {
                    const double hl = tid <= j ? yv[tid] + tot[tid] : 0.0;
                    const double cl = tid < j ? cs[tid] : 0.0, sl = tid < j ? sn[tid] : 0.0;
                    double t = readlane_d(hl, 0), rl = 0.0;
#pragma unroll 4
                    for (int i = 1; i <= j; ++i) {
                        const double c = readlane_d(cl, i - 1), sv = readlane_d(sl, i - 1);
                        const double hi = readlane_d(hl, i);
                        const double rrv = c * t + sv * hi;
                        t = -sv * t + c * hi;
                        if (tid == i - 1) rl = rrv;
                    }
                    if (tid < j) Rp[(j * (j + 1)) / 2 + tid] = rl;
                    if (tid == 0) {
                        const double den = sqrt(t * t + hn * hn);
                        const double rden = 1.0 / den;
                        Rp[(j * (j + 1)) / 2 + j] = den;
                        cs[j] = t * rden;
                        sn[j] = hn * rden;
                        gv[j] = t * rden * gcur;
                    }
                }
                // the neighbours' rows into the halos; the round's barrier also publishes the
                // rotation to every thread
                get_halo();
                if (!(alive = X.end_round())) break;
                gcur = -sn[j] * gcur;
                kk = j + 1;
                if (fabs(gcur) <= P.tol * bnorm || brk) break;
            }
            if (!alive) break;
            res_est = fabs(gcur) / bnorm;
            // y = R^{-1} g by one wavefront (lane c holds g_c and 1 / R_cc)
            if (tid < 64) {
                double gl = (tid < kk) ? gv[tid] : 0.0;
                const double rdiag = (tid < kk) ? 1.0 / Rp[(tid * (tid + 1)) / 2 + tid] : 0.0;
                for (int c = kk - 1; c >= 0; --c) {
                    const double yc = readlane_d(gl, c) * readlane_d(rdiag, c);
                    if (tid < c) gl -= Rp[(c * (c + 1)) / 2 + tid] * yc;
                    if (tid == 0) yv[c] = yc;
                }
            }
            __syncthreads();
            for (int c = 0; c < kk; ++c) x += yv[c] * Vl[c * NT + tid];
            if (own) s.x[p] = x;
            if (first) {
                kfirst = kk;
                first = false;
            }
            // the new x's boundary rows, then the true residual in FP64
            __syncthreads();   // every thread has read yv
            if (!(alive = exchange_row(x))) break;
            if (!(alive = residual(false))) break;
            res_true = beta / bnorm;
            if (beta <= P.tol * bnorm) break;
            if (!isfinite(beta)) {
                status = XKP_EINVAL;
                break;
            }
            if (restarts >= P.max_restarts) {
                status = XKP_ENOCONV;
                break;
            }
            ++restarts;
        }
    } else if (alive && status == XKP_OK) {
        if (own) s.x[p] = 0.0;   // b = 0: x = 0
    }
    if (!alive) status = XKP_EDEVICE;
    if (g == 0 && tid == 0) {
        hdr->n = n;
        hdr->m = m;
        hdr->k = kfirst;
        hdr->status = status;
        hdr->beta = beta_first;
        hdr->ldv = ldv;
        hdr->bf16 = Vb ? 1 : 0;
        hdr->kind = XKP_BASIS_ARNOLDI;
        info->status = status;
        info->iters = iters;
        info->restarts = restarts;
        info->basis_dim = kfirst;
        info->res_est = res_est;
        info->res_true = res_true;
        info->guess_res = 1.0;
        info->guess_source = 0;
        info->pad = 0;
    }
}

// Sets every unit of the launch's exchange areas to tag 0xFFFFFFFF (no round matches it).
__global__ void clear_exchange_kernel(unsigned char *xch, size_t bytes) {
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(xch, (short)0, (int)bytes, 0x00020000);
    for (unsigned i = blockIdx.x * blockDim.x + threadIdx.x; i < bytes / 16;
         i += gridDim.x * blockDim.x)
        __builtin_amdgcn_raw_buffer_store_b128(u32x4_t{0u, 0xFFFFFFFFu, 0u, 0xFFFFFFFFu}, rs,
                                               i * 16u, 0, kAux);
}

size_t lds_bytes(int mmax) { return sizeof(double) * lds_doubles(mmax) + 16; }

// Raises the kernel's dynamic-LDS limit once per device (to the largest size asked for), so
// that a launch inside a graph capture makes no attribute call.
static hipError_t set_lds(size_t bytes) {
    static std::mutex mu;
    static std::vector<std::pair<int, size_t>> done;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    for (auto &d : done)
        if (d.first == dev) {
            if (d.second >= bytes) return hipSuccess;
            e = hipFuncSetAttribute((const void *)wide_seed_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
            if (e == hipSuccess) d.second = bytes;
            return e;
        }
    e = hipFuncSetAttribute((const void *)wide_seed_kernel,
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (e == hipSuccess) done.push_back({dev, bytes});
    return e;
}

hipError_t launch_wide_seed(hipStream_t st, const xkp_system *sys, int nsys, xkp_params P,
                            void *const *keep_bases, xkp_info *infos, unsigned char *xch,
                            size_t xch_stride, int gmax, int nmax, long long limit) {
    const int mpol = P.polish_m > 0 ? P.polish_m : P.m;
    const size_t lds = lds_bytes(P.m > mpol ? P.m : mpol);
    hipError_t e = set_lds(lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(clear_exchange_kernel, dim3(256), dim3(256), 0, st, xch,
                       xch_stride * nsys);
    // up to 32 workgroups of a seed fit one XCD (one per compute unit)
    const int packed = gmax <= 32 ? 1 : 0;
    const dim3 grid(packed ? 8 * gmax * ((nsys + 7) / 8) : gmax * nsys);
    hipLaunchKernelGGL(wide_seed_kernel, grid, dim3(NT), lds, st, sys, nsys, P, keep_bases,
                       infos, xch, xch_stride, gmax, packed, nmax, limit);
    return hipGetLastError();
}

}  // namespace wide
}  // namespace xkp
