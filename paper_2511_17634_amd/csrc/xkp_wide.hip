// Seed solve spread over several workgroups (gfx950).
//
// A seed is one system per timestep on the projected chain's critical path (Section 3, Phase 1:
// every target of the timestep waits for its basis), so one workgroup per seed leaves the chip
// idle while it runs.  Here each seed is split into G contiguous row blocks of NB = 512 R rows,
// one workgroup per block (thread t owns rows t, t + 512, ... of its block), all G on one XCD
// (workgroup ids congruent mod 8) so that their exchanges stay in one L2.  Per Arnoldi step:
//   operator   w = A v_j on the owned rows; the neighbours H rows away come from the adjacent
//              blocks' boundary rows (exchanged), the rest from the block's own LDS copy
//   Gram-Schmidt  two classical passes (CGS2): pass k forms the owned rows' share of V^T w
//              (and of ||w||^2), the G shares are exchanged and summed in block order (the same
//              order in every workgroup, so every workgroup holds bitwise the same sums and takes
//              the same decisions), w -= V h; ||w2||^2 = ||w1||^2 - ||h2||^2
//   then       v_{j+1} = w2 / ||w2|| on the owned rows, its boundary rows exchanged for the next
//              operator application; Givens rotations and the Hessenberg column computed
//              identically by every workgroup
// i.e. three exchanges per step.  The basis, Hessenberg matrix, header, solution and info are
// those of the single-workgroup seed solve (restarted GMRES from x0, first cycle kept); the two
// classical passes give an orthonormal basis to working precision as two modified passes do.
//
// An exchange: every thread publishes its values with device-coherent stores and waits for them
// to complete, workgroup barrier, then one thread adds 1 to the seed's arrival counter and waits
// until G arrivals of this round are counted; readers use device-coherent loads.  Exchange
// buffers alternate between rounds.  Every wait is bounded in time: a workgroup whose partners
// do not arrive (they must all be resident at once) gives up, and the seed gets XKP_EDEVICE.
#define XKP_NT 512
#define XKP_VARIANT wdev
#include "xkp_device.h"
#include "xkp_internal.h"

namespace xkp {
namespace wide {

using namespace xkp::wdev;

constexpr int NT = 512, NW = NT / 64;
constexpr int HM = 128;                    // largest grid side (halo rows on each side)
constexpr int kMM = 64;                    // largest restart length
constexpr int kWV = kMM + 4;               // values of one exchange (j + 2 <= kMM + 1)

// Per-seed exchange area (bytes): the arrival counter, then two rounds of per-workgroup value
// slots, then two rounds of per-workgroup boundary rows (low H rows, high H rows).
__host__ __device__ inline size_t xch_part_off() { return 256; }
__host__ __device__ inline size_t xch_bnd_off(int gmax) {
    return xch_part_off() + sizeof(double) * 2 * (size_t)gmax * kWV;
}
size_t xch_bytes(int gmax) {
    return (xch_bnd_off(gmax) + sizeof(double) * 2 * (size_t)gmax * 2 * HM + 255) & ~(size_t)255;
}

__device__ __forceinline__ void pub(double *p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get(const double *p) {
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

struct Wide {
    unsigned *cnt;
    double *part, *bnd;
    int gmax, G, g, H, nb, n;
    unsigned round;
    long long limit;
    int *abort_lds;
    double *red, *tot, *vbuf;   // LDS

    // Round of exchange: publishes nothing itself (callers stored with pub()), orders every
    // thread's stores, counts this workgroup's arrival and waits for the others.
    __device__ bool sync() {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(cnt, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const unsigned target = (round + 1u) * (unsigned)G;
            const long long t0 = __builtin_amdgcn_s_memrealtime();
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__builtin_amdgcn_s_memrealtime() - t0 > limit) {
                    *abort_lds = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
        ++round;
        return *abort_lds == 0;
    }
    __device__ double *my_part() { return part + ((size_t)(round & 1) * gmax + g) * kWV; }
    __device__ const double *part_of(int gg) const {
        return part + ((size_t)(round & 1) * gmax + gg) * kWV;
    }
    __device__ double *bnd_of(unsigned rnd, int gg, int side) const {
        return bnd + (((size_t)(rnd & 1) * gmax + gg) * 2 + side) * HM;
    }

    // The workgroup's share of nv values, already summed per wave in red[v * NW + wave], is
    // published; after the exchange tot[v] holds the sums over the G blocks in block order.
    __device__ bool reduce(int nv) {
        __syncthreads();
        double *mp = my_part();
        for (int v = threadIdx.x; v < nv; v += NT) pub(mp + v, tree_sum<NW>(red + v * NW));
        const unsigned rnd = round;
        if (!sync()) return false;
        for (int v = threadIdx.x; v < nv; v += NT) {
            double t = 0.0;
            for (int gg = 0; gg < G; ++gg)
                t += get(part + ((size_t)(rnd & 1) * gmax + gg) * kWV + v);
            tot[v] = t;
        }
        __syncthreads();
        return true;
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

template <int R>
__global__ __launch_bounds__(NT) void wide_seed_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                       xkp_params P, void *const *keep_bases,
                                                       xkp_info *infos, unsigned char *xch,
                                                       size_t xch_stride, double *mws,
                                                       size_t mws_stride, int gmax, int nmax,
                                                       long long limit) {
    constexpr int NB = NT * R;
    const int tid = threadIdx.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int si = xcd + 8 * (slot / gmax), g = slot % gmax;
    if (si >= nsys) return;
    const xkp_system s = sys[si];
    xkp_info *info = infos + si;
    const int H = s.H;
    const bool ok = H > 0 && H <= HM && (long)H * H <= nmax && s.mt && s.b && s.x &&
                    s.dt > 0.0 && keep_bases[si] != nullptr && P.m >= 1 && P.m <= kMM &&
                    P.polish_m >= 0 && P.polish_m <= kMM;
    if (!ok) {
        if (g == 0 && tid == 0) info->status = XKP_EINVAL;
        return;
    }
    const int n = H * H, G = (n + NB - 1) / NB;
    if (g >= G) return;

    extern __shared__ __attribute__((aligned(16))) double lds[];
    double *vbuf = lds;                               // [HM | NB owned | HM]
    double *red = vbuf + NB + 2 * HM;                 // kWV x NW
    double *tot = red + kWV * NW;                     // kWV
    double *Rp = tot + kWV;                           // kMM (kMM + 1) / 2
    double *cs = Rp + kMM * (kMM + 1) / 2, *sn = cs + kMM, *gv = sn + kMM, *yv = gv + kMM + 1;
    int *flags = (int *)(yv + kMM);                   // [0] abort

    if (tid == 0) flags[0] = 0;
    for (int t = tid; t < NB + 2 * HM; t += NT) vbuf[t] = 0.0;
    __syncthreads();
    unsigned char *xs = xch + (size_t)si * xch_stride;
    Wide X{(unsigned *)xs, (double *)(xs + xch_part_off()), (double *)(xs + xch_bnd_off(gmax)),
           gmax, G, g, H, NB, n, 0u, limit, flags, red, tot, vbuf};

    // rows owned: local r_q = tid + NT q, global p_q = g NB + r_q; the last block's rows at or
    // past n are zero and are never read from a basis column (the kept basis ends at row n)
    const int base = g * NB;
    bool own[R];
#pragma unroll
    for (int q = 0; q < R; ++q) own[q] = base + tid + NT * q < n;
    const OpConst o = op_const(s);
    double cE[R], cW[R], cN[R], cS[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int p = base + tid + NT * q;
        double e = 0.0, w = 0.0, nn = 0.0, ss = 0.0;
        if (p < n) {
            const int i = p / H, j = p - (p / H) * H;
            const double mE = (i + 1 < H) ? s.mt[p + H] : 0.0;
            const double mW = (i > 0) ? s.mt[p - H] : 0.0;
            const double mN = (j + 1 < H) ? s.mt[p + 1] : 0.0;
            const double mS = (j > 0) ? s.mt[p - 1] : 0.0;
            const double fxp = s.fx ? s.fx[p] : 0.0;
            const double fyp = s.fy ? s.fy[p] : 0.0;
            const double ex = fxp * o.inv2h - o.c8 * (mE - mW);
            const double ey = fyp * o.inv2h - o.c8 * (mN - mS);
            e = (i + 1 < H) ? -o.a + ex : 0.0;
            w = (i > 0) ? -o.a - ex : 0.0;
            nn = (j + 1 < H) ? -o.a + ey : 0.0;
            ss = (j > 0) ? -o.a - ey : 0.0;
        }
        cE[q] = e;
        cW[q] = w;
        cN[q] = nn;
        cS[q] = ss;
    }
    // y = A u for the owned rows, u in vbuf (owned rows at HM + r, halos around them)
    auto apply = [&](double (&y)[R]) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const double *u = vbuf + HM + tid + NT * q;
            y[q] = o.cd * u[0] + cE[q] * u[H] + cW[q] * u[-H] + cN[q] * u[1] + cS[q] * u[-1];
        }
    };
    auto put_own = [&](const double (&v)[R]) {
#pragma unroll
        for (int q = 0; q < R; ++q) vbuf[HM + tid + NT * q] = v[q];
    };
    // boundary rows of the owned block (low H rows, high H rows) published for the neighbours
    auto pub_bnd = [&](const double (&v)[R]) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int r = tid + NT * q;
            if (r < H) pub(X.bnd_of(X.round, g, 0) + r, v[q]);
            if (r >= NB - H) pub(X.bnd_of(X.round, g, 1) + (r - (NB - H)), v[q]);
        }
    };
    // after the exchange of round rnd: the halos from the neighbours' boundary rows
    auto get_halo = [&](unsigned rnd) {
        for (int t = tid; t < H; t += NT) {
            vbuf[HM - H + t] = g > 0 ? get(X.bnd_of(rnd, g - 1, 1) + t) : 0.0;
            vbuf[HM + NB + t] = g + 1 < G ? get(X.bnd_of(rnd, g + 1, 0) + t) : 0.0;
        }
    };

    const int m = P.m, mpol = P.polish_m > 0 ? P.polish_m : P.m;
    xkp_basis_header *hdr = (xkp_basis_header *)keep_bases[si];
    const int ldv = (n + 8) & ~7;
    double *Vk = (double *)((char *)hdr + 256);
    double *Hb = (double *)((char *)hdr + basis_off_h(n, m));
    unsigned short *Vb = P.precision == XKP_MIXED
                             ? (unsigned short *)((char *)hdr + basis_off_vb(n, m))
                             : nullptr;
    double *Vw = mws + (size_t)(si * gmax + g) * mws_stride;   // later cycles: own rows, NB each
    if (g == 0)
        for (int t = tid; t < (m + 1) * m; t += NT) Hb[t] = 0.0;

    double b[R], x[R], w[R], r[R];
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int p = base + tid + NT * q;
        b[q] = p < n ? s.b[p] : 0.0;
        x[q] = (p < n && s.x0) ? s.x0[p] : 0.0;
    }
    // x halo for the first residual: straight from the input x0 (or zero)
    for (int t = tid; t < H; t += NT) {
        const int pl = base - H + t, ph = base + NB + t;
        vbuf[HM - H + t] = (s.x0 && pl >= 0 && pl < n) ? s.x0[pl] : 0.0;
        vbuf[HM + NB + t] = (s.x0 && ph < n) ? s.x0[ph] : 0.0;
    }
    put_own(x);
    __syncthreads();

    int iters = 0, restarts = 0, kfirst = 0, status = XKP_OK;
    double res_est = 0.0, res_true = 0.0, beta_first = 0.0, bnorm = 0.0, beta = 0.0;
    bool alive = true, first = true;
    // r = b - A x, its norm (and ||b|| on the first call) and its boundary rows: one exchange
    auto residual = [&](bool with_b) -> bool {
        apply(w);
        double rr = 0.0, bb = 0.0;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            r[q] = b[q] - w[q];
            rr += r[q] * r[q];
            bb += b[q] * b[q];
        }
        wave_put4(rr, bb, 0.0, 0.0, red, 0, 2);
        pub_bnd(r);
        const unsigned rnd = X.round;
        if (!X.reduce(2)) return false;
        get_halo(rnd);
        beta = sqrt(tot[0]);
        if (with_b) bnorm = sqrt(tot[1]);
        return true;
    };
    alive = residual(true);
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int p = base + tid + NT * q;
        if (p < n) s.x[p] = x[q];
    }
    // data that are not finite (NaN or Inf in m~, f, b or x0) cannot be solved
    if (alive && (!isfinite(beta) || !isfinite(bnorm))) status = XKP_EINVAL;
    if (alive && status == XKP_OK && bnorm > 0.0) {
        res_true = res_est = beta / bnorm;
        while (alive && beta > P.tol * bnorm) {
            const bool keep = first;
            const int mc = keep ? m : mpol;
            double *V = keep ? Vk : Vw;
            const size_t ld = keep ? (size_t)ldv : (size_t)NB;
            const int coff = keep ? base : 0;   // row offset of the owned block in a column
            auto col = [&](int c) { return V + (size_t)c * ld + coff; };
            // v_0 = r / beta (owned rows and halos)
            const double rb0 = 1.0 / beta;
#pragma unroll
            for (int q = 0; q < R; ++q) {
                w[q] = r[q] * rb0;
                const int p = base + tid + NT * q;
                if (p < n || !keep) col(0)[tid + NT * q] = (p < n) ? w[q] : 0.0;
            }
            if (keep) {
                if (g + 1 == G)
                    for (int p = n + tid; p < ldv; p += NT) Vk[p] = 0.0;
                beta_first = beta;
            }
            put_own(w);
            for (int t = tid; t < H; t += NT) {
                vbuf[HM - H + t] *= rb0;
                vbuf[HM + NB + t] *= rb0;
            }
            if (keep && Vb) {
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int p = base + tid + NT * q;
                    if (p < n) {
                        const unsigned u = __builtin_bit_cast(unsigned, (float)w[q]);
                        Vb[p] = (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
                    }
                }
            }
            __syncthreads();
            double gcur = beta;
            int kk = 0;
            for (int j = 0; j < mc; ++j) {
                apply(w);
                ++iters;
                // pass 1: shares of V_{j+1}^T w and ||w||^2
                for (int c0 = 0; c0 <= j + 1; c0 += 4) {
                    double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = c0 + e;
                        if (c <= j) {
                            const double *vc = col(c);
#pragma unroll
                            for (int q = 0; q < R; ++q) d[e] += (own[q] ? vc[tid + NT * q] : 0.0) * w[q];
                        } else if (c == j + 1) {
#pragma unroll
                            for (int q = 0; q < R; ++q) d[e] += w[q] * w[q];
                        }
                    }
                    wave_put4(d[0], d[1], d[2], d[3], red, c0, j + 2);
                }
                if (!(alive = X.reduce(j + 2))) break;
                const double wn0 = sqrt(tot[j + 1]);
                for (int c = 0; c <= j; ++c) {
                    const double hc = tot[c];
                    const double *vc = col(c);
#pragma unroll
                    for (int q = 0; q < R; ++q) w[q] -= hc * (own[q] ? vc[tid + NT * q] : 0.0);
                }
                // keep pass 1's coefficients: tot is overwritten by pass 2
                for (int c = tid; c <= j; c += NT) yv[c] = tot[c];
                // pass 2: shares of V_{j+1}^T w1 and ||w1||^2
                for (int c0 = 0; c0 <= j + 1; c0 += 4) {
                    double d[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int c = c0 + e;
                        if (c <= j) {
                            const double *vc = col(c);
#pragma unroll
                            for (int q = 0; q < R; ++q) d[e] += (own[q] ? vc[tid + NT * q] : 0.0) * w[q];
                        } else if (c == j + 1) {
#pragma unroll
                            for (int q = 0; q < R; ++q) d[e] += w[q] * w[q];
                        }
                    }
                    wave_put4(d[0], d[1], d[2], d[3], red, c0, j + 2);
                }
                if (!(alive = X.reduce(j + 2))) break;
                double c2 = 0.0;
                for (int c = 0; c <= j; ++c) {
                    const double hc = tot[c];
                    c2 += hc * hc;
                    const double *vc = col(c);
#pragma unroll
                    for (int q = 0; q < R; ++q) w[q] -= hc * (own[q] ? vc[tid + NT * q] : 0.0);
                }
                const double hn = sqrt(fmax(tot[j + 1] - c2, 0.0));
                const bool brk = !(hn > 1e-14 * wn0);
                const double rhn = brk ? 0.0 : 1.0 / hn;
#pragma unroll
                for (int q = 0; q < R; ++q) w[q] = w[q] * rhn;
                // v_{j+1}: owned rows into the basis, boundary rows to the neighbours
                double *vn = col(j + 1);
#pragma unroll
                for (int q = 0; q < R; ++q) {
                    const int p = base + tid + NT * q;
                    if (p < n || !keep) vn[tid + NT * q] = (p < n) ? w[q] : 0.0;
                    if (keep && Vb && p < n) {
                        const unsigned u = __builtin_bit_cast(unsigned, (float)w[q]);
                        Vb[(size_t)(j + 1) * ldv + p] =
                            (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
                    }
                }
                if (keep && g + 1 == G)
                    for (int p = n + tid; p < ldv; p += NT) Vk[(size_t)(j + 1) * ldv + p] = 0.0;
                // Hessenberg column j (both passes) and its Givens rotations, the same in every
                // workgroup; the kept cycle's unrotated column is written by block 0
                if (keep && g == 0)
                    for (int rr = tid; rr <= m; rr += NT)
                        Hb[(size_t)j * (m + 1) + rr] =
                            rr <= j ? yv[rr] + tot[rr] : (rr == j + 1 ? hn : 0.0);
                double t = yv[0] + tot[0];
                for (int i = 1; i <= j; ++i) {
                    const double hi = yv[i] + tot[i];
                    const double c = cs[i - 1], sv = sn[i - 1];
                    const double rrv = c * t + sv * hi;
                    t = -sv * t + c * hi;
                    if (tid == 0) Rp[(j * (j + 1)) / 2 + i - 1] = rrv;
                }
                const double den = sqrt(t * t + hn * hn);
                const double rden = 1.0 / den;
                const double cj = t * rden, sj = hn * rden;
                pub_bnd(w);
                const unsigned rnd = X.round;
                __syncthreads();   // every thread has read cs, sn, yv, tot
                if (tid == 0) {
                    Rp[(j * (j + 1)) / 2 + j] = den;
                    cs[j] = cj;
                    sn[j] = sj;
                    gv[j] = cj * gcur;
                }
                gcur = -sj * gcur;
                kk = j + 1;
                put_own(w);
                if (!(alive = X.sync())) break;
                get_halo(rnd);
                __syncthreads();
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
            for (int c = 0; c < kk; ++c) {
                const double yc = yv[c];
                const double *vc = col(c);
#pragma unroll
                for (int q = 0; q < R; ++q) x[q] += yc * (own[q] ? vc[tid + NT * q] : 0.0);
            }
#pragma unroll
            for (int q = 0; q < R; ++q) {
                const int p = base + tid + NT * q;
                if (p < n) s.x[p] = x[q];
            }
            if (first) {
                kfirst = kk;
                first = false;
            }
            // the new x's boundary rows, then the true residual in FP64
            put_own(x);
            pub_bnd(x);
            const unsigned rnd = X.round;
            if (!(alive = X.sync())) break;
            get_halo(rnd);
            __syncthreads();
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
        // b = 0: x = 0
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int p = base + tid + NT * q;
            if (p < n) s.x[p] = 0.0;
        }
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

__global__ void clear_counters_kernel(unsigned char *xch, size_t stride, int nsys) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nsys) *(unsigned *)(xch + (size_t)i * stride) = 0u;
}

size_t lds_bytes(int R) {
    return sizeof(double) * ((size_t)NT * R + 2 * HM + kWV * NW + kWV + kMM * (kMM + 1) / 2 +
                             4 * kMM + 1) + 16;
}

hipError_t launch_wide_seed(hipStream_t st, int R, const xkp_system *sys, int nsys,
                            xkp_params P, void *const *keep_bases, xkp_info *infos,
                            unsigned char *xch, size_t xch_stride, double *mws,
                            size_t mws_stride, int gmax, int nmax, long long limit) {
    hipLaunchKernelGGL(clear_counters_kernel, dim3((nsys + 63) / 64), dim3(64), 0, st, xch,
                       xch_stride, nsys);
    const dim3 grid(8 * gmax * ((nsys + 7) / 8));
    const size_t lds = lds_bytes(R);
    switch (R) {
    case 1:
        hipLaunchKernelGGL(wide_seed_kernel<1>, grid, dim3(NT), lds, st, sys, nsys, P,
                           keep_bases, infos, xch, xch_stride, mws, mws_stride, gmax, nmax,
                           limit);
        break;
    case 2:
        hipLaunchKernelGGL(wide_seed_kernel<2>, grid, dim3(NT), lds, st, sys, nsys, P,
                           keep_bases, infos, xch, xch_stride, mws, mws_stride, gmax, nmax,
                           limit);
        break;
    case 4:
        hipLaunchKernelGGL(wide_seed_kernel<4>, grid, dim3(NT), lds, st, sys, nsys, P,
                           keep_bases, infos, xch, xch_stride, mws, mws_stride, gmax, nmax,
                           limit);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace wide
}  // namespace xkp
