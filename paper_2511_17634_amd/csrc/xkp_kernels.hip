// HIP kernels (gfx950) of the cross-matrix Krylov projection path.
//
// One workgroup of kNT threads owns one linear system at a time (persistent loop over the
// batch).  Thread t owns rows p = t + k*kNT, k < rmax, of every grid vector: basis columns are
// read and written only by the thread owning the row, so global memory needs no cross-thread
// ordering; the stencil's neighbour values come from an LDS copy of the vector.
//
//   gmres_kernel    restarted GMRES(m): stencil operator (Section 2.3), Arnoldi with modified
//                   Gram-Schmidt done twice, Givens rotations, restart on the FP64 true
//                   residual; optionally keeps the first cycle as the seed basis (Section 3,
//                   Phase 1) or starts from the projected guess (Phase 2 polish).
//   project_kernel  Phase 2 projection of each target onto its seed basis: the k x k system
//                   V^T A' V (FP64 matrix cores), H_k, or the least-squares Hessenberg problem,
//                   solved by one wavefront; x0 = x_base + V alpha.
//   residual_kernel ||b - A x|| / ||b|| in FP64;  apply_kernel y = A u.
#include "xkp_device.h"
#include "xkp_internal.h"

namespace xkp {

constexpr int kLdA = 81;   // leading dimension of the projected matrix in LDS (<= 80 columns)

// ----------------------------------------------------------------------------------------
// Vector helpers over the rows a thread owns.

template <int RMAX>
__device__ __forceinline__ void load_rows(const double *__restrict__ v, int n, double (&r)[RMAX]) {
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = (int)threadIdx.x + k * kNT;
        r[k] = (p < n) ? v[p] : 0.0;
    }
}

template <int RMAX>
__device__ __forceinline__ void store_rows(double *__restrict__ v, int n, const double (&r)[RMAX]) {
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = (int)threadIdx.x + k * kNT;
        if (p < n) v[p] = r[k];
    }
}

template <int RMAX>
__device__ __forceinline__ double dot_rows(const double (&a)[RMAX], const double (&b)[RMAX]) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) s += a[k] * b[k];
    return s;
}

// ex, ey per row: C_east = -a + ex, C_west = -a - ex, C_north = -a + ey, C_south = -a - ey with
// ex = f_x/(2h) - g^2/(8h^2) (m~_{i+1,j} - m~_{i-1,j}) and ey likewise along j (Section 2.3).
template <int RMAX>
__device__ void build_coeffs(const xkp_system &s, const OpConst &o, double *__restrict__ ex,
                             double *__restrict__ ey) {
    RowIdx ri;
    ri.init(o.H);
    int i = ri.i0, j = ri.j0;
    const int H = o.H;
    const double *__restrict__ mt = s.mt;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = (int)threadIdx.x + k * kNT;
        if (p < o.n) {
            const double mE = (i + 1 < H) ? mt[p + H] : 0.0;
            const double mW = (i > 0) ? mt[p - H] : 0.0;
            const double mN = (j + 1 < H) ? mt[p + 1] : 0.0;
            const double mS = (j > 0) ? mt[p - 1] : 0.0;
            const double fxp = s.fx ? s.fx[p] : 0.0;
            const double fyp = s.fy ? s.fy[p] : 0.0;
            ex[p] = fxp * o.inv2h - o.c8 * (mE - mW);
            ey[p] = fyp * o.inv2h - o.c8 * (mN - mS);
        }
        j += ri.dj;
        i += ri.di;
        if (j >= H) { j -= H; ++i; }
    }
}

// w = A u with u read from `u` (LDS copy or global), zero outside the grid.
template <int RMAX>
__device__ __forceinline__ void stencil(const double *u, const double *__restrict__ ex,
                                        const double *__restrict__ ey, const OpConst &o,
                                        double (&w)[RMAX]) {
    RowIdx ri;
    ri.init(o.H);
    int i = ri.i0, j = ri.j0;
    const int H = o.H;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = (int)threadIdx.x + k * kNT;
        double s = 0.0;
        if (p < o.n) {
            const double uc = u[p];
            const double uE = (i + 1 < H) ? u[p + H] : 0.0;
            const double uW = (i > 0) ? u[p - H] : 0.0;
            const double uN = (j + 1 < H) ? u[p + 1] : 0.0;
            const double uS = (j > 0) ? u[p - 1] : 0.0;
            s = o.cd * uc - o.a * ((uE + uW) + (uN + uS)) + ex[p] * (uE - uW) + ey[p] * (uN - uS);
        }
        w[k] = s;
        j += ri.dj;
        i += ri.di;
        if (j >= H) { j -= H; ++i; }
    }
}

// Same operator with the coefficients formed on the fly from m~ (no workspace).
template <int RMAX>
__device__ __forceinline__ void stencil_direct(const double *u, const xkp_system &s,
                                               const OpConst &o, double (&w)[RMAX]) {
    RowIdx ri;
    ri.init(o.H);
    int i = ri.i0, j = ri.j0;
    const int H = o.H;
    const double *__restrict__ mt = s.mt;
#pragma unroll
    for (int k = 0; k < RMAX; ++k) {
        const int p = (int)threadIdx.x + k * kNT;
        double r = 0.0;
        if (p < o.n) {
            const bool e = i + 1 < H, wv = i > 0, nn = j + 1 < H, ss = j > 0;
            const double ex = (s.fx ? s.fx[p] : 0.0) * o.inv2h
                              - o.c8 * ((e ? mt[p + H] : 0.0) - (wv ? mt[p - H] : 0.0));
            const double ey = (s.fy ? s.fy[p] : 0.0) * o.inv2h
                              - o.c8 * ((nn ? mt[p + 1] : 0.0) - (ss ? mt[p - 1] : 0.0));
            const double uc = u[p];
            const double uE = e ? u[p + H] : 0.0;
            const double uW = wv ? u[p - H] : 0.0;
            const double uN = nn ? u[p + 1] : 0.0;
            const double uS = ss ? u[p - 1] : 0.0;
            r = o.cd * uc - o.a * ((uE + uW) + (uN + uS)) + ex * (uE - uW) + ey * (uN - uS);
        }
        w[k] = r;
        j += ri.dj;
        i += ri.di;
        if (j >= H) { j -= H; ++i; }
    }
}

__device__ __forceinline__ bool desc_ok(const xkp_system &s, int nmax) {
    return s.H > 0 && (long)s.H * s.H <= nmax && s.mt != nullptr && s.b != nullptr &&
           s.x != nullptr && s.dt > 0.0;
}

// ----------------------------------------------------------------------------------------
// LDS layout of the GMRES kernel: vbuf[nlds] | Rp[kMMax*(kMMax+1)/2] | cs | sn | gv | h1 | yv | red
struct GmresLds {
    double *vbuf, *Rp, *cs, *sn, *gv, *h1, *yv, *red;
    __device__ GmresLds(double *base, int nlds) {
        vbuf = base;
        Rp = vbuf + nlds;
        cs = Rp + kMMax * (kMMax + 1) / 2;
        sn = cs + kMMax;
        gv = sn + kMMax;
        h1 = gv + kMMax + 1;
        yv = h1 + kMMax + 1;
        red = yv + kMMax;
    }
};

__device__ __forceinline__ int tri(int c) { return c * (c + 1) / 2; }

template <int RMAX>
__device__ void gmres_one(const xkp_system &s, const xkp_params &P, int flags, int prestatus,
                          xkp_basis_header *hdr, double *Vfirst, double *Hb, double *Vws,
                          double *ex, double *ey, xkp_info *info, GmresLds &L) {
    const OpConst o = op_const(s);
    const int n = o.n, m = P.m, tid = threadIdx.x;
    const bool keep = hdr != nullptr;
    BlockRed br{L.red, 0};

    build_coeffs<RMAX>(s, o, ex, ey);
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
            store_rows<RMAX>(L.vbuf, n, nxt);
            if (xs != s.x) store_rows<RMAX>(s.x, n, nxt);
            lds_barrier();
            stencil<RMAX>(L.vbuf, ex, ey, o, w);
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
        if (beta > P.tol * bnorm) {
            for (;;) {
                double *V = first ? Vfirst : Vws;
                // v_0 = r / beta; the LDS copy feeds the stencil
#pragma unroll
                for (int k = 0; k < RMAX; ++k) cur[k] = cur[k] / beta;
                store_rows<RMAX>(V, n, cur);
                store_rows<RMAX>(L.vbuf, n, cur);
                if (first) beta_first = beta;
                lds_barrier();
                double gcur = beta;
                int kk = 0;
                for (int j = 0; j < m; ++j) {
                    stencil<RMAX>(L.vbuf, ex, ey, o, w);
                    ++iters;
                    const double wsq = dot_rows<RMAX>(w, w);
                    double wn0 = 0.0, t = 0.0;
                    for (int pass = 0; pass < 2; ++pass) {
                        load_rows<RMAX>(V, n, cur);
                        for (int i = 0; i <= j; ++i) {
                            if (i < j) load_rows<RMAX>(V + (size_t)(i + 1) * n, n, nxt);
                            double d;
                            if (pass == 0 && i == 0) {
                                double two[2] = {dot_rows<RMAX>(w, cur), wsq};
                                br.sum_multi<2>(two);
                                d = two[0];
                                wn0 = sqrt(two[1]);
                            } else {
                                d = br.sum(dot_rows<RMAX>(w, cur));
                            }
#pragma unroll
                            for (int k = 0; k < RMAX; ++k) w[k] -= d * cur[k];
                            if (pass == 0) {
                                if (tid == 0) L.h1[i] = d;
                            } else {
                                // final h_{i,j}; fold the Givens rotations in as entries arrive
                                const double hf = L.h1[i] + d;
                                if (keep && first && tid == 0) Hb[(size_t)j * (m + 1) + i] = hf;
                                if (i == 0) {
                                    t = hf;
                                } else {
                                    const double c = L.cs[i - 1], sn = L.sn[i - 1];
                                    const double rr = c * t + sn * hf;
                                    t = -sn * t + c * hf;
                                    if (tid == 0) L.Rp[tri(j) + i - 1] = rr;
                                }
                            }
                            if (i < j) {
#pragma unroll
                                for (int k = 0; k < RMAX; ++k) cur[k] = nxt[k];
                            }
                        }
                    }
                    const double hn = sqrt(br.sum(dot_rows<RMAX>(w, w)));
                    const bool brk = !(hn > 1e-14 * wn0);
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) w[k] = brk ? 0.0 : w[k] / hn;
                    store_rows<RMAX>(V + (size_t)(j + 1) * n, n, w);
                    store_rows<RMAX>(L.vbuf, n, w);
                    if (keep && first && tid == 0) Hb[(size_t)j * (m + 1) + j + 1] = hn;
                    const double den = sqrt(t * t + hn * hn);
                    const double cj = t / den, sj = hn / den;
                    if (tid == 0) {
                        L.Rp[tri(j) + j] = den;
                        L.cs[j] = cj;
                        L.sn[j] = sj;
                        L.gv[j] = cj * gcur;
                    }
                    gcur = -sj * gcur;
                    kk = j + 1;
                    res_est = fabs(gcur) / bnorm;
                    lds_barrier();
                    if (fabs(gcur) <= P.tol * bnorm || brk) break;
                }
                // y = R^{-1} g by one wavefront (lane c holds g_c), column-oriented
                if (tid < 64) {
                    double gl = (tid < kk) ? L.gv[tid] : 0.0;
                    for (int c = kk - 1; c >= 0; --c) {
                        const double yc = readlane_d(gl, c) / L.Rp[tri(c) + c];
                        if (tid < c) gl -= L.Rp[tri(c) + tid] * yc;
                        if (tid == 0) L.yv[c] = yc;
                    }
                }
                lds_barrier();
                // x += V_k y
                load_rows<RMAX>(s.x, n, w);
                load_rows<RMAX>(V, n, cur);
                for (int c = 0; c < kk; ++c) {
                    if (c + 1 < kk) load_rows<RMAX>(V + (size_t)(c + 1) * n, n, nxt);
                    const double yc = L.yv[c];
#pragma unroll
                    for (int k = 0; k < RMAX; ++k) w[k] += yc * cur[k];
                    if (c + 1 < kk) {
#pragma unroll
                        for (int k = 0; k < RMAX; ++k) cur[k] = nxt[k];
                    }
                }
                store_rows<RMAX>(s.x, n, w);
                store_rows<RMAX>(L.vbuf, n, w);
                if (first) {
                    kfirst = kk;
                    first = false;
                }
                lds_barrier();
                // true residual in FP64
                stencil<RMAX>(L.vbuf, ex, ey, o, w);
                load_rows<RMAX>(s.b, n, cur);
#pragma unroll
                for (int k = 0; k < RMAX; ++k) cur[k] -= w[k];
                beta = sqrt(br.sum(dot_rows<RMAX>(cur, cur)));
                res_true = beta / bnorm;
                if (beta <= P.tol * bnorm) break;
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
    }
    // no wave may start the next system (and overwrite LDS / workspace) while others still
    // read this one's values
    __syncthreads();
}

template <int RMAX>
__global__ __launch_bounds__(kNT) void gmres_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                    xkp_params P, int flags, void *const *bases,
                                                    xkp_info *infos, double *ws, WsLayout Lw,
                                                    int nmax, int nlds) {
    extern __shared__ double lds[];
    GmresLds L(lds, nlds);
    double *slot = ws + (size_t)blockIdx.x * Lw.stride;
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        xkp_info *info = infos + si;
        int pre = XKP_OK;
        if (flags & kTarget) pre = info->status;
        if (!desc_ok(s, nmax) || P.m < 1 || P.m > kMMax) {
            if (threadIdx.x == 0) info->status = XKP_EINVAL;
            continue;
        }
        if (pre == XKP_EINVAL) continue;
        xkp_basis_header *hdr = nullptr;
        double *Vfirst = slot + Lw.v, *Hb = nullptr;
        if (flags & kKeepBasis) {
            char *base = (char *)bases[si];
            hdr = (xkp_basis_header *)base;
            Vfirst = (double *)(base + 256);
            Hb = (double *)(base + 256 + sizeof(double) * (size_t)s.H * s.H * (P.m + 1));
        }
        gmres_one<RMAX>(s, P, flags, pre, hdr, Vfirst, Hb, slot + Lw.v, slot + Lw.ex, slot + Lw.ey,
                        info, L);
    }
}

// ----------------------------------------------------------------------------------------
// Projection (Section 3, Phase 2)

// LU with partial pivoting of the kk x kk row-major LDS matrix A (leading dimension lda) by
// wavefront 0, lane r owning row r; zr is lane r's right-hand side entry.  Rows are not moved:
// the pivot of column c is the largest remaining |A[r][c]| (lowest lane on ties).  A pivot
// <= 1e-13 max|A| reports singular.  The solution goes to out[0..kk).
__device__ bool lu_solve_wave(double *A, int lda, int kk, double zr, double *out, int *pivl) {
    const int r = threadIdx.x;
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
            for (int q = c + 1; q < kk; ++q) A[r * lda + q] -= l * A[pl * lda + q];
            zr -= l * zp;
        }
        wave_lds_sync();
    }
    for (int c = kk - 1; c >= 0; --c) {
        const int pl = __builtin_amdgcn_readfirstlane(pivl[c]);
        const double xc = readlane_d(zr, pl) / A[pl * lda + c];
        if (pc < c) zr -= A[r * lda + c] * xc;
        if (r == 0) out[c] = xc;
    }
    wave_lds_sync();
    return false;
}

// Least squares min ||z - Hbar alpha|| for the (kk+1) x kk upper Hessenberg matrix in LDS (row
// major) by Givens rotations, wavefront 0, lane q owning column q.  z is in LDS (kk+1 values).
__device__ bool lsq_hessenberg_wave(double *A, int lda, int kk, double *z, double *out) {
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

template <int RMAX>
__global__ __launch_bounds__(kNT) void project_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                      int n_bases, const void *const *bases,
                                                      xkp_params P, xkp_info *infos, double *ws,
                                                      WsLayout Lw, int nmax, int nlds) {
    extern __shared__ double lds[];
    // vbuf and the projected matrix share the front of LDS; they are never live together.
    double *vbuf = lds;
    double *Ap = lds;
    double *zv = lds + nlds;           // kMMax + 1
    double *alpha = zv + kMMax + 1;    // kMMax
    int *pivl = (int *)(alpha + kMMax);
    double *red = alpha + kMMax + kMMax / 2;
    double *slot = ws + (size_t)blockIdx.x * Lw.stride;
    double *ex = slot + Lw.ex, *ey = slot + Lw.ey, *W = slot + Lw.w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;

    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        xkp_info *info = infos + si;
        const int n = s.H * s.H;
        const xkp_basis_header *hdr = nullptr;
        int k = 0;
        bool ok = desc_ok(s, nmax) && P.m >= 1 && P.m <= kMMax && s.basis_id >= 0 &&
                  s.basis_id < n_bases;
        if (ok) {
            hdr = (const xkp_basis_header *)bases[s.basis_id];
            ok = hdr != nullptr && hdr->n == n && hdr->m == P.m && hdr->k >= 0 && hdr->k <= P.m;
            if (ok) k = hdr->k;
        }
        if (!ok) {
            if (tid == 0) {
                info->status = XKP_EINVAL;
                info->basis_dim = 0;
            }
            continue;
        }
        const int m = P.m;
        const double *V = (const double *)((const char *)hdr + 256);
        const double *Hb = V + (size_t)n * (m + 1);
        const OpConst o = op_const(s);
        BlockRed br{red, 0};
        build_coeffs<RMAX>(s, o, ex, ey);

        // r_base = b - A' x_base
        double rb[RMAX], xr[RMAX], cur[RMAX];
        load_rows<RMAX>(s.b, n, rb);
        if (s.x0) {
            load_rows<RMAX>(s.x0, n, xr);
            store_rows<RMAX>(vbuf, n, xr);
            lds_barrier();
            stencil<RMAX>(vbuf, ex, ey, o, cur);
#pragma unroll
            for (int q = 0; q < RMAX; ++q) rb[q] -= cur[q];
        } else {
#pragma unroll
            for (int q = 0; q < RMAX; ++q) xr[q] = 0.0;
        }
        bool singular = false;
        if (k > 0) {
            if (P.mode == XKP_PROJ_TARGET_GALERKIN) {
                // W = [A' V_k | r_base] in the workspace, then [V_k^T A' V_k | V_k^T r_base] by
                // FP64 matrix-core tiles (16x16 outputs, 4-deep inner steps over the rows).
                for (int c = 0; c < k; ++c) {
                    stencil<RMAX>(V + (size_t)c * n, ex, ey, o, cur);
                    store_rows<RMAX>(W + (size_t)c * n, n, cur);
                }
                store_rows<RMAX>(W + (size_t)k * n, n, rb);
                __syncthreads();   // W rows written by other threads are read below
                const int ktr = (k + 15) / 16, ktc = (k + 16) / 16;
                for (int tl = wave; tl < ktr * ktc; tl += kNW) {
                    const int ta = tl / ktc, tc = tl % ktc;
                    const int ia = ta * 16 + (lane & 15), jc = tc * 16 + (lane & 15);
                    const int kq = lane >> 4;
                    const double *Va = V + (size_t)(ia < k ? ia : 0) * n;
                    const double *Wc = W + (size_t)(jc <= k ? jc : 0) * n;
                    const bool va = ia < k, wb = jc <= k;
                    double4_t acc = {0.0, 0.0, 0.0, 0.0};
                    for (int p0 = 0; p0 < n; p0 += 4) {
                        const int p = p0 + kq;
                        const double av = (va && p < n) ? Va[p] : 0.0;
                        const double bv = (wb && p < n) ? Wc[p] : 0.0;
                        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
                    }
                    // FP64 16x16x4 output layout: lane l, register r holds D[4r + l/16][l%16]
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int a = ta * 16 + 4 * r + (lane >> 4), c = tc * 16 + (lane & 15);
                        if (a < k && c <= k) Ap[a * kLdA + c] = acc[r];
                    }
                }
                lds_barrier();
                if (wave == 0) {
                    const double zr = (lane < k) ? Ap[lane * kLdA + k] : 0.0;
                    singular = lu_solve_wave(Ap, kLdA, k, zr, alpha, pivl);
                }
            } else {
                // z = V_{k(+1)}^T r_base, eight columns per reduction
                const int nz = (P.mode == XKP_PROJ_SEED_LSQ) ? k + 1 : k;
                for (int c0 = 0; c0 < nz; c0 += kRedSlots) {
                    double part[kRedSlots];
#pragma unroll
                    for (int q = 0; q < kRedSlots; ++q) {
                        part[q] = 0.0;
                        if (c0 + q < nz) {
                            load_rows<RMAX>(V + (size_t)(c0 + q) * n, n, cur);
                            part[q] = dot_rows<RMAX>(cur, rb);
                        }
                    }
                    br.sum_multi<kRedSlots>(part);
                    if (tid == 0)
                        for (int q = 0; q < kRedSlots && c0 + q < nz; ++q) zv[c0 + q] = part[q];
                }
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
            if (!singular) {
                // x0 = x_base + V_k alpha
                load_rows<RMAX>(V, n, cur);
                for (int c = 0; c < k; ++c) {
                    if (c + 1 < k) load_rows<RMAX>(V + (size_t)(c + 1) * n, n, rb);
                    const double al = alpha[c];
#pragma unroll
                    for (int q = 0; q < RMAX; ++q) xr[q] += al * cur[q];
                    if (c + 1 < k) {
#pragma unroll
                        for (int q = 0; q < RMAX; ++q) cur[q] = rb[q];
                    }
                }
            }
        }
        store_rows<RMAX>(s.x, n, xr);
        if (tid == 0) {
            info->status = singular ? XKP_ESINGULAR : XKP_OK;
            info->basis_dim = k;
        }
        __syncthreads();
    }
}

// ----------------------------------------------------------------------------------------

template <int RMAX>
__global__ __launch_bounds__(kNT) void residual_kernel(const xkp_system *__restrict__ sys, int nsys,
                                                       double *rel, int nmax, int nlds) {
    extern __shared__ double lds[];
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
        store_rows<RMAX>(vbuf, o.n, x);
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
    extern __shared__ double lds[];
    for (int si = blockIdx.x; si < nsys; si += gridDim.x) {
        const xkp_system s = sys[si];
        if (!desc_ok(s, nmax) || s.x0 == nullptr) continue;
        const OpConst o = op_const(s);
        double u[RMAX], w[RMAX];
        load_rows<RMAX>(s.x0, o.n, u);
        store_rows<RMAX>(lds, o.n, u);
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
        RowIdx ri;
        ri.init(o.H);
        int i = ri.i0, j = ri.j0;
        const int H = o.H;
#pragma unroll
        for (int k = 0; k < RMAX; ++k) {
            const int p = (int)threadIdx.x + k * kNT;
            if (p < o.n) {
                double div = 0.0;
                if (s.fx) div += ((i + 1 < H) ? s.fx[p + H] : 0.0) - ((i > 0) ? s.fx[p - H] : 0.0);
                if (s.fy) div += ((j + 1 < H) ? s.fy[p + 1] : 0.0) - ((j > 0) ? s.fy[p - 1] : 0.0);
                b[p] = s.mt[p] / s.dt - div * o.inv2h;
            }
            j += ri.dj;
            i += ri.di;
            if (j >= H) { j -= H; ++i; }
        }
    }
}

// ----------------------------------------------------------------------------------------
// Host launchers

WsLayout ws_layout(int nmax, int mmax) {
    auto up = [](size_t v) { return (v + 63) & ~(size_t)63; };
    WsLayout L;
    L.v = 0;
    L.ex = up((size_t)nmax * (mmax + 1));
    L.ey = L.ex + up(nmax);
    L.w = L.ey + up(nmax);
    L.stride = L.w + up((size_t)nmax * (mmax + 1));
    return L;
}

size_t basis_off_v() { return 256; }
size_t basis_off_h(int n, int m) { return 256 + sizeof(double) * (size_t)n * (m + 1); }
size_t basis_off_vb(int n, int m) {
    size_t o = basis_off_h(n, m) + sizeof(double) * (size_t)(m + 1) * m;
    return (o + 255) & ~(size_t)255;
}
size_t basis_bytes(int n, int m) {
    size_t o = basis_off_vb(n, m) + 2 * (size_t)n * (m + 1);
    return (o + 255) & ~(size_t)255;
}

int rmax_for(int n) {
    if (n <= kNT * 2) return 2;
    if (n <= kNT * 8) return 8;
    if (n <= kNT * 32) return 32;
    return 0;
}

static size_t gmres_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + kMMax * (kMMax + 1) / 2 + 5 * kMMax + 2 +
                             2 * kRedSlots * kNW);
}
static size_t project_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + (kMMax + 1) + kMMax + kMMax / 2 + 2 * kRedSlots * kNW);
}
static size_t small_lds_bytes(int nlds) {
    return sizeof(double) * ((size_t)nlds + 2 * kRedSlots * kNW);
}

template <typename K>
static hipError_t set_lds(K kern, size_t bytes) {
    return hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

#define XKP_DISPATCH(RM, CALL)                     \
    switch (RM) {                                  \
    case 2: { constexpr int R = 2; CALL; } break;  \
    case 8: { constexpr int R = 8; CALL; } break;  \
    case 32: { constexpr int R = 32; CALL; } break; \
    default: return hipErrorInvalidValue;          \
    }

hipError_t launch_gmres(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys,
                        int nsys, xkp_params P, int flags, void *const *bases, xkp_info *infos,
                        double *ws, WsLayout L, int nmax) {
    const size_t lds = gmres_lds_bytes(nlds);
    XKP_DISPATCH(rmax, {
        hipError_t e = set_lds(gmres_kernel<R>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(gmres_kernel<R>, dim3(grid), dim3(kNT), lds, st, sys, nsys, P, flags,
                           bases, infos, ws, L, nmax, nlds);
    });
    return hipGetLastError();
}

hipError_t launch_project(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys,
                          int nsys, int n_bases, const void *const *bases, xkp_params P,
                          xkp_info *infos, double *ws, WsLayout L, int nmax) {
    const int nl = nlds > (kMMax + 1) * kLdA ? nlds : (kMMax + 1) * kLdA;
    const size_t lds = project_lds_bytes(nl);
    XKP_DISPATCH(rmax, {
        hipError_t e = set_lds(project_kernel<R>, lds);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(project_kernel<R>, dim3(grid), dim3(kNT), lds, st, sys, nsys, n_bases,
                           bases, P, infos, ws, L, nmax, nl);
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

}  // namespace xkp
