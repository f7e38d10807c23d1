// Score and probability-flow embedding of solved log-densities (gfx950): one fused pass per
// batch, bound by HBM bandwidth.
//
// For system i and grid point p = i_x * H + j (i_x the x index, j the y index), with h = 1/H and
// m = 0 outside the grid (zero padding):
//   score  s_x = (m[i_x+1, j] - m[i_x-1, j]) / (2h),  s_y = (m[i_x, j+1] - m[i_x, j-1]) / (2h)
//          (Section 2.3's central difference after the solve)
//   flow   d += (f - g^2/2 s) dt
//          (one explicit step of the probability-flow ODE that embeds the score, Section 4)
// Consecutive lanes take consecutive points, so every plane is read and written in full cache
// lines and each neighbour of m comes from the cache.  With an even grid side a thread takes two
// consecutive points of one grid column (p even, so the pair never crosses a column) and moves
// the score and displacement planes with 16-byte accesses; an odd side (or an output not
// 16-byte aligned) takes one point per thread.
#include "xkp_internal.h"

namespace xkp {
namespace epi {

constexpr int kThreads = 256;

typedef double double2_t __attribute__((ext_vector_type(2)));

// score and flow of one point p = i*H + j
__device__ __forceinline__ void point(const double *__restrict__ m, const xkp_system &s, int H,
                                      int p, double &sx, double &sy) {
    const int i = p / H, j = p - (p / H) * H;
    const double inv2h = 0.5 * (double)H;   // 1 / (2h)
    const double mE = i + 1 < H ? m[p + H] : 0.0, mW = i > 0 ? m[p - H] : 0.0;
    const double mN = j + 1 < H ? m[p + 1] : 0.0, mS = j > 0 ? m[p - 1] : 0.0;
    sx = (mE - mW) * inv2h;
    sy = (mN - mS) * inv2h;
}

__global__ __launch_bounds__(kThreads) void score_flow_kernel(const xkp_system *__restrict__ sys,
                                                               int nsys, int field,
                                                               double *const *score,
                                                               double *const *disp, int nmax) {
    const int si = blockIdx.y;
    if (si >= nsys) return;
    const xkp_system s = sys[si];
    if (!(s.H > 0 && (long)s.H * s.H <= nmax && s.dt > 0.0)) return;
    const double *__restrict__ m = field == XKP_FIELD_X ? s.x : s.mt;
    if (m == nullptr) return;
    const int H = s.H, n = H * H;
    double *sc = score ? score[si] : nullptr;
    double *dp = disp ? disp[si] : nullptr;
    const double c = 0.5 * s.g * s.g;
    const unsigned long long al = (unsigned long long)sc | (unsigned long long)dp;
    if ((H & 1) == 0 && (al & 15) == 0) {
        // two points per thread: grid.x covers nmax / 2 pairs
        const int p = 2 * (blockIdx.x * kThreads + (int)threadIdx.x);
        if (p >= n) return;
        double sx0, sy0, sx1, sy1;
        point(m, s, H, p, sx0, sy0);
        point(m, s, H, p + 1, sx1, sy1);
        if (sc) {
            *(double2_t *)(sc + p) = double2_t{sx0, sx1};
            *(double2_t *)(sc + n + p) = double2_t{sy0, sy1};
        }
        if (dp) {
            double2_t fx = {0.0, 0.0}, fy = {0.0, 0.0};
            if (s.fx) fx = double2_t{s.fx[p], s.fx[p + 1]};
            if (s.fy) fy = double2_t{s.fy[p], s.fy[p + 1]};
            double2_t dx = *(double2_t *)(dp + p), dy = *(double2_t *)(dp + n + p);
            dx[0] += (fx[0] - c * sx0) * s.dt;
            dx[1] += (fx[1] - c * sx1) * s.dt;
            dy[0] += (fy[0] - c * sy0) * s.dt;
            dy[1] += (fy[1] - c * sy1) * s.dt;
            *(double2_t *)(dp + p) = dx;
            *(double2_t *)(dp + n + p) = dy;
        }
        return;
    }
    const int p = blockIdx.x * kThreads + (int)threadIdx.x;
    if (p >= n) return;
    double sx, sy;
    point(m, s, H, p, sx, sy);
    if (sc) {
        sc[p] = sx;
        sc[n + p] = sy;
    }
    if (dp) {
        const double fx = s.fx ? s.fx[p] : 0.0, fy = s.fy ? s.fy[p] : 0.0;
        dp[p] += (fx - c * sx) * s.dt;
        dp[n + p] += (fy - c * sy) * s.dt;
    }
}

hipError_t launch_score_flow(hipStream_t st, const xkp_system *sys, int nsys, int field,
                             double *const *score, double *const *disp, int nmax) {
    const dim3 grid((nmax + kThreads - 1) / kThreads, nsys);
    hipLaunchKernelGGL(score_flow_kernel, grid, dim3(kThreads), 0, st, sys, nsys, field, score,
                       disp, nmax);
    return hipGetLastError();
}

}  // namespace epi
}  // namespace xkp
