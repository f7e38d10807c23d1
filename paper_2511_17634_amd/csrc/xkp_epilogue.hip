// Score and probability-flow embedding of solved log-densities (gfx950): one fused pass per
// batch, bound by HBM bandwidth.
//
// For system i and grid point p = i_x * H + j (i_x the x index, j the y index), with h = 1/H and
// m = 0 outside the grid (zero padding):
//   score  s_x = (m[i_x+1, j] - m[i_x-1, j]) / (2h),  s_y = (m[i_x, j+1] - m[i_x, j-1]) / (2h)
//          (Section 2.3's central difference after the solve)
//   flow   d += (f - g^2/2 s) dt
//          (one explicit step of the probability-flow ODE that embeds the score, Section 4)
// One thread per grid point; consecutive lanes take consecutive points, so every plane is read
// and written in full cache lines and each neighbour of m comes from the cache.
#include "xkp_internal.h"

namespace xkp {
namespace epi {

constexpr int kThreads = 256;

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
    const int p = blockIdx.x * kThreads + (int)threadIdx.x;
    if (p >= n) return;
    double *sc = score ? score[si] : nullptr;
    double *dp = disp ? disp[si] : nullptr;
    const int i = p / H, j = p - (p / H) * H;
    const double inv2h = 0.5 * (double)H;   // 1 / (2h)
    const double mE = i + 1 < H ? m[p + H] : 0.0, mW = i > 0 ? m[p - H] : 0.0;
    const double mN = j + 1 < H ? m[p + 1] : 0.0, mS = j > 0 ? m[p - 1] : 0.0;
    const double sx = (mE - mW) * inv2h, sy = (mN - mS) * inv2h;
    if (sc) {
        sc[p] = sx;
        sc[n + p] = sy;
    }
    if (dp) {
        const double c = 0.5 * s.g * s.g;
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
