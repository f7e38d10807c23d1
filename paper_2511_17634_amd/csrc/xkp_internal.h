// Host-side launch interface between the C ABI (xkp_api.hip) and the kernels (xkp_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

#include "xkp.h"

namespace xkp {

// Per-workgroup workspace, in doubles, for systems of at most nmax unknowns and restart m;
// npad is the padded row count (threads x rows per thread) of the kernel variant used.
struct WsLayout {
    size_t v, cE, cW, cN, cS, c32, w, stride;   // c32: four FP32 coefficient arrays of npad
    int npad;   // rows covered by the kernel variant, coefficient array length
};
WsLayout ws_layout(int nmax, int mmax, int npad);

// Byte offsets inside a seed basis buffer (the layout documented in xkp.h): V columns have
// leading dimension ldv = roundup(n + 1, 8) doubles, element n (and the rest of the column
// padding) being zero.
size_t basis_off_v();
int basis_ldv(int n);
__host__ __device__ inline size_t basis_off_h(int n, int m) {
    return 256 + sizeof(double) * (size_t)((n + 8) & ~7) * (m + 1);
}
__host__ __device__ inline size_t basis_off_vb(int n, int m) {
    const size_t o = basis_off_h(n, m) + sizeof(double) * (size_t)(m + 1) * m;
    return (o + 255) & ~(size_t)255;
}
size_t basis_bytes(int n, int m);

enum GmresFlags {
    kStartFromX = 1,   // initial guess is the descriptor's x (the projected x0)
    kKeepBasis = 2,    // seed build: write the first cycle into bases[i]
    kTarget = 4,       // project onto the seed basis first, then polish from the projection
    kLearned = 8,      // try the learned guess first; project only if it fails the gate
    kDcgs = 16,        // seeds: the kept cycle by DCGS2 (set by the launcher when the LDS fits)
    kRegBasis = 32,    // discarded cycles with the basis in registers where it fits
    kPreProjected = 64,   // targets projected by the projection launches (xkp_project.hip): x
                          // holds x0, pre[i] the projection's status
    kCorrection = 128,    // with kLearned: the prediction corrects the projected guess
    kRedo = 256           // seeds: solve only those whose info status is XKP_EDEVICE (a
                          // spread-out solve gave up), skip the rest
};

// Learned-guess inputs of a solve launch: target i's predicted residual coordinates at
// alpha + i*ld (FP32, k+1 used), multiplied by scale; the guess is kept when its relative
// residual is <= gate.
struct Learned {
    const float *alpha;
    int ld;
    double scale, gate;
};

// The kernel file can be compiled once per workgroup size into its own namespace; the build
// uses v512 (512 threads; 2, 8 or 32 rows per thread).  A variant reports the rows per thread
// it would use for n unknowns (0: too large), and the zero-padded LDS vector length.
#define XKP_DECLARE_VARIANT(NS)                                                                  \
    namespace NS {                                                                               \
    int threads();                                                                               \
    int rmax_for(int n);                                                                         \
    int lds_vec_len(int nmax);                                                                   \
    int solve_per_cu(int nmax);                                                                  \
    hipError_t launch_solve(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys, \
                            int nsys, xkp_params P, int flags, int n_bases,                      \
                            const void *const *bases, void *const *keep_bases,                   \
                            xkp_info *infos, double *ws, WsLayout L, int nmax,                   \
                            unsigned *queue, Learned lg, const int *pre);                        \
    hipError_t launch_coeffs(hipStream_t st, int grid, int rmax, const xkp_system *sys,         \
                             int nsys, int n_bases, const void *const *bases, int m_out,         \
                             int kind, double *alpha, int nmax);                                 \
    hipError_t launch_residual(hipStream_t st, int grid, int rmax, int nlds,                     \
                               const xkp_system *sys, int nsys, double *rel, int nmax);          \
    hipError_t launch_rhs(hipStream_t st, int grid, int rmax, const xkp_system *sys, int nsys,   \
                          int nmax);                                                             \
    hipError_t launch_apply(hipStream_t st, int grid, int rmax, int nlds, const xkp_system *sys, \
                            int nsys, int nmax);                                                 \
    hipError_t launch_accum(hipStream_t st, int rmax, int n, int nsrc, const void *const *srcs,  \
                            void *const *outs, int per_source, int cap, int *out_k);             \
    }

XKP_DECLARE_VARIANT(v512)
XKP_DECLARE_VARIANT(v1024)
XKP_DECLARE_VARIANT(v256)

// Seeds spread over several workgroups (xkp_wide.hip): blocks of rows_per_block() rows, up to
// gmax workgroups per seed; xch: per-seed exchange areas of xch_stride bytes (xch_bytes(gmax)).
namespace wide {
size_t xch_bytes(int gmax);
int rows_per_block();
hipError_t launch_wide_seed(hipStream_t st, const xkp_system *sys, int nsys, xkp_params P,
                            void *const *keep_bases, xkp_info *infos, unsigned char *xch,
                            size_t xch_stride, int gmax, int nmax, long long limit);
}  // namespace wide

// Target projection in launches of its own (xkp_project.hip): every target split into at most
// tiles_cap row tiles (0: about one round of items on the cus compute units), then x0 written
// to the targets' x; per target, the status (XKP_OK, XKP_ESINGULAR, XKP_EINVAL, -1 for a
// rejected descriptor) goes to stat for the polish launch (kPreProjected).  part: slots partial
// slots of slot_doubles(mmax) doubles (uncached memory); ctr: one zeroed counter per target;
// alpha: 64 per target.
namespace proj {
int slot_doubles(int mmax);
int tiles_per_target(int nsys, int nmax, int slots, int tiles_cap, int cus);
hipError_t launch_project(hipStream_t st, const xkp_system *sys, int nsys, int n_bases,
                          const void *const *bases, xkp_params P, int nmax, double *part,
                          int slots, int sstride, unsigned *ctr, double *alpha, int *stat,
                          xkp_info *infos, int tiles_cap, int cus);
}  // namespace proj

// Score and probability-flow embedding (xkp_epilogue.hip).
namespace epi {
hipError_t launch_score_flow(hipStream_t st, const xkp_system *sys, int nsys, int field,
                             double *const *score, double *const *disp, int nmax);
}  // namespace epi

// Clustered seed selection (xkp_cluster.hip).
namespace clu {
hipError_t pool(hipStream_t st, const double *img, int N, int H, int pool, double *feat);
hipError_t distances(hipStream_t st, const double *feat, int N, int d, const double *cent, int k,
                     int *assign, double *dist);
hipError_t update(hipStream_t st, const double *feat, int N, int d, const int *assign, int K,
                  double *cent);
}  // namespace clu

// The learned-guess network (xkp_cnn.hip).
namespace cnn {
size_t param_count(int k);
size_t workspace_bytes(int B, int k);
hipError_t forward(hipStream_t st, int B, int k, const float *prm, const double *img,
                   const int *img_idx, const int *steps, float *alpha, float *ws);
hipError_t backward(hipStream_t st, int B, int k, const float *prm, const double *img,
                    const int *img_idx, const int *steps, const double *target, int ld,
                    const int *tidx, double scale, float *alpha, float *g, float *loss,
                    float *ws);
hipError_t adam(hipStream_t st, int count, float *prm, const float *g, float *m, float *v, int t,
                float lr, float b1, float b2, float eps);
}  // namespace cnn

}  // namespace xkp
