// Clustered seed selection (gfx950): k-means on block-mean image features, so that each group
// of similar images gets its own seed (the remedy the paper suggests for diverse datasets).
//
//   pool_kernel    features: each image's pool x pool block means
//   dist_kernel    squared distance of every image to each of k centroids (one workgroup per
//                  image, a fixed-shape reduction tree per centroid, so results do not depend
//                  on scheduling); nearest centroid (lowest index on ties) and its distance
//   update_kernel  each centroid the mean of its members, summed in image order
// The host drives the farthest-first start and the Lloyd iterations (xkp_cluster_seeds).
#include "xkp_internal.h"

namespace xkp {
namespace clu {

constexpr int kThreads = 256;

__global__ __launch_bounds__(kThreads) void pool_kernel(const double *__restrict__ img, int N,
                                                         int H, int pool, double *feat) {
    const int Hp = H / pool, d = Hp * Hp;
    const int i = blockIdx.y;
    const int f = blockIdx.x * kThreads + (int)threadIdx.x;
    if (i >= N || f >= d) return;
    const int fi = f / Hp, fj = f - (f / Hp) * Hp;
    const double *x = img + (size_t)i * H * H;
    double s = 0.0;
    for (int a = 0; a < pool; ++a)
        for (int b = 0; b < pool; ++b) s += x[(fi * pool + a) * H + fj * pool + b];
    feat[(size_t)i * d + f] = s / (double)(pool * pool);
}

// Sum over the workgroup in a fixed order: per-thread partials into LDS, then halving.
__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = kThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double s = red[0];
    __syncthreads();
    return s;
}

__global__ __launch_bounds__(kThreads) void dist_kernel(const double *__restrict__ feat, int N,
                                                         int d, const double *__restrict__ cent,
                                                         int k, int *assign, double *dist) {
    __shared__ double red[kThreads];
    const int i = blockIdx.x;
    if (i >= N) return;
    const double *x = feat + (size_t)i * d;
    double best = 0.0;
    int arg = -1;
    for (int c = 0; c < k; ++c) {
        const double *y = cent + (size_t)c * d;
        double part = 0.0;
        for (int f = threadIdx.x; f < d; f += kThreads) {
            const double t = x[f] - y[f];
            part += t * t;
        }
        const double s = block_sum(part, red);
        if (arg < 0 || s < best) {
            best = s;
            arg = c;
        }
    }
    if (threadIdx.x == 0) {
        if (assign) assign[i] = arg;
        dist[i] = best;
    }
}

__global__ __launch_bounds__(kThreads) void update_kernel(const double *__restrict__ feat, int N,
                                                           int d, const int *__restrict__ assign,
                                                           int K, double *cent) {
    const int c = blockIdx.y;
    const int f = blockIdx.x * kThreads + (int)threadIdx.x;
    if (c >= K || f >= d) return;
    double s = 0.0;
    int cnt = 0;
    for (int i = 0; i < N; ++i)
        if (assign[i] == c) {
            s += feat[(size_t)i * d + f];
            ++cnt;
        }
    if (cnt > 0) cent[(size_t)c * d + f] = s / (double)cnt;
}

hipError_t pool(hipStream_t st, const double *img, int N, int H, int pool_, double *feat) {
    const int d = (H / pool_) * (H / pool_);
    hipLaunchKernelGGL(pool_kernel, dim3((d + kThreads - 1) / kThreads, N), dim3(kThreads), 0,
                       st, img, N, H, pool_, feat);
    return hipGetLastError();
}

hipError_t distances(hipStream_t st, const double *feat, int N, int d, const double *cent,
                     int k, int *assign, double *dist) {
    hipLaunchKernelGGL(dist_kernel, dim3(N), dim3(kThreads), 0, st, feat, N, d, cent, k, assign,
                       dist);
    return hipGetLastError();
}

hipError_t update(hipStream_t st, const double *feat, int N, int d, const int *assign, int K,
                  double *cent) {
    hipLaunchKernelGGL(update_kernel, dim3((d + kThreads - 1) / kThreads, K), dim3(kThreads), 0,
                       st, feat, N, d, assign, K, cent);
    return hipGetLastError();
}

}  // namespace clu
}  // namespace xkp
