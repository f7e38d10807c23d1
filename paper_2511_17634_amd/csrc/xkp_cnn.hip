// Learned starting guess: the small network mapping a target's initial image and the timestep
// index to coefficients in the seed subspace, forward and backward, and Adam (gfx950).
//
// Network: 64x64 image -> 2x2 average pool -> 32x32; three 3x3 stride-2 convolutions with
// padding 1 (1 -> 16 -> 32 -> 64 channels, 32 -> 16 -> 8 -> 4 positions), each + bias and GELU;
// mean over the 4x4 positions (64 features) concatenated with a 32-wide sinusoidal embedding of
// the timestep; linear 96 -> k.  Parameters are FP32 (the master copy), one flat array:
// conv1.W[16][1*9], conv1.b[16], conv2.W[32][16*9], conv2.b[32], conv3.W[64][32*9], conv3.b[64],
// lin.W[k][96], lin.b[k]; a convolution weight's column index is ci*9 + ky*3 + kx.
//
// The convolutions (forward, weight gradient and input gradient) run as GEMMs on BF16 matrix
// cores with FP32 accumulation (v_mfma_f32_16x16x32_bf16): operands are gathered straight from
// the FP32 activations (im2col on the fly) and rounded to BF16.  Pooling, the head (96 x k), the
// loss and Adam are FP32.  Reductions over the batch go through per-slice partial sums added in a
// fixed order, so results are deterministic.
#include <hip/hip_runtime.h>
#include <math.h>

#include "xkp.h"
#include "xkp_internal.h"

namespace xkp {
namespace cnn {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int kEmb = 32, kFeat = 96, kImg = 64, kIn = 32;
constexpr int kCh[4] = {1, 16, 32, 64};

// Parameter offsets (floats).
__host__ __device__ constexpr int off_w(int l) {
    return l == 0 ? 0 : (l == 1 ? 16 * 9 + 16 : 16 * 9 + 16 + 32 * 144 + 32);
}
__host__ __device__ constexpr int off_b(int l) { return off_w(l) + kCh[l + 1] * kCh[l] * 9; }
constexpr int kOffLin = 16 * 9 + 16 + 32 * 144 + 32 + 64 * 288 + 64;

size_t param_count(int k) { return (size_t)kOffLin + (size_t)k * kFeat + k; }

// BF16 bits of an FP32 value, round to nearest even (finite values).
__device__ __forceinline__ __bf16 bf(float f) {
    const unsigned u = __builtin_bit_cast(unsigned, f);
    return __builtin_bit_cast(__bf16, (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16));
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678f)); }
__device__ __forceinline__ float gelu_grad(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678f)) + z * 0.39894228f * expf(-0.5f * z * z);
}

// One 16x16 tile of sum_{q < K} A(r, q) B(q, c) for rows r0.., columns c0..: lane l gathers
// A(r0 + l%16, q0 + 8(l/16) + i) and B(q0 + 8(l/16) + i, c0 + l%16), i < 8, per 32-wide step;
// register r of the result is element (r0 + 4(l/16) + r, c0 + l%16).  Out-of-range q read 0.
template <typename FA, typename FB>
__device__ __forceinline__ f32x4_t mfma_tile(int r0, int c0, int K, FA fa, FB fb) {
    const int lane = threadIdx.x & 63;
    const int r = r0 + (lane & 15), c = c0 + (lane & 15), kq = 8 * (lane >> 4);
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int q0 = 0; q0 < K; q0 += 32) {
        bf16x8_t a, b;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int q = q0 + kq + i;
            a[i] = bf(q < K ? fa(r, q) : 0.f);
            b[i] = bf(q < K ? fb(q, c) : 0.f);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
    return acc;
}

// Input of a stride-2 3x3 convolution at column q = ci*9 + ky*3 + kx for output position
// (oy, ox): x[ci][2oy+ky-1][2ox+kx-1], zero outside the S x S input.
template <int S>
__device__ __forceinline__ float conv_in(const float *x, int q, int oy, int ox) {
    const int ci = q / 9, t = q - 9 * ci, ky = t / 3, kx = t - 3 * ky;
    const int y = 2 * oy + ky - 1, xx = 2 * ox + kx - 1;
    return (y >= 0 && y < S && xx >= 0 && xx < S) ? x[(ci * S + y) * S + xx] : 0.f;
}

// 2x2 average pooling of the FP64 64x64 images (index [i][j], p = 64 i + j) to FP32 32x32.
__global__ void prep_kernel(int B, const double *__restrict__ img, const int *__restrict__ idx,
                            float *__restrict__ a0) {
    const int b = blockIdx.x;
    const size_t src = idx ? (size_t)idx[b] : (size_t)b;
    for (int t = threadIdx.x; t < kIn * kIn; t += blockDim.x) {
        const int i = t / kIn, j = t - kIn * i;
        const double *p = img + src * kImg * kImg + (2 * i) * kImg + 2 * j;
        a0[(size_t)b * kIn * kIn + t] = (float)(0.25 * ((p[0] + p[1]) + (p[kImg] + p[kImg + 1])));
    }
}

// z = W * x + b, a = GELU(z): rows co (M = CO), columns n = b*So*So + pos, one wave per tile.
template <int CI, int CO, int S>
__global__ __launch_bounds__(256) void conv_fwd_kernel(int B, const float *__restrict__ x,
                                                       const float *__restrict__ prm, int l,
                                                       float *__restrict__ z,
                                                       float *__restrict__ a) {
    constexpr int So = S / 2, NP = So * So, K = CI * 9;
    const float *W = prm + off_w(l), *bias = prm + off_b(l);
    const int tiles_m = CO / 16, tiles_n = (B * NP + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles_m * tiles_n) return;
    const int r0 = (tile % tiles_m) * 16, c0 = (tile / tiles_m) * 16;
    const int N = B * NP;
    auto fa = [&](int co, int q) { return W[co * K + q]; };
    auto fb = [&](int q, int n) {
        if (n >= N) return 0.f;
        const int b = n / NP, pos = n - NP * b;
        return conv_in<S>(x + (size_t)b * CI * S * S, q, pos / So, pos % So);
    };
    const f32x4_t acc = mfma_tile(r0, c0, K, fa, fb);
    const int lane = threadIdx.x & 63;
    const int n = c0 + (lane & 15);
    if (n < N) {
        const int b = n / NP, pos = n - NP * b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int co = r0 + 4 * (lane >> 4) + r;
            const float v = acc[r] + bias[co];
            const size_t o = ((size_t)b * CO + co) * NP + pos;
            z[o] = v;
            a[o] = gelu(v);
        }
    }
}

// Head: u = [mean over positions of a3 | embedding of the timestep], alpha = Wl u + bl.
__global__ void head_fwd_kernel(int B, int k, const float *__restrict__ a3,
                                const int *__restrict__ steps, const float *__restrict__ prm,
                                float *__restrict__ u, float *__restrict__ alpha) {
    __shared__ float us[kFeat];
    const int b = blockIdx.x, t = threadIdx.x;
    if (t < kCh[3]) {
        const float *p = a3 + ((size_t)b * kCh[3] + t) * 16;
        float s = 0.f;
        for (int q = 0; q < 16; ++q) s += p[q];
        us[t] = s / 16.f;
    } else if (t < kFeat) {
        const int e = t - kCh[3], i = e >> 1;
        const double w = pow(10000.0, -(double)i / (kEmb / 2));
        const double arg = (double)steps[b] * w;
        us[t] = (float)((e & 1) ? cos(arg) : sin(arg));
    }
    __syncthreads();
    if (t < kFeat) u[(size_t)b * kFeat + t] = us[t];
    const float *Wl = prm + kOffLin, *bl = prm + kOffLin + k * kFeat;
    for (int o = t; o < k; o += blockDim.x) {
        float s = bl[o];
        for (int c = 0; c < kFeat; ++c) s += Wl[o * kFeat + c] * us[c];
        alpha[(size_t)b * k + o] = s;
    }
}

// Mean squared error over B x k and its gradient d alpha = 2 (alpha - target) / (B k), the
// target of sample b being scale * target[tidx[b] * ld + o] (FP64 rows); one workgroup, fixed
// summation order.
__global__ void loss_kernel(int B, int k, const float *__restrict__ alpha,
                            const double *__restrict__ target, int ld,
                            const int *__restrict__ tidx, double scale,
                            float *__restrict__ dalpha, float *__restrict__ loss) {
    __shared__ float part[256];
    const int cnt = B * k;
    float s = 0.f;
    for (int i = threadIdx.x; i < cnt; i += 256) {
        const int b = i / k, o = i - k * b;
        const size_t row = tidx ? (size_t)tidx[b] : (size_t)b;
        const float d = alpha[i] - (float)(scale * target[row * ld + o]);
        dalpha[i] = 2.f * d / (float)cnt;
        s += d * d;
    }
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = part[0] / (float)cnt;
}

// Head gradients: dWl[o][c] = sum_b dalpha[b][o] u[b][c], dbl[o] = sum_b dalpha[b][o].
__global__ void head_wgrad_kernel(int B, int k, const float *__restrict__ dalpha,
                                  const float *__restrict__ u, float *__restrict__ g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= k * (kFeat + 1)) return;
    const int o = i / (kFeat + 1), c = i - (kFeat + 1) * o;
    float s = 0.f;
    for (int b = 0; b < B; ++b)
        s += dalpha[(size_t)b * k + o] * (c < kFeat ? u[(size_t)b * kFeat + c] : 1.f);
    if (c < kFeat) g[kOffLin + o * kFeat + c] = s;
    else g[kOffLin + k * kFeat + o] = s;
}

// dz3[b][c][pos] = GELU'(z3) * (sum_o Wl[o][c] dalpha[b][o]) / 16 for the 64 pooled features.
__global__ void head_dgrad_kernel(int B, int k, const float *__restrict__ dalpha,
                                  const float *__restrict__ prm, const float *__restrict__ z3,
                                  float *__restrict__ dz3) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * kCh[3] * 16) return;
    const int b = i / (kCh[3] * 16), c = (i / 16) % kCh[3];
    const float *Wl = prm + kOffLin;
    float s = 0.f;
    for (int o = 0; o < k; ++o) s += Wl[o * kFeat + c] * dalpha[(size_t)b * k + o];
    dz3[i] = gelu_grad(z3[i]) * s / 16.f;
}

// Partial weight and bias gradients of one convolution over a slice of samples:
// part[slice][co][q] = sum_{b in slice, pos} dz[b][co][pos] * col(b, pos, q), q = K the bias
// (column of ones).  Tiles (co, q) are spread over the waves.
template <int CI, int CO, int S>
__global__ __launch_bounds__(256) void conv_wgrad_kernel(int B, int per_slice,
                                                         const float *__restrict__ x,
                                                         const float *__restrict__ dz,
                                                         float *__restrict__ part) {
    constexpr int So = S / 2, NP = So * So, K = CI * 9, KB = K + 1;
    constexpr int tiles_m = CO / 16, tiles_q = (KB + 15) / 16;
    const int b0 = blockIdx.x * per_slice;
    const int nb = (B - b0) < per_slice ? (B - b0) : per_slice;
    const int N = nb * NP;
    float *out = part + (size_t)blockIdx.x * CO * KB;
    auto fa = [&](int co, int n) {
        const int b = b0 + n / NP, pos = n % NP;
        return dz[((size_t)b * CO + co) * NP + pos];
    };
    auto fb = [&](int n, int q) {
        if (q > K) return 0.f;
        if (q == K) return 1.f;
        const int b = b0 + n / NP, pos = n % NP;
        return conv_in<S>(x + (size_t)b * CI * S * S, q, pos / So, pos % So);
    };
    const int lane = threadIdx.x & 63;
    for (int tile = threadIdx.x >> 6; tile < tiles_m * tiles_q; tile += 4) {
        const int r0 = (tile % tiles_m) * 16, c0 = (tile / tiles_m) * 16;
        const f32x4_t acc = mfma_tile(r0, c0, N, fa, fb);
        const int q = c0 + (lane & 15);
        if (q < KB) {
#pragma unroll
            for (int r = 0; r < 4; ++r) out[(size_t)(r0 + 4 * (lane >> 4) + r) * KB + q] = acc[r];
        }
    }
}

// grad[W(l)][co][q] / grad[b(l)][co] = sum over slices of the partials, in slice order.
__global__ void wgrad_reduce_kernel(int nslices, int CO, int K, const float *__restrict__ part,
                                    float *__restrict__ g, int ow, int ob) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int KB = K + 1;
    if (i >= CO * KB) return;
    float s = 0.f;
    for (int sl = 0; sl < nslices; ++sl) s += part[(size_t)sl * CO * KB + i];
    const int co = i / KB, q = i - KB * co;
    if (q < K) g[ow + co * K + q] = s;
    else g[ob + co] = s;
}

// Input gradient of a convolution as a GEMM: dcol[n][q] = sum_co dz[b][co][pos] W[co][q],
// n = b*NP + pos, rows n (tiles of 16), columns q < K.
template <int CI, int CO, int S>
__global__ __launch_bounds__(256) void conv_dgrad_kernel(int B, const float *__restrict__ dz,
                                                         const float *__restrict__ prm, int l,
                                                         float *__restrict__ dcol) {
    constexpr int So = S / 2, NP = So * So, K = CI * 9;
    constexpr int tiles_q = (K + 15) / 16;
    const float *W = prm + off_w(l);
    const int N = B * NP, tiles_n = (N + 15) / 16;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (tile >= tiles_n * tiles_q) return;
    const int r0 = (tile / tiles_q) * 16, c0 = (tile % tiles_q) * 16;
    auto fa = [&](int n, int co) {
        if (n >= N) return 0.f;
        const int b = n / NP, pos = n - NP * b;
        return dz[((size_t)b * CO + co) * NP + pos];
    };
    auto fb = [&](int co, int q) { return q < K ? W[co * K + q] : 0.f; };
    const f32x4_t acc = mfma_tile(r0, c0, CO, fa, fb);
    const int lane = threadIdx.x & 63, q = c0 + (lane & 15);
    if (q < K) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int n = r0 + 4 * (lane >> 4) + r;
            if (n < N) dcol[(size_t)n * K + q] = acc[r];
        }
    }
}

// dz_prev[b][ci][y][x] = GELU'(z_prev) * sum over the taps (ky, kx) with y = 2oy+ky-1,
// x = 2ox+kx-1 of dcol[b*NP + oy*So + ox][ci*9 + ky*3 + kx].
template <int CI, int S>
__global__ void col2im_gelu_kernel(int B, const float *__restrict__ dcol,
                                   const float *__restrict__ zp, float *__restrict__ dzp) {
    constexpr int So = S / 2, NP = So * So, K = CI * 9;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= B * CI * S * S) return;
    const int x = i % S, y = (i / S) % S, ci = (i / (S * S)) % CI, b = i / (CI * S * S);
    float s = 0.f;
    for (int ky = 0; ky < 3; ++ky) {
        const int ty = y + 1 - ky;
        if (ty < 0 || (ty & 1) || ty / 2 >= So) continue;
        for (int kx = 0; kx < 3; ++kx) {
            const int tx = x + 1 - kx;
            if (tx < 0 || (tx & 1) || tx / 2 >= So) continue;
            s += dcol[((size_t)b * NP + (ty / 2) * So + tx / 2) * K + ci * 9 + ky * 3 + kx];
        }
    }
    dzp[i] = gelu_grad(zp[i]) * s;
}

// Adam on the FP32 master parameters (bias-corrected moments).
__global__ void adam_kernel(int count, float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float lr, float b1,
                            float b2, float eps, float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------------------------
// Workspace plan for a batch of B (floats, 64-float aligned pieces).

struct Plan {
    size_t a0, z1, a1, z2, a2, z3, a3, u, dal, dz3, dz2, dz1, dcol, part, total;
    int nslices, per_slice;
};

static Plan plan(int B, int k) {
    auto up = [](size_t v) { return (v + 63) & ~(size_t)63; };
    Plan p;
    size_t o = 0;
    auto take = [&](size_t n) { size_t r = o; o += up(n); return r; };
    p.a0 = take((size_t)B * kIn * kIn);
    p.z1 = take((size_t)B * 16 * 256);
    p.a1 = take((size_t)B * 16 * 256);
    p.z2 = take((size_t)B * 32 * 64);
    p.a2 = take((size_t)B * 32 * 64);
    p.z3 = take((size_t)B * 64 * 16);
    p.a3 = take((size_t)B * 64 * 16);
    p.u = take((size_t)B * kFeat);
    p.dal = take((size_t)B * k);
    p.dz3 = take((size_t)B * 64 * 16);
    p.dz2 = take((size_t)B * 32 * 64);
    p.dz1 = take((size_t)B * 16 * 256);
    const size_t dc3 = (size_t)B * 16 * 288, dc2 = (size_t)B * 64 * 144;
    p.dcol = take(dc3 > dc2 ? dc3 : dc2);
    p.per_slice = 8;
    p.nslices = (B + p.per_slice - 1) / p.per_slice;
    p.part = take((size_t)p.nslices * 64 * 289);
    p.total = o;
    return p;
}

size_t workspace_bytes(int B, int k) { return plan(B, k).total * sizeof(float); }

static int blocks(size_t n, int t) { return (int)((n + t - 1) / t); }

hipError_t forward(hipStream_t st, int B, int k, const float *prm, const double *img,
                   const int *img_idx, const int *steps, float *alpha, float *ws) {
    const Plan p = plan(B, k);
    hipLaunchKernelGGL(prep_kernel, dim3(B), dim3(256), 0, st, B, img, img_idx, ws + p.a0);
    hipLaunchKernelGGL((conv_fwd_kernel<1, 16, 32>), dim3(blocks(1 * (B * 256 / 16), 4)),
                       dim3(256), 0, st, B, ws + p.a0, prm, 0, ws + p.z1, ws + p.a1);
    hipLaunchKernelGGL((conv_fwd_kernel<16, 32, 16>), dim3(blocks(2 * (B * 64 / 16), 4)),
                       dim3(256), 0, st, B, ws + p.a1, prm, 1, ws + p.z2, ws + p.a2);
    hipLaunchKernelGGL((conv_fwd_kernel<32, 64, 8>), dim3(blocks(4 * (B * 16 / 16), 4)),
                       dim3(256), 0, st, B, ws + p.a2, prm, 2, ws + p.z3, ws + p.a3);
    hipLaunchKernelGGL(head_fwd_kernel, dim3(B), dim3(128), 0, st, B, k, ws + p.a3, steps, prm,
                       ws + p.u, alpha);
    return hipGetLastError();
}

template <int CI, int CO, int S>
static void wgrad(hipStream_t st, const Plan &p, int B, const float *x, const float *dz,
                  float *ws, float *g, int l) {
    hipLaunchKernelGGL((conv_wgrad_kernel<CI, CO, S>), dim3(p.nslices), dim3(256), 0, st, B,
                       p.per_slice, x, dz, ws + p.part);
    hipLaunchKernelGGL(wgrad_reduce_kernel, dim3(blocks((size_t)CO * (CI * 9 + 1), 256)),
                       dim3(256), 0, st, p.nslices, CO, CI * 9, ws + p.part, g, off_w(l),
                       off_b(l));
}

hipError_t backward(hipStream_t st, int B, int k, const float *prm, const double *img,
                    const int *img_idx, const int *steps, const double *target, int ld,
                    const int *tidx, double scale, float *alpha, float *g, float *loss,
                    float *ws) {
    hipError_t e = forward(st, B, k, prm, img, img_idx, steps, alpha, ws);
    if (e != hipSuccess) return e;
    const Plan p = plan(B, k);
    hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(256), 0, st, B, k, alpha, target, ld, tidx,
                       scale, ws + p.dal, loss);
    hipLaunchKernelGGL(head_wgrad_kernel, dim3(blocks((size_t)k * (kFeat + 1), 128)), dim3(128),
                       0, st, B, k, ws + p.dal, ws + p.u, g);
    hipLaunchKernelGGL(head_dgrad_kernel, dim3(blocks((size_t)B * 1024, 256)), dim3(256), 0, st,
                       B, k, ws + p.dal, prm, ws + p.z3, ws + p.dz3);
    // layer 3
    wgrad<32, 64, 8>(st, p, B, ws + p.a2, ws + p.dz3, ws, g, 2);
    hipLaunchKernelGGL((conv_dgrad_kernel<32, 64, 8>),
                       dim3(blocks((size_t)((B * 16 + 15) / 16) * 18, 4)), dim3(256), 0, st, B,
                       ws + p.dz3, prm, 2, ws + p.dcol);
    hipLaunchKernelGGL((col2im_gelu_kernel<32, 8>), dim3(blocks((size_t)B * 32 * 64, 256)),
                       dim3(256), 0, st, B, ws + p.dcol, ws + p.z2, ws + p.dz2);
    // layer 2
    wgrad<16, 32, 16>(st, p, B, ws + p.a1, ws + p.dz2, ws, g, 1);
    hipLaunchKernelGGL((conv_dgrad_kernel<16, 32, 16>),
                       dim3(blocks((size_t)((B * 64 + 15) / 16) * 9, 4)), dim3(256), 0, st, B,
                       ws + p.dz2, prm, 1, ws + p.dcol);
    hipLaunchKernelGGL((col2im_gelu_kernel<16, 16>), dim3(blocks((size_t)B * 16 * 256, 256)),
                       dim3(256), 0, st, B, ws + p.dcol, ws + p.z1, ws + p.dz1);
    // layer 1 (no input gradient)
    wgrad<1, 16, 32>(st, p, B, ws + p.a0, ws + p.dz1, ws, g, 0);
    return hipGetLastError();
}

hipError_t adam(hipStream_t st, int count, float *prm, const float *g, float *m, float *v,
                int t, float lr, float b1, float b2, float eps) {
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks((size_t)count, 256)), dim3(256), 0, st, count,
                       prm, g, m, v, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

}  // namespace cnn
}  // namespace xkp
