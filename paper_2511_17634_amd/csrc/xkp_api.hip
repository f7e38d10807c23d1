// C ABI of libxkp: context, workspace and argument checks around the kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <vector>

#include "xkp.h"
#include "xkp_internal.h"

struct xkp_ctx {
    int device;
    hipStream_t stream;
    int max_n, max_m, max_batch;
    int slots;          // workgroups that own a workspace slot (the largest grid launched)
    xkp::WsLayout L;
    double *ws;
    unsigned *queue;    // work-queue counters of the solve kernels (reset by each launch)
    int cus;            // compute units of the device
    int per_cu;         // workgroups per compute unit used for the grid (autotuned)
    int variant;        // kernel variant (workgroup size) of the solve launches (autotuned)
    // seeds spread over several workgroups (xkp_ctx_set_seed_width): on (1) or off (0),
    // workgroups per seed at max_n, seeds per call, exchange areas
    int wide_R, wide_gmax, wide_cap;
    unsigned char *xch;
    size_t xch_stride;
    long long wide_limit;   // give-up time of a spread-out seed's waits, 100 MHz ticks
    // targets projected in launches of their own (xkp_ctx_set_projection_split): on, tiles per
    // target at most (0: as many as the slots allow), partial slots, per-target counters,
    // coefficients and statuses
    int split, split_tiles, pj_slots, pj_stride;
    double *pj_part, *pj_alpha;
    unsigned *pj_ctr;
    int *pj_stat;
    // phase timing of target calls (xkp_ctx_set_timing): before the projection launches, before
    // the solve launch, after it; recorded once a call has run
    int timing, timed;
    hipEvent_t tev[3];
};

namespace {

xkp_status from_hip(hipError_t e) { return e == hipSuccess ? XKP_OK : XKP_EDEVICE; }

// One compiled kernel variant (workgroup size) and its launchers.
struct Variant {
    int (*threads)();
    int (*rmax_for)(int);
    int (*lds_vec_len)(int);
    int (*solve_per_cu)(int);
    decltype(&xkp::v512::launch_solve) solve;
    decltype(&xkp::v512::launch_coeffs) coeffs;
    decltype(&xkp::v512::launch_residual) residual;
    decltype(&xkp::v512::launch_rhs) rhs;
    decltype(&xkp::v512::launch_apply) apply;
    decltype(&xkp::v512::launch_accum) accum;
};
#define XKP_VARIANT_TABLE(NS)                                                          \
    Variant {                                                                          \
        xkp::NS::threads, xkp::NS::rmax_for, xkp::NS::lds_vec_len, xkp::NS::solve_per_cu, \
            xkp::NS::launch_solve, xkp::NS::launch_coeffs, xkp::NS::launch_residual,   \
            xkp::NS::launch_rhs, xkp::NS::launch_apply, xkp::NS::launch_accum          \
    }
// Kernel variants by workgroup size: 8 wave64s (2, 8 or 32 rows per thread for up to 1024, 4096,
// 16384 unknowns), 16 (4 or 16 rows per thread for up to 4096, 16384) and 4 (4 or 16 rows per
// thread for up to 1024, 4096).  Variant 0 serves every size and the single-pass kernels
// (residual, rhs, apply, accumulation).
const Variant kVariants[] = {XKP_VARIANT_TABLE(v512), XKP_VARIANT_TABLE(v1024),
                             XKP_VARIANT_TABLE(v256)};
constexpr int kNumVariants = 3;

const Variant *choose(int nmax) { return kVariants[0].rmax_for(nmax) ? &kVariants[0] : nullptr; }

// The context's solve variant if it covers nmax, else variant 0.
const Variant *choose_solve(const xkp_ctx *ctx, int nmax) {
    const Variant &v = kVariants[ctx->variant];
    return v.rmax_for(nmax) ? &v : choose(nmax);
}

// Rows covered by the workspace's coefficient arrays: the most any variant uses for nmax.
int npad_for(int nmax) {
    int best = 0;
    for (const Variant &v : kVariants) {
        const int r = v.rmax_for(nmax) * v.threads();
        if (r > best) best = r;
    }
    return best;
}

// Exchange areas of spread-out seeds and the partial slots of split projections live in
// uncached device memory: workgroups on different XCDs read each other's stores within one
// launch, and a line of ordinary (coarse-grained) memory held in one XCD's L2 need not see
// another XCD's store.  Uncached memory once read by a kernel must not be freed while the
// process runs (later allocations could then read wrong values), so released areas go back to
// this per-device pool and are reused, never freed.
struct XchBuf {
    int device;
    size_t bytes;
    unsigned char *ptr;
    bool used;
};
std::mutex g_xch_mu;
std::vector<XchBuf> g_xch_pool;

unsigned char *xch_acquire(int device, size_t bytes) {
    std::lock_guard<std::mutex> g(g_xch_mu);
    XchBuf *best = nullptr;
    for (XchBuf &b : g_xch_pool)
        if (!b.used && b.device == device && b.bytes >= bytes && (!best || b.bytes < best->bytes))
            best = &b;
    if (best) {
        best->used = true;
        return best->ptr;
    }
    void *p = nullptr;
    if (hipExtMallocWithFlags(&p, bytes, hipDeviceMallocUncached) != hipSuccess || !p)
        return nullptr;
    g_xch_pool.push_back(XchBuf{device, bytes, (unsigned char *)p, true});
    return (unsigned char *)p;
}

void xch_release(unsigned char *ptr) {
    std::lock_guard<std::mutex> g(g_xch_mu);
    for (XchBuf &b : g_xch_pool)
        if (b.ptr == ptr) b.used = false;
}

// Host checks of a call's parameters against the restart and size limits of its workspace.
xkp_status check_params(const xkp_params *P, int max_m, int max_n) {
    if (!P) return XKP_EINVAL;
    if (P->m < 1 || P->m > max_m || !(P->tol >= 0.0) || P->max_restarts < 0 ||
        P->polish_m < 0 || P->polish_m > max_m || P->batch_max_n < 0 || P->batch_max_n > max_n ||
        (P->reorth != XKP_REORTH_AUTO && P->reorth != XKP_REORTH_ALWAYS))
        return XKP_EINVAL;
    if (P->precision != XKP_FP64 && P->precision != XKP_MIXED) return XKP_EINVAL;
    if (P->mode < XKP_PROJ_TARGET_GALERKIN || P->mode > XKP_PROJ_NONE) return XKP_EINVAL;
    return XKP_OK;
}

// Shared host checks of a batched call; fills the effective n limit and kernel variant.
xkp_status check_call(const xkp_ctx *ctx, int32_t count, const void *arr, const xkp_params *P,
                      int *nmax, int *rmax, const Variant **var) {
    if (!ctx || count < 0 || (count > 0 && !arr) || !P) return XKP_EINVAL;
    const xkp_status pst = check_params(P, ctx->max_m, ctx->max_n);
    if (pst != XKP_OK) return pst;
    *nmax = P->batch_max_n > 0 ? P->batch_max_n : ctx->max_n;
    *var = choose_solve(ctx, *nmax);
    if (!*var) return XKP_EUNSUPPORTED;
    *rmax = (*var)->rmax_for(*nmax);
    return XKP_OK;
}

// Workgroups of a solve launch over `count` systems.
int solve_grid(const xkp_ctx *ctx, int count) {
    int g = ctx->per_cu * ctx->cus;
    if (g > ctx->slots) g = ctx->slots;
    return count < g ? count : g;
}

// Workspace of the allocation-free target solve: one fixed device array per GPU, held until the
// process ends.  Bytes [0, 256) hold the work-queue counters, the per-workgroup solve slots
// follow.  Host code never passes `scratch` itself to a kernel (in host code it names a host-side
// stand-in); it uses the device address hipGetSymbolAddress returns on each device.
constexpr size_t kScratchBytes = (size_t)XKP_NOALLOC_SCRATCH_MIB << 20;
constexpr size_t kScratchHead = 256;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];   // device address of `scratch` on each device, once set up

// The device address of this device's `scratch` (the device must be current).
xkp_status scratch_on(int device, unsigned char **out) {
    if (device < 0 || device >= kMaxDevices) return XKP_EINVAL;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return XKP_EDEVICE;
        g_scratch_ptr[device] = p;
    }
    *out = (unsigned char *)g_scratch_ptr[device];
    return XKP_OK;
}

// Clears the work-queue counters before a launch (a kernel node, so the call can be captured).
__global__ void clear_queue_kernel(unsigned *q) {
    if (threadIdx.x < 2) q[threadIdx.x] = 0u;
}

}  // namespace

extern "C" {

xkp_status xkp_ctx_create(xkp_ctx **out, int device, void *hip_stream, int32_t max_n,
                          int32_t max_m, int32_t max_batch) {
    if (!out || max_n < 1 || max_m < 1 || max_batch < 1) return XKP_EINVAL;
    *out = nullptr;
    if (max_m > 64 || !choose(max_n)) return XKP_EUNSUPPORTED;
    if (hipSetDevice(device) != hipSuccess) return XKP_EDEVICE;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return XKP_EDEVICE;
    xkp_ctx *c = new (std::nothrow) xkp_ctx();
    if (!c) return XKP_ENOMEM;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->max_n = max_n;
    c->max_m = max_m;
    c->max_batch = max_batch;
    // one workspace slot per workgroup that can be resident at once: a larger grid would only
    // add workgroups that find the work queue empty
    int per_cu = 0;
    for (const Variant &v : kVariants) {
        if (!v.rmax_for(max_n)) continue;
        const int p = v.solve_per_cu(max_n);
        if (p < 1) {
            delete c;
            return XKP_EDEVICE;
        }
        if (p > per_cu) per_cu = p;
    }
    c->slots = max_batch < per_cu * cus ? max_batch : per_cu * cus;
    c->cus = cus;
    c->per_cu = choose(max_n)->solve_per_cu(max_n);
    c->variant = 0;
    c->wide_limit = 10000000LL;   // 100 ms (a 128x128 seed takes about 2 ms)
    c->L = xkp::ws_layout(max_n, max_m, npad_for(max_n));
    if (hipMalloc((void **)&c->ws, sizeof(double) * c->L.stride * (size_t)c->slots) != hipSuccess) {
        delete c;
        return XKP_ENOMEM;
    }
    if (hipMalloc((void **)&c->queue, 2 * sizeof(unsigned)) != hipSuccess) {
        hipFree(c->ws);
        delete c;
        return XKP_ENOMEM;
    }
    if (hipMemset(c->queue, 0, 2 * sizeof(unsigned)) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        hipFree(c->queue);
        hipFree(c->ws);
        delete c;
        return XKP_EDEVICE;
    }
    *out = c;
    return XKP_OK;
}

xkp_status xkp_ctx_destroy(xkp_ctx *ctx) {
    if (!ctx) return XKP_EINVAL;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    hipError_t f = hipFree(ctx->ws);
    hipError_t q = hipFree(ctx->queue);
    if (ctx->xch) xch_release(ctx->xch);
    if (ctx->pj_part) xch_release((unsigned char *)ctx->pj_part);
    if (ctx->pj_alpha) hipFree(ctx->pj_alpha);
    if (ctx->pj_ctr) hipFree(ctx->pj_ctr);
    if (ctx->pj_stat) hipFree(ctx->pj_stat);
    if (ctx->tev[0])
        for (hipEvent_t ev : ctx->tev) hipEventDestroy(ev);
    delete ctx;
    return (e == hipSuccess && f == hipSuccess && q == hipSuccess) ? XKP_OK : XKP_EDEVICE;
}

xkp_status xkp_ctx_set_launch(xkp_ctx *ctx, int32_t waves, int32_t wg_per_cu) {
    if (!ctx || wg_per_cu < 1) return XKP_EINVAL;
    for (int vi = 0; vi < kNumVariants; ++vi) {
        if (kVariants[vi].threads() != 64 * waves) continue;
        if (!kVariants[vi].rmax_for(ctx->max_n)) return XKP_EUNSUPPORTED;
        if (wg_per_cu * ctx->cus > ctx->slots && wg_per_cu > 1) return XKP_EINVAL;
        ctx->variant = vi;
        ctx->per_cu = wg_per_cu;
        return XKP_OK;
    }
    return XKP_EINVAL;
}

xkp_status xkp_ctx_set_seed_width(xkp_ctx *ctx, int32_t rows_per_thread) {
    if (!ctx || (rows_per_thread != 0 && rows_per_thread != 1)) return XKP_EINVAL;
    if (rows_per_thread == 0) {
        ctx->wide_R = 0;
        return XKP_OK;
    }
    int h = 1;
    while (h * h < ctx->max_n) ++h;
    if (h > 128 || ctx->max_m > 64) return XKP_EUNSUPPORTED;
    const int nb = xkp::wide::rows_per_block();
    const int gmax = (ctx->max_n + nb - 1) / nb;
    const int cap = ctx->max_batch < 64 ? ctx->max_batch : 64;
    if (ctx->xch && ctx->wide_gmax == gmax && ctx->wide_cap == cap) {
        ctx->wide_R = 1;
        return XKP_OK;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return XKP_EDEVICE;
    if (ctx->xch) xch_release(ctx->xch);
    ctx->xch = nullptr;
    ctx->wide_R = 0;
    const size_t xs = xkp::wide::xch_bytes(gmax);
    ctx->xch = xch_acquire(ctx->device, xs * cap);
    if (!ctx->xch) return XKP_ENOMEM;
    ctx->xch_stride = xs;
    ctx->wide_gmax = gmax;
    ctx->wide_cap = cap;
    ctx->wide_R = 1;
    return XKP_OK;
}

xkp_status xkp_ctx_set_timing(xkp_ctx *ctx, int32_t on) {
    if (!ctx || (on != 0 && on != 1)) return XKP_EINVAL;
    if (on && !ctx->tev[0]) {
        if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
        for (int i = 0; i < 3; ++i) {
            if (hipEventCreate(&ctx->tev[i]) != hipSuccess) {
                for (int q = 0; q < i; ++q) hipEventDestroy(ctx->tev[q]);
                ctx->tev[0] = nullptr;
                return XKP_EDEVICE;
            }
        }
    }
    ctx->timing = on;
    ctx->timed = 0;
    return XKP_OK;
}

xkp_status xkp_ctx_last_timing(xkp_ctx *ctx, float *ms_projection, float *ms_solve) {
    if (!ctx || !ms_projection || !ms_solve || !ctx->timing || !ctx->timed) return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    if (hipEventSynchronize(ctx->tev[2]) != hipSuccess ||
        hipEventElapsedTime(ms_projection, ctx->tev[0], ctx->tev[1]) != hipSuccess ||
        hipEventElapsedTime(ms_solve, ctx->tev[1], ctx->tev[2]) != hipSuccess)
        return XKP_EDEVICE;
    return XKP_OK;
}

xkp_status xkp_ctx_set_seed_wait(xkp_ctx *ctx, int64_t microseconds) {
    if (!ctx || microseconds < 0 || microseconds > 60000000LL) return XKP_EINVAL;
    ctx->wide_limit = 100LL * microseconds;
    return XKP_OK;
}

xkp_status xkp_ctx_set_projection_split(xkp_ctx *ctx, int32_t max_tiles) {
    if (!ctx || max_tiles < -1) return XKP_EINVAL;
    if (max_tiles < 0) {
        ctx->split = 0;
        return XKP_OK;
    }
    ctx->split_tiles = max_tiles;
    if (ctx->pj_part) {
        ctx->split = 1;
        return XKP_OK;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    // one slot per 256-row tile of a full batch of the largest systems, 2048 at most: a batch
    // with more tiles than slots splits its targets into fewer tiles, down to one per target
    const int tiles = (ctx->max_n + 255) / 256;
    long slots = (long)ctx->max_batch * tiles;
    if (slots > 2048) slots = 2048;
    const int stride = xkp::proj::slot_doubles(ctx->max_m);
    // the slots from the uncached pool: a target's last tile reads what tiles on other XCDs
    // stored in the same launch
    double *part = (double *)xch_acquire(ctx->device, sizeof(double) * stride * (size_t)slots);
    double *alpha = nullptr;
    unsigned *ctr = nullptr;
    int *stat = nullptr;
    if (!part ||
        hipMalloc((void **)&alpha, sizeof(double) * 64 * (size_t)ctx->max_batch) != hipSuccess ||
        hipMalloc((void **)&ctr, sizeof(unsigned) * (size_t)ctx->max_batch) != hipSuccess ||
        hipMalloc((void **)&stat, sizeof(int) * (size_t)ctx->max_batch) != hipSuccess) {
        if (part) xch_release((unsigned char *)part);
        if (alpha) hipFree(alpha);
        if (ctr) hipFree(ctr);
        return XKP_ENOMEM;
    }
    if (hipMemset(ctr, 0, sizeof(unsigned) * (size_t)ctx->max_batch) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        xch_release((unsigned char *)part);
        hipFree(alpha);
        hipFree(ctr);
        hipFree(stat);
        return XKP_EDEVICE;
    }
    ctx->pj_part = part;
    ctx->pj_alpha = alpha;
    ctx->pj_ctr = ctr;
    ctx->pj_stat = stat;
    ctx->pj_slots = (int)slots;
    ctx->pj_stride = stride;
    ctx->split = 1;
    return XKP_OK;
}

size_t xkp_basis_bytes(int32_t n, int32_t m) {
    if (n < 1 || m < 1) return 0;
    return xkp::basis_bytes(n, m);
}

xkp_status xkp_seed_build(xkp_ctx *ctx, int32_t n_seeds, const xkp_system *seeds,
                          void *const *bases, const xkp_params *params, xkp_info *infos) {
    int nmax = 0, rmax = 0;
    const Variant *v = nullptr;
    xkp_status st = check_call(ctx, n_seeds, seeds, params, &nmax, &rmax, &v);
    if (st != XKP_OK) return st;
    if (n_seeds > 0 && (!bases || !infos)) return XKP_EINVAL;
    if (n_seeds == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    if (ctx->wide_R > 0 && n_seeds <= ctx->wide_cap && params->reorth == XKP_REORTH_AUTO) {
        // each seed over ceil(n / 256) workgroups; a wait gives up after ctx->wide_limit, and a
        // seed that gave up (XKP_EDEVICE) is solved again by one workgroup in a second launch
        // that skips every other seed
        hipError_t e = xkp::wide::launch_wide_seed(ctx->stream, seeds, n_seeds, *params, bases,
                                                   infos, ctx->xch, ctx->xch_stride,
                                                   ctx->wide_gmax, nmax, ctx->wide_limit);
        if (e != hipSuccess) return XKP_EDEVICE;
        const int grid = solve_grid(ctx, n_seeds);
        return from_hip(v->solve(ctx->stream, grid, rmax, v->lds_vec_len(nmax), seeds, n_seeds,
                                 *params, xkp::kKeepBasis | xkp::kRedo, 0, nullptr, bases, infos,
                                 ctx->ws, ctx->L, nmax, ctx->queue,
                                 xkp::Learned{nullptr, 0, 0.0, 0.0}, nullptr));
    }
    const int grid = solve_grid(ctx, n_seeds);
    return from_hip(v->solve(ctx->stream, grid, rmax, v->lds_vec_len(nmax), seeds, n_seeds,
                             *params, xkp::kKeepBasis, 0, nullptr, bases, infos, ctx->ws, ctx->L,
                             nmax, ctx->queue, xkp::Learned{nullptr, 0, 0.0, 0.0}, nullptr));
}

xkp_status xkp_target_project_solve(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                                    int32_t n_bases, const void *const *bases,
                                    const xkp_params *params, xkp_info *infos) {
    int nmax = 0, rmax = 0;
    const Variant *v = nullptr;
    xkp_status st = check_call(ctx, n_targets, targets, params, &nmax, &rmax, &v);
    if (st != XKP_OK) return st;
    if (n_targets > 0 && !infos) return XKP_EINVAL;
    if (params->mode != XKP_PROJ_NONE && n_targets > 0 && (n_bases < 1 || !bases))
        return XKP_EINVAL;
    if (n_targets == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = solve_grid(ctx, n_targets);
    int flags = (params->mode != XKP_PROJ_NONE ? xkp::kTarget : 0) | xkp::kRegBasis;
    if (ctx->timing && hipEventRecord(ctx->tev[0], ctx->stream) != hipSuccess) return XKP_EDEVICE;
    if (ctx->split && params->mode != XKP_PROJ_NONE && n_targets <= ctx->max_batch) {
        // the projection over row tiles across the chip, then the polish from x0 (the
        // per-target buffers hold max_batch targets: a larger batch projects in the solve
        // launch)
        const hipError_t e = xkp::proj::launch_project(
            ctx->stream, targets, n_targets, n_bases, bases, *params, nmax, ctx->pj_part,
            ctx->pj_slots, ctx->pj_stride, ctx->pj_ctr, ctx->pj_alpha, ctx->pj_stat, infos,
            ctx->split_tiles, ctx->cus);
        if (e != hipSuccess) return XKP_EDEVICE;
        flags |= xkp::kPreProjected;
    }
    if (ctx->timing && hipEventRecord(ctx->tev[1], ctx->stream) != hipSuccess) return XKP_EDEVICE;
    st = from_hip(v->solve(ctx->stream, grid, rmax, v->lds_vec_len(nmax), targets, n_targets,
                           *params, flags, n_bases, bases, nullptr, infos, ctx->ws, ctx->L,
                           nmax, ctx->queue, xkp::Learned{nullptr, 0, 0.0, 0.0}, ctx->pj_stat));
    if (st == XKP_OK && ctx->timing) {
        if (hipEventRecord(ctx->tev[2], ctx->stream) != hipSuccess) return XKP_EDEVICE;
        ctx->timed = 1;
    }
    return st;
}

xkp_status xkp_learned_solve(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                             int32_t n_bases, const void *const *bases, const xkp_params *params,
                             const float *alpha, int32_t alpha_ld, double alpha_scale,
                             double gate, xkp_info *infos) {
    int nmax = 0, rmax = 0;
    const Variant *v = nullptr;
    xkp_status st = check_call(ctx, n_targets, targets, params, &nmax, &rmax, &v);
    if (st != XKP_OK) return st;
    if (n_targets > 0 && (!infos || !alpha || alpha_ld < 1 || n_bases < 1 || !bases))
        return XKP_EINVAL;
    if (!(gate >= 0.0) || !(alpha_scale == alpha_scale)) return XKP_EINVAL;
    if (n_targets == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = solve_grid(ctx, n_targets);
    const int flags = xkp::kLearned | (params->mode != XKP_PROJ_NONE ? xkp::kTarget : 0) |
                      xkp::kRegBasis;
    return from_hip(v->solve(ctx->stream, grid, rmax, v->lds_vec_len(nmax), targets, n_targets,
                             *params, flags, n_bases, bases, nullptr, infos, ctx->ws, ctx->L,
                             nmax, ctx->queue, xkp::Learned{alpha, alpha_ld, alpha_scale, gate},
                             nullptr));
}

xkp_status xkp_learned_correction_solve(xkp_ctx *ctx, int32_t n_targets,
                                        const xkp_system *targets, int32_t n_bases,
                                        const void *const *bases, const xkp_params *params,
                                        const float *alpha, int32_t alpha_ld, double alpha_scale,
                                        double gate, xkp_info *infos) {
    int nmax = 0, rmax = 0;
    const Variant *v = nullptr;
    xkp_status st = check_call(ctx, n_targets, targets, params, &nmax, &rmax, &v);
    if (st != XKP_OK) return st;
    if (params->mode == XKP_PROJ_NONE) return XKP_EINVAL;
    if (n_targets > 0 && (!infos || !alpha || alpha_ld < 1 || n_bases < 1 || !bases))
        return XKP_EINVAL;
    if (!(gate >= 0.0) || !(alpha_scale == alpha_scale)) return XKP_EINVAL;
    if (n_targets == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = solve_grid(ctx, n_targets);
    const int flags = xkp::kLearned | xkp::kCorrection | xkp::kTarget | xkp::kRegBasis;
    return from_hip(v->solve(ctx->stream, grid, rmax, v->lds_vec_len(nmax), targets, n_targets,
                             *params, flags, n_bases, bases, nullptr, infos, ctx->ws, ctx->L,
                             nmax, ctx->queue, xkp::Learned{alpha, alpha_ld, alpha_scale, gate},
                             nullptr));
}

xkp_status xkp_basis_coeffs(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems,
                            int32_t n_bases, const void *const *bases, int32_t m_out,
                            int32_t kind, double *alpha) {
    if (!ctx || n_sys < 0 || (n_sys > 0 && (!systems || !bases || n_bases < 1 || !alpha)) ||
        m_out < 1 || m_out > 65 || (kind != 0 && kind != 1) || (kind == 0 && m_out > 64))
        return XKP_EINVAL;
    if (n_sys == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const Variant *v = choose(ctx->max_n);
    const int grid = n_sys < 4096 ? n_sys : 4096;
    return from_hip(v->coeffs(ctx->stream, grid, v->rmax_for(ctx->max_n), systems, n_sys, n_bases,
                              bases, m_out, kind, alpha, ctx->max_n));
}

xkp_status xkp_residual(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems, double *rel_res) {
    if (!ctx || n_sys < 0 || (n_sys > 0 && (!systems || !rel_res))) return XKP_EINVAL;
    if (n_sys == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = n_sys < 4096 ? n_sys : 4096;
    const Variant *v = choose(ctx->max_n);
    return from_hip(v->residual(ctx->stream, grid, v->rmax_for(ctx->max_n),
                                v->lds_vec_len(ctx->max_n), systems, n_sys, rel_res, ctx->max_n));
}

xkp_status xkp_basis_accumulate(xkp_ctx *ctx, int32_t n, int32_t n_src,
                                const void *const *src_bases, void *const *out_bases,
                                int32_t per_source, int32_t cap, int32_t *out_k) {
    if (!ctx || !src_bases || !out_bases || n_src < 1 || per_source < 1 || cap < 1 ||
        cap > ctx->max_m || n < 1 || n > ctx->max_n)
        return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const Variant *v = choose(n);
    if (!v) return XKP_EINVAL;
    return from_hip(v->accum(ctx->stream, v->rmax_for(n), n, n_src, src_bases, out_bases,
                             per_source, cap, out_k));
}

xkp_status xkp_score_flow(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems, int32_t field,
                          double *const *score, double *const *disp) {
    if (!ctx || n_sys < 0 || (n_sys > 0 && !systems) ||
        (field != XKP_FIELD_MT && field != XKP_FIELD_X) || n_sys > 65535)
        return XKP_EINVAL;
    if (n_sys == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    return from_hip(xkp::epi::launch_score_flow(ctx->stream, systems, n_sys, field, score, disp,
                                                ctx->max_n));
}

xkp_status xkp_cluster_seeds(xkp_ctx *ctx, int32_t n_img, int32_t H, const double *images,
                             int32_t pool, int32_t K, int32_t max_iters, int32_t *assign,
                             int32_t *seeds, int32_t *iters) {
    if (!ctx || n_img < 1 || H < 1 || (long)H * H > ctx->max_n || !images || pool < 1 ||
        H % pool != 0 || K < 1 || K > 64 || K > n_img || max_iters < 1 || !assign || !seeds)
        return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int N = n_img, d = (H / pool) * (H / pool);
    hipStream_t st = ctx->stream;
    double *feat = nullptr;
    const size_t bytes = sizeof(double) * ((size_t)N * d + (size_t)K * d + N) + sizeof(int) * N;
    if (hipMalloc((void **)&feat, bytes) != hipSuccess) return XKP_ENOMEM;
    double *cent = feat + (size_t)N * d, *dist = cent + (size_t)K * d;
    int *asg = (int *)(dist + N);
    std::vector<double> hd(N);
    std::vector<int> ha(N), prev(N);
    int it = 0;
    auto run = [&]() -> xkp_status {
        if (xkp::clu::pool(st, images, N, H, pool, feat) != hipSuccess) return XKP_EDEVICE;
        // farthest-first start
        if (hipMemcpyAsync(cent, feat, sizeof(double) * d, hipMemcpyDeviceToDevice, st) !=
            hipSuccess)
            return XKP_EDEVICE;
        for (int k = 1; k < K; ++k) {
            if (xkp::clu::distances(st, feat, N, d, cent, k, nullptr, dist) != hipSuccess ||
                hipMemcpyAsync(hd.data(), dist, sizeof(double) * N, hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return XKP_EDEVICE;
            int arg = 0;
            for (int i = 1; i < N; ++i)
                if (hd[i] > hd[arg]) arg = i;
            if (hipMemcpyAsync(cent + (size_t)k * d, feat + (size_t)arg * d, sizeof(double) * d,
                               hipMemcpyDeviceToDevice, st) != hipSuccess)
                return XKP_EDEVICE;
        }
        // Lloyd iterations
        bool have = false;
        while (it < max_iters) {
            if (xkp::clu::distances(st, feat, N, d, cent, K, asg, dist) != hipSuccess ||
                hipMemcpyAsync(ha.data(), asg, sizeof(int) * N, hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return XKP_EDEVICE;
            ++it;
            if (have && ha == prev) break;
            prev = ha;
            have = true;
            if (xkp::clu::update(st, feat, N, d, asg, K, cent) != hipSuccess) return XKP_EDEVICE;
        }
        // final assignment and the seed of each cluster
        if (xkp::clu::distances(st, feat, N, d, cent, K, asg, dist) != hipSuccess ||
            hipMemcpyAsync(ha.data(), asg, sizeof(int) * N, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipMemcpyAsync(hd.data(), dist, sizeof(double) * N, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return XKP_EDEVICE;
        std::vector<int> hs(K, -1);
        for (int i = 0; i < N; ++i) {
            const int c = ha[i];
            if (hs[c] < 0 || hd[i] < hd[hs[c]]) hs[c] = i;
        }
        if (hipMemcpyAsync(assign, ha.data(), sizeof(int) * N, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(seeds, hs.data(), sizeof(int) * K, hipMemcpyHostToDevice, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
            return XKP_EDEVICE;
        return XKP_OK;
    };
    const xkp_status r = run();
    hipStreamSynchronize(st);
    hipFree(feat);
    if (r == XKP_OK && iters) *iters = it;
    return r;
}

xkp_status xkp_build_rhs(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems) {
    if (!ctx || n_sys < 0 || (n_sys > 0 && !systems)) return XKP_EINVAL;
    if (n_sys == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = n_sys < 4096 ? n_sys : 4096;
    const Variant *v = choose(ctx->max_n);
    return from_hip(v->rhs(ctx->stream, grid, v->rmax_for(ctx->max_n), systems, n_sys,
                           ctx->max_n));
}

xkp_status xkp_apply(xkp_ctx *ctx, int32_t n_sys, const xkp_system *systems) {
    if (!ctx || n_sys < 0 || (n_sys > 0 && !systems)) return XKP_EINVAL;
    if (n_sys == 0) return XKP_OK;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int grid = n_sys < 4096 ? n_sys : 4096;
    const Variant *v = choose(ctx->max_n);
    return from_hip(v->apply(ctx->stream, grid, v->rmax_for(ctx->max_n),
                             v->lds_vec_len(ctx->max_n), systems, n_sys, ctx->max_n));
}

// Shared timing loop of the autotuners: for each kernel variant covering nmax, each candidate
// restart length and each workgroup count per compute unit, one untimed and `timed` timed calls
// of `call(P)`; keeps the fastest candidate whose every system ended with an accepted status.
// The chosen variant and workgroup count stay in the context.
extern "C++" template <typename Call>
static xkp_status tune_loop(xkp_ctx *ctx, int nmax, int nsys, xkp_info *infos,
                            const xkp_params *params, const int *cand_m, int ncand, bool seeds,
                            int timed, Call call, xkp_tuning *out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return XKP_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return XKP_EDEVICE;
    }
    std::vector<xkp_info> host(nsys);
    const int saved_w = ctx->per_cu, saved_v = ctx->variant;
    xkp_status result = XKP_OK;
    float best = -1.f, def = -1.f;
    int best_m = cand_m[ncand - 1], best_w = saved_w, best_v = saved_v, tried = 0;
    for (int vi = 0; vi < kNumVariants && result == XKP_OK; ++vi) {
        const Variant &var = kVariants[vi];
        if (!var.rmax_for(nmax)) continue;
        int nb = var.solve_per_cu(nmax);
        if (nb < 1) {
            result = XKP_EDEVICE;
            break;
        }
        if (nb * ctx->cus > ctx->slots) nb = (ctx->slots + ctx->cus - 1) / ctx->cus;
        ctx->variant = vi;
        for (int ci = 0; ci < ncand && result == XKP_OK; ++ci) {
            if (ci > 0 && cand_m[ci] == cand_m[ci - 1]) continue;
            for (int w = 1; w <= nb && result == XKP_OK; ++w) {
                xkp_params P = *params;
                if (!seeds) P.polish_m = cand_m[ci];
                ctx->per_cu = w;
                float ms = 0.f;
                for (int rep = 0; rep <= timed && result == XKP_OK; ++rep) {
                    if (rep == 1 && hipEventRecord(e0, ctx->stream) != hipSuccess)
                        result = XKP_EDEVICE;
                    xkp_status st = call(P);
                    if (st != XKP_OK) result = st;
                }
                if (result != XKP_OK) break;
                if (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                    hipEventSynchronize(e1) != hipSuccess ||
                    hipEventElapsedTime(&ms, e0, e1) != hipSuccess ||
                    hipMemcpy(host.data(), infos, sizeof(xkp_info) * nsys,
                              hipMemcpyDeviceToHost) != hipSuccess) {
                    result = XKP_EDEVICE;
                    break;
                }
                ms /= (float)timed;
                ++tried;
                bool ok = true;
                for (const xkp_info &i : host)
                    ok = ok && (i.status == XKP_OK || (!seeds && i.status == XKP_ESINGULAR));
                if (vi == 0 && ci == ncand - 1 && w == nb) def = ms;
                if (ok && (best < 0.f || ms < best)) {
                    best = ms;
                    best_m = cand_m[ci];
                    best_w = w;
                    best_v = vi;
                }
            }
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (result != XKP_OK || best < 0.f) {
        ctx->per_cu = saved_w;
        ctx->variant = saved_v;
        return result != XKP_OK ? result : XKP_ENOCONV;
    }
    out->polish_m = best_m;
    out->wg_per_cu = best_w;
    out->ms_best = best;
    out->ms_default = def;
    out->n_tried = tried;
    out->waves = kVariants[best_v].threads() / 64;
    ctx->per_cu = best_w;
    ctx->variant = best_v;
    return XKP_OK;
}

xkp_status xkp_autotune(xkp_ctx *ctx, int32_t n_targets, const xkp_system *targets,
                        int32_t n_bases, const void *const *bases, const xkp_params *params,
                        xkp_info *infos, xkp_tuning *out) {
    if (!ctx || !params || !out || n_targets < 1 || !targets || !infos) return XKP_EINVAL;
    {
        int nmax = 0, rmax = 0;
        const Variant *v = nullptr;
        xkp_status st = check_call(ctx, n_targets, targets, params, &nmax, &rmax, &v);
        if (st != XKP_OK) return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int m = params->m;
    const int nmax = params->batch_max_n > 0 ? params->batch_max_n : ctx->max_n;
    // short restarts whose basis fits the registers (6, 8, 9), then fractions of m (>= 8)
    int cand_m[7] = {6, 8, 9, m / 4 < 8 ? 8 : m / 4, m / 2, (3 * m) / 4, m};
    for (int &c : cand_m)
        if (c > m) c = m;
    std::sort(cand_m, cand_m + 7);
    auto run = [&](xkp_tuning *t) {
        return tune_loop(ctx, nmax, n_targets, infos, params, cand_m, 7, false, 2,
                         [&](const xkp_params &P) {
                             return xkp_target_project_solve(ctx, n_targets, targets, n_bases,
                                                             bases, &P, infos);
                         },
                         t);
    };
    // every candidate with the projection inside the solve launch, then (projected batches the
    // per-target buffers hold) with the projection in launches of its own; the faster stays
    const int saved_split = ctx->split;
    ctx->split = 0;
    xkp_tuning t_in = *out;
    xkp_status st = run(&t_in);
    if (st != XKP_OK) {
        ctx->split = saved_split;
        return st;
    }
    *out = t_in;
    out->split = -1;
    if (params->mode == XKP_PROJ_NONE || n_targets > ctx->max_batch) return XKP_OK;
    const int in_w = ctx->per_cu, in_v = ctx->variant;
    const int tiles = ctx->pj_part ? ctx->split_tiles : 0;
    st = xkp_ctx_set_projection_split(ctx, tiles);
    if (st != XKP_OK) {
        ctx->split = 0;
        return st == XKP_ENOMEM ? XKP_OK : st;   // no room for the split buffers: stay in-launch
    }
    xkp_tuning t_sp = t_in;
    st = run(&t_sp);
    if (st == XKP_OK && t_sp.ms_best < t_in.ms_best) {
        // the two winners timed again, five calls each, alternating: the split stays only if
        // it is still the faster
        const int sp_w = ctx->per_cu, sp_v = ctx->variant;
        auto timed = [&](int split, int w, int vi, int pm, float *ms) {
            ctx->split = split;
            ctx->per_cu = w;
            ctx->variant = vi;
            xkp_params P = *params;
            P.polish_m = pm;
            hipEvent_t e0, e1;
            if (hipEventCreate(&e0) != hipSuccess) return XKP_EDEVICE;
            if (hipEventCreate(&e1) != hipSuccess) {
                hipEventDestroy(e0);
                return XKP_EDEVICE;
            }
            xkp_status r = xkp_target_project_solve(ctx, n_targets, targets, n_bases, bases, &P,
                                                    infos);
            if (r == XKP_OK && hipEventRecord(e0, ctx->stream) != hipSuccess) r = XKP_EDEVICE;
            for (int q = 0; q < 5 && r == XKP_OK; ++q)
                r = xkp_target_project_solve(ctx, n_targets, targets, n_bases, bases, &P, infos);
            if (r == XKP_OK && (hipEventRecord(e1, ctx->stream) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess ||
                                hipEventElapsedTime(ms, e0, e1) != hipSuccess))
                r = XKP_EDEVICE;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            return r;
        };
        float ms_in = 0.f, ms_sp = 0.f;
        st = timed(0, in_w, in_v, t_in.polish_m, &ms_in);
        if (st == XKP_OK) st = timed(1, sp_w, sp_v, t_sp.polish_m, &ms_sp);
        if (st != XKP_OK) return st;
        if (ms_sp < ms_in) {
            t_sp.ms_best = ms_sp / 5.f;
            t_sp.ms_default = t_in.ms_default;
            t_sp.n_tried += t_in.n_tried;
            t_sp.split = tiles;
            *out = t_sp;
            return XKP_OK;   // the split winner's variant and workgroup count stay set
        }
        out->ms_best = ms_in / 5.f;
    }
    out->n_tried += st == XKP_OK ? t_sp.n_tried : 0;
    ctx->split = 0;
    ctx->per_cu = in_w;
    ctx->variant = in_v;
    return st == XKP_OK || st == XKP_ENOCONV ? XKP_OK : st;
}

xkp_status xkp_autotune_seeds(xkp_ctx *ctx, int32_t n_seeds, const xkp_system *seeds,
                              void *const *bases, const xkp_params *params, xkp_info *infos,
                              xkp_tuning *out) {
    if (!ctx || !params || !out || n_seeds < 1 || !seeds || !bases || !infos) return XKP_EINVAL;
    {
        int nmax = 0, rmax = 0;
        const Variant *v = nullptr;
        xkp_status st = check_call(ctx, n_seeds, seeds, params, &nmax, &rmax, &v);
        if (st != XKP_OK) return st;
    }
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    const int nmax = params->batch_max_n > 0 ? params->batch_max_n : ctx->max_n;
    const int cand_m[1] = {params->m};
    const int saved_R = ctx->wide_R;
    ctx->wide_R = 0;
    auto call = [&](const xkp_params &P) {
        return xkp_seed_build(ctx, n_seeds, seeds, bases, &P, infos);
    };
    xkp_status st = tune_loop(ctx, nmax, n_seeds, infos, params, cand_m, 1, true, 5, call, out);
    out->seed_rows = 0;
    if (st != XKP_OK) {
        ctx->wide_R = saved_R;
        return st;
    }
    // then each seed over several workgroups (256-row blocks) when that gives it at least
    // two; kept if faster with every seed converged
    int h = 1;
    while (h * h < nmax) ++h;
    if (n_seeds > 64 || h > 128 || params->reorth != XKP_REORTH_AUTO) return XKP_OK;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess) return XKP_EDEVICE;
    if (hipEventCreate(&e1) != hipSuccess) {
        hipEventDestroy(e0);
        return XKP_EDEVICE;
    }
    std::vector<xkp_info> host(n_seeds);
    int best_R = 0;
    for (int R : {1}) {
        if ((nmax + 255) / 256 < 2) continue;
        if (xkp_ctx_set_seed_width(ctx, R) != XKP_OK) continue;
        float ms = 0.f;
        bool ok = call(*params) == XKP_OK && hipEventRecord(e0, ctx->stream) == hipSuccess;
        for (int rep = 0; ok && rep < 5; ++rep) ok = call(*params) == XKP_OK;
        ok = ok && hipEventRecord(e1, ctx->stream) == hipSuccess &&
             hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess &&
             hipMemcpy(host.data(), infos, sizeof(xkp_info) * n_seeds,
                       hipMemcpyDeviceToHost) == hipSuccess;
        if (!ok) {
            st = XKP_EDEVICE;
            break;
        }
        ms /= 5.f;
        ++out->n_tried;
        bool conv = true;
        for (const xkp_info &i : host) conv = conv && i.status == XKP_OK;
        if (conv && ms < out->ms_best) {
            out->ms_best = ms;
            best_R = R;
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st != XKP_OK) {
        xkp_ctx_set_seed_width(ctx, 0);
        return st;
    }
    st = xkp_ctx_set_seed_width(ctx, best_R);
    if (st != XKP_OK) return st;
    out->seed_rows = best_R;
    // the last candidate's results are in the outputs: recompute them with the choice
    return call(*params);
}

size_t xkp_cnn_param_count(int32_t k) {
    if (k < 1 || k > 64) return 0;
    return xkp::cnn::param_count(k);
}

size_t xkp_cnn_workspace_bytes(int32_t batch, int32_t k) {
    if (batch < 1 || k < 1 || k > 64) return 0;
    return xkp::cnn::workspace_bytes(batch, k);
}

xkp_status xkp_cnn_forward(xkp_ctx *ctx, int32_t batch, int32_t k, const float *params,
                           const double *images, const int32_t *image_idx, const int32_t *steps,
                           float *alpha, void *work) {
    if (!ctx || batch < 1 || k < 1 || k > 64 || !params || !images || !steps || !alpha || !work)
        return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    return from_hip(xkp::cnn::forward(ctx->stream, batch, k, params, images, image_idx, steps,
                                      alpha, (float *)work));
}

xkp_status xkp_cnn_backward(xkp_ctx *ctx, int32_t batch, int32_t k, const float *params,
                            const double *images, const int32_t *image_idx, const int32_t *steps,
                            const double *target, int32_t target_ld, const int32_t *target_idx,
                            double target_scale, float *alpha, float *grad, float *loss,
                            void *work) {
    if (!ctx || batch < 1 || k < 1 || k > 64 || !params || !images || !steps || !target ||
        target_ld < k || !alpha || !grad || !loss || !work || !(target_scale == target_scale))
        return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    return from_hip(xkp::cnn::backward(ctx->stream, batch, k, params, images, image_idx, steps,
                                       target, target_ld, target_idx, target_scale, alpha, grad,
                                       loss, (float *)work));
}

xkp_status xkp_cnn_adam(xkp_ctx *ctx, int32_t count, float *params, const float *grad, float *m,
                        float *v, int32_t t, float lr, float beta1, float beta2, float eps) {
    if (!ctx || count < 1 || !params || !grad || !m || !v || t < 1 || !(lr > 0.f) ||
        !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return XKP_EINVAL;
    if (hipSetDevice(ctx->device) != hipSuccess) return XKP_EDEVICE;
    return from_hip(xkp::cnn::adam(ctx->stream, count, params, grad, m, v, t, lr, beta1, beta2,
                                   eps));
}

xkp_status xkp_target_project_solve_noalloc(int device, void *hip_stream, int32_t n_targets,
                                            const xkp_system *targets, int32_t n_bases,
                                            const void *const *bases, const xkp_params *params,
                                            xkp_info *infos) {
    // host checks first: nothing is enqueued and no device call is made for a bad argument
    constexpr int kMaxN = XKP_NOALLOC_MAX_N;
    if (n_targets < 0 || (n_targets > 0 && (!targets || !infos))) return XKP_EINVAL;
    xkp_status st = check_params(params, 64, kMaxN);
    if (st != XKP_OK) return st;
    if (params->mode != XKP_PROJ_NONE && n_targets > 0 && (n_bases < 1 || !bases))
        return XKP_EINVAL;
    // the 8-wave kernels cover every size up to kMaxN
    const int nmax = params->batch_max_n > 0 ? params->batch_max_n : kMaxN;
    const int rmax = xkp::v512::rmax_for(nmax);
    if (!rmax) return XKP_EUNSUPPORTED;
    const int mm = params->polish_m > params->m ? params->polish_m : params->m;
    const xkp::WsLayout L = xkp::ws_layout(nmax, mm, rmax * xkp::v512::threads());
    const size_t slot_bytes = sizeof(double) * L.stride;
    const size_t fit = (kScratchBytes - kScratchHead) / slot_bytes;
    if (fit < 1) return XKP_EINVAL;   // one system of this size does not fit the array
    if (n_targets == 0) return XKP_OK;
    if (hipSetDevice(device) != hipSuccess) return XKP_EDEVICE;
    unsigned char *base = nullptr;
    st = scratch_on(device, &base);
    if (st != XKP_OK) return st;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess)
        return XKP_EDEVICE;
    const int per_cu = xkp::v512::solve_per_cu(nmax);
    if (per_cu < 1) return XKP_EDEVICE;
    long grid = (long)per_cu * cus;
    if ((long)fit < grid) grid = (long)fit;
    if (n_targets < grid) grid = n_targets;
    hipStream_t stream = (hipStream_t)hip_stream;
    unsigned *queue = (unsigned *)base;
    hipLaunchKernelGGL(clear_queue_kernel, dim3(1), dim3(64), 0, stream, queue);
    if (hipGetLastError() != hipSuccess) return XKP_EDEVICE;
    const int flags = (params->mode != XKP_PROJ_NONE ? xkp::kTarget : 0) | xkp::kRegBasis;
    return from_hip(xkp::v512::launch_solve(stream, (int)grid, rmax,
                                            xkp::v512::lds_vec_len(nmax), targets, n_targets,
                                            *params, flags, n_bases, bases, nullptr, infos,
                                            (double *)(base + kScratchHead), L, nmax, queue,
                                            xkp::Learned{nullptr, 0, 0.0, 0.0}, nullptr));
}

const char *xkp_status_string(xkp_status s) {
    switch (s) {
    case XKP_OK: return "ok";
    case XKP_EINVAL: return "invalid argument";
    case XKP_ENOMEM: return "out of device memory";
    case XKP_EDEVICE: return "HIP runtime error";
    case XKP_ENOCONV: return "no convergence within max_restarts";
    case XKP_ESINGULAR: return "projected system singular; base vector used";
    case XKP_EUNSUPPORTED: return "unsupported size";
    }
    return "unknown status";
}

}  // extern "C"
