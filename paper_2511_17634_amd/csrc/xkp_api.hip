// C ABI of libxkp: context, workspace and argument checks around the kernels.
#include <hip/hip_runtime.h>

#include <new>

#include "xkp.h"
#include "xkp_internal.h"

struct xkp_ctx {
    int device;
    hipStream_t stream;
    int max_n, max_m, max_batch;
    int slots;          // workgroups that own a workspace slot
    xkp::WsLayout L;
    double *ws;
};

namespace {

xkp_status from_hip(hipError_t e) { return e == hipSuccess ? XKP_OK : XKP_EDEVICE; }

// One compiled kernel variant (workgroup size) and its launchers.
struct Variant {
    int (*threads)();
    int (*rmax_for)(int);
    int (*lds_vec_len)(int);
    decltype(&xkp::v512::launch_gmres) gmres;
    decltype(&xkp::v512::launch_project) project;
    decltype(&xkp::v512::launch_residual) residual;
    decltype(&xkp::v512::launch_rhs) rhs;
    decltype(&xkp::v512::launch_apply) apply;
};
#define XKP_VARIANT_TABLE(NS)                                                          \
    Variant {                                                                          \
        xkp::NS::threads, xkp::NS::rmax_for, xkp::NS::lds_vec_len, xkp::NS::launch_gmres, \
            xkp::NS::launch_project, xkp::NS::launch_residual, xkp::NS::launch_rhs,    \
            xkp::NS::launch_apply                                                      \
    }
const Variant kV512 = XKP_VARIANT_TABLE(v512);

// Kernel variant for systems of up to nmax unknowns (512 threads: 2 rows per thread up to 1024
// unknowns, 8 up to 4096, 32 up to 16384).
const Variant *choose(int nmax) { return kV512.rmax_for(nmax) ? &kV512 : nullptr; }

int npad_for(int nmax) { return kV512.rmax_for(nmax) * kV512.threads(); }

// Shared host checks of a batched call; fills the effective n limit and kernel variant.
xkp_status check_call(const xkp_ctx *ctx, int32_t count, const void *arr, const xkp_params *P,
                      int *nmax, int *rmax, const Variant **var) {
    if (!ctx || count < 0 || (count > 0 && !arr) || !P) return XKP_EINVAL;
    if (P->m < 1 || P->m > ctx->max_m || !(P->tol >= 0.0) || P->max_restarts < 0 ||
        P->reserved != 0 || P->batch_max_n < 0 || P->batch_max_n > ctx->max_n)
        return XKP_EINVAL;
    if (P->precision != XKP_FP64 && P->precision != XKP_MIXED) return XKP_EINVAL;
    if (P->mode < XKP_PROJ_TARGET_GALERKIN || P->mode > XKP_PROJ_NONE) return XKP_EINVAL;
    *nmax = P->batch_max_n > 0 ? P->batch_max_n : ctx->max_n;
    *var = choose(*nmax);
    if (!*var) return XKP_EUNSUPPORTED;
    *rmax = (*var)->rmax_for(*nmax);
    return XKP_OK;
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
    c->slots = max_batch < 4 * cus ? max_batch : 4 * cus;
    c->L = xkp::ws_layout(max_n, max_m, npad_for(max_n));
    if (hipMalloc((void **)&c->ws, sizeof(double) * c->L.stride * (size_t)c->slots) != hipSuccess) {
        delete c;
        return XKP_ENOMEM;
    }
    *out = c;
    return XKP_OK;
}

xkp_status xkp_ctx_destroy(xkp_ctx *ctx) {
    if (!ctx) return XKP_EINVAL;
    hipError_t e = hipStreamSynchronize(ctx->stream);
    hipError_t f = hipFree(ctx->ws);
    delete ctx;
    return (e == hipSuccess && f == hipSuccess) ? XKP_OK : XKP_EDEVICE;
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
    const int grid = n_seeds < ctx->slots ? n_seeds : ctx->slots;
    return from_hip(v->gmres(ctx->stream, grid, rmax, v->lds_vec_len(nmax), seeds, n_seeds,
                             *params, xkp::kKeepBasis, bases, infos, ctx->ws, ctx->L, nmax));
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
    const int grid = n_targets < ctx->slots ? n_targets : ctx->slots;
    int flags = 0;
    if (params->mode != XKP_PROJ_NONE) {
        hipError_t e = v->project(ctx->stream, grid, rmax, v->lds_vec_len(nmax), targets,
                                  n_targets, n_bases, bases, *params, infos, ctx->ws, ctx->L,
                                  nmax);
        if (e != hipSuccess) return XKP_EDEVICE;
        flags = xkp::kStartFromX | xkp::kTarget;
    }
    return from_hip(v->gmres(ctx->stream, grid, rmax, v->lds_vec_len(nmax), targets, n_targets,
                             *params, flags, nullptr, infos, ctx->ws, ctx->L, nmax));
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
