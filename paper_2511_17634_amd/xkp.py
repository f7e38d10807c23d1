"""ctypes binding of libxkp.so (argument marshalling only).

Every step of the method runs in the HIP library; torch provides device memory (tensor data
pointers) and the stream.  Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# XKP_LIB selects another build of the library (e.g. one compiled with other tuning macros)
LIB_PATH = os.environ.get("XKP_LIB") or os.path.join(HERE, "libxkp.so")

OK, EINVAL, ENOMEM, EDEVICE, ENOCONV, ESINGULAR, EUNSUPPORTED = range(7)
FP64, MIXED = 0, 1
TARGET_GALERKIN, SEED_GALERKIN, SEED_LSQ, NONE = 0, 1, 2, 3
REORTH_AUTO, REORTH_ALWAYS = 0, 1
FIELD_MT, FIELD_X = 0, 1
MODES = {"target_galerkin": TARGET_GALERKIN, "seed_galerkin": SEED_GALERKIN,
         "seed_lsq": SEED_LSQ, "none": NONE}

# Device-side structs, byte-compatible with include/xkp.h.
SYSTEM_DTYPE = np.dtype([("H", "<i4"), ("basis_id", "<i4"), ("dt", "<f8"), ("g", "<f8"),
                         ("mt", "<u8"), ("fx", "<u8"), ("fy", "<u8"), ("b", "<u8"),
                         ("x0", "<u8"), ("x", "<u8")])
INFO_DTYPE = np.dtype([("status", "<i4"), ("iters", "<i4"), ("restarts", "<i4"),
                       ("basis_dim", "<i4"), ("res_est", "<f8"), ("res_true", "<f8"),
                       ("guess_res", "<f8"), ("guess_source", "<i4"), ("pad", "<i4")])
HEADER_BYTES = 256


class Params(ct.Structure):
    _fields_ = [("m", ct.c_int32), ("max_restarts", ct.c_int32), ("tol", ct.c_double),
                ("precision", ct.c_int32), ("mode", ct.c_int32), ("batch_max_n", ct.c_int32),
                ("polish_m", ct.c_int32), ("reorth", ct.c_int32)]


class Tuning(ct.Structure):
    _fields_ = [("polish_m", ct.c_int32), ("wg_per_cu", ct.c_int32), ("ms_best", ct.c_float),
                ("ms_default", ct.c_float), ("n_tried", ct.c_int32), ("waves", ct.c_int32),
                ("seed_rows", ct.c_int32), ("split", ct.c_int32)]


class XkpError(RuntimeError):
    pass


_lib = None


def load():
    """Load libxkp.so; raises if it is missing (build it with paper_2511_17634_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise XkpError(f"{LIB_PATH} not found: build the HIP library first "
                           "(python -m paper_2511_17634_amd.build)")
        try:
            import torch  # noqa: F401  (load torch's HIP runtime first so libxkp binds to it)
        except ImportError:
            pass
        lib = ct.CDLL(LIB_PATH)
        P = ct.c_void_p
        lib.xkp_ctx_create.argtypes = [ct.POINTER(P), ct.c_int, P, ct.c_int32, ct.c_int32,
                                       ct.c_int32]
        lib.xkp_ctx_destroy.argtypes = [P]
        lib.xkp_ctx_set_launch.argtypes = [P, ct.c_int32, ct.c_int32]
        lib.xkp_ctx_set_seed_width.argtypes = [P, ct.c_int32]
        lib.xkp_ctx_set_seed_wait.argtypes = [P, ct.c_int64]
        lib.xkp_ctx_set_projection_split.argtypes = [P, ct.c_int32]
        lib.xkp_ctx_set_timing.argtypes = [P, ct.c_int32]
        lib.xkp_ctx_last_timing.argtypes = [P, ct.POINTER(ct.c_float), ct.POINTER(ct.c_float)]
        lib.xkp_basis_bytes.argtypes = [ct.c_int32, ct.c_int32]
        lib.xkp_basis_bytes.restype = ct.c_size_t
        lib.xkp_seed_build.argtypes = [P, ct.c_int32, P, P, ct.POINTER(Params), P]
        lib.xkp_target_project_solve.argtypes = [P, ct.c_int32, P, ct.c_int32, P,
                                                 ct.POINTER(Params), P]
        lib.xkp_residual.argtypes = [P, ct.c_int32, P, P]
        lib.xkp_apply.argtypes = [P, ct.c_int32, P]
        lib.xkp_build_rhs.argtypes = [P, ct.c_int32, P]
        lib.xkp_autotune.argtypes = [P, ct.c_int32, P, ct.c_int32, P, ct.POINTER(Params), P,
                                     ct.POINTER(Tuning)]
        lib.xkp_autotune_seeds.argtypes = [P, ct.c_int32, P, P, ct.POINTER(Params), P,
                                           ct.POINTER(Tuning)]
        lib.xkp_basis_accumulate.argtypes = [P, ct.c_int32, ct.c_int32, P, P, ct.c_int32,
                                             ct.c_int32, P]
        lib.xkp_score_flow.argtypes = [P, ct.c_int32, P, ct.c_int32, P, P]
        lib.xkp_cluster_seeds.argtypes = [P, ct.c_int32, ct.c_int32, P, ct.c_int32, ct.c_int32,
                                          ct.c_int32, P, P, ct.POINTER(ct.c_int32)]
        lib.xkp_cnn_param_count.argtypes = [ct.c_int32]
        lib.xkp_cnn_param_count.restype = ct.c_size_t
        lib.xkp_cnn_workspace_bytes.argtypes = [ct.c_int32, ct.c_int32]
        lib.xkp_cnn_workspace_bytes.restype = ct.c_size_t
        lib.xkp_cnn_forward.argtypes = [P, ct.c_int32, ct.c_int32, P, P, P, P, P, P]
        lib.xkp_cnn_backward.argtypes = [P, ct.c_int32, ct.c_int32, P, P, P, P, P, ct.c_int32, P,
                                         ct.c_double, P, P, P, P]
        lib.xkp_cnn_adam.argtypes = [P, ct.c_int32, P, P, P, P, ct.c_int32, ct.c_float,
                                     ct.c_float, ct.c_float, ct.c_float]
        lib.xkp_learned_solve.argtypes = [P, ct.c_int32, P, ct.c_int32, P, ct.POINTER(Params),
                                          P, ct.c_int32, ct.c_double, ct.c_double, P]
        lib.xkp_learned_correction_solve.argtypes = lib.xkp_learned_solve.argtypes
        lib.xkp_basis_coeffs.argtypes = [P, ct.c_int32, P, ct.c_int32, P, ct.c_int32, ct.c_int32,
                                         P]
        lib.xkp_target_project_solve_noalloc.argtypes = [ct.c_int, P, ct.c_int32, P, ct.c_int32,
                                                         P, ct.POINTER(Params), P]
        lib.xkp_status_string.argtypes = [ct.c_int]
        lib.xkp_status_string.restype = ct.c_char_p
        for f in ("xkp_ctx_create", "xkp_ctx_destroy", "xkp_seed_build",
                  "xkp_target_project_solve", "xkp_residual", "xkp_apply", "xkp_build_rhs",
                  "xkp_autotune", "xkp_autotune_seeds", "xkp_basis_accumulate",
                  "xkp_score_flow", "xkp_cluster_seeds",
                  "xkp_cnn_forward", "xkp_cnn_backward", "xkp_cnn_adam",
                  "xkp_learned_solve", "xkp_basis_coeffs", "xkp_ctx_set_launch",
                  "xkp_target_project_solve_noalloc", "xkp_ctx_set_seed_width",
                  "xkp_ctx_set_seed_wait", "xkp_ctx_set_projection_split",
                  "xkp_ctx_set_timing", "xkp_ctx_last_timing",
                  "xkp_learned_correction_solve"):
            getattr(lib, f).restype = ct.c_int
        _lib = lib
    return _lib


def status_string(code: int) -> str:
    return load().xkp_status_string(int(code)).decode()


def _check(code: int, what: str):
    if code != OK:
        raise XkpError(f"{what}: {status_string(code)} ({code})")


def target_project_solve_noalloc(systems, n_sys, n_bases, bases_ptrs, params, infos, stream=None,
                                 device=0):
    """xkp_target_project_solve without a context: the library's fixed per-GPU workspace, no
    allocation (calls on one GPU must not overlap)."""
    import torch
    st = stream if stream is not None else torch.cuda.current_stream(device)
    _check(load().xkp_target_project_solve_noalloc(device, ct.c_void_p(st.cuda_stream), n_sys,
                                                   _ptr(systems), n_bases, _ptr(bases_ptrs),
                                                   ct.byref(params), _ptr(infos)),
           "xkp_target_project_solve_noalloc")


def basis_bytes(n: int, m: int) -> int:
    return int(load().xkp_basis_bytes(n, m))


def _ptr(t):
    return 0 if t is None else int(t.data_ptr())


@dataclass
class SystemSpec:
    """Host description of one system; tensors are CUDA float64 of n = H*H elements."""
    H: int
    dt: float
    g: float
    mt: object
    b: object
    x: object
    x0: object = None
    fx: object = None
    fy: object = None
    basis_id: int = 0


def pack_systems(specs, device):
    """Device array of xkp_system descriptors (uint8 tensor)."""
    import torch
    a = np.zeros(len(specs), dtype=SYSTEM_DTYPE)
    keep = []
    for i, s in enumerate(specs):
        a[i] = (s.H, s.basis_id, s.dt, s.g, _ptr(s.mt), _ptr(s.fx), _ptr(s.fy), _ptr(s.b),
                _ptr(s.x0), _ptr(s.x))
        keep += [t for t in (s.mt, s.fx, s.fy, s.b, s.x0, s.x) if t is not None]
    d = torch.from_numpy(a.view(np.uint8).copy()).to(device)
    d._xkp_keep = keep          # the descriptors hold device addresses: keep their owners alive
    return d


def pack_batch(H, dt, g, mt, b, x, x0=None, basis_id=None, device=None):
    """Descriptors for a batch stored as (N, n) CUDA float64 tensors (rows are systems)."""
    import torch
    N = mt.shape[0]
    n = H * H
    a = np.zeros(N, dtype=SYSTEM_DTYPE)
    a["H"] = H
    a["dt"] = dt
    a["g"] = g
    st = 8 * n
    for f, t in (("mt", mt), ("b", b), ("x", x), ("x0", x0)):
        if t is not None:
            assert t.is_contiguous() and t.dtype == torch.float64 and t.shape[-1] == n
            a[f] = t.data_ptr() + st * np.arange(N, dtype=np.uint64)
    if basis_id is not None:
        a["basis_id"] = basis_id
    d = torch.from_numpy(a.view(np.uint8).copy()).to(device or mt.device)
    d._xkp_keep = [t for t in (mt, b, x, x0) if t is not None]
    return d


def infos_to_numpy(t) -> np.ndarray:
    return t.cpu().numpy().view(INFO_DTYPE)


class Context:
    """A libxkp context bound to one device and stream, with its fixed workspace."""

    def __init__(self, max_n: int, max_m: int, max_batch: int, device: int = 0, stream=None):
        import torch
        lib = load()
        self.device = device
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = ct.c_void_p()
        _check(lib.xkp_ctx_create(ct.byref(h), device, ct.c_void_p(self.stream.cuda_stream),
                                  max_n, max_m, max_batch), "xkp_ctx_create")
        self._h = h
        self.max_n, self.max_m, self.max_batch = max_n, max_m, max_batch
        self.seed_width = 0        # 1 once seed calls are spread over several workgroups
        self.split = -1            # >= 0 once targets are projected in launches of their own

    def set_launch(self, waves, wg_per_cu=1):
        """Workgroup size (8 or 16 wave64s) and workgroups per compute unit of later solves."""
        _check(load().xkp_ctx_set_launch(self._h, waves, wg_per_cu), "xkp_ctx_set_launch")

    def set_seed_width(self, rows_per_thread):
        """Later seed calls spread each seed over workgroups of 256 rows (1), or one workgroup
        per seed (0)."""
        _check(load().xkp_ctx_set_seed_width(self._h, rows_per_thread),
               "xkp_ctx_set_seed_width")
        self.seed_width = int(rows_per_thread)

    def set_seed_wait(self, microseconds):
        """Give-up time of a spread-out seed's waits (default two seconds)."""
        _check(load().xkp_ctx_set_seed_wait(self._h, int(microseconds)), "xkp_ctx_set_seed_wait")

    def set_projection_split(self, max_tiles=0):
        """Later target calls project in launches of their own over at most max_tiles row tiles
        per target (0: as many as fit); -1 projects inside the solve launch again."""
        _check(load().xkp_ctx_set_projection_split(self._h, int(max_tiles)),
               "xkp_ctx_set_projection_split")
        self.split = int(max_tiles)

    def set_timing(self, on=True):
        """Record phase events around later target calls (see last_timing)."""
        _check(load().xkp_ctx_set_timing(self._h, int(bool(on))), "xkp_ctx_set_timing")

    def last_timing(self):
        """(projection ms, solve ms) of the last target call recorded with timing on."""
        a, b = ct.c_float(), ct.c_float()
        _check(load().xkp_ctx_last_timing(self._h, ct.byref(a), ct.byref(b)),
               "xkp_ctx_last_timing")
        return float(a.value), float(b.value)

    def close(self):
        if getattr(self, "_h", None):
            _check(load().xkp_ctx_destroy(self._h), "xkp_ctx_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def params(m, tol=1e-8, max_restarts=1000, precision=FP64, mode=TARGET_GALERKIN,
               batch_max_n=0, polish_m=0, reorth=REORTH_AUTO):
        if isinstance(mode, str):
            mode = MODES[mode]
        if isinstance(reorth, str):
            reorth = {"auto": REORTH_AUTO, "always": REORTH_ALWAYS}[reorth]
        return Params(m, max_restarts, tol, precision, mode, batch_max_n, polish_m, reorth)

    def new_infos(self, count):
        import torch
        return torch.zeros(count * INFO_DTYPE.itemsize, dtype=torch.uint8,
                           device=f"cuda:{self.device}")

    def seed_build(self, systems, n_sys, bases_ptrs, params, infos):
        """systems: packed descriptors; bases_ptrs: int64 CUDA tensor of basis buffer addresses."""
        _check(load().xkp_seed_build(self._h, n_sys, _ptr(systems), _ptr(bases_ptrs),
                                     ct.byref(params), _ptr(infos)), "xkp_seed_build")

    def target_project_solve(self, systems, n_sys, n_bases, bases_ptrs, params, infos):
        _check(load().xkp_target_project_solve(self._h, n_sys, _ptr(systems), n_bases,
                                               _ptr(bases_ptrs), ct.byref(params), _ptr(infos)),
               "xkp_target_project_solve")

    def autotune(self, systems, n_sys, n_bases, bases_ptrs, params, infos) -> Tuning:
        """Times candidate polish restart lengths and workgroups per compute unit on this batch
        (host-synchronous); the workgroup count is kept by the context, the returned
        polish_m goes into later params."""
        t = Tuning()
        _check(load().xkp_autotune(self._h, n_sys, _ptr(systems), n_bases, _ptr(bases_ptrs),
                                   ct.byref(params), _ptr(infos), ct.byref(t)), "xkp_autotune")
        self.split = int(t.split)
        return t

    def basis_accumulate(self, n, n_src, src_ptrs, out_ptrs, per_source, cap, out_k=None):
        """out_j = orthonormal basis gathered from source bases 0..j (int64 CUDA tensors of basis
        buffer addresses); out_k: optional int32 CUDA tensor of n_src column counts."""
        _check(load().xkp_basis_accumulate(self._h, n, n_src, _ptr(src_ptrs), _ptr(out_ptrs),
                                           per_source, cap, _ptr(out_k)),
               "xkp_basis_accumulate")

    def score_flow(self, systems, n_sys, field, score_ptrs=None, disp_ptrs=None):
        """Score (2n per system) and one probability-flow step of the displacement (2n, in
        place); pointer arrays are int64 CUDA tensors or None."""
        _check(load().xkp_score_flow(self._h, n_sys, _ptr(systems), field, _ptr(score_ptrs),
                                     _ptr(disp_ptrs)), "xkp_score_flow")

    def cluster_seeds(self, images, H, pool, K, max_iters=50):
        """k-means seed selection on (N, H*H) CUDA float64 images: returns (assign (N,) int32,
        seeds (K,) int32 CUDA tensors, assignment count); host-synchronous."""
        import torch
        N = images.shape[0]
        assign = torch.empty(N, dtype=torch.int32, device=images.device)
        seeds = torch.empty(K, dtype=torch.int32, device=images.device)
        it = ct.c_int32(0)
        _check(load().xkp_cluster_seeds(self._h, N, H, _ptr(images), pool, K, max_iters,
                                        _ptr(assign), _ptr(seeds), ct.byref(it)),
               "xkp_cluster_seeds")
        return assign, seeds, it.value

    def autotune_seeds(self, systems, n_sys, bases_ptrs, params, infos) -> Tuning:
        """Times the seed call over the kernel variants and workgroup counts (host-synchronous);
        the choice is kept by the context (one that serves seed calls)."""
        t = Tuning()
        _check(load().xkp_autotune_seeds(self._h, n_sys, _ptr(systems), _ptr(bases_ptrs),
                                         ct.byref(params), _ptr(infos), ct.byref(t)),
               "xkp_autotune_seeds")
        self.seed_width = int(t.seed_rows)
        return t

    def learned_solve(self, systems, n_sys, n_bases, bases_ptrs, params, alpha, alpha_ld,
                      alpha_scale, gate, infos):
        """Polish from the guess rebuilt from the predicted residual coordinates alpha (times
        alpha_scale) when its residual is <= gate, else the projection path of params.mode."""
        _check(load().xkp_learned_solve(self._h, n_sys, _ptr(systems), n_bases, _ptr(bases_ptrs),
                                        ct.byref(params), _ptr(alpha), alpha_ld, alpha_scale,
                                        gate, _ptr(infos)), "xkp_learned_solve")

    def learned_correction_solve(self, systems, n_sys, n_bases, bases_ptrs, params, alpha,
                                 alpha_ld, alpha_scale, gate, infos):
        """Projection, then the predicted correction of its residual coordinates (times
        alpha_scale), kept when its residual is <= gate and below the projected guess's."""
        _check(load().xkp_learned_correction_solve(
            self._h, n_sys, _ptr(systems), n_bases, _ptr(bases_ptrs), ct.byref(params),
            _ptr(alpha), alpha_ld, alpha_scale, gate, _ptr(infos)), "xkp_learned_correction_solve")

    def basis_coeffs(self, systems, n_sys, n_bases, bases_ptrs, m_out, alpha, kind=0):
        """kind 0: alpha[i][c] = v_c . x_i on each system's seed basis; kind 1: the residual
        coordinates Hbar (V^T x_i) / beta (float64 device, (n_sys, m_out))."""
        _check(load().xkp_basis_coeffs(self._h, n_sys, _ptr(systems), n_bases, _ptr(bases_ptrs),
                                       m_out, kind, _ptr(alpha)), "xkp_basis_coeffs")

    def residual(self, systems, n_sys, rel_out):
        _check(load().xkp_residual(self._h, n_sys, _ptr(systems), _ptr(rel_out)), "xkp_residual")

    def build_rhs(self, systems, n_sys):
        _check(load().xkp_build_rhs(self._h, n_sys, _ptr(systems)), "xkp_build_rhs")

    def apply(self, systems, n_sys):
        _check(load().xkp_apply(self._h, n_sys, _ptr(systems)), "xkp_apply")


class Bases:
    """Device storage for `count` seed bases of restart length m; n is the number of unknowns of
    every basis, or a sequence giving each basis its own (batches of uneven sizes)."""

    def __init__(self, count, n, m, device=0):
        import torch
        ns = [int(n)] * count if np.isscalar(n) else [int(v) for v in n]
        assert len(ns) == count
        self.count, self.m, self.ns = count, m, ns
        self.n = ns[0] if len(set(ns)) == 1 else None
        self.offsets = []
        off = 0
        for v in ns:
            self.offsets.append(off)
            off += (basis_bytes(v, m) + 255) & ~255
        self.buf = torch.zeros(max(off, 256), dtype=torch.uint8, device=f"cuda:{device}")
        base = self.buf.data_ptr()
        assert base % 256 == 0
        self.ptrs = torch.tensor([base + o for o in self.offsets], dtype=torch.int64,
                                 device=f"cuda:{device}")

    def ldv(self, i=0):
        """Leading dimension of basis i's V: roundup(n + 1, 8) doubles (zeros past row n)."""
        return (self.ns[i] + 8) & ~7

    def header(self, i):
        o = self.offsets[i]
        h = self.buf[o:o + 36].cpu().numpy().view(np.int32)
        return {"n": int(h[0]), "m": int(h[1]), "k": int(h[2]), "status": int(h[3]),
                "ldv": int(h[6]), "bf16": int(h[7]), "kind": int(h[8])}

    def V_padded(self, i):
        """(ldv, m+1) view of basis i's FP64 columns including the zero rows."""
        import torch
        off = self.offsets[i] + HEADER_BYTES
        ldv = self.ldv(i)
        raw = self.buf[off:off + 8 * ldv * (self.m + 1)]
        return raw.view(torch.float64).view(self.m + 1, ldv).T

    def V(self, i):
        """(n, m+1) view of basis i's FP64 columns."""
        return self.V_padded(i)[:self.ns[i]]

    def Vb_bits(self, i):
        """(ldv, m+1) view of basis i's BF16 copy as raw 16-bit patterns (int16)."""
        import torch
        ldv, m = self.ldv(i), self.m
        o = 256 + 8 * ldv * (m + 1) + 8 * (m + 1) * m
        off = self.offsets[i] + ((o + 255) & ~255)
        raw = self.buf[off:off + 2 * ldv * (m + 1)]
        return raw.view(torch.int16).view(m + 1, ldv).T

    def Hbar(self, i):
        import torch
        off = self.offsets[i] + HEADER_BYTES + 8 * self.ldv(i) * (self.m + 1)
        raw = self.buf[off:off + 8 * (self.m + 1) * self.m]
        return raw.view(torch.float64).view(self.m, self.m + 1).T


class Net:
    """The learned-guess network's FP32 parameters, Adam moments and workspace on the device,
    driven through the library's kernels (forward, backward, Adam)."""

    def __init__(self, ctx, k, batch, params=None):
        import torch
        lib = load()
        self.ctx, self.k, self.batch = ctx, k, batch
        self.count = int(lib.xkp_cnn_param_count(k))
        dev = f"cuda:{ctx.device}"
        if params is None:
            self.params = torch.zeros(self.count, dtype=torch.float32, device=dev)
        else:
            self.params = torch.as_tensor(params, dtype=torch.float32).to(dev).contiguous()
            assert self.params.numel() == self.count
        self.grad = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.t = 0
        self.work = torch.empty(int(lib.xkp_cnn_workspace_bytes(batch, k)), dtype=torch.uint8,
                                device=dev)
        self.loss = torch.zeros(1, dtype=torch.float32, device=dev)

    def forward(self, images, steps, alpha, image_idx=None, B=None):
        """images: (M, 4096) float64 (sample b uses row image_idx[b], or row b), steps: (B,)
        int32, alpha: (B, k) float32 output."""
        B = B or steps.shape[0]
        assert B <= self.batch
        _check(load().xkp_cnn_forward(self.ctx._h, B, self.k, _ptr(self.params), _ptr(images),
                                      _ptr(image_idx), _ptr(steps), _ptr(alpha),
                                      _ptr(self.work)), "xkp_cnn_forward")

    def backward(self, images, steps, target, alpha, image_idx=None, target_idx=None,
                 target_scale=1.0, B=None):
        """Gradient of the mean squared error against target_scale * target rows (float64,
        (R, ld)) into self.grad, the loss into self.loss."""
        B = B or steps.shape[0]
        assert B <= self.batch
        _check(load().xkp_cnn_backward(self.ctx._h, B, self.k, _ptr(self.params), _ptr(images),
                                       _ptr(image_idx), _ptr(steps), _ptr(target),
                                       target.shape[-1], _ptr(target_idx), target_scale,
                                       _ptr(alpha), _ptr(self.grad), _ptr(self.loss),
                                       _ptr(self.work)), "xkp_cnn_backward")

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        self.t += 1
        _check(load().xkp_cnn_adam(self.ctx._h, self.count, _ptr(self.params), _ptr(self.grad),
                                   _ptr(self.m), _ptr(self.v), self.t, lr, beta1, beta2, eps),
               "xkp_cnn_adam")
