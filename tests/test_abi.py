"""CPU checks of the C ABI: the library loads, exports every function include/xkp.h declares,
its structs have the layout the binding packs, and host-side argument errors come back without
touching a GPU."""
import ctypes as ct
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xkp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(xkp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2511_17634_amd import xkp
    if not os.path.exists(xkp.LIB_PATH):
        from paper_2511_17634_amd import build
        build.build()
    return xkp.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"xkp_seed_build", "xkp_target_project_solve", "xkp_residual"} <= set(names)
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layouts_match_binding(tmp_path):
    from paper_2511_17634_amd import xkp
    probe = tmp_path / "probe.c"
    probe.write_text(r'''
#include <stdio.h>
#include <stddef.h>
#include "xkp.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(xkp_system), offsetof(xkp_system, dt),
         offsetof(xkp_system, mt), offsetof(xkp_system, x), sizeof(xkp_info), sizeof(xkp_params));
  printf("%zu %zu %zu\n", sizeof(xkp_basis_header), offsetof(xkp_info, res_est),
         offsetof(xkp_params, tol));
  printf("%zu %zu %zu %zu %zu\n", offsetof(xkp_params, polish_m), sizeof(xkp_tuning),
         offsetof(xkp_tuning, ms_default), offsetof(xkp_params, reorth),
         offsetof(xkp_basis_header, kind));
  return 0;
}''')
    exe = tmp_path / "probe"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(probe),
                           "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    v = list(map(int, out))
    S, I = xkp.SYSTEM_DTYPE, xkp.INFO_DTYPE
    assert v[0] == S.itemsize and v[1] == S.fields["dt"][1] and v[2] == S.fields["mt"][1]
    assert v[3] == S.fields["x"][1] and v[4] == I.itemsize and v[5] == ct.sizeof(xkp.Params)
    assert v[6] == xkp.HEADER_BYTES and v[7] == I.fields["res_est"][1]
    assert v[8] == xkp.Params.tol.offset
    assert v[9] == xkp.Params.polish_m.offset and v[10] == ct.sizeof(xkp.Tuning)
    assert v[11] == xkp.Tuning.ms_default.offset and v[12] == xkp.Params.reorth.offset
    assert v[13] == 32    # Bases.header reads kind as the ninth int32


def test_host_side_errors_without_gpu(lib):
    from paper_2511_17634_amd import xkp
    h = ct.c_void_p()
    assert lib.xkp_ctx_create(ct.byref(h), 0, None, 0, 10, 1) == xkp.EINVAL
    assert lib.xkp_ctx_create(ct.byref(h), 0, None, 4096, 65, 1) == xkp.EUNSUPPORTED
    assert lib.xkp_ctx_create(ct.byref(h), 0, None, 1 << 20, 10, 1) == xkp.EUNSUPPORTED
    P = xkp.Context.params(10)
    assert lib.xkp_seed_build(None, 1, None, None, ct.byref(P), None) == xkp.EINVAL
    assert lib.xkp_target_project_solve(None, 1, None, 0, None, ct.byref(P), None) == xkp.EINVAL
    assert lib.xkp_residual(None, 1, None, None) == xkp.EINVAL
    t = xkp.Tuning()
    assert lib.xkp_autotune(None, 1, None, 0, None, ct.byref(P), None, ct.byref(t)) == xkp.EINVAL
    assert lib.xkp_ctx_set_launch(None, 8, 1) == xkp.EINVAL
    assert lib.xkp_ctx_set_projection_split(None, 0) == xkp.EINVAL
    assert lib.xkp_ctx_set_seed_wait(None, 1000) == xkp.EINVAL
    assert lib.xkp_learned_solve(None, 1, None, 1, None, ct.byref(P), None, 41, 1.0, 1e-6,
                                 None) == xkp.EINVAL
    assert lib.xkp_basis_coeffs(None, 1, None, 1, None, 40, 0, None) == xkp.EINVAL
    assert lib.xkp_autotune_seeds(None, 1, None, None, ct.byref(P), None, ct.byref(t)) == xkp.EINVAL
    assert lib.xkp_basis_accumulate(None, 4096, 2, None, None, 20, 40, None) == xkp.EINVAL
    assert lib.xkp_score_flow(None, 1, None, 0, None, None) == xkp.EINVAL
    assert lib.xkp_cluster_seeds(None, 8, 16, None, 4, 2, 10, None, None, None) == xkp.EINVAL
    # the allocation-free target solve: argument errors before any device call
    noalloc = lib.xkp_target_project_solve_noalloc
    assert noalloc(0, None, 1, None, 0, None, ct.byref(P), None) == xkp.EINVAL
    assert noalloc(0, None, -1, None, 0, None, ct.byref(P), None) == xkp.EINVAL
    assert noalloc(0, None, 0, None, 0, None, None, None) == xkp.EINVAL
    for bad in (xkp.Context.params(65), xkp.Context.params(40, polish_m=65),
                xkp.Context.params(40, batch_max_n=16385), xkp.Context.params(40, tol=-1.0)):
        assert noalloc(0, None, 0, None, 0, None, ct.byref(bad), None) == xkp.EINVAL
    assert noalloc(0, None, 0, None, 0, None, ct.byref(P), None) == xkp.OK
    # the network's sizes and argument checks
    assert lib.xkp_cnn_param_count(40) == 16 * 9 + 16 + 32 * 144 + 32 + 64 * 288 + 64 + 40 * 97
    assert lib.xkp_cnn_param_count(0) == 0 and lib.xkp_cnn_param_count(65) == 0
    assert lib.xkp_cnn_workspace_bytes(0, 40) == 0
    assert lib.xkp_cnn_workspace_bytes(512, 41) > lib.xkp_cnn_workspace_bytes(256, 41) > 0
    assert lib.xkp_cnn_forward(None, 1, 40, None, None, None, None, None, None) == xkp.EINVAL
    assert lib.xkp_cnn_backward(None, 1, 40, None, None, None, None, None, 40, None, 1.0, None,
                                None, None, None) == xkp.EINVAL
    assert lib.xkp_cnn_adam(None, 1, None, None, None, None, 1, 1e-3, 0.9, 0.999,
                            1e-8) == xkp.EINVAL
    assert xkp.basis_bytes(0, 10) == 0
    n, m = 4096, 40
    assert xkp.basis_bytes(n, m) >= 256 + 8 * n * (m + 1) + 8 * (m + 1) * m + 2 * n * (m + 1)
    assert xkp.basis_bytes(n, m) % 256 == 0
    assert xkp.status_string(xkp.ESINGULAR).startswith("projected")


def test_single_hip_runtime_in_process(lib):
    """libxkp binds to the HIP runtime torch already loaded: one libamdhip64 mapping."""
    import torch  # noqa: F401
    maps = open("/proc/self/maps").read().splitlines()
    paths = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    assert len(paths) == 1, paths
