"""Build libxkp.so (HIP, gfx950) in-tree with hipcc.

Objects are compiled by hipcc and linked by a plain host link against a link-time stub named
libamdhip64.so that carries no SONAME.  The library therefore records a dependency on
"libamdhip64.so" (not "libamdhip64.so.7"): inside a process that already loaded a HIP runtime
under that name (PyTorch's bundled one) the dynamic linker reuses it, so the library and torch
share one runtime, one device context and one set of streams; standalone, the RUNPATH finds the
ROCm installation's runtime.
"""
from __future__ import annotations

import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libxkp.so")
# (source, object, extra flags): the kernel file is compiled once per workgroup size
UNITS = [("xkp_kernels.hip", "xkp_kernels_512.o", ["-DXKP_NT=512", "-DXKP_VARIANT=v512"]),
         ("xkp_kernels.hip", "xkp_kernels_1024.o", ["-DXKP_NT=1024", "-DXKP_VARIANT=v1024"]),
         ("xkp_kernels.hip", "xkp_kernels_256.o", ["-DXKP_NT=256", "-DXKP_VARIANT=v256",
                                                   "-DXKP_DEPTH16=2"]),
         ("xkp_common.hip", "xkp_common.o", []),
         ("xkp_wide.hip", "xkp_wide.o", []),
         ("xkp_project.hip", "xkp_project.o", []),
         ("xkp_cnn.hip", "xkp_cnn.o", []),
         ("xkp_epilogue.hip", "xkp_epilogue.o", []),
         ("xkp_cluster.hip", "xkp_cluster.o", []),
         ("xkp_api.hip", "xkp_api.o", [])]
ARCH = os.environ.get("XKP_OFFLOAD_ARCH", "gfx950")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # no packed FP32 instructions anywhere in the device code
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]))
    return r.stdout


def build(verbose: bool = False, out_lib: str = LIB, build_dir: str = OUT,
          extra_flags=(), csrc: str = CSRC) -> str:
    """Compile every unit (sources from `csrc`) and link `out_lib`.  extra_flags (e.g. -D tuning
    macros) are added to every hipcc line."""
    os.makedirs(build_dir, exist_ok=True)
    hipcc = os.environ.get("HIPCC", os.path.join(ROCM, "bin", "hipcc"))
    objs = []
    procs = []
    for src, objname, extra in UNITS:
        obj = os.path.join(build_dir, objname)
        cmd = [hipcc, *FLAGS, *extra, *extra_flags, "-I", os.path.join(ROOT, "include"), "-I",
               csrc, "-c", os.path.join(csrc, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
        objs.append(obj)
    for cmd, pr in procs:
        out, err = pr.communicate()
        if pr.returncode != 0:
            sys.stderr.write(out + err)
            raise RuntimeError("build step failed: " + " ".join(cmd[:3]))
    # link-time stub: every HIP runtime symbol the objects use, no SONAME
    undef = set()
    for o in objs:
        for line in _run(["nm", "-u", o], False).splitlines():
            name = line.split()[-1]
            if re.match(r"^(__)?hip", name):
                undef.add(name)
    stubdir = os.path.join(build_dir, "linkstub")
    os.makedirs(stubdir, exist_ok=True)
    stub_c = os.path.join(stubdir, "stub.c")
    with open(stub_c, "w") as f:
        f.write("/* link-time stand-in for the HIP runtime's exported names; never loaded */\n")
        for name in sorted(undef):
            f.write(f"void {name}(void) {{}}\n")
    _run(["gcc", "-shared", "-fPIC", "-o", os.path.join(stubdir, "libamdhip64.so"), stub_c],
         verbose)
    tmp = out_lib + ".tmp%d" % os.getpid()
    rocm_lib = os.path.realpath(os.path.join(ROCM, "lib"))
    _run(["g++", "-shared", "-o", tmp, *objs, "-L" + stubdir, "-lamdhip64",
          "-Wl,-rpath," + rocm_lib, "-Wl,--no-undefined"], verbose)
    needed = _run(["readelf", "-d", tmp], False)
    if "[libamdhip64.so]" not in needed:
        raise RuntimeError("libxkp.so does not depend on the unversioned HIP runtime name")
    os.replace(tmp, out_lib)
    return out_lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
