"""Build libgrmhd.so (HIP for gfx950 + host C++) in the package directory.

    python -m paper_2508_18221_amd.build        # or build.build()

Every HIP translation unit is compiled with hipcc for --offload-arch=gfx950;
packed FP32 instructions are disabled for all device code.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgrmhd.so")
SOURCES = ["contract.hip", "contract_mixed.hip", "pointwise.hip", "xcts.hip", "operators.cpp", "init_data.cpp",
           "abi.cpp", "server.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         # MFMA accumulators in ordinary VGPRs: no per-loop-trip copies
         # through the accumulation registers
         "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I", INCLUDE, "-I", CSRC]


# host-only sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer on the
# host pass; the device code is built as usual): a separate library for the
# CPU tests of the C-ABI and the job server, loaded with the sanitizer runtime
# preloaded
HOSTSAN_LIB = os.path.join(HERE, "libgrmhd_hostsan.so")
HOSTSAN_FLAGS = ("-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined "
                 "-Xarch_host -fno-omit-frame-pointer -Xarch_host -fno-sanitize-recover=undefined").split()


def build(verbose=False, jobs=5, hostsan=False):
    objdir = os.path.join(HERE, "_build_hostsan" if hostsan else "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src + ".o")
        # every translation unit goes through hipcc as HIP: the host sources
        # include the HIP runtime header and launch the kernels
        cmd = [HIPCC] + FLAGS + (HOSTSAN_FLAGS if hostsan else []) + ["-x", "hip", "-c",
                                                                     os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the packed-fp32 feature: harmless
        lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l and l.strip()]
        if lines and (verbose or p.returncode):
            print("\n".join(lines), file=sys.stderr)
        if p.returncode:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed for: " + ", ".join(failed))
    lib = HOSTSAN_LIB if hostsan else LIB
    tmp = lib + ".tmp"
    # roctx: the ranges around each RK stage and the filter (rocprofv3 --marker-trace)
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lrocprofiler-sdk-roctx"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, hostsan="--hostsan" in sys.argv))
