"""Compiles tests/capi/vlp_capi_demo.c (plain C, gcc) against include/vlp.h,
the built libvlp.so and the HIP runtime's C API."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_2506_12761_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SRC = os.path.join(HERE, "vlp_capi_demo.c")
EXE = os.path.join(HERE, "vlp_capi_demo")


def missing():
    """Why the program cannot be built here, or None."""
    if shutil.which("gcc") is None:
        return "gcc not found"
    if not os.path.exists(os.path.join(PKG, "libvlp.so")):
        return "libvlp.so not built"
    if not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        return "HIP headers not found"
    return None


def build(out=EXE):
    why = missing()
    if why:
        raise RuntimeError("cannot build the C ABI example: " + why)
    cmd = ["gcc", "-std=c11", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-L", PKG, "-lvlp", "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           "-Wl,-rpath," + PKG, "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        raise RuntimeError("gcc failed:\n" + r.stderr[-4000:])
    return out


if __name__ == "__main__":
    print(build())
