"""Compile libphi.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libphi.so")
SOURCES = [os.path.join(CSRC, "phi_kernels.hip"), os.path.join(CSRC, "phi_host.cpp"),
           os.path.join(CSRC, "phi_dr.cpp"), os.path.join(CSRC, "phi_static.cpp")]
ARCH = os.environ.get("PHI_OFFLOAD_ARCH", "gfx950")


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, out=None, defines=()):
    """Compile every source into libphi.so (always recompiles)."""
    objs = []
    lib = out or LIB
    for src in SOURCES:
        obj = os.path.join(os.path.dirname(lib), os.path.basename(lib) + "." + os.path.basename(src) + ".o")
        cmd = [hipcc(), "-c", "-fPIC", "-O3", "-std=c++17", "--offload-arch=" + ARCH,
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wall", "-Wno-unused-function",
               "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", obj] + ["-D" + d for d in defines]
        if src.endswith(".cpp"):
            cmd[1:1] = ["-x", "hip"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose=True))
