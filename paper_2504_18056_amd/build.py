"""Build the HIP library libmcslam.so for gfx950 in-tree with hipcc."""

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmcslam.so")
ARCH = os.environ.get("MCSLAM_OFFLOAD_ARCH", "gfx950")

# Packed FP32 VALU ops are disabled for all device code.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result"]


def _hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build libmcslam.so")
    return exe


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(line for line in r.stdout.splitlines()
                    if "packed-fp32-ops" not in line or "error" in line)
    if r.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (r.returncode, " ".join(cmd), out))
    if verbose and out.strip():
        print(out)


def build(verbose=False, save_temps=False):
    """Compile kernels.hip, mcslam.cpp, server.cpp and rates.hip and link libmcslam.so (always rebuilds)."""
    hipcc = _hipcc()
    obj_dir = os.path.join(HERE, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    k_obj = os.path.join(obj_dir, "kernels.o")
    h_obj = os.path.join(obj_dir, "mcslam.o")
    s_obj = os.path.join(obj_dir, "server.o")
    r_obj = os.path.join(obj_dir, "rates.o")
    extra = ["-save-temps=obj"] if save_temps else []
    _run([hipcc, "-x", "hip", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS + extra +
         ["-c", os.path.join(CSRC, "kernels.hip"), "-o", k_obj], verbose)
    _run([hipcc, "-x", "hip", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS +
         ["-c", os.path.join(CSRC, "mcslam.cpp"), "-o", h_obj], verbose)
    _run([hipcc, "-x", "hip", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS +
         ["-c", os.path.join(CSRC, "server.cpp"), "-o", s_obj], verbose)
    _run([hipcc, "-x", "hip", "--offload-arch=" + ARCH] + COMMON + DEVICE_FLAGS +
         ["-c", os.path.join(CSRC, "rates.hip"), "-o", r_obj], verbose)
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-pthread", "-o", tmp, k_obj, h_obj,
          s_obj, r_obj], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, save_temps="--save-temps" in sys.argv)
