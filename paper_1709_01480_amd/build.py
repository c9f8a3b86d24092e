"""Build the HIP library libfbim.so for gfx950 (in-tree).

    python paper_1709_01480_amd/build.py
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfbim.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

SOURCES = ["kernels_geom.hip", "kernels_real.hip", "kernels_wave.hip", "kernels_la.hip", "kernels_mlp.hip", "kernels_fft.hip", "kernels_rng.hip", "kernels_sk.hip", "fbim_api.hip", "batch_api.hip", "tune.hip", "second_kind.hip",
           "host_math.cpp"]

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-result", "-Wno-unused-value",
          "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(HERE, "..", "include")]
# device code for gfx950 only; packed FP32 instructions disabled
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics"]


def _compile(src):
    path = os.path.join(CSRC, src)
    obj = os.path.join(OBJ, src + ".o")
    if src.endswith(".hip"):
        cmd = [os.path.join(ROCM, "bin", "hipcc"), "-x", "hip"] + HIP_FLAGS + COMMON + ["-c", path, "-o", obj]
    else:
        cmd = ["g++"] + COMMON + ["-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return src, r.returncode, r.stdout + r.stderr, obj


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    objs = []
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        for src, rc, out, obj in ex.map(_compile, SOURCES):
            if rc != 0:
                raise RuntimeError("compiling %s failed:\n%s" % (src, out))
            if verbose and out.strip():
                print(out)
            objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [os.path.join(ROCM, "bin", "hipcc"), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + \
          ["-L" + os.path.join(ROCM, "lib"), "-lrocfft", "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("linking failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
