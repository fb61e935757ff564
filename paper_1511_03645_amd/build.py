"""Build the HIP library libwavepatch.so in-tree for gfx950.

    python -m paper_1511_03645_amd.build

Every HIP source under csrc/ is compiled with hipcc into one shared library
next to this file.  Packed FP32 instructions are disabled for all device code.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwavepatch.so")
ARCH = os.environ.get("WP_OFFLOAD_ARCH", "gfx950")


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")) + glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def _compile(hipcc, src, verbose):
    obj = os.path.join(HERE, "_build", os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [hipcc, f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return obj, cmd, r.returncode, err


def build(verbose=False, jobs=None):
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 1)
    with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(hipcc, s, verbose), sources()))
    objs = []
    for src, (obj, cmd, rc, err) in zip(sources(), results):
        if verbose:
            print(" ".join(cmd), flush=True)
        if rc != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
        if err.strip() and verbose:
            sys.stderr.write(err + "\n")
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
