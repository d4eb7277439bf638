"""Build libbp.so (HIP kernels for gfx950 + the C ABI) in the package directory."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbp.so")
LIB_SRBP = os.path.join(HERE, "libsrbp.so")
SRBP_SOURCE = os.path.join(CSRC, "srbp.cpp")
SOURCES = [os.path.join(CSRC, "bp_kernels.hip"), os.path.join(CSRC, "bp_api.cpp")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compile (the sources in parallel) and link libbp.so.  ``defines`` (e.g. a
    tile size) and ``out`` produce an alternative build; the default is the
    shipped one."""
    from concurrent.futures import ThreadPoolExecutor
    tag = "" if out == LIB else "." + os.path.basename(out)
    jobs = []
    if out == LIB:
        # serial residual BP: host code only
        jobs.append((["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-Wall",
                      "-I" + os.path.join(ROOT, "include"), "-o", LIB_SRBP + ".tmp", SRBP_SOURCE],
                     None))
    for src in SOURCES:
        obj = os.path.join(CSRC, os.path.basename(src) + tag + ".o")
        cmd = [HIPCC] + COMMON + DEVICE_FLAGS + ["-D" + d for d in defines] + ["-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        jobs.append((cmd, obj))
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for f in [ex.submit(subprocess.run, cmd, check=True) for cmd, _ in jobs]:
            f.result()
    if out == LIB:
        os.replace(LIB_SRBP + ".tmp", LIB_SRBP)
    objs = [obj for _, obj in jobs if obj is not None]
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
