"""Build libporedvm.so (HIP kernels + host C ABI of the solver and of the
warm-start network) for gfx950, in-tree."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libporedvm.so")
SOURCES = ["dvm_sweep_strips_f64.hip", "dvm_sweep_strips_f32.hip", "dvm_sweep_rows.hip", "dvm_sweep_diag.hip", "dvm_iter.hip", "dvm_host.cpp", "unet_kernels.hip", "unet_host.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # no packed FP32 instructions: FP32 arithmetic stays scalar
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _compile(src, verbose):
    obj = os.path.join(CSRC, src + ".o")
    cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC, "-x", "hip"] + cmd[1:]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    return obj


def _fresh(src):
    """The object of `src` is newer than the source and every header here."""
    obj = os.path.join(CSRC, src + ".o")
    if not os.path.exists(obj):
        return False
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    deps.append(os.path.join(HERE, "..", "include", "poredvm.h"))
    deps.append(os.path.join(HERE, "..", "include", "poredvm_unet.h"))
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in deps if os.path.exists(d))


def build(verbose=False, incremental=False):
    """Compile every source (incremental: only those whose object is stale)."""
    # the translation units are independent: compile them concurrently
    from concurrent.futures import ThreadPoolExecutor
    todo = [src for src in SOURCES if not (incremental and _fresh(src))]
    with ThreadPoolExecutor(max_workers=max(1, len(todo))) as ex:
        list(ex.map(lambda src: _compile(src, verbose), todo))
    objs = [os.path.join(CSRC, src + ".o") for src in SOURCES]
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv, incremental="-i" in sys.argv)
    print(LIB)
