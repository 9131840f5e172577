"""Build the gfx950 shared library ``liblindhard.so`` in-tree with hipcc."""
import glob
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "liblindhard.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-mcode-object-version=5",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source into liblindhard.so.

    Each source is compiled to an object of its own, in parallel (the
    sources share no device symbols), then the objects are linked.  By
    default every source is recompiled; with ``incremental`` an object newer
    than its source and every header is reused."""
    from concurrent.futures import ThreadPoolExecutor

    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = "%d" % os.getpid()
    compile_flags = [f for f in FLAGS if f != "-shared"]
    headers = glob.glob(os.path.join(CSRC, "*.h")) + glob.glob(os.path.join(INCLUDE, "*.h"))
    newest_header = max((os.path.getmtime(h) for h in headers), default=0.0)

    def obj(src):
        keep = os.path.join(objdir, os.path.basename(src) + ".o")
        if incremental and os.path.exists(keep) and os.path.getmtime(keep) > max(os.path.getmtime(src),
                                                                                  newest_header):
            return keep
        o = keep + "." + tag
        cmd = [HIPCC] + compile_flags + ["-I", INCLUDE, "-I", CSRC, "-c", src, "-o", o]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(o, keep)
        return keep

    with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
        objs = list(ex.map(obj, sources()))
    tmp = LIB + ".tmp" + tag
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys

    print(build(verbose=True, incremental="--incremental" in sys.argv))
