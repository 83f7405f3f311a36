"""Build libfehx.so (HIP for gfx950) in-tree with hipcc.

Every translation unit is compiled to an object in parallel, then linked into
paper_2512_08571_amd/libfehx.so.  Packed-FP32 instructions are disabled for
all device code.  Run ``python -m paper_2512_08571_amd.build`` or call
``build()``.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libfehx.so")
ARCH = os.environ.get("FEHX_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I", os.path.join(HERE, "..", "include"), "-Wno-unused-result"]


def _sources():
    return sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))


def _deps(path, seen=None):
    """The source and every local header it includes (recursively)."""
    seen = set() if seen is None else seen
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    for line in open(path, errors="replace"):
        line = line.strip()
        if line.startswith("#include \""):
            name = line.split('"')[1]
            for d in (os.path.dirname(path), os.path.join(HERE, "..", "include")):
                _deps(os.path.normpath(os.path.join(d, name)), seen)
    return seen


def _stale(src):
    out = os.path.join(OBJ, src + ".o")
    if not os.path.exists(out):
        return True
    t = os.path.getmtime(out)
    return any(os.path.getmtime(d) > t for d in _deps(os.path.join(CSRC, src)))


def _compile(src):
    out = os.path.join(OBJ, src + ".o")
    # the object is dated when its inputs were read, so an input edited while
    # it compiles leaves it stale for the next incremental build
    t_read = max(os.path.getmtime(d) for d in _deps(os.path.join(CSRC, src)))
    cmd = [HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", out] + FLAGS
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stderr[-6000:]}")
    os.utime(out, (t_read, t_read))
    return out


def build(jobs=None, verbose=True, incremental=False):
    """Compile every source (incremental=True: only those whose object is
    older than the source or a local header it includes) and link."""
    os.makedirs(OBJ, exist_ok=True)
    srcs = _sources()
    todo = [s for s in srcs if _stale(s)] if incremental else srcs
    jobs = jobs or min(max(len(todo), 1), max(1, (os.cpu_count() or 2)))
    with cf.ThreadPoolExecutor(jobs) as ex:
        list(ex.map(_compile, todo))
    objs = [os.path.join(OBJ, s + ".o") for s in srcs]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-o", tmp] + objs + [f"--offload-arch={ARCH}", "-L/opt/rocm/lib",
                                                   "-lrocblas", "-lrocsolver", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(incremental="--incremental" in sys.argv)
    sys.exit(0)
