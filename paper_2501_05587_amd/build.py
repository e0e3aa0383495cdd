"""Build libkkm.so (gfx950) in-tree with hipcc.

Every source under csrc/ is compiled for gfx950 only, with packed-FP32
instructions disabled, and linked into paper_2501_05587_amd/libkkm.so.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libkkm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-ffp-contract=fast", "-I", os.path.join(HERE, "..", "include")]


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _includes(path, seen):
    """Every header `path` includes with #include "...", transitively."""
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("#include \""):
                h = os.path.normpath(os.path.join(os.path.dirname(path), line.split('"')[1]))
                if h not in seen and os.path.exists(h):
                    seen.add(h)
                    _includes(h, seen)
    return seen


def _object(src):
    return os.path.join(BUILD, os.path.basename(src) + ".o")


def _stale(src):
    obj = _object(src)
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(t < os.path.getmtime(p) for p in [src, *_includes(src, set())])


def _compile(src):
    obj = _object(src)
    cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every HIP source and link libkkm.so; returns its path.  With
    incremental=True only sources whose object is older than the source or any
    header are compiled again."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    todo = srcs
    if incremental:
        todo = [s for s in srcs if _stale(s)]
    results = []
    if todo:
        with cf.ThreadPoolExecutor(max_workers=min(8, len(todo))) as ex:
            results = list(ex.map(_compile, todo))
    objs = [_object(s) for s in srcs]
    if verbose:
        for (_, w), s in zip(results, todo):
            if w:
                print("[%s]\n%s" % (os.path.basename(s), w), file=sys.stderr)
    tmp = LIB + ".tmp%d" % os.getpid()
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, incremental="--incremental" in sys.argv))
