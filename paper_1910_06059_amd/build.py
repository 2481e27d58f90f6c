"""Build libopm_gpu.so for gfx950 with hipcc (host part and kernels in one
shared library next to this file).

Each source is compiled to its own object in parallel (no kernel or device
variable is referenced across sources, so no relocatable device code is
needed) and the objects are linked into the library."""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libopm_gpu.so")
OBJ_DIR = os.path.join(ROOT, "_build", "obj")

HIPCC_FLAGS = [
    "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip"))) + sorted(
        glob.glob(os.path.join(HERE, "csrc", "*.cpp")))


def _headers():
    return glob.glob(os.path.join(HERE, "csrc", "*.h")) + glob.glob(
        os.path.join(ROOT, "include", "*.h"))


def _compile(hipcc, src, force, newest_header):
    obj = os.path.join(OBJ_DIR, os.path.basename(src) + ".o")
    if (not force and os.path.exists(obj)
            and os.path.getmtime(obj) >= max(os.path.getmtime(src), newest_header)):
        return obj, None
    tmp = obj + ".tmp"
    cmd = [hipcc] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"), "-c", "-o", tmp, src]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        return obj, f"hipcc failed on {os.path.basename(src)}:\n" + res.stderr[-8000:]
    os.replace(tmp, obj)
    return obj, None


def build(verbose: bool = False, force: bool = True, jobs: int = 8) -> str:
    """Compile every source (``force=False``: only those older than their
    object or a header) and link the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ_DIR, exist_ok=True)
    newest_header = max((os.path.getmtime(h) for h in _headers()), default=0.0)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        results = list(ex.map(lambda s: _compile(hipcc, s, force, newest_header), srcs))
    errors = [e for _, e in results if e]
    if errors:
        raise RuntimeError("\n".join(errors))
    tmp = LIB + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _ in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("link failed:\n" + res.stderr[-8000:])
    if verbose:
        print(res.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    import sys
    print(build(verbose=True, force="--incremental" not in sys.argv))
