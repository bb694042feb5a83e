"""Builds libslh.so (HIP for gfx950) in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libslh.so")
SOURCES = ["mc.hip", "dg.hip", "diffusion.hip", "util.hip", "capi.hip", "server.hip"]
ARCH = os.environ.get("SLH_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH,
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result"]


# Host-side AddressSanitizer and UBSan for a CPU-only check of the host code
# (validation, sizes, checkpoint parsing, the server's admission logic); the
# device code is built as usual.  Each -fsanitize applies to the host pass only.
SAN_OBJ = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_OBJ, "libslh_san.so")
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _compile(src: str, san: bool = False) -> str:
    out = os.path.join(SAN_OBJ if san else OBJ, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, *(SAN_FLAGS if san else []), "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return out


def build(verbose: bool = False, sanitize_host: bool = False) -> str:
    """Compiles every source and links libslh.so; always rebuilds.
    sanitize_host: _build_san/libslh_san.so with host-side ASan and UBSan."""
    obj_dir, lib = (SAN_OBJ, SAN_LIB) if sanitize_host else (OBJ, LIB)
    os.makedirs(obj_dir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, sanitize_host), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    # the sanitized library leaves the runtime's symbols to the preloaded
    # sanitizer runtime of the process that loads it
    cmd = ["hipcc", "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


def sanitized_is_current() -> bool:
    """The host-sanitized library exists and is newer than every source."""
    if not os.path.exists(SAN_LIB):
        return False
    t = os.path.getmtime(SAN_LIB)
    srcs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)]
    srcs.append(os.path.join(HERE, "..", "include", "slh.h"))
    return all(os.path.getmtime(f) <= t for f in srcs)


if __name__ == "__main__":
    import sys
    build(verbose=True, sanitize_host="--sanitize-host" in sys.argv)
