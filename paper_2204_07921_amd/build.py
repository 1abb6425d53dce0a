"""Build libmgcurv.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2204_07921_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmgcurv.so")

SOURCES = ["mgc_kernels.hip", "mgc_split.hip", "mgc_runtime.hip", "mgc_batch.hip", "mgc_cnn.hip", "mgc_fbs.hip", "mgc_recon.hip"]
HEADERS = ["mgc_device.h", "mgc_internal.h", "mgc_sweep.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # packed FP32 instructions stay off (plain scalar/vector FP32 and FP64 only)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def source_hash() -> str:
    """Hash of everything the library is compiled from (csrc/ and include/mgcurv.h); the build
    embeds it and the binding refuses a library built from other sources."""
    import hashlib
    h = hashlib.sha256()
    paths = sorted(os.path.join(CSRC, n) for n in os.listdir(CSRC)) + [os.path.join(ROOT, "include", "mgcurv.h")]
    for p in paths:
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link libmgcurv.so; always recompiles."""
    from concurrent.futures import ThreadPoolExecutor
    objs = []
    cmds = []
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    tag = f'-DMGC_SOURCE_HASH="{source_hash()}"'
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmds.append([hipcc(), *HIPCC_FLAGS, tag, "-I", os.path.join(ROOT, "include"), "-c",
                     os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        for rc in ex.map(subprocess.call, cmds):
            if rc != 0:
                raise subprocess.CalledProcessError(rc, "hipcc")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
