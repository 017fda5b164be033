"""Build libfractal.so for gfx950 with hipcc (in-tree, no JIT cache).

Every translation unit under csrc/ is compiled to an object in _build/ and
the objects are linked into paper_2004_13475_amd/libfractal.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libfractal.so")
BUILD_DIR = os.path.join(HERE, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -packed-fp32-ops off: no packed float32 VALU instructions are generated.
# Denormals are kept (the heat field decays through the float32 subnormal
# range), so no flush-to-zero and no fast-math.
HIP_FLAGS = [
    "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-x", "hip",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fno-gpu-flush-denormals-to-zero", "-ffp-contract=fast-honor-pragmas",
    "-Wall", "-Wno-unused-function",
]
SOURCES = ["api.cpp", "step_kernels.hip", "step_lambda.hip", "step_bb.hip", "step_mfma.hip",
           "step_march.hip", "step_march_ca.hip", "step_march_heat.hip",
           "step_march_mid_ca.hip", "step_march_mid_heat.hip", "block_heat.hip", "block_ca.hip", "batch_block.hip",
           "seed.hip", "batch.hip", "batch_ca.hip", "batch_heat.hip", "batch_march_ca.hip", "batch_march_heat.hip",
           "sw_rd.hip", "compact.hip", "compact_ca.hip", "compact_heat.hip", "compact_block.hip", "nbb.hip",
           "serve.cpp"]


def _local_deps(path: str, seen: set) -> set:
    """The file and every project header it includes (quoted includes,
    followed recursively)."""
    path = os.path.normpath(path)
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path, encoding="utf-8") as fh:
        for line in fh:
            m = re.match(r'\s*#\s*include\s+"([^"]+)"', line)
            if m:
                _local_deps(os.path.join(os.path.dirname(path), m.group(1)), seen)
    return seen


def _up_to_date(src: str, obj: str) -> bool:
    """The object is newer than its source and every header it includes."""
    if not os.path.exists(obj):
        return False
    t = os.path.getmtime(obj)
    return all(os.path.getmtime(d) < t for d in _local_deps(os.path.join(CSRC, src), set()))


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and _up_to_date(src, obj):
        return obj
    cmd = [HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every translation unit (or, with incremental, those whose
    object is older than a source or header) and link libfractal.so."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, incremental), srcs))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
           "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build(verbose=True, incremental="--incremental" in sys.argv[1:])
    sys.exit(0)
