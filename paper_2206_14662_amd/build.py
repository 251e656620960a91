"""Build libpicmcc.so (HIP for gfx950) in-tree.

Every .hip source compiles with hipcc for gfx950 with packed-FP32 instruction
selection off; the FP64 form and the host code also turn floating-point
contraction off, so every multiply and add rounds as written.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libpicmcc.so")
# streaming-bandwidth probes (a measurement tool beside the library)
PROBE_SRC = "stream_probe.hip"
PROBE_LIB = os.path.join(PKG, "libstreamprobe.so")
ARCH = os.environ.get("PIC_OFFLOAD_ARCH", "gfx950")

# source -> extra flags
SOURCES = {
    "api.hip": ["-ffp-contract=off"],
    "k_fp64.hip": ["-ffp-contract=off"],
    "k_field.hip": [],
    "fp32.hip": [],
    "insert.hip": ["-ffp-contract=off"],
    "insert3.hip": ["-ffp-contract=off"],
    "noalloc.hip": [],
}

COMMON = [
    "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unknown-warning-option",
]


def _compile(src, flags, verbose):
    obj = os.path.join(OUT, src.replace(".hip", ".o"))
    cmd = COMMON + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    # the host pass does not know the packed-fp32 feature; drop that warning only
    msgs = [l for l in (r.stderr or "").splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if msgs and verbose:
        print("\n".join(msgs), flush=True)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(OUT, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 1)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda kv: _compile(kv[0], kv[1], verbose), SOURCES.items()))
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    probe = _compile(PROBE_SRC, [], verbose)
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", PROBE_LIB + ".tmp", probe]
    subprocess.run(cmd, check=True)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
