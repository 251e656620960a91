"""Streaming-bandwidth probes of the particle loop's access patterns (see
csrc/stream_probe.hip): the HBM rate a kernel that only moves the particle
loop's bytes reaches on this GPU, for comparison with the particle kernel.

Run: python -m paper_2206_14662_amd.stream_probe [--n N] [--reps R]
Prints one JSON line: per pattern the average launch time and GB/s."""
import argparse
import ctypes as C
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
PATTERNS = ("copy", "read6", "write5", "soa", "soa_pers", "aosoa", "aosoa8", "aosoa8_pers", "aosoa_pers",
            "aosoa_pers2")


def run(n=128_000_000, reps=10):
    lib = C.CDLL(os.path.join(HERE, "libstreamprobe.so"))
    lib.sp_run.argtypes = [C.c_int, C.c_longlong, C.c_int, C.POINTER(C.c_double)]
    lib.sp_run.restype = C.c_double
    out = {}
    for k, name in enumerate(PATTERNS):
        gb = C.c_double()
        ms = lib.sp_run(k, int(n), int(reps), C.byref(gb))
        if ms <= 0.0:
            raise RuntimeError(f"stream probe {name} failed ({ms})")
        out[name] = {"ms": ms, "GB": gb.value, "GB_per_s": gb.value / (ms * 1e-3)}
        print(f"# {name}: {ms:.4f} ms, {gb.value / (ms * 1e-3):.1f} GB/s", flush=True)
    return out


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=128_000_000)
    ap.add_argument("--reps", type=int, default=10)
    a = ap.parse_args()
    print(json.dumps({"elements": a.n, "reps": a.reps, "patterns": run(a.n, a.reps)}), flush=True)
