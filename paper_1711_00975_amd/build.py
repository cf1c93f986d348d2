"""Build libcsk.so (the HIP library behind include/csk.h) for gfx950 with hipcc.

Each source is compiled to its own object in parallel (no relocatable device code: every
kernel is launched from the translation unit that defines it), then the objects are
linked into one shared library.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcsk.so")
PROBE_LIB = os.path.join(HERE, "libcsk_probe.so")   # measurement probes for the benchmark
OBJ_DIR = os.path.join(ROOT, "_build")
SOURCES = ["csk_api.hip", "csk_update.hip", "csk_sortbin.hip", "csk_sortbin_rows.hip", "csk_collect.hip", "csk_kernels.hip", "csk_router.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
GPU_FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd, what, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns that it does not know the packed-fp32 feature: harmless
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        sys.stderr.write(err + "\n")
        raise RuntimeError("hipcc failed building " + what)
    if verbose and err.strip():
        sys.stderr.write(err + "\n")


def build(verbose: bool = False) -> str:
    os.makedirs(OBJ_DIR, exist_ok=True)
    objs = [os.path.join(OBJ_DIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    common = GPU_FLAGS + ["-ffp-contract=off", "-Wall", "-Wno-unused-result",
                          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = [([HIPCC] + common + ["-c", os.path.join(CSRC, s), "-o", o], s) for s, o in zip(SOURCES, objs)]
    jobs.append(([HIPCC] + GPU_FLAGS + ["-shared", "-o", PROBE_LIB + ".tmp", os.path.join(CSRC, "csk_probe.hip")],
                 "libcsk_probe.so"))
    with ThreadPoolExecutor(max_workers=len(jobs)) as ex:
        for f in [ex.submit(_run, c, w, verbose) for c, w in jobs]:
            f.result()
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs, "libcsk.so", verbose)
    os.replace(LIB + ".tmp", LIB)
    os.replace(PROBE_LIB + ".tmp", PROBE_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
