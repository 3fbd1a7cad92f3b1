"""Build the HIP library libgt.so in place (hipcc, gfx950).

Every source is compiled to an object file of its own (in parallel), then
the objects are linked into one shared library.
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["gt_api.hip", "gt_kernels.hip", "gt_persistent.hip", "gt_devplan.hip", "gt_policy.hip", "gt_sample.hip", "gt_mlp.hip", "gt_unordered.hip",
           "gt_microbench.hip"]
LIB = os.path.join(HERE, "libgt.so")
OBJDIR = os.path.join(HERE, "_build")
HIPCC = "/opt/rocm/bin/hipcc"

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # no packed fp32 instructions in any HIP code of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _filtered(r):
    return [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops' is not a recognized" not in l]


# per-source flags: the persistent kernel runs every body inside one loop;
# without machine-level loop-invariant code motion the compiler keeps no
# body's constants live across the others
EXTRA_FLAGS = {"gt_persistent.hip": ["-mllvm", "-disable-machine-licm"]}


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.splitext(os.path.basename(src))[0] + ".o")
    cmd = [HIPCC] + HIPCC_FLAGS + EXTRA_FLAGS.get(os.path.basename(src), []) + ["-c", "-o", obj, src]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    return obj, r.returncode, _filtered(r)


def build(verbose=False, jobs=None):
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    jobs = jobs or min(len(srcs), max(1, min(16, os.cpu_count() or 1)))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        results = list(pool.map(lambda s: _compile(s, verbose), srcs))
    failed = [(o, msgs) for o, rc, msgs in results if rc != 0]
    for _, _, msgs in results:
        if msgs:
            sys.stderr.write("\n".join(msgs) + "\n")
    if failed:
        raise RuntimeError("hipcc failed: " + ", ".join(os.path.basename(o) for o, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [o for o, _, _ in results]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write("\n".join(_filtered(r)) + "\n")
        raise RuntimeError("hipcc link failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
