"""Build libspr.so (HIP for gfx950) in-tree.

Every per-size kernel object is compiled from kernels_n.hip with -DSPR_N=<n>
(and -DSPR_VARIANT=<v> for the sizes with a tunable alternative plan);
objects are compiled in parallel and linked with hipcc into
paper_2409_07413_amd/libspr.so.  Run ``python -m paper_2409_07413_amd.build``.
"""

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libspr.so")

SIZES = (8, 12, 16, 24, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024)
# sizes compiled with an alternative plan (variant 1) for the run-time tuner
VARIANT_SIZES = (128, 256, 384, 512, 768, 1024)
ARCH = os.environ.get("SPR_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# extra compile definitions and an alternative output path (tuning builds)
EXTRA = os.environ.get("SPR_EXTRA_FLAGS", "").split()
if os.environ.get("SPR_LIB_OUT"):
    LIB = os.environ["SPR_LIB_OUT"]
    OBJ = LIB + ".objs"

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # code object v5 loads under every ROCm 7.x runtime, including the one PyTorch ships
    "-mcode-object-version=5",
    # keep the compiler from emitting packed-FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-function", "-Wno-unknown-pragmas",
]


def _jobs():
    jobs = []
    for n in SIZES:
        for v in ((0, 1) if n in VARIANT_SIZES else (0,)):
            # no automatic contraction: kernel results follow the source alone
            jobs.append((os.path.join(CSRC, "kernels_n.hip"), os.path.join(OBJ, f"kernels_{n}_{v}.o"),
                         [f"-DSPR_N={n}", f"-DSPR_VARIANT={v}", "-ffp-contract=off"]))
    jobs.append((os.path.join(CSRC, "kernels_common.hip"), os.path.join(OBJ, "kernels_common.o"), []))
    jobs.append((os.path.join(CSRC, "runtime.cpp"), os.path.join(OBJ, "runtime.o"), ["-x", "hip"]))
    jobs.append((os.path.join(CSRC, "server.cpp"), os.path.join(OBJ, "server.o"), ["-x", "hip"]))
    jobs.append((os.path.join(CSRC, "graph.cpp"), os.path.join(OBJ, "graph.o"), ["-x", "hip"]))
    jobs.append((os.path.join(CSRC, "noalloc.cpp"), os.path.join(OBJ, "noalloc.o"), ["-x", "hip"]))
    return jobs


def _compile(job):
    src, obj, extra = job
    cmd = [HIPCC] + FLAGS + EXTRA + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    # source warnings (the host pass's notice about the packed-FP32 target
    # feature it does not know is expected and left out)
    warns = [l for l in r.stderr.splitlines() if "warning:" in l and "packed-fp32-ops" not in l]
    return obj, sorted(set(warns))


def build(jobs_parallel=None, verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = _jobs()
    workers = jobs_parallel or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        done = list(ex.map(_compile, jobs))
    objs = [o for o, _ in done]
    if verbose:
        for w in sorted({w for _, ws in done for w in ws}):
            print(w)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
