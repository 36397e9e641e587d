"""Build libqds.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqds.so")
SOURCES = ["qds_api.hip", "qds_batch.hip", "qds_stages.hip", "qds_fused.hip", "qds_current.hip", "qds_adjoint.hip", "qds_noalloc.hip", "qds_particles.hip", "qds_copy.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

OBJDIR = os.path.join(HERE, "_build")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds fused within a source expression only: a step computes the
    # same bits whichever kernel it is inlined into (the one-step and two-step
    # marches, the kernel that advances the axion)
    "-ffp-contract=on",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]
if os.environ.get("QDS_RESOURCE_USAGE"):
    FLAGS.append("-Rpass-analysis=kernel-resource-usage")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libqds.so: " + " ".join(cmd[-3:]))
    return r.stderr


def build(verbose: bool = False) -> str:
    """Compile every source (in parallel) and link libqds.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [[HIPCC] + FLAGS + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(SOURCES, objs)]
    jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
    with ThreadPoolExecutor(jobs) as ex:
        for err in ex.map(lambda c: _run(c, verbose), cmds):
            if verbose and err:
                sys.stderr.write(err)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + objs + ["-o", tmp], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
