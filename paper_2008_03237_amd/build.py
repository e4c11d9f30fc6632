"""Compile the HIP sources of the library (and the workload generator) for gfx950.

Every source is compiled on every call (hipcc, in parallel) and linked into
shared objects next to the Python modules that load them.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ARCH = os.environ.get("DLPNO_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# packed FP32 instructions are disabled in all device code
FLAGS = ["-O3", "--offload-arch=" + ARCH, "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]

LIB_SOURCES = ["grouped_f64.hip", "grouped_f32.hip", "split.hip", "adjoint.hip", "elementwise.hip", "plan.hip",
               "mixed.hip", "tune.hip", "noalloc.hip", "solve.hip", "pno.hip", "quadratic.hip", "ring.hip"]
GEN_SOURCES = [os.path.join(ROOT, "workload", "csrc", "gen.hip")]


def _compile(src, obj, extra=()):
    cmd = [HIPCC] + FLAGS + list(extra) + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("compile failed: %s\n%s\n%s" % (" ".join(cmd), r.stdout, r.stderr))
    return obj


def _link(objs, out):
    tmp = out + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed: %s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, out)


def build(verbose=True, jobs=None):
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)
    srcs = [os.path.join(HERE, "csrc", s) for s in LIB_SOURCES if os.path.exists(os.path.join(HERE, "csrc", s))]
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, s, os.path.join(bdir, os.path.basename(s) + ".o")): s for s in srcs}
        gfut = {ex.submit(_compile, s, os.path.join(bdir, "gen_" + os.path.basename(s) + ".o"),
                          ("-ffp-contract=off",)): s for s in GEN_SOURCES}
        objs = [f.result() for f in futs]
        gobjs = [f.result() for f in gfut]
    _link(sorted(objs), os.path.join(HERE, "libdlpno.so"))
    _link(gobjs, os.path.join(ROOT, "workload", "libdlpno_gen.so"))
    if verbose:
        print("built", os.path.join(HERE, "libdlpno.so"), "and workload/libdlpno_gen.so", file=sys.stderr)


if __name__ == "__main__":
    build()
