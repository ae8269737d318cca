"""Builds libcoex.so (HIP kernels for gfx950 + host runtime + C ABI) in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcoex.so")


FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed fp32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError("compile failed:\n" + err)
    if verbose and err.strip():
        print(err, file=sys.stderr)


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Always recompiles (the driver's build check calls this): the host-only
    compiler with g++, the kernels and runtime with hipcc for gfx950."""
    inc = ["-I", os.path.join(ROOT, "include")]
    tag = ".tmp%d_%d" % (os.getpid(), abs(hash((out, tuple(defines)))) % 100000)
    sfx = tag.replace(".", "_")
    obj_host = os.path.join(CSRC, "compile%s.o" % sfx)
    obj_serve = os.path.join(CSRC, "serve%s.o" % sfx)
    obj_hm = os.path.join(CSRC, "host_method%s.o" % sfx)
    obj_fa = os.path.join(CSRC, "fasta%s.o" % sfx)
    dev_srcs = ["coex.hip", "batch.hip", "sort.hip", "partition.hip"] + ["tail_%s_%s.hip" % (e, k) for e in ("byte", "2bit")
                                            for k in ("count", "hist", "pos")]
    obj_dev = [os.path.join(CSRC, "%s%s.o" % (os.path.splitext(f)[0], sfx)) for f in dev_srcs]
    tmp = out + tag
    try:
        jobs = [subprocess.Popen(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c", "-o", obj_host] + inc +
                                 [os.path.join(CSRC, "compile.cpp")],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
                subprocess.Popen(["g++", "-O2", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-D__HIP_PLATFORM_AMD__",
                                  "-I/opt/rocm/include", "-c", "-o", obj_serve] + inc +
                                 [os.path.join(CSRC, "serve.cpp")],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
                subprocess.Popen(["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-c", "-o", obj_hm] + inc +
                                 [os.path.join(CSRC, "host_method.cpp")],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True),
                subprocess.Popen(["g++", "-O3", "-std=c++17", "-fPIC", "-Wall", "-pthread", "-c", "-o", obj_fa] + inc +
                                 [os.path.join(CSRC, "fasta.cpp")],
                                 stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)]
        for src, obj in zip(dev_srcs, obj_dev):
            cmd = [hipcc()] + FLAGS + ["-D" + d for d in defines] + inc + ["-c", "-o", obj, os.path.join(CSRC, src)]
            if verbose:
                print(" ".join(cmd), flush=True)
            jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
        errs = []
        for j in jobs:
            _, err = j.communicate()
            err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l)
            if j.returncode != 0:
                errs.append(err)
            elif verbose and err.strip():
                print(err, file=sys.stderr)
        if errs:
            raise RuntimeError("compile failed:\n" + "\n".join(errs))
        rocm_lib = "/opt/rocm/lib"
        _run(["g++", "-shared", "-pthread", "-o", tmp] + obj_dev + [obj_host, obj_serve, obj_hm, obj_fa, "-L" + rocm_lib,
              "-lamdhip64", "-Wl,-rpath," + rocm_lib], verbose)
        os.replace(tmp, out)
    finally:
        for f in [obj_host, obj_serve, obj_hm, obj_fa, tmp] + obj_dev:
            if os.path.exists(f):
                os.remove(f)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
