"""Build the gfx950 HIP library libfciqmc.so in-tree with hipcc.

The host runtime (fq_lib.hip) and the merge/spawn kernel instantiations
(fq_inst.hip, once per address-word count and model variant) are compiled
as separate objects in parallel, then linked into one shared library.
"""
import concurrent.futures
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfciqmc.so")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off",                      # no FMA contraction: bit-exact parity
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
    "-I", os.path.join(ROOT, "include"),
]

# (address words, model variant): 0 real-space ring, 1 momentum space with
# M <= 16, 2 momentum space with M <= 32, 3 square lattice / importance sampling
INSTANCES = [(w, m) for w in (1, 2) for m in (0, 1, 2, 3)]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the packed-fp32 feature
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return r.returncode, " ".join(cmd), err


def build(verbose=False, jobs=None):
    jobs = jobs or min(len(INSTANCES) + 1, os.cpu_count() or 1, 16)
    with tempfile.TemporaryDirectory(prefix="fq_build_") as td:
        cmds, objs = [], []
        obj = os.path.join(td, "fq_lib.o")
        cmds.append(["hipcc", *FLAGS, "-c", os.path.join(CSRC, "fq_lib.hip"), "-o", obj])
        objs.append(obj)
        for w, m in INSTANCES:
            obj = os.path.join(td, f"fq_inst_w{w}_m{m}.o")
            cmds.append(["hipcc", *FLAGS, f"-DFQ_INST_W={w}", f"-DFQ_INST_MODEL={m}", "-c",
                         os.path.join(CSRC, "fq_inst.hip"), "-o", obj])
            objs.append(obj)
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(_run, cmds))
        failed = False
        for rc, cmd, err in results:
            if verbose:
                print(cmd, flush=True)
            if rc != 0:
                failed = True
                sys.stderr.write(err + "\n")
            elif verbose and err.strip():
                sys.stderr.write(err + "\n")
        if failed:
            raise RuntimeError("hipcc failed")
        rc, cmd, err = _run(["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", LIB + ".tmp"])
        if verbose:
            print(cmd, flush=True)
        if rc != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError("hipcc link failed")
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
