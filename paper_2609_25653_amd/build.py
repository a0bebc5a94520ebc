"""Build the HIP library (gfx950) in-tree: paper_2609_25653_amd/libipc_hip.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SO = os.path.join(HERE, "libipc_hip.so")
SOURCES = ["ipc_create.hip", "ipc_elastic.hip", "ipc_contact.hip", "ipc_solver.hip", "ipc_coarse.hip", "ipc_adjoint.hip", "ipc_api.hip", "ipc_dualmesh.hip", "ipc_halfspace.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast-honor-pragmas",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result"]


def build(jobs=8, verbose=False):
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_obj_" + src.replace(".hip", ".o"))
        objs.append(obj)
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            failed.append(src)
            sys.stderr.write(out.decode(errors="replace"))
        elif verbose and out:
            sys.stderr.write(out.decode(errors="replace"))
    if failed:
        raise RuntimeError("hipcc failed for " + ", ".join(failed))
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", SO + ".tmp", *objs]
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    for o in objs:
        os.remove(o)
    return SO


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(SO)
