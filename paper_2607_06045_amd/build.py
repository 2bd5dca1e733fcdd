"""Build libdgidp.so (HIP kernels for gfx950 + host code) in place with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdgidp.so")
SOURCES = ["dgidp_kernels.hip", "dgidp_tables.cpp", "dgidp_host.cpp", "dgidp_amr.cpp", "dgidp_mlp.hip",
           "dgidp_noalloc.hip"]
# packed FP32 instructions are disabled: hipcc would otherwise emit them from
# ordinary float code.  The feature is a device one: the host (x86) pass of
# hipcc reports that it does not know it, once per function; that line alone
# is dropped from the build output.
HIPFLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-Wno-pass-failed",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
HOST_PASS_NOTE = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"


def build(verbose=False, jobs=4):
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src + ".o")
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = ["hipcc"] + HIPFLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    failed = []
    for p, src in procs:
        err = p.communicate()[1]
        rest = [l for l in err.splitlines() if l.strip() != HOST_PASS_NOTE]
        if rest:
            print("\n".join(rest), file=sys.stderr, flush=True)
        if p.returncode != 0:
            failed.append(src)
    if failed:
        raise RuntimeError("hipcc failed on " + ", ".join(failed))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
