"""Build the hpdg shared library (C ABI) for gfx950 with hipcc, in-tree.

    python -m paper_1907_01572_amd.build        # writes paper_1907_01572_amd/libhpdg.so
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhpdg.so")
SOURCES = ["basis.cpp", "geom.cpp", "topo.cpp", "setup.cpp", "schwarz.cpp", "api.cpp", "kernels.hip", "apply.hip", "fastapply.hip", "newton.hip", "rhs.hip", "schwarz.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose=False, jobs=6):
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    flags = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(HERE, "..", "include"), "-Wall", "-Wno-unused-function"]
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        objs.append(obj)
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        cmd = [HIPCC] + flags + lang + ["-c", os.path.join(SRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs)
            procs = []
    _wait(procs)
    cmd = [HIPCC, "-shared", "--offload-arch=gfx950", "-o", OUT + ".tmp"] + objs + \
        ["-L/opt/rocm/lib", "-lrocsolver", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout.decode())
    os.replace(OUT + ".tmp", OUT)
    return OUT


def _wait(procs):
    errs = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode()
        if p.returncode != 0:
            errs.append("%s:\n%s" % (src, text))
        elif text.strip() and "warning" in text and "packed-fp32-ops" not in text:
            sys.stderr.write(text)
    if errs:
        raise RuntimeError("compile failed:\n" + "\n".join(errs))


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
