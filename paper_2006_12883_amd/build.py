"""Builds libstmg.so (HIP for gfx950) in-tree with hipcc.

Run as ``python -m paper_2006_12883_amd.build`` or call ``build()``.
``--host-sanitize`` builds libstmg_hostsan.so instead: the host code with
AddressSanitizer and UndefinedBehaviorSanitizer (device code unchanged), for
loading through ``binding.LIB_PATH`` with the ASan runtime preloaded on a
machine without a GPU (the setup paths: hierarchies, tables, Galerkin
stencils, PFASST levels, windows, batch sizing).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libstmg.so")
SOURCES = ["inst_smooth_f64.hip", "inst_smooth_f32.hip", "inst_restrict_f64.hip", "inst_restrict_f32.hip",
           "inst_resid.hip", "inst_prolong.hip", "inst_fft.hip", "inst_galerkin.hip", "smooth_restrict.hip", "kernels_misc.hip", "krylov.hip", "coarse_coef.hip", "coarse_scan.hip", "solver.hip", "pfasst.hip", "capi.hip", "batch.hip", "tables.cpp"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions are kept out of generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-result",
]


HOST_SANITIZE = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer"]


def build(verbose=False, jobs=None, host_sanitize=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    bdir = os.path.join(HERE, "_build_hostsan" if host_sanitize else "_build")
    lib = os.path.join(HERE, "libstmg_hostsan.so") if host_sanitize else LIB
    flags = [f for f in FLAGS if f != "-shared" and not (host_sanitize and f == "-O3")]
    if host_sanitize:
        flags += HOST_SANITIZE
    os.makedirs(bdir, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(bdir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
        if src.endswith(".cpp"):
            cmd = [hipcc, "-x", "hip"] + cmd[1:]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and text.strip():
            sys.stdout.write(text)
    if failed:
        for src, text in failed:
            sys.stderr.write("---- %s ----\n%s\n" % (src, text))
        raise RuntimeError("hipcc failed for " + ", ".join(s for s, _ in failed))
    tmp = lib + ".tmp"
    cmd = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    if host_sanitize:
        cmd[4:4] = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, host_sanitize="--host-sanitize" in sys.argv))
