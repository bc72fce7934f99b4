"""Build libirk.so (HIP, gfx950) in-tree, the host-only test library and its
address/undefined-behaviour sanitizer build.

``python -m paper_2010_11377_amd.build`` or ``build()``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)

HIP_SOURCES = ["host_setup.cpp", "kernels.hip", "vcycle.hip", "wtile.hip", "wsplit.hip",
               "wfine.hip", "ws9.hip", "tail2.hip", "left.hip", "solver.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include")]


def _run(cmd):
    proc = subprocess.run(cmd, cwd=CSRC, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in proc.stdout.splitlines() if "packed-fp32-ops" not in l)
    if proc.returncode != 0:
        raise RuntimeError("build failed: %s\n%s" % (" ".join(cmd), out))
    return out


def _compile_objects(objdir):
    """One hipcc process per source, in parallel; returns the object paths."""
    from concurrent.futures import ThreadPoolExecutor
    flags = [f for f in HIP_FLAGS if f != "-shared"]
    objs = [os.path.join(objdir, os.path.splitext(src)[0] + ".o") for src in HIP_SOURCES]
    with ThreadPoolExecutor(max_workers=min(len(HIP_SOURCES), os.cpu_count() or 1)) as ex:
        outs = list(ex.map(lambda so: _run([HIPCC] + flags + ["-c", so[0], "-o", so[1]]),
                           zip(HIP_SOURCES, objs)))
    return objs, "\n".join(outs)


def build(verbose=False):
    """Compile libirk.so (gfx950) and libirk_host_test.so (host C++ only)."""
    import tempfile
    lib = os.path.join(HERE, "libirk.so")
    tmp = lib + ".tmp"
    with tempfile.TemporaryDirectory(prefix="irk_build_") as objdir:
        objs, out = _compile_objects(objdir)
        out += _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, lib)
    host = os.path.join(HERE, "libirk_host_test.so")
    out2 = _run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-o", host + ".tmp",
                 "host_setup.cpp", "host_test_api.cpp"])
    os.replace(host + ".tmp", host)
    # the same host code under AddressSanitizer + UBSan (g++ only, no GPU code)
    asan = os.path.join(HERE, "libirk_host_asan.so")
    out3 = _run(["g++", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                 "-fno-sanitize-recover=undefined", "-std=c++17", "-fPIC", "-shared", "-o",
                 asan + ".tmp", "host_setup.cpp", "host_test_api.cpp"])
    os.replace(asan + ".tmp", asan)
    if verbose:
        print(out, out2, out3, sep="\n")
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
