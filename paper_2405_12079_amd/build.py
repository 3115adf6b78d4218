"""Build libphos.so: the gfx950 HIP kernels and the C-ABI runtime, in-tree."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["csrc/kernels.hip", "csrc/runtime.cpp", "csrc/batch.cpp", "csrc/serve.cpp"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose: bool = False, jobs: int = 4) -> str:
    out = os.path.join(HERE, "libphos.so")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        path = os.path.join(HERE, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(objdir, os.path.basename(src) + ".o")
        lang = [] if src.endswith(".hip") else ["-x", "hip"]
        cmd = [HIPCC, *FLAGS, *lang, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-lhsa-runtime64",
           "-o", out + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def _wait(item, verbose):
    src, p = item
    text, _ = p.communicate()
    text = text.decode(errors="replace")
    noise = "'-packed-fp32-ops' is not a recognized feature for this target (ignoring feature)"
    lines = [l for l in text.splitlines() if noise not in l]
    if p.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n" + "\n".join(lines))
    if verbose and lines:
        print("\n".join(lines))


if __name__ == "__main__":
    print(build(verbose=True))
