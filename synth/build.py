"""Build the synthetic-workload generators: host C (gcc) and device HIP (gfx950)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False, device: bool = True):
    host = os.path.join(HERE, "libsynth_host.so")
    cmd = ["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC",
           os.path.join(HERE, "synth_host.c"), "-o", host + ".tmp"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(host + ".tmp", host)
    outs = [host]
    if device:
        dev = os.path.join(HERE, "libsynth_dev.so")
        cmd = [HIPCC, *HIP_FLAGS, os.path.join(HERE, "synth_dev.hip"), "-o", dev + ".tmp"]
        if verbose:
            print(" ".join(cmd))
        subprocess.run(cmd, check=True)
        os.replace(dev + ".tmp", dev)
        outs.append(dev)
    return outs


if __name__ == "__main__":
    print(build(verbose=True))
