"""Builds libglint.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["api.hip", "partition.hip", "prefilter.hip", "lut.hip", "shade.hip", "batched.hip", "mlp.hip", "profile.hip"]
ARCH = os.environ.get("GLINT_OFFLOAD_ARCH", "gfx950")


def library_path() -> str:
    return os.path.join(HERE, "libglint.so")


def hipcc_flags():
    return ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
            # packed FP32 instructions stay off (they have given wrong results on these parts)
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]


# Per-source additions: the network kernels keep their matrix-core
# accumulators in ordinary vector registers (the backend's VGPR form of
# MFMA), so the elementwise epilogue reads them without a copy out of the
# accumulation registers per value.
SOURCE_FLAGS = {"mlp.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form=true"]}


def build_library(verbose: bool = False, jobs: int = 8) -> str:
    out = library_path()
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = ["hipcc", "-c", *hipcc_flags(), *SOURCE_FLAGS.get(src, []), os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((src, subprocess.Popen(cmd)))
        objs.append(obj)
        while sum(p.poll() is None for _, p in procs) >= jobs:
            procs[0][1].wait()
    for src, p in procs:
        if p.wait() != 0:
            raise RuntimeError(f"hipcc failed on {src}")
    tmp = out + ".tmp"
    cmd = ["hipcc", "-shared", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
