"""Compile libpr.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
SOURCES = ["csrc/pr_kernels.hip", "csrc/pr_batch.hip", "csrc/pr_set.hip", "csrc/pr_warm.hip", "csrc/pr_sort.hip",
           "csrc/pr_upload.hip", "csrc/pr_solve.hip", "csrc/pr_set_host.hip", "csrc/pr_host.hip",
           "csrc/pr_serve.hip", "csrc/pr_probe.hip", "csrc/pr_noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-munsafe-fp-atomics",  # FP atomics as hardware instructions, not CAS loops
    # no packed FP32 arithmetic anywhere in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall",
]


def build(verbose: bool = False, jobs: int = 4) -> str:
    out = os.path.join(_HERE, "libpr.so")
    objdir = os.path.join(_ROOT, "_build", "pr")
    os.makedirs(objdir, exist_ok=True)
    procs, objs = [], []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.basename(src).replace(".hip", ".o"))
        cmd = ["hipcc", *HIPCC_FLAGS, "-I", os.path.join(_ROOT, "include"), "-c", os.path.join(_HERE, src),
               "-o", obj]
        if verbose:
            print(" ".join(cmd))
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    errs = []
    for p, src in procs:
        _, err = p.communicate()
        noise = "is not a recognized feature for this target"
        lines = [ln for ln in err.splitlines() if noise not in ln]
        if lines and verbose:
            print("\n".join(lines))
        if p.returncode != 0:
            errs.append(f"{src}:\n" + "\n".join(lines))
    if errs:
        raise RuntimeError("hipcc failed:\n" + "\n".join(errs))
    tmp = out + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
