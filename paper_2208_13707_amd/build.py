"""Build libmpixs.so (and the native program driver) for gfx950 with hipcc.

Run ``python -m paper_2208_13707_amd.build`` or call ``build()``.  The
shared libraries are written next to this file, in-tree.
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
ARCH = os.environ.get("MPIXS_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    "-O3", f"--offload-arch={ARCH}", "-std=c++17", "-fPIC",
    # packed fp32 instructions stay off; reductions and user kernels must
    # round every operation separately and keep subnormals
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Wall", "-Wno-unused-function",
]

LIBS = {
    "libmpixs.so": ["k_sync.hip", "k_copy.hip", "k_reduce.hip", "k_batch.hip", "k_batch_nt.hip",
                    "batch_static.hip", "runtime.cpp", "types.cpp"],
    "libmpixs_driver.so": ["driver.cpp", "serve.hip", "hostrate.cpp"],
}


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(name, sources, extra, verbose):
    objs = []
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    procs = []
    for src in sources:
        obj = os.path.join(build_dir, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc()] + HIP_FLAGS + ["-I", os.path.join(ROOT, "include"), "-c",
                                       os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    for src, p in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        text = "\n".join(line for line in text.splitlines()
                         if "packed-fp32-ops' is not a recognized feature" not in line)
        if p.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{text}")
        if text.strip() and verbose:
            print(text)
    target = os.path.join(HERE, name)
    tmp = target + ".tmp"
    cmd = [hipcc(), "-shared", f"--offload-arch={ARCH}", "-fPIC", "-o", tmp] + objs + extra
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    if r.returncode != 0:
        raise RuntimeError(f"link of {name} failed:\n{r.stdout.decode(errors='replace')}")
    os.replace(tmp, target)
    return target


def build(verbose: bool = False):
    out = []
    out.append(_compile("libmpixs.so", LIBS["libmpixs.so"], [], verbose))
    if os.path.exists(os.path.join(CSRC, "driver.cpp")):
        out.append(_compile("libmpixs_driver.so", LIBS["libmpixs_driver.so"],
                            ["-L" + HERE, "-lmpixs", "-Wl,-rpath,$ORIGIN"], verbose))
    return out


if __name__ == "__main__":
    for p in build(verbose="-v" in sys.argv):
        print(p)
