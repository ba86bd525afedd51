"""Build libperm.so (HIP kernels for gfx950 + host C++ library) in-tree.

Device translation units (csrc/*.hip) are compiled by hipcc for gfx950; host
translation units (csrc/*.cpp) by g++ against the HIP runtime headers; both in
parallel, then linked into paper_2602_10141_amd/libperm.so next to this file.
Every HIP compile carries -ffp-contract=off (the Kahan compensation and the
exact Barrett steps must not be re-fused) and disables packed FP32 ops.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libperm.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-fno-fast-math", "-mcode-object-version=5",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + CSRC, "-I" + os.path.join(HERE, "..", "include")]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-Wno-unused-parameter",
             "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include"), "-I" + CSRC,
             "-I" + os.path.join(HERE, "..", "include")]


def _sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _compile(cmd, log):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "feature flag" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    return log


def _deps(path, seen=None):
    """The file and every quoted #include it reaches, recursively."""
    seen = set() if seen is None else seen
    path = os.path.normpath(path)
    if path in seen or not os.path.exists(path):
        return seen
    seen.add(path)
    with open(path) as f:
        for line in f:
            line = line.strip()
            if line.startswith("#include \""):
                inc = line.split('"')[1]
                _deps(os.path.join(os.path.dirname(path), inc), seen)
    return seen


def _stale(src, obj):
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    return any(os.path.getmtime(d) > t for d in _deps(src))


def build(jobs: int = None, verbose: bool = False, force: bool = True) -> str:
    """Compile the sources and link libperm.so; returns the library path.

    force=False recompiles only objects older than their source or any header.
    """
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    os.makedirs(BUILD, exist_ok=True)
    hip, cpp = _sources()
    tasks = []
    for f in hip:
        obj = os.path.join(BUILD, f + ".o")
        tasks.append(([hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj], obj))
    for f in cpp:
        obj = os.path.join(BUILD, f + ".o")
        tasks.append((["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, f), "-o", obj], obj))
    jobs = jobs or min(len(tasks), max(1, os.cpu_count() or 1), 16)
    # longest translation units first
    order = sorted(tasks, key=lambda t: ("fused" not in t[1], "c128" not in t[1], t[1]))
    if not force:
        order = [(c, o) for c, o in order if _stale(c[-3], o)]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, cmd, obj) for cmd, obj in order]
        for fu in cf.as_completed(futs):
            done = fu.result()
            if verbose:
                print("built", os.path.basename(done), flush=True)
    tmp = LIB + ".tmp"
    link = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp,
            *[o for _, o in tasks], "-L" + os.path.join(ROCM, "lib"), "-lamdhip64",
            "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lpthread"]
    subprocess.run(link, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, force="-f" in sys.argv))
