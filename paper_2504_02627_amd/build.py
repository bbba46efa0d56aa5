"""Build libchees_smc.so (HIP, gfx950) in-tree with hipcc."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libchees_smc.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("smc_kernels.hip", "flow_kernels.hip", "target_kernels.hip", "smc_api.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions off: some of their forms have given wrong
    # results on this hardware without an error
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


def build(verbose=False):
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(ROOT, "include"),
                                     "-I", os.path.join(HERE, "csrc")] + SOURCES + ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitized(out):
    """The same library with the host code under AddressSanitizer and
    UndefinedBehaviorSanitizer (device code unchanged), for CPU tests of the
    validation and planning paths.  Load it with the ASan runtime preloaded
    (sanitizer_runtime())."""
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + [
        "-O1", "-g",
        "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-omit-frame-pointer",
    ]
    cmd = [hipcc()] + flags + ["-I", os.path.join(ROOT, "include"),
                               "-I", os.path.join(HERE, "csrc")] + SOURCES + ["-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    return str(out)


def sanitizer_runtime():
    """Path of the compiler's AddressSanitizer runtime, or None."""
    import glob
    base = os.path.join(os.path.dirname(os.path.dirname(hipcc())) if os.path.isabs(hipcc())
                        else "/opt/rocm", "llvm", "lib", "clang")
    hits = sorted(glob.glob(os.path.join(base, "*", "lib", "linux", "libclang_rt.asan-x86_64.so")))
    return hits[-1] if hits else None


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
