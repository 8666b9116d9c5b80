"""Build the HIP library ``liblbm.so`` in-tree for gfx950 with hipcc.

``build()`` keeps its object files in ``_build/``.  ``build_host_sanitized``
links another copy of the library whose host code in ``lbm_host.hip`` (the
C ABI and its argument checks) carries AddressSanitizer and
UndefinedBehaviorSanitizer; the kernel objects are those of ``build()``.
That copy loads only in a process with clang's ASan runtime preloaded
(``asan_runtime()``), through ``LBM_LIBRARY``.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["kernels.hip", "adjoint.hip", "lbm_host.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    # keep the compiler from emitting packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one source expression, so that every
    # instantiation of a kernel (pointer or buffer addressing, with or without
    # the density and velocity record of the adjoint's recompute) rounds the
    # same arithmetic the same way and their results are bit-identical
    "-ffp-contract=on",
    "-Wno-unused-result",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    os.makedirs(OBJDIR, exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd, stderr=subprocess.PIPE, text=True), src))
        objs.append(obj)
    for p, src in procs:
        _, err = p.communicate()
        err = "\n".join(l for l in err.splitlines() if "packed-fp32-ops" not in l and "ignoring feature" not in l)
        if p.returncode != 0:
            sys.stderr.write(err + "\n")
            raise RuntimeError("hipcc failed on " + src)
        if verbose and err.strip():
            print(err)
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", LIB + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


# host code only: -Xarch_host keeps the sanitizers out of the device code
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
                 "-Xarch_host", "-g"]


def _objects_current() -> bool:
    inputs = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.abspath(__file__)]
    newest = max(os.path.getmtime(f) for f in inputs)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    return all(os.path.exists(o) and os.path.getmtime(o) >= newest for o in objs)


def build_host_sanitized(outdir: str, verbose: bool = False) -> str:
    """Write ``outdir/liblbm.so`` with the sanitized host code (builds the
    kernel objects first when they are missing or older than a source)."""
    if not _objects_current():
        build(verbose)
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    obj = os.path.join(outdir, "lbm_host_san.o")
    cmd = [hipcc, *HIPCC_FLAGS, *SANITIZE_HOST, "-c", os.path.join(CSRC, "lbm_host.hip"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    p = subprocess.run(cmd, capture_output=True, text=True)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on lbm_host.hip (host sanitizers):\n" + p.stderr)
    out = os.path.join(outdir, "liblbm.so")
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES if s != "lbm_host.hip"]
    subprocess.run([hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out, *objs, obj], check=True)
    return out


def asan_runtime() -> str:
    """Path of the ASan runtime of hipcc's compiler."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise FileNotFoundError("no libclang_rt.asan-x86_64.so under /opt/rocm/llvm")
    return hits[-1]


if __name__ == "__main__":
    build(verbose=True)
