"""Build libtantrg.so (HIP for gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libtantrg.so")

SOURCES = ["model.cpp", "layout.cpp", "kernels.hip", "bgemm.hip", "engine.hip"]

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result", "-Wno-unused-function",
]


def build(verbose=False):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in SOURCES:
        obj = os.path.join(HERE, "_build", src + ".o")
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        if src.endswith(".cpp"):
            # host-only sources: no device code, plain C++
            cmd = [hipcc, "-O3", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", obj, "-Wall"]
        else:
            cmd = [hipcc] + FLAGS + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = [hipcc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


def build_host_sanitized(out_dir, verbose=False):
    """The library's host code with AddressSanitizer and
    UndefinedBehaviorSanitizer: the planners, the MPO and start builders and
    the host-side bounds checks run instrumented.  The HIP sources are
    compiled for the host only, in relocatable-device-code mode so that the
    device link supplies the (empty) code-object symbols: the build takes
    seconds, and the library serves the host-only entry points
    (tt_check_plans, tt_model_bond_sectors, argument checks) but holds no
    kernels and must not launch any.  Load it in a process that preloads the
    ASan runtime (asan_runtime())."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
    os.makedirs(out_dir, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        if src.endswith(".cpp"):
            cmd = [hipcc, "-O1", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, src), "-o", obj] + san
        else:
            cmd = ([hipcc, "-O1", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-fgpu-rdc",
                    "--offload-host-only", "-Wno-unused-result", "-Wno-unused-function", "-x", "hip", "-c",
                    os.path.join(CSRC, src), "-o", obj] + san)
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    out = os.path.join(out_dir, "libtantrg.so")
    cmd = [hipcc, "-shared", "-fPIC", "-fgpu-rdc", "--hip-link", "--offload-arch=gfx950", "-o", out] + objs + san
    subprocess.run(cmd, check=True)
    return out


def host_sanitized_cached(verbose=False):
    """build_host_sanitized into _build_asan/<digest of the sources and
    flags>, reusing an earlier build of the same sources."""
    import hashlib
    h = hashlib.sha256(" ".join(FLAGS + ["host-only-rdc"]).encode())
    names = sorted(os.listdir(CSRC)) + [os.path.join("..", "..", "include", "tantrg.h")]
    for n in names:
        path = os.path.join(CSRC, n)
        if os.path.isfile(path):
            h.update(n.encode())
            with open(path, "rb") as f:
                h.update(f.read())
    out_dir = os.path.join(HERE, "_build_asan", h.hexdigest()[:16])
    lib = os.path.join(out_dir, "libtantrg.so")
    if not os.path.exists(lib):
        build_host_sanitized(out_dir, verbose)
    return lib


def asan_runtime():
    """Path of the compiler's shared ASan runtime (for LD_PRELOAD)."""
    clang = os.path.join(os.path.dirname(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")), "..", "lib", "llvm",
                         "bin", "clang")
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
