"""Build libfftnk.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1603_08893_amd.build
"""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libfftnk.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
SOURCES = ["fftnk_fft_kernels.hip", "fftnk_solver_kernels.hip", "fftnk_api.hip", "fftnk_stream.hip"]
HEADERS = ["fftnk_internal.h", "fftnk_device.h", "fftnk_j2.h"]

# -packed-fp32-ops: no v_pk_*_f32 instructions anywhere in the device code.
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.isabs(c) and os.path.exists(c) or not os.path.isabs(c)):
            return c
    return "hipcc"


# host code instrumented with AddressSanitizer and UndefinedBehaviorSanitizer
# (each -fsanitize= right after -Xarch_host: the device code is built as usual)
SANITIZE_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(force=True, verbose=False, out=None, sanitize=False):
    """Compile every source to an object in parallel (one hipcc per file), then
    link the shared library (to `out`, default the in-tree library).  With
    sanitize, the host code is built with ASan and UBSan (for the CPU tests of
    the host logic; load it with the compiler's ASan runtime preloaded)."""
    lib_path = out or LIB
    os.makedirs(os.path.dirname(lib_path), exist_ok=True)
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    deps = srcs + [os.path.join(CSRC, h) for h in HEADERS] + [os.path.join(ROOT, "include", "fftnk.h")]
    if not force and os.path.exists(lib_path) and os.path.getmtime(lib_path) >= max(os.path.getmtime(d) for d in deps):
        return lib_path
    objs = [os.path.join(os.path.dirname(lib_path), os.path.basename(s) + ".%d.o" % os.getpid()) for s in srcs]
    compile_flags = [f for f in HIPFLAGS if f != "-shared"] + (SANITIZE_FLAGS if sanitize else [])
    procs = []
    for src, obj in zip(srcs, objs):
        cmd = [hipcc()] + compile_flags + ["-c", "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    failed = False
    for p in procs:
        out, _ = p.communicate()
        if p.returncode != 0:
            sys.stderr.write(out)
            failed = True
    try:
        if failed:
            raise RuntimeError("hipcc failed building libfftnk")
        tmp = lib_path + ".tmp%d" % os.getpid()
        cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + [
            "-L" + os.path.join(ROCM, "lib"), "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + os.path.join(ROCM, "lib")] + (
            ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"] if sanitize else [])
        if verbose:
            print(" ".join(cmd), flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True)
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError("hipcc failed linking libfftnk")
        os.replace(tmp, lib_path)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return lib_path


if __name__ == "__main__":
    print(build(force=True, verbose=True))
