"""Builds libmact.so (the HIP library behind the C ABI of include/mact.h) in
place, for gfx950, with hipcc.

    python -m paper_1009_0854_amd.build [--jobs N] [--sanitize]

Sources are compiled in parallel to objects under _build/ and linked into
paper_1009_0854_amd/libmact.so.  Every call rebuilds every object.

--sanitize builds libmact_san.so instead (objects under _build_san/): the
host code (the C++ sources and the host side of the HIP sources) with
AddressSanitizer and UndefinedBehaviorSanitizer, UB fatal; device code as
usual.  A process loads it with MACT_LIB_VARIANT=san and the clang ASan
runtime preloaded (``sanitizer_runtime()``).
"""
import argparse
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libmact.so")
BUILD = os.path.join(ROOT, "_build")
OUT_SAN = os.path.join(HERE, "libmact_san.so")
BUILD_SAN = os.path.join(ROOT, "_build_san")
# host-only sanitizers: each flag behind -Xarch_host, so no device code is instrumented
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

HIP_SOURCES = ["xform.hip", "gather.hip", "lut.hip", "batch.hip", "serve.hip", "inverse.hip", "exact.hip"]
CPP_SOURCES = ["remez.cpp", "host.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include")]
# Device code: no packed-FP32 instructions (see the build notes in the design document).
HIP_FLAGS = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-fno-gpu-rdc", "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    # the host pass does not know the device-only target feature: drop that warning only
    lines = [l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l and "unknown target feature" not in l]
    return r.returncode, "\n".join(lines)


def sources():
    return [s for s in HIP_SOURCES + CPP_SOURCES if os.path.exists(os.path.join(CSRC, s))]


def sanitizer_runtime():
    """Path of the clang AddressSanitizer runtime that a process loading
    libmact_san.so must preload (it carries the UB handlers too)."""
    import glob
    hits = sorted(glob.glob(os.path.join(os.path.dirname(os.path.dirname(HIPCC)), "llvm", "lib", "clang", "*", "lib",
                                         "linux", "libclang_rt.asan-x86_64.so")))
    return hits[-1] if hits else None


def build(jobs=8, verbose=False, sanitize=False):
    build_dir, out = (BUILD_SAN, OUT_SAN) if sanitize else (BUILD, OUT)
    extra = SAN_FLAGS if sanitize else []
    os.makedirs(build_dir, exist_ok=True)
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_gamma.py"), os.path.join(CSRC, "gamma_table.inc")])
    cmds = []
    objs = []
    for s in sources():
        src = os.path.join(CSRC, s)
        obj = os.path.join(build_dir, s + ".o")
        objs.append(obj)
        if s.endswith(".hip"):
            cmd = [HIPCC] + COMMON + HIP_FLAGS + extra + ["-c", src, "-o", obj]
        else:
            cmd = [HIPCC, "-x", "c++"] + COMMON + extra + ["-c", src, "-o", obj]
        cmds.append(cmd)
    with cf.ThreadPoolExecutor(max(1, jobs)) as ex:
        results = list(ex.map(_run, cmds))
    failed = False
    for cmd, (rc, text) in zip(cmds, results):
        if verbose or rc != 0:
            print(" ".join(cmd))
        if text.strip():
            print(text)
        failed |= rc != 0
    if failed:
        raise RuntimeError("libmact: compilation failed")
    tmp = out + ".tmp"
    link = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if sanitize:
        link += ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libasan"]
    rc, msg = _run(link)
    if msg.strip():
        print(msg)
    if rc != 0:
        raise RuntimeError("libmact: link failed")
    os.replace(tmp, out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("-v", "--verbose", action="store_true")
    ap.add_argument("--sanitize", action="store_true")
    a = ap.parse_args()
    print(build(a.jobs, a.verbose, a.sanitize))


if __name__ == "__main__":
    main()
