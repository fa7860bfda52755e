"""Build libsrpr.so (the HIP library behind include/sr.h) for gfx950.

Compiles every translation unit under csrc/ with hipcc (the per-length pass
kernels once per supported FFT length, in parallel) and links them into
paper_2409_05734_amd/libsrpr.so.  Run as a script or call build().
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libsrpr.so")

FFT_LENGTHS = (16, 32, 64, 96, 128, 192, 256, 384, 512, 768, 1024, 2048)
SOURCES = ("sr_api.hip", "plan.hip", "dispatch.hip", "util_kernels.hip", "dense.hip", "vjp.hip", "persist.hip", "batched.hip", "fused2d.hip")

ARCH = os.environ.get("SR_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libsrpr)")


def common_flags() -> list:
    return [
        "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
        # keep the compiler from forming packed-FP32 instructions
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
        "-Wno-unused-command-line-argument",
    ]


def _compile(src: str, obj: str, extra: list) -> tuple:
    cmd = [hipcc()] + common_flags() + extra + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    # hipcc's host pass warns about the device-only target feature; drop that noise
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l)
    return r.returncode, " ".join(cmd), err


def build(verbose: bool = False, jobs: int | None = None) -> str:
    os.makedirs(BUILD, exist_ok=True)
    tasks = []
    for n in FFT_LENGTHS:
        for pset in (0, 1):
            tasks.append((os.path.join(CSRC, "passes_inst.hip"), os.path.join(BUILD, f"passes_{n}_{pset}.o"),
                          [f"-DSR_FFT_N={n}", f"-DSR_PASS_SET={pset}"]))
    for s in SOURCES:
        tasks.append((os.path.join(CSRC, s), os.path.join(BUILD, s.replace(".hip", ".o")), []))
    for k in range(4):  # the level kernel, one pass set per translation unit
        tasks.append((os.path.join(CSRC, "batched.hip"), os.path.join(BUILD, f"batched_set{k}.o"),
                      [f"-DSR_LEVEL_SET={k}"]))
    for k, c in ((0, 1), (0, 2), (1, 1), (1, 2)):  # the GD and spectral sets' two length classes
        tasks.append((os.path.join(CSRC, "batched.hip"), os.path.join(BUILD, f"batched_set{k}_cls{c}.o"),
                      [f"-DSR_LEVEL_SET={k}", f"-DSR_LEVEL_CLS={c}"]))
    jobs = jobs or min(16, os.cpu_count() or 4)
    failures = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = {ex.submit(_compile, *t): t for t in tasks}
        for f in cf.as_completed(futs):
            rc, cmd, err = f.result()
            if rc != 0:
                failures.append((cmd, err))
            elif verbose and err.strip():
                print(err, file=sys.stderr)
    if failures:
        msg = "\n\n".join(f"$ {c}\n{e}" for c, e in failures)
        raise RuntimeError("libsrpr build failed:\n" + msg)
    objs = [t[1] for t in tasks]
    tmp = LIB + ".tmp"
    # hipBLASLt: the dense baseline's products where the library GEMM is faster
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "lib")
    cmd = ([hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs +
           ["-L" + rocm_lib, "-lhipblaslt", "-Wl,-rpath," + rocm_lib])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("libsrpr link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


# Host sanitizers (AddressSanitizer, UndefinedBehaviorSanitizer) on the host
# code only: each -fsanitize= applies to the host compilation (-Xarch_host);
# device code is built as usual.  The host-side translation units are rebuilt
# instrumented and linked, with the ordinary pass-kernel objects, into a
# check program that drives the C ABI (csrc/host_check.cpp).
SAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
CHECK = os.path.join(PKG, "sr_host_check")


def build_host_check(jobs: int | None = None) -> str:
    """Build csrc/host_check.cpp against host-sanitized objects (needs build() first)."""
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    tasks = [(os.path.join(CSRC, s), os.path.join(san, s.replace(".hip", ".o")), SAN_FLAGS) for s in SOURCES]
    tasks.append((os.path.join(CSRC, "host_check.cpp"), os.path.join(san, "host_check.o"),
                  SAN_FLAGS + ["-x", "hip"]))
    plain = [os.path.join(BUILD, f"passes_{n}_{pset}.o") for n in FFT_LENGTHS for pset in (0, 1)]
    plain += [os.path.join(BUILD, f"batched_set{k}.o") for k in range(4)]
    plain += [os.path.join(BUILD, f"batched_set{k}_cls{c}.o") for k, c in ((0, 1), (0, 2), (1, 1), (1, 2))]
    missing = [o for o in plain if not os.path.exists(o)]
    if missing:
        raise RuntimeError("run build() first: missing " + ", ".join(missing[:3]))
    jobs = jobs or min(16, os.cpu_count() or 4)
    failures = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for rc, cmd, err in ex.map(lambda t: _compile(*t), tasks):
            if rc != 0:
                failures.append((cmd, err))
    if failures:
        raise RuntimeError("host check build failed:\n" + "\n\n".join(f"$ {c}\n{e}" for c, e in failures))
    rocm_lib = os.path.join(os.path.dirname(os.path.dirname(os.path.realpath(hipcc()))), "lib")
    cmd = ([hipcc(), f"--offload-arch={ARCH}"] + SAN_FLAGS + ["-o", CHECK] + [t[1] for t in tasks] + plain +
           ["-L" + rocm_lib, "-lhipblaslt", "-Wl,-rpath," + rocm_lib])
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("host check link failed:\n" + r.stderr)
    return CHECK


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--host-check" in sys.argv:
        print(build_host_check())
