"""Build libpw.so in-tree with hipcc for gfx950.

Usage: python -m paper_2102_08384_amd.build  [--jobs N]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libpw.so")
BUILD_DIR = os.path.join(HERE, "_build")

SOURCES = ["generated.hip", "kernels.hip", "inverse.hip", "paint.hip", "coeffs.cpp", "plan.cpp", "api.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

COMMON = ["-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
          "-I", os.path.join(ROOT, "include"), "-I", BUILD_DIR,
          # no packed-FP32 instructions in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wno-unused-command-line-argument"]


def _deps_mtime() -> float:
    """Newest mtime of the headers every translation unit may include."""
    paths = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    paths += [os.path.join(ROOT, "include", "pw.h"), os.path.join(BUILD_DIR, "contract_gen.inc"),
              os.path.abspath(__file__)]  # compile flags live here
    return max(os.path.getmtime(p) for p in paths if os.path.exists(p))


def _compile(src: str, incremental: bool = False) -> str:
    obj = os.path.join(BUILD_DIR, os.path.basename(src) + ".o")
    if incremental and os.path.exists(obj):
        newest = max(os.path.getmtime(os.path.join(CSRC, src)), _deps_mtime())
        if os.path.getmtime(obj) > newest:
            return obj
    cmd = [HIPCC] + COMMON + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd = [HIPCC] + COMMON + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def _generate():
    """Build and run the host-only generator of the register-resident contraction."""
    exe = os.path.join(BUILD_DIR, "gen_contract")
    cmd = ["g++", "-O2", "-std=c++17", os.path.join(CSRC, "coeffs.cpp"),
           os.path.join(CSRC, "gen_contract.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"generator build failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    out = os.path.join(BUILD_DIR, "contract_gen.inc")
    tmp = out + ".new"
    r = subprocess.run([exe, tmp], capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"generator failed\n{r.stdout}\n{r.stderr}")
    # keep the old file (and its mtime) when nothing changed
    if os.path.exists(out) and open(out).read() == open(tmp).read():
        os.remove(tmp)
    else:
        os.replace(tmp, out)


def build(jobs: int | None = None, verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source for gfx950 and link libpw.so (incremental: reuse up-to-date
    objects; the default rebuilds everything)."""
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        raise RuntimeError("hipcc not found")
    os.makedirs(BUILD_DIR, exist_ok=True)
    _generate()
    jobs = jobs or min(8, os.cpu_count() or 4)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, incremental), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libpw_san.so")
# host code under AddressSanitizer and UndefinedBehaviorSanitizer (device code is built as usual;
# the sanitized library serves host-only checks on a machine without a GPU)
SAN_FLAGS = ["-O1", "-g", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-shared-libsan", "-I", os.path.join(ROOT, "include"), "-I", BUILD_DIR,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-command-line-argument"]


def sanitizer_runtime() -> str:
    """The compiler's shared AddressSanitizer runtime (to preload into a host process)."""
    r = subprocess.run([os.path.join(os.path.dirname(HIPCC), "..", "llvm", "bin", "clang"),
                        "--print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path):
        import glob
        cands = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        path = cands[0] if cands else ""
    if not os.path.exists(path):
        raise RuntimeError("AddressSanitizer runtime not found")
    return path


def build_sanitized(jobs: int | None = None) -> str:
    """Host-only build of every source with AddressSanitizer + UndefinedBehaviorSanitizer into
    _build_san/libpw_san.so (rebuilt when a source or header is newer)."""
    os.makedirs(SAN_DIR, exist_ok=True)
    os.makedirs(BUILD_DIR, exist_ok=True)
    _generate()
    newest = max([_deps_mtime()] + [os.path.getmtime(os.path.join(CSRC, f)) for f in SOURCES])

    def one(src):
        obj = os.path.join(SAN_DIR, os.path.basename(src) + ".o")
        if os.path.exists(obj) and os.path.getmtime(obj) > newest:
            return obj
        cmd = [HIPCC] + SAN_FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=jobs or min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(one, SOURCES))
    if os.path.exists(SAN_LIB) and os.path.getmtime(SAN_LIB) > max(os.path.getmtime(o) for o in objs):
        return SAN_LIB
    tmp = SAN_LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--incremental", action="store_true")
    ap.add_argument("--sanitized", action="store_true",
                    help="host-only AddressSanitizer/UBSan build into _build_san/ (no device code)")
    a = ap.parse_args()
    if a.sanitized:
        print("built", build_sanitized(a.jobs))
    else:
        build(a.jobs, verbose=True, incremental=a.incremental)
    sys.exit(0)
