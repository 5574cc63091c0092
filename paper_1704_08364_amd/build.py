"""Build the HIP library libbst.so in-tree for gfx950 with hipcc.

Usage: python -m paper_1704_08364_amd.build   (or call build())

`--host-sanitize` (or build(host_sanitize=True)) builds a second library,
_build_hostsan/libbst_hostsan.so: the host sources (C ABI, argument checks,
workspace arithmetic, plan tables, batch graphs) compiled by g++ with
AddressSanitizer and UndefinedBehaviorSanitizer, linked with the ordinary
kernel objects (device code is never instrumented). GCC's ASan runtime leaves
the HSA allocator alone, so the library also runs kernels on a GPU. Load it
in a process started with the variables of host_sanitizer_env().

`--checked` (or build(checked=True)) builds _build_checked/libbst_checked.so
with BST_CHECKED defined: the kernels verify their computed global indices and
record failures for bst_debug_check (load it with BST_LIBRARY=<path>).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJDIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libbst.so")
SAN_DIR = os.path.join(HERE, "_build_hostsan")
SAN_LIB = os.path.join(SAN_DIR, "libbst_hostsan.so")
CHECK_DIR = os.path.join(HERE, "_build_checked")
CHECK_LIB = os.path.join(CHECK_DIR, "libbst_checked.so")

SOURCES = ["bst_api.cpp", "plan_adjoint.cpp", "batch.cpp", "noalloc.hip", "k_spectrum.hip", "k_gather_colifft.hip", "k_row_c2r.hip",
           "k_bruteforce.hip", "k_project.hip", "k_fp64.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ROCM_LIB = "/opt/rocm/lib"   # roctx (trace ranges)
ARCH = os.environ.get("BST_OFFLOAD_ARCH", "gfx950")
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function"]

# host sources only, compiled by g++ (no .hip file on these lines)
GXX = os.environ.get("BST_HOST_CXX", "g++")
SAN_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]
SAN_COMPILE = ["-O1", "-g", "-std=c++17", "-fPIC", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
               f"-I{INCLUDE}", f"-I{CSRC}", "-Wall", "-Wno-unused-function"] + SAN_FLAGS
HOST_SOURCES = [s for s in SOURCES if s.endswith(".cpp")]


def _stale(obj: str, src: str) -> bool:
    """True when obj is missing or older than its source or any header it may include."""
    if not os.path.exists(obj):
        return True
    deps = [os.path.join(CSRC, src)] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")] + [
        os.path.join(INCLUDE, h) for h in os.listdir(INCLUDE)]
    return os.path.getmtime(obj) < max(os.path.getmtime(d) for d in deps)


def _compile(src: str, sanitize: bool = False, checked: bool = False) -> str:
    objdir = SAN_DIR if sanitize else (CHECK_DIR if checked else OBJDIR)
    obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
    if sanitize:
        cmd = [GXX] + SAN_COMPILE + ["-c", os.path.join(CSRC, src), "-o", obj]
    else:
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        extra = ["-DBST_CHECKED"] if checked else []
        cmd = [HIPCC] + COMMON + extra + lang + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed for {src}:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def host_sanitizer_preload() -> str:
    """LD_PRELOAD value for a process that loads the host-sanitizer library: the
    ASan runtime of the g++ that built it, then libstdc++ (ASan resolves its
    C++ exception interceptor at start-up, and Python does not load libstdc++
    itself)."""
    paths = []
    for name in ("libasan.so", "libstdc++.so.6"):
        r = subprocess.run([GXX, f"-print-file-name={name}"], capture_output=True, text=True)
        path = r.stdout.strip()
        if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
            raise RuntimeError(f"{name} of {GXX} not found")
        paths.append(path)
    return " ".join(paths)


def host_sanitizer_env(log_dir: str | None = None) -> dict:
    """Environment additions for a process that runs the host-sanitizer library.

    Besides BST_LIBRARY and LD_PRELOAD: torch's lib directory goes on
    LD_LIBRARY_PATH, because under ASan's dlopen interceptor torch's own
    $ORIGIN-relative dlopen calls (its runtime-compiler stub) no longer find
    their files; leak checking is off (Python is not instrumented and keeps its
    arenas to the end); every report ends the process with status 86 (ASan) or
    a non-zero status (UBSan), written to log_dir when given."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    torch_lib = os.path.join(os.path.dirname(spec.origin), "lib") if spec and spec.origin else ""
    asan = "detect_leaks=0:exitcode=86"
    ubsan = "print_stacktrace=1:halt_on_error=1"
    if log_dir:
        asan += f":log_path={os.path.join(log_dir, 'asan')}"
        ubsan += f":log_path={os.path.join(log_dir, 'ubsan')}"
    ld = os.environ.get("LD_LIBRARY_PATH", "")
    # the ASan runtime must come first; anything already preloaded stays
    pre = " ".join(x for x in (host_sanitizer_preload(), os.environ.get("LD_PRELOAD", "")) if x)
    return {"BST_LIBRARY": SAN_LIB, "LD_PRELOAD": pre,
            "LD_LIBRARY_PATH": ":".join(x for x in (torch_lib, ld) if x),
            "ASAN_OPTIONS": asan, "UBSAN_OPTIONS": ubsan}


def build(verbose: bool = False, host_sanitize: bool = False, checked: bool = False) -> str:
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    out = SAN_LIB if host_sanitize else (CHECK_LIB if checked else LIB)
    os.makedirs(SAN_DIR if host_sanitize else (CHECK_DIR if checked else OBJDIR), exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    if host_sanitize:
        # instrumented host sources + the ordinary kernel objects (rebuilt only when stale)
        os.makedirs(OBJDIR, exist_ok=True)
        kern = [s for s in SOURCES if s not in HOST_SOURCES]
        todo = [s for s in kern if _stale(os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o"), s)]
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            list(ex.map(_compile, todo))
            objs = list(ex.map(lambda src: _compile(src, True), HOST_SOURCES))
        objs += [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in kern]
    else:
        with ThreadPoolExecutor(max_workers=jobs) as ex:
            objs = list(ex.map(lambda src: _compile(src, checked=checked), SOURCES))
    tmp = out + ".tmp"
    libs = [f"-L{ROCM_LIB}", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM_LIB}"]
    if host_sanitize:
        cmd = [GXX, "-shared", "-fPIC", "-o", tmp] + objs + libs + ["-lamdhip64"] + SAN_FLAGS
    else:
        cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs + libs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, out)
    if verbose:
        print(f"built {out}")
    return out


if __name__ == "__main__":
    build(verbose=True, host_sanitize="--host-sanitize" in sys.argv[1:], checked="--checked" in sys.argv[1:])
    sys.exit(0)
