"""Build libseg.so (HIP kernels + C ABI) for gfx950 in the package directory.

    python paper_2403_16438_amd/build.py      (or __graft_entry__.build())

Every call compiles from source: the compare-exchange network header is
regenerated, then hipcc compiles and links all sources into one shared library.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libseg.so")
SOURCES = ["seg_api.cpp", "k_stream.hip", "k_finalize.hip", "k_nmf.hip", "k_nmf_split.hip", "k_traces.hip", "k_motion.hip", "mc_api.cpp", "nn_api.cpp", "k_nn.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build(verbose: bool = False) -> str:
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_selnet.py"),
                    os.path.join(CSRC, "selnet_gen.h")], check=True,
                   stdout=None if verbose else subprocess.DEVNULL)
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in (r.stdout + r.stderr).splitlines()
                     if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + errs)
    if verbose and errs.strip():
        print(errs)
    os.replace(tmp, LIB)
    return LIB


def asan_runtime() -> str:
    """Path of the toolchain's address-sanitizer runtime (to preload into a
    Python process that loads the sanitized library)."""
    return subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                          text=True, check=True).stdout.strip()


def build_sanitized(out: str) -> str:
    """The same library with its host code instrumented by the address and
    undefined-behaviour sanitizers (device code unchanged), for the CPU
    checks of the host logic; load it with SEG_LIBRARY=<out> and the runtime
    of asan_runtime() preloaded."""
    subprocess.run([sys.executable, os.path.join(CSRC, "gen_selnet.py"), os.path.join(CSRC, "selnet_gen.h")],
                   check=True, stdout=subprocess.DEVNULL)
    host_only = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined"
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + host_only.split() + [
        "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan"]
    cmd = [HIPCC] + flags + [os.path.join(CSRC, s) for s in SOURCES] + ["-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + r.stdout + r.stderr)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
