"""The host logic of the C-ABI library under the address and undefined-
behaviour sanitizers: the library rebuilt with instrumented host code, then
the CPU ABI tests (configuration checks, workspace sizes, the motion
corrector's geometry, every exported symbol) run against it in a child
process with the sanitizer runtime preloaded; any report aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_abi_host_code_under_sanitizers(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_2403_16438_amd"))
    import build
    lib = build.build_sanitized(str(tmp_path / "libseg_san.so"))
    env = dict(os.environ, LD_PRELOAD=build.asan_runtime(), SEG_LIBRARY=lib,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    # the child really runs the instrumented library
    probe = subprocess.run([sys.executable, "-c",
                            "from paper_2403_16438_amd import abi; abi.seg_default_config(8, 8, 100); "
                            "m = open('/proc/self/maps').read(); "
                            "print(int('libseg_san.so' in m and 'libclang_rt.asan' in m))"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert probe.returncode == 0 and probe.stdout.strip().endswith("1"), probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "tests/test_abi_cpu.py", "tests/test_mc_cpu.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
