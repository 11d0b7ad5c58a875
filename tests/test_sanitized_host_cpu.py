"""The host code (ligand preparation and the C ABI's validation) under
AddressSanitizer and UBSan: the sanitizer build (build_lib.build_sanitized:
g++ -fsanitize=address,undefined, kernel launchers replaced by host
stand-ins) runs every CPU test of the C ABI (tests/test_abi_cpu.py: the
named workloads, the 64 ligands of the uneven batch, the hand-worked
goldens, the edge sizes 1..128 and every validation path) in a child
process; any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    gcc = shutil.which("gcc")
    if not gcc:
        return None
    p = subprocess.run([gcc, f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_host_code_under_asan_and_ubsan():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan and shutil.which("g++")):
        pytest.skip("g++ with the ASan/UBSan runtimes is not available")
    from paper_2410_10447_amd import build_lib
    lib = build_lib.build_sanitized()
    env = dict(os.environ)
    env.update({"DOCKMI_LIB": lib, "LD_PRELOAD": f"{asan} {ubsan}",
                "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1",
                "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"})
    probe = subprocess.run([sys.executable, "-c", "from paper_2410_10447_amd import dock; dock.lib(); "
                            "print(dock._LIB_PATH)"], cwd=ROOT, env=env, capture_output=True, text=True,
                           timeout=300)
    assert probe.returncode == 0 and probe.stdout.strip() == lib, probe.stdout + probe.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    print(out[-2000:])
    assert "AddressSanitizer" not in out and "runtime error" not in out
    assert r.returncode == 0 and " passed" in out
