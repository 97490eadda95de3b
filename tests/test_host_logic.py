"""Host-side checks that need no GPU: the closed-form tile count of the prefix
scans (compiled from the library's own header with hipcc and run on the CPU), and
the CPU oracle built with AddressSanitizer and UndefinedBehaviorSanitizer and
driven through every entry point."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and not shutil.which("hipcc"), reason="hipcc not available")
def test_closed_form_tile_count_equals_bucket_walk(tmp_path):
    exe = str(tmp_path / "tiles_for_check")
    src = os.path.join(ROOT, "tests", "host", "tiles_for_check.cpp")
    cmd = [HIPCC, "-O2", "-std=c++17", "-x", "hip", "--offload-arch=gfx950",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2209_00103_amd", "csrc"),
           src, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("ok"), r.stdout + r.stderr


def _sanitizers_available(tmp_path) -> bool:
    probe = tmp_path / "probe.c"
    probe.write_text("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", str(probe), "-o", str(tmp_path / "probe")],
                       capture_output=True, text=True)
    return r.returncode == 0


def test_oracle_under_address_and_ub_sanitizers(tmp_path):
    if not shutil.which("gcc") or not _sanitizers_available(tmp_path):
        pytest.skip("gcc with sanitizer runtimes not available")
    exe = str(tmp_path / "oracle_sanitize_driver")
    src = os.path.join(ROOT, "tests", "host", "oracle_sanitize_driver.c")
    r = subprocess.run(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-Wall", "-Wextra", src, "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout + r.stderr)[-3000:]
