"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the C
oracle (key generation, every gate, transforms) and the netlist builder of the
library's host runtime (many shapes, structural checks).  Built with the host
compilers only; no GPU code is involved."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _run(cmd, tmp_path, name, timeout):
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([str(tmp_path / name)], capture_output=True, text=True, timeout=timeout, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-4000:])
    return run.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    out = _run(["gcc", "-std=c11", *SAN, "-o", str(tmp_path / "oracle_san"),
                os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                os.path.join(ROOT, "oracle", "tfhe_oracle.c"), "-lm"], tmp_path, "oracle_san", 600)
    assert "oracle OK" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_netlist_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_2506_12761_amd", "csrc")
    out = _run(["g++", "-std=c++17", *SAN, "-I", csrc, "-o", str(tmp_path / "netlist_san"),
                os.path.join(ROOT, "tests", "sanitize", "netlist_driver.cpp"), os.path.join(csrc, "netlist.cpp")],
               tmp_path, "netlist_san", 300)
    assert "netlist OK" in out
