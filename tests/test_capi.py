"""The C ABI used from C: a plain C program against include/vlp.h and
libvlp.so (no Python in the path).  The CPU suite compiles and links it; on
the GPU the program built by the build step runs and checks bootstrap and key
switching of trivial ciphertexts against their closed form, plus the error
paths of context creation and of a gate call."""
import os
import subprocess
import sys

import pytest

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "capi"))
import capi_build as capi  # noqa: E402


def test_c_program_builds_against_the_abi(tmp_path):
    if capi.missing():
        pytest.skip(capi.missing())
    assert os.path.exists(capi.build(str(tmp_path / "vlp_capi_demo")))


@pytest.mark.gpu
def test_c_program_runs():
    assert os.path.exists(capi.EXE), "run the build step first (it compiles tests/capi/vlp_capi_demo)"
    r = subprocess.run([capi.EXE], capture_output=True, text=True, timeout=240)
    assert r.returncode == 0 and "C ABI OK" in r.stdout, (r.stdout[-2000:], r.stderr[-2000:])
