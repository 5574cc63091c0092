"""The host side of the library (C ABI, argument checks, workspace arithmetic,
status strings) under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the host-instrumented library (`build(host_sanitize=True)`: host
sources compiled by g++ with -fsanitize=address,undefined, ordinary kernel
objects) and runs the ABI tests against it in a child process with the
ASan runtime preloaded. Any sanitizer report ends the child with a
non-zero status (UBSan is built with -fno-sanitize-recover). CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_1704_08364_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime_or_skip():
    """Skip where hipcc or g++'s sanitizer runtimes are missing."""
    if shutil.which(B.HIPCC) is None and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    try:
        return B.host_sanitizer_preload()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_abi_tests_pass_under_asan_and_ubsan(tmp_path):
    _runtime_or_skip()
    lib = B.build(host_sanitize=True)
    assert lib == B.SAN_LIB
    env = dict(os.environ)
    env.update(B.host_sanitizer_env())
    log = tmp_path / "abi_sanitized.log"
    with open(log, "w") as f:
        r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_abi.py"), "-x", "-q",
                            "-p", "no:cacheprovider", "-m", "not gpu"], cwd=ROOT, env=env, stdout=f,
                           stderr=subprocess.STDOUT, timeout=600)
    text = log.read_text()
    assert "AddressSanitizer" not in text and "runtime error" not in text, text[-4000:]
    assert r.returncode == 0, text[-4000:]
    assert " passed" in text


def test_status_string_takes_any_integer():
    """Regression: the status argument is an integer, so codes outside the
    enumerators are defined behaviour and map to a fixed text."""
    import paper_1704_08364_amd as P
    L = P.lib()
    for code in (-1, 11, 99, 2**31 - 1):
        assert L.bst_status_string(code) == b"unknown status"
