"""The host side of the library (C ABI, argument checks, workspace arithmetic,
status strings) under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds the host-instrumented library (`build(host_sanitize=True)`: host
sources with -fsanitize=address,undefined on the host pass only, ordinary
kernel objects) and runs the ABI tests against it in a child process with the
clang ASan runtime preloaded. Any sanitizer report ends the child with a
non-zero status (UBSan is built with -fno-sanitize-recover). CPU only."""
import os
import shutil
import subprocess
import sys

import pytest

from paper_1704_08364_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime_or_skip():
    if shutil.which(B.HIPCC) is None and not os.path.exists(B.HIPCC):
        pytest.skip("hipcc not available")
    try:
        return B.host_sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))


def test_abi_tests_pass_under_asan_and_ubsan(tmp_path):
    rt = _runtime_or_skip()
    lib = B.build(host_sanitize=True)
    env = dict(os.environ)
    env.update({
        "BST_LIBRARY": lib,
        "LD_PRELOAD": rt,
        # Python itself is not instrumented and keeps its arenas to the end
        "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:exitcode=86",
        "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1",
    })
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
