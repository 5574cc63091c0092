"""Collected last: with the checked build loaded (BST_LIBRARY pointing at
`python -m paper_1704_08364_amd.build --checked`'s library), no kernel index
check may have failed during the GPU tests that ran before. With the ordinary
build the entry point reports BST_E_UNSUPPORTED and the test is skipped."""
import ctypes as C

import pytest

import paper_1704_08364_amd as P


@pytest.mark.gpu
def test_no_kernel_index_check_failed():
    flags = C.c_uint32(0)
    st = P.lib().bst_debug_check(0, C.byref(flags))
    if st == 8:  # BST_E_UNSUPPORTED: ordinary build
        pytest.skip("ordinary build: the kernels carry no index checks")
    assert st == 0
    assert flags.value == 0, f"index checks failed: 0x{flags.value:08x}"
