"""The C-ABI library loads and exports every function include/msc.h
declares (no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msc.h")
LIB = os.path.join(ROOT, "paper_2409_03771_amd", "libmsc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"#define.*", "", text)
    return sorted(set(re.findall(r"MSC_API\s+[\w\s\*]*?\b(\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("msc_segment", "cc_label_grid", "cc_label_csr",
                 "msc_create", "msc_destroy", "msc_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("libmsc.so not built: python -m paper_2409_03771_amd.build")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    from paper_2409_03771_amd import msc
    assert set(msc.EXPORTS) == set(declared_functions())


def test_strerror_without_gpu():
    from paper_2409_03771_amd import msc
    assert msc._lib.msc_strerror(msc.MSC_ENAN).decode() == "NaN in scalar field"
    assert msc._lib.msc_strerror(12345).decode() == "unknown error"


def test_null_arguments_rejected_before_any_device_call():
    from paper_2409_03771_amd import msc
    assert msc._lib.msc_segment(None, None, None, None, None, None,
                                None) == msc.MSC_EINVAL
    assert msc._lib.cc_label_grid(None, None, None, None, None) == msc.MSC_EINVAL
    assert msc._lib.cc_label_csr(None, 5, None, None, None, None,
                                 None) == msc.MSC_EINVAL
    assert msc._lib.msc_pointer_jump(None, None, 3, 0, 0, None) == msc.MSC_EINVAL
    assert msc._lib.msc_create(None, 0) == msc.MSC_EINVAL
    assert msc._lib.cc_label_grid_batched(None, 1, None, None) == msc.MSC_EINVAL
    assert msc._lib.msc_set_workspace(None, None, 0) == msc.MSC_EINVAL
    assert msc._lib.msc_workspace_size(None, 1, 0, None, None) == msc.MSC_EINVAL


def test_fault_injection_hook_without_gpu():
    """Arming and disarming touch no device; unknown kinds are rejected."""
    from paper_2409_03771_amd import msc
    assert msc._lib.msc_debug_inject(msc.INJECT_ENOMEM, 3) == msc.MSC_OK
    assert msc._lib.msc_debug_inject(msc.INJECT_EHIP, 0) == msc.MSC_OK
    assert msc._lib.msc_debug_inject(7, 0) == msc.MSC_EINVAL
    assert msc._lib.msc_debug_inject(msc.INJECT_ENOMEM, -1) == msc.MSC_OK
    assert msc._lib.msc_debug_inject(msc.INJECT_EHIP, -1) == msc.MSC_OK
