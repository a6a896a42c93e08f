"""The C-ABI library loads on a machine without a GPU and exports every entry
point include/qcemu.h declares; host-side argument checks need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "qcemu.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(qce_[a-z0-9_]+)\s*\(", text)))


def test_header_declarations_match_binding():
    from paper_2303_08989_amd import _lib
    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    from paper_2303_08989_amd import _lib
    lib = _lib.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_status_strings_and_workspace_size():
    from paper_2303_08989_amd import _lib
    lib = _lib.load()
    assert lib.qce_status_string(0) == b"QCE_SUCCESS"
    assert lib.qce_status_string(2) == b"QCE_ERR_NOT_SUPPORTED"
    assert lib.qce_cgemm_workspace_size(0, 5, 5) == 0
    # two panel buffers, padded to 128 rows and 16 k, 12 bytes per element,
    # and one 144-byte statistics record per operand (rounded to 256 bytes)
    assert lib.qce_cgemm_workspace_size(100, 200, 40) == 128 * 48 * 12 + 256 * 48 * 12 + 512


def test_null_arguments_rejected_without_device():
    from paper_2303_08989_amd import _lib
    lib = _lib.load()
    assert lib.qce_create(None, 0) == 1          # INVALID_VALUE
    assert lib.qce_destroy(None) == 0            # no-op
    assert lib.qce_set_mode(None, 0) == 1
    assert lib.qce_cgemm_emulated(None, 0, 0, 1, 1, 1, None, None, 1, None, 1, None, None, 1) == 1
