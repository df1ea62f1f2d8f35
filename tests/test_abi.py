"""Host side of the C ABI (no GPU needed): the library loads, exports every
entry point the header declares, and the host-only paths behave."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bcts.h")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(bcts_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2107_01715_amd import bcts
    return bcts


def test_header_declares_the_binding(lib):
    assert declared() == sorted(lib.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in declared():
        assert hasattr(so, name), name


def test_null_context_is_rejected(lib):
    assert lib._reset(None) == lib.E_INVAL
    assert lib._set_precision(None, 0) == lib.E_INVAL
    assert lib._search(None, 1, None, None, 1, 4, 0.9, lib.correction(), None, None) == lib.E_INVAL
    assert lib.bcts_last_error(None) == "null context"


def test_request_bytes(lib):
    assert lib.bcts_request_bytes(7, 4) == 0 and lib.bcts_request_bytes(2, 19) == 0
    b = [lib.bcts_request_bytes(d, 6) for d in range(0, 5)]
    assert all(y > x for x, y in zip(b, b[1:]))
    # an A=18, d=3 tree holds 18 + 324 + 5832 new frames of 7056 bytes
    assert lib.bcts_request_bytes(3, 18) >= (18 + 324 + 5832) * 7056


def test_create_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(lib.BctsError) as e:
        lib.bcts_create(0)
    assert e.value.status == lib.E_HIP
