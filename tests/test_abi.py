"""The C-ABI library builds for gfx950, loads, and exports every declared entry point."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "turboreg.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:tr_status|const char \*)\s*(tr_\w+)\s*\(", txt, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared()
    for n in ("tr_create", "tr_destroy", "tr_register", "tr_register_batch", "tr_scorer_load",
              "tr_train_step", "tr_debug_copy", "tr_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2507_01439_amd import turboreg as T
    L = ct.CDLL(T.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing
    assert set(T.EXPORTS) == set(declared())


def test_status_strings_without_gpu():
    from paper_2507_01439_amd import turboreg as T
    assert T.tr_status_string(T.TR_OK) == "ok"
    assert "TurboClique" in T.tr_status_string(T.TR_ERR_NO_HYPOTHESIS)
    assert T.tr_status_string(99) == "unknown status"


def test_code_object_targets_gfx950():
    from paper_2507_01439_amd import turboreg as T
    blob = open(T.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_binding_refuses_host_tensors():
    torch = pytest.importorskip("torch")
    from paper_2507_01439_amd import turboreg as T
    with pytest.raises(ValueError):
        T._ptr(torch.zeros(3))
