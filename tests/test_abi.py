"""The C-ABI library loads and exports every function include/gosma.h declares
(no compute calls: this runs without a GPU)."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def _declared():
    names = set()
    for h in (ROOT / "include").glob("*.h"):
        text = re.sub(r"/\*.*?\*/", "", h.read_text(), flags=re.S)
        names |= set(re.findall(r"\b(gosma_[A-Za-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    for must in ["gosma_create", "gosma_eval_bounds", "gosma_solve", "gosma_set_mixtures"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1812_01232_amd import gosma
    if not gosma.LIB_PATH.exists():
        pytest.skip("libgosma.so not built")
    lib = ctypes.CDLL(str(gosma.LIB_PATH))
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(gosma.EXPORTS) <= set(_declared())


def test_create_rejects_bad_device_without_gpu():
    from paper_1812_01232_amd import gosma
    if not gosma.LIB_PATH.exists():
        pytest.skip("libgosma.so not built")
    h = ctypes.c_void_p()
    assert gosma.lib().gosma_create(-1, ctypes.byref(h)) == -1
    assert gosma.lib().gosma_last_error(None) == b"null context"
