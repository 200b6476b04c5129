"""CPU-side checks of the C ABI: the library loads and exports every function
that include/gcme.h declares; the Python binding uses the same names; the
package refuses to run without the built library."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gcme.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gcme_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["gcme_create", "gcme_set_params", "gcme_forces_energy", "gcme_step"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2403_08148_amd import _binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(B.LIB_PATH)
    for n in declared_functions():
        assert hasattr(lib, n), n
    assert sorted(B.EXPORTED) == declared_functions()


def test_status_codes_match_header():
    from paper_2403_08148_amd import _binding as B
    src = open(HEADER).read()
    for name, val in re.findall(r"(GCME_E[A-Z]+|GCME_OK)\s*=\s*(\d+)", src):
        if name.startswith("GCME_E_"):
            continue
        assert getattr(B, name) == int(val), name
    for name, val in re.findall(r"(GCME_E_[A-Z]+)\s*=\s*(\d+)", src):
        assert getattr(B, name) == int(val), name


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2403_08148_amd import _binding as B
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError):
        B.load()
