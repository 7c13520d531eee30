"""The C ABI library loads and exports every function include/sfhe.h declares
(no GPU needed: nothing here calls into the device)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sfhe.h")
LIB = os.path.join(ROOT, "paper_2503_09184_amd", "libsfhe.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfhe_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("sfhe_ctx_create", "sfhe_keygen", "sfhe_encrypt_matrix", "sfhe_matmul", "sfhe_decrypt_matrix",
              "sfhe_export_ct", "sfhe_ntt", "sfhe_keyswitch", "sfhe_rescale", "sfhe_tensor"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_lists_every_declared_symbol():
    from paper_2503_09184_amd import sfhe
    assert sorted(sfhe.EXPORTED) == declared_functions()
    assert sfhe.lib() is not None


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2503_09184_amd import sfhe
    monkeypatch.setattr(sfhe, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sfhe, "_lib", None)
    with pytest.raises(ImportError):
        sfhe.lib()
