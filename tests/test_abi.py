"""The C-ABI library loads on any machine and exports every symbol include/ihmc.h declares."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ihmc.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ihmc_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1912_03278_amd import ihmc
    if not os.path.exists(ihmc.LIB_PATH):
        from paper_1912_03278_amd import build
        build.build()
    lib = ctypes.CDLL(ihmc.LIB_PATH)
    names = declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding covers the same set
    assert set(ihmc.EXPORTS) <= set(names)
    assert set(names) <= set(ihmc.EXPORTS), sorted(set(names) - set(ihmc.EXPORTS))


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_1912_03278_amd import ihmc
    monkeypatch.setattr(ihmc, "_lib", None)
    monkeypatch.setattr(ihmc, "LIB_PATH", str(tmp_path / "missing.so"))
    import pytest
    with pytest.raises(ImportError):
        ihmc.load()


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_1912_03278_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ihmc_oracle" not in text, f
