"""CPU checks of the C-ABI library: it loads and exports every declared entry
point (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "alsncg.h")
LIB = os.path.join(ROOT, "paper_1508_03110_amd", "libalsncg.so")


def declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^ALS_API\s+[\w\s\*]*?\b(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_four_hot_path_calls():
    names = declared()
    for n in ("als_sweep", "ncg_gradient", "linesearch_coeffs", "fold_in"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libalsncg.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libalsncg.so not built")
def test_binding_signatures_cover_the_header():
    from paper_1508_03110_amd import _lib
    assert sorted(_lib.EXPORTS) == declared()
    assert _lib.strerror(0) == "ok"
    assert "positive definite" in _lib.strerror(_lib.E_NOT_SPD)


def test_oracle_and_product_share_no_code():
    """The oracle never imports the product and the product never imports
    the oracle (only the seeded generators are shared)."""
    for dirpath, _, files in os.walk(os.path.join(ROOT, "paper_1508_03110_amd")):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.findall(r"^\s*(?:import|from)\s+(\w+)", src, flags=re.M)
                assert "als_oracle" not in src
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c")):
            src = open(os.path.join(ROOT, "oracle", f)).read()
            assert "paper_1508_03110_amd" not in src
            assert "alsncg" not in src
