"""The C-ABI library loads and exports every function include/boltzmc.h declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "boltzmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(bmc_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("bmc_create", "bmc_collision", "bmc_step", "bmc_vjp", "bmc_workspace_bind", "bmc_set_f"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2603_28848_amd import boltzmc
    if not os.path.exists(boltzmc.LIB_PATH):
        pytest.skip("libboltzmc.so not built")
    lib = ctypes.CDLL(boltzmc.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(boltzmc.exported_symbols())
    lib.bmc_version.restype = ctypes.c_char_p
    assert lib.bmc_version().startswith(b"boltzmc")


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2603_28848_amd import boltzmc
    monkeypatch.setattr(boltzmc, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(boltzmc, "_lib", None)
    with pytest.raises(RuntimeError):
        boltzmc.lib()
