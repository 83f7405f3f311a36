"""The C-ABI library loads and exports every entry point include/fe_hx.h declares."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fe_hx.h")).read()
    return sorted(set(re.findall(r"^\s*(?:fe_status|int32_t|const char \*)\s*(fe_\w+)\(", txt, re.M)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("fe_mesh_create", "fe_set_potential", "fe_set_projectors", "fe_apply_H", "fe_cheb_filter"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2512_08571_amd import fehx
    if not os.path.exists(fehx.LIB_PATH):
        pytest.skip("library not built")
    L = fehx.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert set(_declared()) == set(fehx.EXPORTS)
    assert fehx.abi_version() == 2


def test_missing_library_fails_loudly(monkeypatch):
    from paper_2512_08571_amd import fehx
    monkeypatch.setattr(fehx, "_lib", None)
    monkeypatch.setattr(fehx, "LIB_PATH", "/nonexistent/libfehx.so")
    with pytest.raises(RuntimeError):
        fehx.lib()
