"""Host-side checks of the boundary (no GPU needed): the C-ABI library loads,
exports every entry point its header declares, and the product package never
reaches the oracle."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "liblabs.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(labs_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_2504_00987_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2504_00987_amd import build
        build.build()
    return _lib.load()


def test_header_declares_the_boundary():
    names = _declared()
    for want in ("labs_energy_batch", "labs_tabu_batch", "labs_memetic_run", "labs_create",
                 "labs_server_submit"):
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    from paper_2504_00987_amd import _lib
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTED) == _declared()


def test_library_reports_without_a_device(lib):
    import ctypes
    assert lib.labs_version().startswith(b"liblabs")
    assert lib.labs_status_name(1) == b"LABS_E_INVAL"
    h = ctypes.c_void_p()
    # a device ordinal that does not exist is rejected, never a crash
    assert lib.labs_create(ctypes.byref(h), 999) == 1


def test_struct_layouts_match_header():
    import ctypes
    from paper_2504_00987_amd import _lib
    assert ctypes.sizeof(_lib.TabuParams) == 56
    assert ctypes.sizeof(_lib.Launch) == 20
    # K, p_comb, mut_rule, p_mut (16) + tabu (56) + generations (8, aligned at 72) + 7 ints, padded to 8
    assert ctypes.sizeof(_lib.MemeticParams) == 112


def test_limits_match_header():
    import re
    from paper_2504_00987_amd import _lib
    text = open(os.path.join(ROOT, "include", "liblabs.h")).read()
    val = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define (LABS_\w+) (\d+)", text)}
    assert (val["LABS_MIN_N"], val["LABS_MAX_N"], val["LABS_MAX_K"]) == (_lib.MIN_N, _lib.MAX_N, _lib.MAX_K)


def test_product_package_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2504_00987_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h", ".hpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "inputs.py", f
