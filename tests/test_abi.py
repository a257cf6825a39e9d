"""Host-side checks of the C ABI: the library builds/loads, exports every symbol
include/negf.h declares, and rejects bad arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "negf.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(negf_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_1510_04686_amd import build, negf
    if not os.path.exists(build.LIB_PATH):
        build.build(verbose=False)
    return negf.lib()


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for fn in ("negf_lead_selfenergy", "negf_rgf_forward", "negf_rgf_backward", "negf_scba_selfenergy",
               "negf_observables", "negf_create", "negf_bind"):
        assert fn in names


def test_every_declared_symbol_is_exported(lib):
    for fn in _declared():
        assert hasattr(lib, fn), fn


def test_binding_covers_every_declared_symbol():
    from paper_1510_04686_amd import negf
    assert sorted(negf.EXPORTS) == _declared()


def test_create_rejects_bad_config_without_gpu(lib):
    from paper_1510_04686_amd import negf
    h = ctypes.c_void_p()
    for cfg in (negf.negf_config(0, 1, 1, 0), negf.negf_config(8, 0, 1, 0), negf.negf_config(8, 1, 0, 0),
                negf.negf_config(8, 1, 1, 7)):
        assert lib.negf_create(ctypes.byref(cfg), ctypes.byref(h)) == -1
    assert lib.negf_create(None, ctypes.byref(h)) == -1


def test_calls_reject_null_context(lib):
    assert lib.negf_rgf_forward(None, None, 0, 1, None, None, None, None, 0) == -1
    assert lib.negf_rgf_backward(None, None, 0, 1, None, None, None, 0, 1, None, None) == -1
    assert lib.negf_bind(None, None, 1, None) == -1
    assert lib.negf_lead_selfenergy(None, None, 1, None, None, None, 1, None, 0.0, 1e-14, 10, None, None) == -1
    assert lib.negf_lead_selfenergy_pair(None, None, 1, None, None, None, None, None, 1, None, 0.0, 1e-14, 10,
                                         None, None, None, None, None) == -1
    assert lib.negf_scba_selfenergy(None, None, None, None, 1, None, 0, 0, 0, 0, None, None, None) == -1
    assert lib.negf_observables(None, None, None, None, 1, None, None, 2.0, 1, None, None, None, 1) == -1
    assert lib.negf_set_scattering_blocks(None, 10) == -1
    assert lib.negf_zgemm_batched(None, None, 4, 1, 0, 0, None, None, None, 0) == -1
    assert lib.negf_zinv_batched(None, None, 4, 1, None, None, 0) == -1
    assert lib.negf_set_mixed_threshold(None, ctypes.c_double(1e-2)) == -1


def test_error_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, 1, 2, 3, 4):
        assert lib.negf_error_string(code)
    assert lib.negf_error_string(999) == b"unknown status"


def test_library_matches_its_sources(lib):
    """The loaded library was built from the sources in the tree (a stale build
    is refused by negf.lib())."""
    from paper_1510_04686_amd import build
    assert lib.negf_build_id().decode() == build.sources_sha1()


def test_stale_library_is_refused(monkeypatch, lib):
    from paper_1510_04686_amd import negf
    monkeypatch.setattr(negf, "sources_sha1", lambda: "0" * 40)
    monkeypatch.setattr(negf, "_lib", None)
    with pytest.raises(RuntimeError, match="stale"):
        negf.lib()
