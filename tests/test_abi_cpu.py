"""CPU-side checks of the C ABI library (no GPU needed).

* the built library loads and exports every function ``include/mskm.h`` declares;
* calls that need no device fail cleanly with the documented status codes.
"""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mskm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mskm_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2503_04914_amd as m

    try:
        return m.lib()
    except m.MskmLibraryMissing:
        pytest.fail("libmskm.so is not built (run python -m paper_2503_04914_amd.build)")


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mskm_create", "mskm_destroy", "mskm_hier_create", "mskm_hier_destroy", "mskm_export_block",
                     "mskm_solve", "mskm_residual", "mskm_evaluate", "mskm_apply", "mskm_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    import paper_2503_04914_amd as m

    for n in declared_functions():
        assert hasattr(m, n), n


def test_abi_version(lib):
    import paper_2503_04914_amd as m

    assert m.mskm_abi_version() == 3


def test_null_arguments_are_rejected(lib):
    import paper_2503_04914_amd as m

    assert lib.mskm_create(0, None, None) == m.MSKM_EINVAL
    assert "NULL" in m.mskm_last_error()
    assert lib.mskm_solve(None, None, None, 1, None, None, None) == m.MSKM_EINVAL
    assert lib.mskm_hier_stats_get(None, None) == m.MSKM_EINVAL
    assert lib.mskm_destroy(None) == m.MSKM_OK
    assert lib.mskm_hier_destroy(None) == m.MSKM_OK


def test_create_without_device_reports_edevice(lib):
    import paper_2503_04914_amd as m

    try:
        import torch

        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    out = C.c_void_p()
    assert lib.mskm_create(0, None, C.byref(out)) == m.MSKM_EDEVICE
    assert out.value is None


def test_solve_opts_defaults(lib):
    import paper_2503_04914_amd as m

    o = m.mskm_solve_opts_default()
    assert o.precision == m.MSKM_PREC_FP64 and o.algorithm == m.MSKM_ALG_MONOLITHIC
    assert o.cg_rtol == 1e-12 and o.sweeps == 0 and o.target_rel_residual == 1e-8


def test_torch_stream_must_not_be_the_default_stream(lib, monkeypatch):
    """stream="torch" shares torch's current stream with the library; torch's
    default stream has a null handle, which the C ABI reads as "create a
    stream of your own" (unordered with torch's work), so the binding refuses
    it before any call into the library."""
    import paper_2503_04914_amd as m
    import torch

    class _Default:
        cuda_stream = 0

    monkeypatch.setattr(torch.cuda, "current_stream", lambda device=None: _Default())
    with pytest.raises(ValueError, match="default stream"):
        m.mskm_create(0, stream="torch")
