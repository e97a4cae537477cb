"""C-ABI contract checks that need no GPU: the library loads, exports every
symbol include/scmd.h declares, and rejects bad calls on the host side."""
import ctypes
import os
import re

import pytest

from paper_1210_3559_amd import scmd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "scmd.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(scmd_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(scmd.LIB_PATH):
        pytest.fail("libscmd.so is not built: run `python -m paper_1210_3559_amd.build`")
    return scmd.load()


def test_header_declarations_match_binding_list():
    assert _declared() == sorted(scmd.EXPORTS)


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_abi_version(lib):
    text = open(HEADER).read()
    v = int(re.search(r"#define SCMD_ABI_VERSION (\d+)", text).group(1))
    assert scmd.scmd_abi_version() == v


def test_status_strings(lib):
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert scmd.scmd_status_string(code) not in ("", "unknown status")
    assert scmd.scmd_status_string(-99) == "unknown status"


def test_null_context_is_rejected(lib):
    i64 = ctypes.c_int64()
    assert lib.scmd_get_step(None, ctypes.byref(i64)) == scmd.SCMD_EINVAL
    assert lib.scmd_step(None, 1) == scmd.SCMD_EINVAL
    assert lib.scmd_compute(None) == scmd.SCMD_EINVAL
    assert lib.scmd_set_potential(None, None) == scmd.SCMD_EINVAL
    assert lib.scmd_set_integrator(None, 1.0, 0, 0) == scmd.SCMD_EINVAL
    assert lib.scmd_init_clusters(None, 1, None, None, None, 1.0) == scmd.SCMD_EINVAL
    assert lib.scmd_destroy(None) == scmd.SCMD_OK
    assert lib.scmd_create(None, 0, None) == scmd.SCMD_EINVAL


def test_create_without_gpu_reports_device_error(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(scmd.ScmdError) as e:
        scmd.scmd_create(0)
    assert e.value.status == scmd.SCMD_EDEVICE
    assert "device" in e.value.message.lower()


def test_binding_refuses_missing_library(tmp_path):
    saved = scmd._lib
    scmd._lib = None
    try:
        with pytest.raises(RuntimeError, match="build"):
            scmd.load(str(tmp_path / "nope.so"))
    finally:
        scmd._lib = saved
