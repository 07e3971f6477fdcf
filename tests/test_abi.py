"""The C ABI library builds and exports every entry point include/spvgpu.h
declares (no GPU needed; no compute calls)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "include", "spvgpu.h")
LIB = os.path.join(ROOT, "paper_2305_09493_amd", "libspvgpu.so")


def _declared():
    text = open(HDR).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(spv_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib_path():
    if not os.path.exists(LIB):
        from paper_2305_09493_amd import build
        build.build()
    return LIB


def test_header_declares_the_abi():
    names = _declared()
    for n in ("spv_create", "spv_destroy", "spv_workspace_size", "spv_decode", "spv_validate", "spv_encode",
              "spv_encode_bound"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    out = subprocess.check_output(["nm", "-D", "--defined-only", lib_path], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_library_loads_and_binding_matches(lib_path):
    lib = ctypes.CDLL(lib_path)
    import paper_2305_09493_amd as spv
    for n in _declared():
        assert hasattr(lib, n)
        assert n in spv.EXPORTS


def test_encode_bound_is_host_only(lib_path):
    import paper_2305_09493_amd as spv
    assert spv.encode_bound(2, 10, 20, 3, 41) == 5 * 2 + 10 + 20 + 3 + 10


def test_gpu_tests_are_marked():
    """Every test module that calls into the GPU library marks its tests gpu."""
    tdir = os.path.join(ROOT, "tests")
    for f in os.listdir(tdir):
        if f.startswith("test_gpu") and f.endswith(".py"):
            assert "pytestmark = pytest.mark.gpu" in open(os.path.join(tdir, f)).read(), f


def test_binding_codes_match_header():
    """The binding's result and encode-status constants equal the header's."""
    import re

    import paper_2305_09493_amd as spv
    hdr = open(os.path.join(ROOT, "include", "spvgpu.h")).read()
    defs = {m.group(1): int(m.group(2), 0) for m in re.finditer(r"#define (SPV_E_\w+|SPV_ENC_\w+|SPV_OK)\s+(\w+)", hdr)}
    for name, value in defs.items():
        py = name[len("SPV_"):]
        assert getattr(spv, py) == value, name
    assert {"SPV_E_SPIN_LIMIT", "SPV_ENC_CAPACITY", "SPV_E_UNDEFINED_ID"} <= set(defs)
