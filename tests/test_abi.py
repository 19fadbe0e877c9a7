"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and rejects bad arguments before touching the device."""

import ctypes
import os
import re
import subprocess
import sys

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "sbbf.h")
LIB = os.path.join(ROOT, "paper_2101_01719_amd", "libsbbf.so")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(sbbf_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2101_01719_amd import build

        build.build()
    import paper_2101_01719_amd._lib as L

    return L.load()


def test_header_declares_the_core_api():
    names = _declared_functions()
    for must in ("sbbf_create", "sbbf_insert_batch", "sbbf_lookup_batch", "sbbf_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\bT (sbbf_[a-z0-9_]+)$", out, flags=re.M))
    missing = [n for n in _declared_functions() if n not in exported]
    assert not missing, f"declared but not exported: {missing}"


def test_binding_covers_every_symbol(lib):
    import paper_2101_01719_amd as P
    from paper_2101_01719_amd._lib import SIGNATURES

    for name in _declared_functions():
        assert name in SIGNATURES, f"{name} has no ctypes signature"
        assert hasattr(P, name), f"{name} has no Python function of the same name"


def test_single_hip_runtime_is_mapped(lib):
    maps = open("/proc/self/maps").read()
    paths = set(re.findall(r"\S*libamdhip64\S*", maps))
    assert len(paths) == 1, paths


def test_status_strings_and_sizing(lib):
    assert lib.sbbf_status_string(0) == b"ok"
    assert lib.sbbf_status_string(1) == b"invalid argument"
    assert lib.sbbf_blocks_for(100_000, 10.5) == (21 * 100_000 + 511) // 512
    assert lib.sbbf_blocks_for(0, 10.5) == 1
    assert lib.sbbf_blocks_for(1, 0.0) == 0
    assert lib.sbbf_blocks_for(1 << 40, 1024.0) == 0  # beyond 2**32 - 1 blocks
    assert lib.sbbf_blocks_for(100_000_000, 10.0) == 3906250
    assert lib.sbbf_blocks_for(100_000_001, 10.0) == 3906251


def test_argument_errors_without_device(lib):
    out = ctypes.c_void_p()
    assert lib.sbbf_create(0, ctypes.byref(out)) == 1
    assert b"num_blocks" in lib.sbbf_last_error()
    assert lib.sbbf_create(4, None) == 1
    assert lib.sbbf_create_wrapped(None, 4, ctypes.byref(out)) == 1
    assert lib.sbbf_create_wrapped(ctypes.c_void_p(0x1010), 4, ctypes.byref(out)) == 1  # not 32-byte aligned
    assert b"aligned" in lib.sbbf_last_error()
    assert lib.sbbf_destroy(None) == 1
    assert lib.sbbf_insert_batch(None, None, 10, None) == 1
    assert lib.sbbf_lookup_batch(None, None, 10, None, None) == 1
    assert lib.sbbf_lookup_select(None, None, 10, None, None, None, None) == 1
    assert lib.sbbf_device_query(None) == 1


def test_missing_library_fails_loudly(tmp_path):
    code = (
        "import sys; sys.path.insert(0, %r)\n"
        "import paper_2101_01719_amd._lib as L\n"
        "L.LIB_PATH = %r\n"
        "import paper_2101_01719_amd as P\n"
        "try:\n"
        "    P.sbbf_blocks_for(1, 1.0)\n"
        "except ImportError as e:\n"
        "    print('IMPORT_ERROR', e)\n"
    ) % (ROOT, str(tmp_path / "nope.so"))
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True)
    assert "IMPORT_ERROR" in r.stdout, r.stdout + r.stderr


def test_binding_rejects_unknown_settings():
    """A misspelt setting in a launch, grouped or server dict is an error in
    the binding (ctypes structures would otherwise take it silently)."""
    import paper_2101_01719_amd as P

    with pytest.raises(ValueError, match="unknown launch settings"):
        P._launch(dict(strategy=1, unrol=4))
    assert P._launch(dict(strategy=1, unroll=4)) is not None
