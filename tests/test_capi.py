"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every entry point that include/fastmusic.h declares, and its pure host
helpers behave."""
import ctypes as C
import os
import re

import pytest

import paper_1911_07434_amd as fm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fastmusic.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fm_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(fm.LIB_PATH):
        pytest.fail("libfastmusic.so is not built (run __graft_entry__.build())")
    return fm.load_library()


def test_header_declares_the_five_stage_calls():
    names = header_functions()
    for n in ("fm_covariance", "fm_subspace_sample", "fm_subspace_project",
              "fm_pseudospectrum", "fm_peaks"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    names = header_functions()
    assert set(names) == set(fm.EXPORTS)
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    assert lib.fm_status_string(0) == b"ok"
    assert lib.fm_status_string(1) == b"invalid argument"
    assert lib.fm_status_string(99) == b"unknown status"


def test_workspace_bytes_grows_with_shape(lib):
    a = lib.fm_workspace_bytes(1024, 16, 8, 18001)
    b = lib.fm_workspace_bytes(4096, 24, 16, 36001)
    assert 0 < a < b
    assert lib.fm_workspace_bytes(0, 16, 8, 100) == 0
    assert a % 256 == 0


def test_null_context_is_rejected(lib):
    assert lib.fm_covariance(None, None, None, 4, 4, 4, None, 4, 0) == fm.FM_E_ARG
    assert lib.fm_peaks(None, None, None, 4, 1, None, None, None) == fm.FM_E_ARG
    assert lib.fm_last_error(None) == b""
    out = C.c_void_p()
    assert lib.fm_create(-1, 0, C.byref(out)) != fm.FM_OK
    assert not out.value


def test_fm_frame_layout_matches_header():
    # the ctypes mirror must list the C struct's fields in order
    text = open(HEADER).read()
    body = re.search(r"typedef struct \{(.*?)\} fm_frame;", text, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        names = decl.split()[-1] if "," not in decl else decl
        for part in re.split(r",", decl):
            fields.append(re.sub(r"[*\s]", " ", part).split()[-1])
    assert fields == [f[0] for f in fm.fm_frame._fields_]
