"""The C-ABI library loads and exports every entry point include/rpmi.h
declares; host-side validation answers without touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rpmi.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    # every function declaration: a return type (rp_status or const char*)
    # followed by the name and its parameter list
    return sorted(set(re.findall(r"^(?:rp_status|const\s+char\s*\*)\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def L():
    import paper_2304_04612_amd as rp
    if not os.path.exists(rp.LIB_PATH):
        from paper_2304_04612_amd import build
        build.build()
    return rp.lib()


def test_header_declares_entry_points():
    names = _declared()
    for n in ("rp_create", "rp_destroy", "rp_project", "rp_omega_generate", "rp_get_device_status", "rsvd",
              "rsvd_batched", "rp_hosvd", "rp_project_grouped", "rp_omega_generate_e4m3"):
        assert n in names


def test_every_declared_symbol_exported(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_status_strings(L):
    import paper_2304_04612_amd as rp
    assert rp.status_string(rp.RP_OK) == "RP_OK"
    assert rp.status_string(rp.RP_ERR_RANGE) == "RP_ERR_RANGE"
    assert rp.status_string(99) == "unknown rp_status"


def test_null_context_rejected_without_gpu(L):
    import paper_2304_04612_amd as rp
    d = rp.rp_desc(0, 4, 4, 4, 4, 1, 0)
    st = L.rp_project(None, ctypes.byref(d), 4, rp.RP_OMEGA_F16, 0, 0, None, 4, None,
                      rp.RP_ALGO_SPLIT_F16, 0, None, 4, None)
    assert st == rp.RP_ERR_INVALID_ARG
    assert b"ctx" in L.rp_last_error(None)
    assert L.rp_omega_generate(None, 0, 0, 4, 4, rp.RP_OMEGA_F16, None, 4, None) == rp.RP_ERR_INVALID_ARG
    assert L.rp_destroy(None) == rp.RP_OK
    out = ctypes.c_void_p()
    assert L.rp_create(None, 0) == rp.RP_ERR_INVALID_ARG


def test_product_path_has_no_oracle_import():
    # the product package must not reach the CPU oracle
    pkg = os.path.join(ROOT, "paper_2304_04612_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
                assert "oracle/" not in src, f
