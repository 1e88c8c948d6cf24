"""The C-ABI library builds for gfx950, loads, and exports every symbol the header declares.
No compute call is made (these run without a GPU)."""
import os
import re

import pytest

import paper_2308_07277_amd as qm


def _declared():
    src = open(qm.HEADER_PATH).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(qm.LIB_PATH):
        from paper_2308_07277_amd import build
        build.build()
    return qm._load()


def test_header_declares_the_entry_points():
    names = _declared()
    for required in ("qm_hpsi_plan_create", "qm_apply_h", "qm_davidson_step", "qm_davidson_solve",
                     "qm_hpsi_plan_destroy", "qm_last_error"):
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_create_rejects_null_out(lib):
    # host-side argument check: no device work is started
    import ctypes
    st = lib.qm_hpsi_plan_create(None, None, None, 1, 0, None, None, None, 0, None, None)
    assert st == qm.QM_E_ARG
    assert b"out" in lib.qm_last_error(None)


def test_binding_names_match_abi():
    for n in ("qm_hpsi_plan_create", "qm_apply_h", "qm_davidson_step", "qm_davidson_solve",
              "qm_mlp_forward", "qm_mlp_loss_grad", "qm_mlp_adam", "qm_hpsi_plan_set_precision"):
        assert callable(getattr(qm, n))


def test_struct_sizes_match_header():
    import ctypes
    # qm_dav_opts: double, 4 x int32, double, pointer
    assert ctypes.sizeof(qm.qm_dav_opts) == 8 + 16 + 8 + 8
    assert ctypes.sizeof(qm.qm_dav_stats) == 4 + 4 + 8 + 8 + 5 * 8
    assert ctypes.sizeof(qm.qm_kset) == 8 + 3 * 8
