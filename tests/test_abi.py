"""The C-ABI library builds for gfx950, loads, and exports every symbol the header declares.
No compute call is made (these run without a GPU)."""
import os
import re

import pytest

import paper_2308_07277_amd as qm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def test_struct_sizes_match_header(tmp_path):
    """The binding's ctypes structures have the sizes and field offsets the C compiler gives
    the header's structures (a small C program built with gcc prints them)."""
    import ctypes
    import subprocess
    structs = {"qm_dav_opts": qm.qm_dav_opts, "qm_dav_stats": qm.qm_dav_stats, "qm_kset": qm.qm_kset,
               "qm_scf_opts": qm.qm_scf_opts, "qm_scf_stats": qm.qm_scf_stats}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "qm_hpsi.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("  return 0;\n}")
    src = tmp_path / "probe.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "probe"
    inc = os.path.join(ROOT, "include")
    subprocess.run(["gcc", "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert ctypes.sizeof(cls) == int(got[name]), name
        for fname, _ in cls._fields_:
            assert getattr(cls, fname).offset == int(got[f"{name}.{fname}"]), (name, fname)


def test_entry_points_fail_loudly_without_the_library(monkeypatch, tmp_path):
    """With no built library every entry point raises before touching its arguments: there is
    no CPU fallback behind the binding."""
    monkeypatch.setattr(qm, "_LIB", None)
    monkeypatch.setattr(qm, "LIB_PATH", str(tmp_path / "libqm_hpsi.so"))
    calls = [
        lambda: qm.lib_loaded_path(),
        lambda: qm.qm_hpsi_plan_create(None, None, None, None, None, 0, 0, None, None, None),
        lambda: qm.qm_mlp_forward(None, None, None, 0),
        lambda: qm.qm_mlp_loss_grad(None, None, None, None, None, 0, None),
        lambda: qm.qm_mlp_adam(None, None, None, None, 1),
    ]
    for call in calls:
        with pytest.raises(RuntimeError, match="is not built"):
            call()
