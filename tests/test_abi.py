"""CPU checks of the C-ABI boundary: the built library loads and exports every
symbol declared in include/pw.h, and the ctypes structures of the Python binding
match the C layout (sizes and field offsets compiled from the header by gcc)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2002_00088_amd import pw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pw.h")


def declared_symbols():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:pw_status|const char \*|void)\s*(pw_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    if not os.path.exists(pw.LIB):
        pytest.fail("libpw.so is not built (run __graft_entry__.build())")
    L = C.CDLL(pw.LIB)
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(L, s), s
    assert sorted(pw.EXPORTS) == syms


def test_ctypes_layout_matches_header(tmp_path):
    fields = {
        "pw_config": [f for f, _ in pw.Config._fields_],
        "pw_patch_desc": [f for f, _ in pw.PatchDesc._fields_],
        "pw_exact_desc": [f for f, _ in pw.ExactDesc._fields_],
        "pw_diag": [f for f, _ in pw.Diag._fields_],
        "pw_counters_t": [f for f, _ in pw.Counters._fields_],
        "pw_tuning": [f for f, _ in pw.Tuning._fields_],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "pw.h"', "int main(void){"]
    for st, fs in fields.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (st, st))
        for f in fs:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (st, f, st, f))
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    out = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    cls = {"pw_config": pw.Config, "pw_patch_desc": pw.PatchDesc, "pw_exact_desc": pw.ExactDesc,
           "pw_diag": pw.Diag, "pw_counters_t": pw.Counters, "pw_tuning": pw.Tuning}
    for st, k in cls.items():
        assert int(out[st]) == C.sizeof(k), st
        for f, _ in k._fields_:
            assert int(out["%s.%s" % (st, f)]) == getattr(k, f).offset, (st, f)


def test_binding_fails_loudly_without_library(monkeypatch):
    monkeypatch.setattr(pw, "_lib", None)
    monkeypatch.setattr(pw, "LIB", "/nonexistent/libpw.so")
    with pytest.raises(RuntimeError):
        pw.load()
