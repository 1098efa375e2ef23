"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function declared in include/dfamin.h, fills default options, and
rejects bad arguments before touching the device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2508_20735_amd import binding as B
from paper_2508_20735_amd import build as hip_build

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include",
                      "dfamin.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dfa_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not hip_build.is_built():
        hip_build.build()
    return B.load()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert len(names) >= 26
    for name in names:
        assert hasattr(lib, name), name
    assert B.EXPORTS == names


def test_default_options(lib):
    o = B.Options()
    lib.dfa_options_default(ctypes.byref(o))
    assert o.tc_mode == B.TC["auto"] and o.loop_mode == B.LOOP["graph"]
    assert o.start == 0 and o.max_rounds == 0 and o.lds_stage == 2
    assert o.algorithm == B.ALGO["signature"] and o.prune == 0
    assert o.equiv_method == B.EQ["union"]


STRUCTS = {
    "dfa_options": "Options", "dfa_stats": "Stats", "dfa_view": "View", "dfa_tuning": "Tuning",
    "dfa_batch_stats": "BatchStats", "dfa_server_config": "ServerConfig",
    "dfa_request": "Request", "dfa_result": "Result", "dfa_server_stats": "ServerStats",
    "dfa_kernel_time": "KernelTime", "dfa_quotient": "Quotient",
}


def test_struct_layouts_match_header(tmp_path):
    """The binding's structures mirror the header's: sizes and the offset of
    every field, as a C compiler lays the header out."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "dfamin.h"',
             'int main(void) {']
    for cname, pyname in STRUCTS.items():
        cls = getattr(B, pyname)
        lines.append(f'printf("{pyname} size %zu\\n", sizeof({cname}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{pyname} {field} %zu\\n", offsetof({cname}, {field}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c11", "-I", os.path.dirname(HEADER), str(src), "-o",
                           str(exe)])
    out = subprocess.check_output([str(exe)], text=True).split("\n")
    seen = 0
    for line in filter(None, out):
        pyname, what, value = line.split()
        cls = getattr(B, pyname)
        want = ctypes.sizeof(cls) if what == "size" else getattr(cls, what).offset
        assert int(value) == want, (pyname, what)
        seen += 1
    assert seen == sum(len(getattr(B, p)._fields_) + 1 for p in STRUCTS.values())


def test_default_tuning(lib):
    t = B.Tuning()
    lib.dfa_tuning_default(ctypes.byref(t))
    assert t.label_rounds == 2 and t.chunk >= 1 and t.cached_probe in (0, 1)


def test_bad_arguments_rejected_on_host(lib):
    d = np.zeros((4, 2), dtype=np.uint32)
    a = np.zeros(4, dtype=np.uint8)
    out = np.zeros(4, dtype=np.uint32)
    # n == 0 and k == 0 are rejected before any device call
    assert lib.dfa_minimise(0, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None, None,
                            None) == B.DFA_EINVAL
    assert lib.dfa_minimise(4, 0, d.ctypes.data, a.ctypes.data, out.ctypes.data, None, None,
                            None) == B.DFA_EINVAL
    assert b"n and k" in lib.dfa_last_error()
    assert lib.dfa_minimise(4, 2, None, a.ctypes.data, out.ctypes.data, None, None,
                            None) == B.DFA_EINVAL
    o = B.Options()
    lib.dfa_options_default(ctypes.byref(o))
    o.start = 4
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    o.start = 0
    o.tc_mode = 7
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    va = B.View(4, 2, 0, d.ctypes.data, a.ctypes.data)
    vb = B.View(4, 3, 0, d.ctypes.data, a.ctypes.data)
    v = ctypes.c_int()
    assert lib.dfa_equivalent(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v), None,
                              None) == B.DFA_EINVAL
    vb = B.View(4, 2, 9, d.ctypes.data, a.ctypes.data)
    assert lib.dfa_included(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v), None, None,
                            None) == B.DFA_EINVAL
    assert b"start" in lib.dfa_last_error()
    # option values out of range, and options a call does not support
    vb = B.View(4, 2, 0, d.ctypes.data, a.ctypes.data)
    o.tc_mode = B.TC["off"]
    o.prune = 1
    assert lib.dfa_equivalent(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                              ctypes.byref(o), None) == B.DFA_EINVAL
    assert b"prune" in lib.dfa_last_error()
    o.prune = 2
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    o.prune = 0
    o.algorithm = 5
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    o.algorithm = B.ALGO["leader"]
    nb = np.zeros(1, dtype=np.uint32)
    assert lib.dfa_minimise_batch(1, ctypes.byref(va), out.ctypes.data, None, nb.ctypes.data,
                                  None, ctypes.byref(o), None) == B.DFA_EINVAL
    # the persistent loop: table grouping or leader rounds (single and
    # batched calls), not sort grouping
    o.algorithm = B.ALGO["sort"]
    o.loop_mode = B.LOOP["persistent"]
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    assert b"persistent" in lib.dfa_last_error()
    assert lib.dfa_minimise_batch(1, ctypes.byref(va), out.ctypes.data, None, nb.ctypes.data,
                                  None, ctypes.byref(o), None) == B.DFA_EINVAL
    o.algorithm = B.ALGO["signature"]
    o.loop_mode = 4
    assert lib.dfa_minimise(4, 2, d.ctypes.data, a.ctypes.data, out.ctypes.data, None,
                            ctypes.byref(o), None) == B.DFA_EINVAL
    # equivalence by product exploration: single pairs only
    o.loop_mode = B.LOOP["graph"]
    o.equiv_method = 7
    assert lib.dfa_equivalent(ctypes.byref(va), ctypes.byref(vb), ctypes.byref(v),
                              ctypes.byref(o), None) == B.DFA_EINVAL
    assert b"equiv_method" in lib.dfa_last_error()
    o.equiv_method = B.EQ["product"]
    verdicts = np.zeros(1, dtype=np.int32)
    assert lib.dfa_equivalent_batch(1, ctypes.byref(va), ctypes.byref(vb), verdicts.ctypes.data,
                                    ctypes.byref(o), None) == B.DFA_EINVAL
    assert b"DFA_EQ_UNION" in lib.dfa_last_error()


def test_profile_only_rejects_long_names(lib):
    assert lib.dfa_profile_only(b"k" * 40) == B.DFA_EINVAL
    assert b"too long" in lib.dfa_last_error()
