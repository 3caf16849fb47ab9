"""The C ABI: libch.so loads on a machine without a GPU and exports every
entry point include/ch.h declares; the binding's structs match the header."""
import ctypes
import os
import re

import pytest

from paper_2502_14589_amd import ch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "ch.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ch_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    if not os.path.exists(ch.LIB_PATH):
        pytest.fail("libch.so is not built (python -m paper_2502_14589_amd.build)")
    lib = ctypes.CDLL(ch.LIB_PATH)
    declared = header_functions()
    assert len(declared) >= 9
    for name in declared:
        assert hasattr(lib, name), name
    assert sorted(ch.EXPORTED) == declared


def test_strerror_without_device():
    lib = ch.load_library()
    assert lib.ch_strerror(ch.CH_OK) == b"ok"
    assert b"trace" in lib.ch_strerror(ch.CH_ETAU_UNDERFLOW)


def test_struct_layouts_match_header(tmp_path):
    """Compile the header with gcc and compare every field offset with ctypes."""
    import shutil
    import subprocess

    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    structs = {"ch_problem": ch.ChProblem, "ch_ee_opts": ch.ChEeOpts, "ch_step_record": ch.ChStepRecord,
               "ch_run_stats": ch.ChRunStats, "ch_batch_item": ch.ChBatchItem, "ch_request": ch.ChRequest,
               "ch_shape": ch.ChShape}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ch.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def test_header_constants_match_binding():
    text = open(os.path.join(ROOT, "include", "ch.h")).read()
    assert f"#define CH_MMAX {ch.CH_MMAX}" in text
    assert f"#define CH_PMAX {ch.CH_PMAX}" in text
    for name in ("CH_OK", "CH_EINVAL", "CH_ENOMEM", "CH_ENONFINITE", "CH_ETAU_UNDERFLOW", "CH_EDEVICE",
                 "CH_ORTH_DCGS2", "CH_ORTH_MGS", "CH_KERNEL_MGS", "CH_KERNEL_MATVEC", "CH_KERNEL_PHI",
                 "CH_KERNEL_DC_MATVEC", "CH_KERNEL_DC_UPDATE", "CH_KERNEL_LIM_STAGE", "CH_KERNEL_DC_ITER",
                 "CH_KERNEL_LIM_STAGE2"):
        m = re.search(rf"{name}\s*=\s*(-?\d+)", text)
        assert m and int(m.group(1)) == getattr(ch, name)


def test_create_fails_cleanly_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = ch.load_library()
    p = ctypes.c_void_p()
    rc = lib.ch_create(ctypes.byref(p), 0, None)
    assert rc == ch.CH_EDEVICE and not p
