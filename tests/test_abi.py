"""Boundary checks that need no GPU: the library loads, exports every entry
point the header declares, and its ctypes mirror matches the C layouts."""

import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tdagw.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(tdg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def tdg():
    import paper_2502_05635_amd as P
    if not os.path.exists(P.LIB_PATH):
        P_build = __import__("paper_2502_05635_amd.build", fromlist=["build"])
        P_build.build()
    return P


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("tdg_create", "tdg_destroy", "tdg_kernel_build", "tdg_kernel_compress", "tdg_propagate",
                 "tdg_observables", "tdg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(tdg):
    handle = tdg.lib()
    for name in _declared():
        assert hasattr(handle, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", tdg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (tdg_\w+)", out))
    assert exported == set(_declared()), exported ^ set(_declared())


def test_ctypes_layouts_match_c(tmp_path, tdg):
    from paper_2502_05635_amd import _abi as abi
    structs = {"tdg_model": abi.Model, "tdg_coulomb": abi.Coulomb, "tdg_trunc": abi.Trunc,
               "tdg_lowrank": abi.LowRank, "tdg_field": abi.Field, "tdg_operator": abi.Operator,
               "tdg_obs": abi.Obs, "tdg_obs_grad": abi.ObsGrad, "tdg_grads": abi.Grads, "tdg_channels": abi.Channels}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "tdagw.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname}.{fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = dict(line.split() for line in subprocess.run([str(exe)], capture_output=True, text=True,
                                                      check=True).stdout.splitlines())
    for cname, py in structs.items():
        assert int(got[cname]) == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert int(got[f"{cname}.{fname}"]) == getattr(py, fname).offset, f"{cname}.{fname}"


def test_constants_match_header():
    """Every integer TDG_* constant the binding defines equals the header's,
    and every option and kernel-class constant of the header is bound."""
    import re

    from paper_2502_05635_amd import _abi as abi
    text = open(os.path.join(ROOT, "include", "tdagw.h")).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(TDG_\w+)\s+\(?(-?\d+)\)?", text)}
    assert defs, "no integer constants found in the header"
    for name, value in defs.items():
        if hasattr(abi, name):
            assert getattr(abi, name) == value, name
    for name in defs:
        if name.startswith(("TDG_OPT_", "TDG_KCLASS_")):
            assert hasattr(abi, name), f"{name} is not in the binding"


def test_host_validation_without_device(tdg):
    from paper_2502_05635_amd import _abi as abi
    L = tdg.lib()
    m = abi.Model(12, 12, 2, 1, 0.5, 6.0, None, None, None, None)
    n = C.c_int64()
    assert L.tdg_kernel_dim(C.byref(m), abi.TDG_BLOCK_ALL, C.byref(n)) == 0 and n.value == 576
    assert L.tdg_kernel_dim(C.byref(m), abi.TDG_BLOCK_EH, C.byref(n)) == 0 and n.value == 144
    assert L.tdg_kernel_dim(C.byref(m), 7, C.byref(n)) == abi.TDG_E_INVAL
    # a NULL context is rejected before any device work
    assert L.tdg_propagate(None, None, None, None, 1, 1.0, None, 1, None) == abi.TDG_E_INVAL
    assert L.tdg_kernel_build(None, None, None, 0, None, 0) == abi.TDG_E_INVAL
    assert L.tdg_kernel_compress(None, None, 0, 0, None, None) == abi.TDG_E_INVAL
    assert L.tdg_kernel_compress_randomized(None, None, 0, 0, None, None, 0, 0, None) == abi.TDG_E_INVAL
    assert L.tdg_propagate_adjoint(None, None, None, None, 1, 1.0, None, 50, None, None) == abi.TDG_E_INVAL
    assert L.tdg_kernel_compress_channels(None, None, 0, 0, None, None) == abi.TDG_E_INVAL
    assert L.tdg_version() >= 100
