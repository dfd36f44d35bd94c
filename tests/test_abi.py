"""Host-only checks of the C-ABI library (no GPU, no kernel launches).

* libsevo.so loads and exports every function include/sevo.h declares;
* the ctypes structs of the binding have the C layout of the header;
* the library's own host instance generator (an independent Householder QR)
  agrees with the oracle's: the shift bit for bit, the rotation to 1e-12;
* invalid arguments are rejected with SEVO_EINVAL and a message.
"""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

import oracle as O
from paper_2505_17430_amd import sevo as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(S.LIB_PATH):
        from paper_2505_17430_amd import build
        build.build(incremental=True)
    return S.lib()


def test_exports_every_declared_function(L):
    names = S.header_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(L, n), n


STRUCTS = {
    "sevo_problem": (S.Problem, ["func", "dim", "lb", "ub", "f_star"]),
    "sevo_eval_item": (S.EvalItem, ["prob", "instance", "n", "ld", "x", "err_out"]),
    "sevo_de_state": (S.DEState, [f for f, _ in S.DEState._fields_]),
    "sevo_de_params": (S.DEParams, ["F", "CR"]),
    "sevo_pso_state": (S.PSOState, [f for f, _ in S.PSOState._fields_]),
    "sevo_pso_params": (S.PSOParams, ["w", "c1", "c2", "vmax"]),
    "sevo_run_desc": (S.RunDesc, [f for f, _ in S.RunDesc._fields_]),
    "sevo_run_result": (S.RunResult, [f for f, _ in S.RunResult._fields_]),
    "sevo_run_state": (S.RunState, [f for f, _ in S.RunState._fields_]),
}


def test_struct_layout_matches_header(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "sevo.h"', 'int main(void){']
    for cname, (_, fields) in STRUCTS.items():
        lines.append(f'printf("{cname} %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname}.{f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    got = dict(l.split() for l in subprocess.check_output([str(exe)]).decode().splitlines())
    for cname, (cls, fields) in STRUCTS.items():
        assert int(got[cname]) == C.sizeof(cls), cname
        for f in fields:
            assert int(got[f"{cname}.{f}"]) == getattr(cls, f).offset, (cname, f)


@pytest.mark.parametrize("func,dim,inst", [(0, 2, 0), (2, 3, 1), (2, 10, 0), (3, 30, 4),
                                           (5, 50, 9), (1, 100, 2), (4, 121, 0), (0, 200, 3)])
def test_instance_generator_matches_oracle(L, func, dim, inst):
    o1, M1 = S.generate_instance(func, dim, inst, 250517431)
    o2, M2 = O.instance(func, dim, inst, 250517431)
    assert np.array_equal(o1, o2)
    assert np.abs(M1 - M2).max() <= 1e-12
    assert np.abs(M1.T @ M1 - np.eye(dim)).max() <= 1e-12


@pytest.mark.slow
def test_instance_generator_matches_oracle_d1000(L):
    o1, M1 = S.generate_instance(0, 1000, 0, 250517431)
    o2, M2 = O.instance(0, 1000, 0, 250517431)
    assert np.array_equal(o1, o2)
    assert np.abs(M1 - M2).max() <= 1e-12


def test_invalid_arguments_rejected(L):
    o = np.zeros(4); M = np.zeros(16)
    for func, dim in ((6, 4), (-1, 4), (0, 1), (0, 1025)):
        rc = L.sevo_generate_instance(func, dim, 0, 1, o.ctypes.data, M.ctypes.data)
        assert rc == S.EINVAL
        assert L.sevo_last_error(None).decode()
    assert L.sevo_generate_instance(0, 4, 0, 1, None, M.ctypes.data) == S.EINVAL
    # a null context is rejected, not dereferenced
    assert L.sevo_sync(None, None) == S.EINVAL
    assert L.sevo_evaluate(None, None, 0, None, 0, 0, None, 1, None) == S.EINVAL
    out = C.c_void_p()
    assert L.sevo_create(None, 0, 1, 1) == S.EINVAL
