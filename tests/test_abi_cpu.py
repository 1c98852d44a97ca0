"""The ctypes binding agrees with include/smg.h: struct sizes and field
offsets (measured by compiling the header with the host C compiler), the
status/precision/smoother constants, and every prototype's return and
argument kinds.  A mismatch here is a silent marshalling bug, so it is
checked on the host, without a GPU."""
import ctypes
import os
import re
import shutil
import subprocess

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "smg.h")

STRUCTS = {
    "smg_pre_opts": ("PreOpts", ["n_levels", "min_coarse", "collapses"]),
    "smg_opts": ("Opts", ["mu_pre", "mu_post", "tail_rows", "lanes_per_row", "team_level", "team_size"]),
    "smg_solve_params": ("SolveParams", ["rtol", "max_cycles", "precision", "fixed_cycles", "use_graph", "timed"]),
    "smg_solve_info": ("SolveInfo", ["cycles", "k", "rel_res", "ms", "ms_phase"]),
    "smg_batch_opts": ("BatchOpts", ["threads", "lanes_level0", "lanes_coarse", "team_max", "cache_file",
                                     "device_teams", "balance"]),
}
CONSTANTS = ["SMG_OK", "SMG_FP64", "SMG_FP32_IR", "SMG_SMOOTH_GS", "SMG_SMOOTH_JACOBI",
             "SMG_COLLAPSE_ALL", "SMG_COLLAPSE_INTERIOR", "SMG_COLLAPSE_STRAIGHT",
             "SMG_PHASE_PREPARE", "SMG_PHASE_RELAX", "SMG_PHASE_TRANSFER", "SMG_PHASE_NORM", "SMG_PHASE_OTHER",
             "SMG_ERR_INVALID_ARG", "SMG_ERR_OOM", "SMG_ERR_HIP", "SMG_ERR_NOT_SPD",
             "SMG_ERR_NO_CONVERGENCE", "SMG_ERR_NONFINITE", "SMG_ERR_STATE", "SMG_ERR_PRECOMPUTE"]


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "smg.h"', "int main(void) {"]
    for cname, (_, fields) in STRUCTS.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    for k in CONSTANTS:
        lines.append(f'printf("const {k} %d\\n", (int){k});')
    lines += ["return 0;", "}"]
    src = d / "abi.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "abi"
    subprocess.run([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True, capture_output=True, timeout=60)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True, timeout=60).stdout
    layout = {}
    for line in out.splitlines():
        a, b, v = line.split()
        layout[(a, b)] = int(v)
    return layout


def test_struct_layouts_match(c_layout):
    from paper_2104_13755_amd import _lib as L
    for cname, (pyname, fields) in STRUCTS.items():
        cls = getattr(L, pyname)
        assert [f[0] for f in cls._fields_] == fields, cname
        assert ctypes.sizeof(cls) == c_layout[(cname, "size")], cname
        for f in fields:
            assert getattr(cls, f).offset == c_layout[(cname, f)], (cname, f)


def test_constants_match(c_layout):
    from paper_2104_13755_amd import _lib as L
    for k in ("SMG_OK", "SMG_FP64", "SMG_FP32_IR", "SMG_SMOOTH_GS", "SMG_SMOOTH_JACOBI",
              "SMG_COLLAPSE_ALL", "SMG_COLLAPSE_INTERIOR", "SMG_COLLAPSE_STRAIGHT"):
        assert getattr(L, k) == c_layout[("const", k)]
    for k in CONSTANTS:
        if k.startswith("SMG_ERR_"):
            assert L.STATUS[c_layout[("const", k)]] == k[len("SMG_ERR_"):], k
    assert [c_layout[("const", "SMG_PHASE_" + p.upper())] for p in L.PHASES] == [0, 1, 2, 3, 4]
    from paper_2104_13755_amd import solver
    assert solver.PRECISION == {"fp64": c_layout[("const", "SMG_FP64")],
                                "fp32ir": c_layout[("const", "SMG_FP32_IR")]}
    assert solver.SMOOTHER == {"gs": c_layout[("const", "SMG_SMOOTH_GS")],
                               "jacobi": c_layout[("const", "SMG_SMOOTH_JACOBI")]}


def _prototypes():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    src = re.sub(r"#[^\n]*", " ", src)
    protos = {}
    for m in re.finditer(r"([A-Za-z_][A-Za-z0-9_ \*]*?)\b(smg_[a-z0-9_]+)\s*\(([^;{}]*?)\)\s*;", src):
        ret, name, args = m.group(1).strip(), m.group(2), m.group(3).strip()
        if ret.startswith("typedef"):
            continue
        params = [] if args in ("", "void") else [a.strip() for a in args.split(",")]
        protos[name] = (ret, params)
    return protos


def _kind_c(decl):
    d = " ".join(decl.replace("*", " * ").split())
    if "*" in d:
        return "ptr"
    base = d.replace("const ", "").split()[0]
    if base in ("smg_hier", "smg_solver", "smg_batch", "smg_stream", "smg_ctx", "smg_alloc_fn", "smg_free_fn"):
        return "ptr"
    return {"int32_t": "i32", "smg_status": "i32", "int64_t": "i64", "double": "f64", "void": "void"}[base]


def _kind_py(t):
    if t is None:
        return "void"
    if t in (ctypes.c_int32, ctypes.c_int):
        return "i32"
    if t is ctypes.c_int64:
        return "i64"
    if t is ctypes.c_double:
        return "f64"
    if t in (ctypes.c_void_p, ctypes.c_char_p) or issubclass(t, (ctypes._Pointer, ctypes.c_void_p, ctypes._CFuncPtr)):
        return "ptr"
    raise AssertionError(t)


def test_prototypes_match_signatures():
    from paper_2104_13755_amd import _lib as L
    protos = _prototypes()
    assert len(protos) >= 30
    assert set(protos) == set(L.SIGNATURES)
    for name, (ret, params) in protos.items():
        res, args = L.SIGNATURES[name]
        want_ret = "ptr" if ret.endswith("*") else _kind_c(ret)
        assert _kind_py(res) == want_ret, name
        assert [_kind_c(p) for p in params] == [_kind_py(a) for a in args], name
