"""The C-ABI library builds, loads and exports every entry point of include/jfnk.h.

CPU only: no call here touches a GPU (argument validation and host-side
helpers return before any HIP call).
"""

import ctypes
import os
import re

import pytest

import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "jfnk.h")
LIB = os.path.join(ROOT, "paper_2605_13378_amd", "libjfnk.so")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(jfnk_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def jlib():
    if not os.path.exists(LIB):
        from paper_2605_13378_amd import build

        build.build()
    from paper_2605_13378_amd import jfnk

    return jfnk.lib()


def test_every_header_function_is_exported(jlib):
    names = header_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(jlib, name), name
    from paper_2605_13378_amd import jfnk

    assert set(jfnk.exported_symbols()) == set(names)


def test_header_compiles_as_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "jfnk.h"\nint main(void){jfnk_options o; jfnk_default_options(0,&o); return o.m != 30;}\n')
    rc = os.system(f"gcc -std=c99 -Wall -Werror -I{ROOT}/include -c {src} -o {tmp_path}/t.o")
    assert rc == 0


def test_problem_size_and_footprint(jlib):
    from paper_2605_13378_amd import jfnk

    gs = W.grayscott_spec(1024)
    assert jfnk.problem_size(gs) == 2 * 1024 * 1024
    assert jfnk.problem_size(W.burgers1d_spec(256)) == 256
    fp = jfnk.footprint_bytes(gs, "f64", 30)
    npad = 2 * 1024 * 1024
    assert fp >= 31 * npad * 8 + 8 * npad * 8
    assert jfnk.footprint_bytes(gs, "f32", 30) < fp
    bad = dict(gs, nx=2)
    assert jfnk.problem_size(bad) == 0
    assert jfnk.footprint_bytes(gs, "f64", 33) == 0


def test_default_options_follow_the_paper(jlib):
    from paper_2605_13378_amd import jfnk

    o64 = jfnk.default_options("f64")
    o32 = jfnk.default_options("f32")
    assert (o64.tol_newton, o64.tol_krylov) == (1e-6, 1e-8)
    assert (o32.tol_newton, o32.tol_krylov) == (1e-4, 1e-6)
    assert o64.max_newton == 15 and o64.max_restarts == 100 and o64.m == 30
    assert o64.krylov == jfnk.KRYLOV["gmres"] and o64.engine == jfnk.ENGINES["auto"]
    assert o64.orth == jfnk.ORTH["dcgs2"] and jfnk.default_options("f16s").orth == jfnk.ORTH["dcgs2"]


def test_invalid_create_is_rejected_without_gpu(jlib):
    from paper_2605_13378_amd import jfnk

    h = ctypes.c_void_p()
    p = jfnk.make_problem(dict(W.grayscott_spec(8), ny=2))
    assert jlib.jfnk_create(ctypes.byref(p), 0, 30, None, ctypes.byref(h)) == 1
    assert b"grid" in jlib.jfnk_last_error(None)
    p = jfnk.make_problem(W.grayscott_spec(8))
    assert jlib.jfnk_create(ctypes.byref(p), 0, 40, None, ctypes.byref(h)) == 1
    assert jlib.jfnk_create(ctypes.byref(p), 7, 30, None, ctypes.byref(h)) == 1
    assert jlib.jfnk_status_string(6) == b"not converged"


def test_null_handles_are_rejected(jlib):
    assert jlib.jfnk_destroy(None) == 1
    assert jlib.jfnk_residual(None, None, None) == 1
    assert jlib.jfnk_newton_solve(None, None, None, None) == 1
    assert jlib.jfnk_bicgstab(None, None, None, None, 1e-8, 10, 0, 0.0, 0, None) == 1


def test_product_path_does_not_import_oracle():
    pkg = os.path.join(ROOT, "paper_2605_13378_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
