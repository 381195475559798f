"""The C ABI as declared in include/bfgsuq.h: every declared function is exported by
libbfgsuq.so and bound by the Python layer with the same number of arguments.
No compute calls: this runs without a GPU."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bfgsuq.h")


def declarations():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    decls = {}
    for m in re.finditer(r"\b(?:const\s+)?(?:int|void|char|int32_t|int64_t)\s*\**\s*(bfgs_\w+)\s*\(([^)]*)\)\s*;", text):
        args = [a for a in m.group(2).split(",") if a.strip() and a.strip() != "void"]
        decls[m.group(1)] = len(args)
    return decls


@pytest.fixture(scope="module")
def lib():
    from paper_2009_12663_amd import _lib, build
    if not os.path.exists(_lib.LIB_PATH):
        build.build()
    return _lib.load()


def test_header_declares_the_path():
    d = declarations()
    for name in ["bfgs_create", "bfgs_push_pair", "bfgs_apply_Hinv", "bfgs_rsvd", "bfgs_posterior_diag",
                 "bfgs_destroy", "bfgs_batch_create", "bfgs_batch_push_pairs", "bfgs_batch_graph_build", "bfgs_mlp_train_step"]:
        assert name in d, name


def test_every_declared_symbol_is_exported(lib):
    missing = [name for name in declarations() if not hasattr(lib, name)]
    assert not missing, missing


def test_binding_matches_header(lib):
    from paper_2009_12663_amd import _lib
    d = declarations()
    assert sorted(d) == sorted(_lib.EXPORTS)
    for name, nargs in d.items():
        assert len(getattr(lib, name).argtypes) == nargs, name


def test_status_strings(lib):
    from paper_2009_12663_amd import _lib
    for code in range(0, -9, -1):
        s = lib.bfgs_status_string(code)
        assert isinstance(s, bytes) and len(s) > 0
