"""The ctypes structures of the binding against the C header: a small C
program built with gcc prints sizeof and offsetof for every field of every
structure the binding mirrors, and each must agree with ctypes.  No GPU."""
import ctypes
import json
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# binding class name -> C type name
STRUCTS = {
    "RelationDesc": "lh_relation_desc",
    "Atom": "lh_atom",
    "Filter": "lh_filter",
    "GroupCol": "lh_group_col",
    "Query": "lh_query",
    "Result": "lh_result",
    "TrieInfo": "lh_trie_info",
    "PlanInfo": "lh_plan_info",
    "Hypergraph": "lh_hypergraph",
    "Ghd": "lh_ghd",
    "ProfileEntry": "lh_profile_entry",
    "FeatureCol": "lh_feature_col",
}
def _binding_module():
    from paper_1708_07859_amd import lh
    return lh


@pytest.fixture(scope="module")
def c_layout():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    b = _binding_module()
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "lh.h"', "int main(void) {", 'printf("{");']
    first = True
    for py, c in STRUCTS.items():
        cls = getattr(b, py)
        for name, _ in cls._fields_:
            sep = "" if first else ","
            first = False
            lines.append(f'printf("{sep}\\"{py}.{name}\\": %zu", offsetof({c}, {name}));')
        lines.append(f'printf(",\\"{py}.__size__\\": %zu", sizeof({c}));')
    lines += ['printf("}");', "return 0; }"]
    d = tempfile.mkdtemp()
    try:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True,
                       capture_output=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
        return b, json.loads(out)
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("py", sorted(STRUCTS))
def test_struct_layout_matches_header(c_layout, py):
    b, layout = c_layout
    cls = getattr(b, py)
    for name, _ in cls._fields_:
        assert getattr(cls, name).offset == layout[f"{py}.{name}"], (py, name)
    assert ctypes.sizeof(cls) == layout[f"{py}.__size__"], py


def test_policy_and_flag_constants_match_header():
    b = _binding_module()
    hdr = open(os.path.join(ROOT, "include", "lh.h")).read()

    def define(name):
        for line in hdr.splitlines():
            parts = line.split()
            if len(parts) >= 3 and parts[0] == "#define" and parts[1] == name:
                return int(parts[2].rstrip("u"), 0)
        raise KeyError(name)
    assert b.GROUP_IMPL == {"auto": define("LH_GROUP_AUTO"), "sort": define("LH_GROUP_SORT"),
                            "hash": define("LH_GROUP_HASH"), "dense": define("LH_GROUP_DENSE")}
    assert b.LH_DENSE_BLAS == define("LH_DENSE_BLAS")
    assert b.POLICY == {"plain": define("LH_POLICY_PLAIN"), "learned": define("LH_POLICY_LEARNED"),
                        "fixed": define("LH_POLICY_FIXED")}
    assert b.LH_GHD_MAX_NODES == define("LH_GHD_MAX_NODES")
