"""The C-ABI library without a GPU: it loads, exports every function that
include/tenso.h declares (and the Python binding declares no other), and its
host-only tree construction (ends, n-ary splits, rank clamping) agrees with
the oracle's trees.  No call here touches a device."""
import os
import re

import numpy as np
import pytest

import workloads
from oracle.ttn import nary_tree, train_tree

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tenso.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tenso_\w+)\s*\(", src)))


def _lib():
    from paper_2603_17711_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib


def test_library_exports_every_declared_function():
    L = _lib()
    names = _declared()
    assert len(names) > 30
    lib = L.lib()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    unbound = [n for n in names if n not in L.SIGS]
    assert not unbound, unbound
    extra = [n for n in L.SIGS if n not in names]
    assert not extra, extra


def _oracle_tree(kind, M, dims, R):
    return train_tree(M, dims, R) if kind == "train" else nary_tree(M, dims, int(kind[4:]), R)


@pytest.mark.parametrize("which", ["spin_boson_train", "exciton_7site", "structured_bath_ternary",
                                   "uneven_batch"])
def test_tree_ranks_match_oracle(which):
    _lib()
    from paper_2603_17711_amd import api
    if which == "uneven_batch":
        insts = workloads.uneven_batch(n_inst=24, seed=2)
    else:
        insts = [getattr(workloads, which)()]
    for inst in insts:
        dims = []
        for b in inst.baths:
            dims += [inst.depth] * b.n_features()
        R = inst.rank
        o = _oracle_tree(inst.tree, inst.M, dims, R)
        t = api.Tree.train(inst.M, dims, R) if inst.tree == "train" else \
            api.Tree.nary(inst.M, dims, int(inst.tree[4:]), R)
        assert t.n_nodes == len(o.parent)
        r = t.ranks()
        assert list(r[1:]) == [o.rank[s] for s in range(1, len(o.parent))], inst.name
