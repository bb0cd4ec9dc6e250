"""Error paths of the C ABI that need no GPU: malformed trees and generators
are EINVAL, unsupported generators and plans are EUNSUPPORTED, and the host-only
plan compiler (tenso_plan_query) agrees with the sizes a plan reports.  Every
call here is host-only; tenso_last_error() carries a message for each failure.
"""
import ctypes as C
import os

import numpy as np
import pytest

import workloads

EINVAL, ENOMEM, EUNSUPPORTED = -1, -2, -5


def _L():
    from paper_2603_17711_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return _lib


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def build_tree(parent, end_node, end_dim, max_rank=4, bond_rank=None):
    L = _L()
    p, pp = _i32(parent)
    e, ep = _i32(end_node)
    d, dp = _i32(end_dim)
    br = None
    if bond_rank is not None:
        b, br = _i32(bond_rank)
    h = C.c_void_p()
    rc = L.lib().tenso_build_tree(len(parent), pp, len(end_node), ep, dp, max_rank, br, C.byref(h))
    if rc == 0:
        L.lib().tenso_tree_destroy(h)
    return rc, L.lib().tenso_last_error().decode()


@pytest.mark.parametrize("case,parent,end_node,end_dim", [
    ("root has a parent", [0, 0], [0, 0, 1], [2, 2, 3]),
    ("parent after child", [-1, 2, 0], [0, 0, 1, 2], [2, 2, 3, 3]),
    ("parent out of range", [-1, 5], [0, 0, 1], [2, 2, 3]),
    ("ket off the root", [-1, 0], [1, 0, 1], [2, 2, 3]),
    ("end on a missing node", [-1, 0], [0, 0, 7], [2, 2, 3]),
    ("zero end dimension", [-1, 0], [0, 0, 1], [2, 2, 0]),
    ("bra neither the ket's size nor 1", [-1, 0], [0, 0, 1], [2, 3, 3]),
    ("fewer than two ends", [-1], [0], [2]),
])
def test_build_tree_rejects_malformed_input(case, parent, end_node, end_dim):
    rc, msg = build_tree(parent, end_node, end_dim)
    assert rc == EINVAL, (case, rc)
    assert msg, case


def test_build_tree_null_and_counts():
    L = _L()
    h = C.c_void_p()
    assert L.lib().tenso_build_tree(0, None, 0, None, None, 4, None, C.byref(h)) == EINVAL
    _, pp = _i32([-1, 0])
    assert L.lib().tenso_build_tree(2, pp, 3, None, None, 4, None, C.byref(h)) == EINVAL
    rc, _ = build_tree([-1, 0], [0, 0, 1], [2, 2, 3], max_rank=0)
    assert rc == EINVAL


def test_tree_builders_reject_bad_sizes():
    L = _L()
    h = C.c_void_p()
    d, dp = _i32([4, 4, 4])
    assert L.lib().tenso_tree_train(0, 3, dp, 4, C.byref(h)) == EINVAL
    assert L.lib().tenso_tree_train(2, -1, dp, 4, C.byref(h)) == EINVAL
    assert L.lib().tenso_tree_train(2, 3, dp, 0, C.byref(h)) == EINVAL
    assert L.lib().tenso_tree_nary(2, 3, dp, 1, 4, C.byref(h)) == EINVAL
    z, zp = _i32([4, 0, 4])
    assert L.lib().tenso_tree_nary(2, 3, zp, 2, 4, C.byref(h)) == EINVAL
    assert L.lib().tenso_tree_train(2, 3, dp, 4, None) == EINVAL


def _tree(M=2, dims=(3, 3, 3), n_ary=2, rank=4):
    from paper_2603_17711_amd import api
    _L()
    return api.Tree.nary(M, list(dims), n_ary, rank)


def gen_rc(tree, coef, slot, nfac, fend, mats):
    L = _L()
    c = np.ascontiguousarray(coef, np.complex128)
    m = np.ascontiguousarray(mats, np.complex128)
    s, sp = _i32(slot)
    n, np_ = _i32(nfac)
    f, fp = _i32(fend)
    h = C.c_void_p()
    rc = L.lib().tenso_build_generator(tree.h, len(c), c.ctypes.data_as(C.POINTER(L.c128)), sp, np_,
                                       fp, m.ctypes.data_as(C.POINTER(L.c128)), C.byref(h))
    if rc == 0:
        L.lib().tenso_gen_destroy(h)
    return rc, L.lib().tenso_last_error().decode()


def test_build_generator_accepts_a_valid_table():
    t = _tree()
    rc, _ = gen_rc(t, [1.0, 2.0], [-1, -1], [1, 2], [0, 1, 2],
                   np.concatenate([np.eye(2).ravel(), np.eye(2).ravel(), np.eye(3).ravel()]))
    assert rc == 0


@pytest.mark.parametrize("case,nfac,fend", [
    ("end out of range", [1], [9]),
    ("negative end", [1], [-1]),
    ("term without factors", [0], []),
    ("same end twice in a term", [2], [2, 2]),
])
def test_build_generator_rejects_bad_terms(case, nfac, fend):
    t = _tree()
    mats = np.concatenate([np.eye(3).ravel()] * max(1, len(fend)))
    rc, msg = gen_rc(t, [1.0], [-1], nfac, fend, mats)
    assert rc == EINVAL, (case, rc, msg)
    assert msg


def test_build_generator_rejects_negative_counts():
    t = _tree()
    rc, _ = gen_rc(t, [1.0], [-1], [-1], [2], np.eye(3).ravel())
    assert rc == EINVAL
    # any negative slot means "no drive" (f = 1)
    rc, _ = gen_rc(t, [1.0], [-2], [1], [2], np.eye(3).ravel())
    assert rc == 0


def _plan_query(tree, gen, precision=1, method=0, max_rank=0):
    L = _L()
    opts = L.PlanOpts(precision, method, max_rank)
    sb, wb, nl, fl = C.c_size_t(), C.c_size_t(), C.c_int64(), C.c_double()
    rc = L.lib().tenso_plan_query(tree.h, gen.h, C.byref(opts), C.byref(sb), C.byref(wb),
                                  C.byref(nl), C.byref(fl))
    return rc, sb.value, wb.value, nl.value, fl.value, L.lib().tenso_last_error().decode()


def _instance_tree_gen(inst, rank=None):
    from paper_2603_17711_amd import api
    from paper_2603_17711_amd.heom import heom_table
    _L()
    table, dims = heom_table(inst.H, inst.baths, inst.depth)
    R = inst.rank if rank is None else rank
    t = api.Tree.train(inst.M, dims, R) if inst.tree == "train" else \
        api.Tree.nary(inst.M, dims, int(inst.tree[4:]), R)
    return t, api.Generator(t, table)


def test_plan_query_sizes_and_launches():
    t, g = _instance_tree_gen(workloads.exciton_7site())
    rc, sb, wb, nl, fl, msg = _plan_query(t, g)
    assert rc == 0, msg
    # 28 cores of the binary tree (root 7x7x16, the rest at most 16^3) in FP64
    assert 28 * 7 * 7 * 16 * 16 <= sb < 28 * 16 ** 3 * 16 + 28 * 256
    assert wb > 0 and nl > 100
    # algorithmic apply work of one step at the 7-site exciton workload
    assert 5e9 < fl < 5e10
    rc64, sb64, wb64, nl64, fl64, _ = _plan_query(t, g, precision=0)
    # same state; wider workspace operands; the FP64 path splits some
    # contractions differently, which moves the credited work by < 1e-4
    assert rc64 == 0 and sb64 == sb and wb64 > wb and abs(fl64 - fl) < 1e-4 * fl


def test_plan_query_rejects_bad_options():
    t, g = _instance_tree_gen(workloads.spin_boson_train())
    assert _plan_query(t, g, precision=7)[0] == EINVAL
    assert _plan_query(t, g, method=3)[0] == EINVAL
    assert _plan_query(t, g, method=1, max_rank=1)[0] == EINVAL
    t2, g2 = _instance_tree_gen(workloads.exciton_7site())
    rc = _L().lib().tenso_plan_query(t.h, g2.h, C.byref(_L().PlanOpts(1, 0, 0)), None, None,
                                     None, None)
    assert rc == EINVAL  # a generator built for another tree


def test_plan_query_ps2_two_site_budget():
    """A ps2 plan sizes every buffer at the rank cap: the structured-bath
    ternary tree fits at caps 8 and 16; from cap 32 its largest two-site tensor
    (4 r^2 x r^3 elements on the edge below the root's child) exceeds the
    2^26-element budget: ENOMEM."""
    t, g = _instance_tree_gen(workloads.structured_bath_ternary(), rank=8)
    for cap in (8, 16):
        rc, sb, wb, _, _, msg = _plan_query(t, g, method=1, max_rank=cap)
        assert rc == 0, (cap, msg)
        assert wb > sb > 0
    for cap in (32, 64):
        rc, _, _, _, _, msg = _plan_query(t, g, method=1, max_rank=cap)
        assert rc == ENOMEM and "two-site" in msg


def test_plan_query_vmf():
    """VMF plans: FP64 only (EUNSUPPORTED otherwise); the query reports one
    evaluation of the derivative: every node's effective generator in one
    contraction launch plus the environments, densities and projections."""
    t, g = _instance_tree_gen(workloads.exciton_7site())
    assert _plan_query(t, g, precision=1, method=2)[0] == EUNSUPPORTED
    rc, sb, wb, nl, fl, msg = _plan_query(t, g, precision=0, method=2)
    assert rc == 0, msg
    rc1, sb1, wb1, nl1, fl1, _ = _plan_query(t, g, precision=0, method=0)
    assert sb == sb1 and wb == wb1          # one layout serves ps1 and vmf
    assert 0 < nl < nl1 and 0 < fl < fl1     # one derivative against a whole ps1 step
