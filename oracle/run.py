"""Oracle driver: build terms and tree for a workload instance and propagate.

Takes the plain parameters of ``workloads.Instance`` (system Hamiltonian, baths,
depth, tree kind, rank, initial state, drive) and runs the oracle's ps1 / ps2
sweep, recording rho_S at every `every`-th step and the final step.
"""
import numpy as np

from .bath import bath_features
from .integrators import Propagator
from .sop import heom_terms
from .ttn import Tree, initial_state, nary_tree, train_tree


def build(inst, rank=None):
    baths = []
    for b in inst.baths:
        baths.append((b.Q, bath_features(b.T, dl=b.dl, bo=b.bo, n_ltc=b.n_ltc,
                                         method=getattr(b, "decomposition", "matsubara"))))
    drives = [] if inst.drive is None else [(0, inst.drive[0])]
    terms, dims = heom_terms(inst.H, baths, inst.depth, drives=drives,
                             metric=getattr(inst, "metric", "abs"))
    K = len(dims) - 2
    R = inst.rank if rank is None else rank
    if inst.method == "ps2":
        from .integrators import PS2_INIT_RANK
        R = PS2_INIT_RANK
    if inst.tree == "train":
        tree = train_tree(inst.M, dims[2:], R)
    else:
        tree = nary_tree(inst.M, dims[2:], int(inst.tree[4:]), R)
    return terms, tree


def propagate(inst, n_steps=None, every=10, rank=None, max_rank=None):
    terms, tree = build(inst, rank)
    drive = None
    if inst.drive is not None:
        drive = lambda t: np.array([inst.drive_value(t)])
    P = Propagator(tree, terms, initial_state(tree, inst.rho0), drive_fn=drive)
    n = inst.n_steps if n_steps is None else n_steps
    rhos, steps, ranks = [P.rho()], [0], []
    for s in range(n):
        t0 = s * inst.dt
        if inst.method == "ps2":
            ranks.append(P.step_ps2(t0, inst.dt, inst.eps,
                                    inst.rank if max_rank is None else max_rank))
        else:
            P.step_ps1(t0, inst.dt)
        if (s + 1) % every == 0 or s + 1 == n:
            rhos.append(P.rho())
            steps.append(s + 1)
    return np.array(steps), np.array(rhos), ranks, P
