"""How much the oracle's truncated-rank trajectories depend on the QR rank rule.

Projector splitting at truncated rank depends on the orthonormal completion of
rank-deficient cores (every bond is rank-deficient at t = 0), and Householder
QR completes them from whatever is left of the dependent columns.  The oracle
fixes the completion by treating residual columns at or below
QR_RANK_TOL * ||A||_F as exact zeros.  This test moves that threshold by two
decades either way and states the spread of rho_S (trace distance, every 10th
step): it bounds how much of a truncated-rank parity result is the shared
convention rather than the dynamics.  Measured on the spin-boson train
(200 steps): 1.1e-7 for 1e-8 against 1e-10, 6e-10 for 1e-12 against 1e-10;
on batch instance 1 (25 steps): 4e-9 and 3e-8.
"""
import numpy as np

import oracle.integrators as integ
import workloads
from oracle.run import propagate
from oracle.ttn import trace_distance


def _spread(inst, n_steps, every):
    old = integ.QR_RANK_TOL
    res = {}
    try:
        for tol in (1e-8, 1e-10, 1e-12):
            integ.QR_RANK_TOL = tol
            res[tol] = propagate(inst, n_steps=n_steps, every=every)[1]
    finally:
        integ.QR_RANK_TOL = old
    return {tol: max(trace_distance(a, b) for a, b in zip(res[tol], res[1e-10]))
            for tol in (1e-8, 1e-12)}


def test_qr_rank_rule_spread_spin_boson_train():
    s = _spread(workloads.spin_boson_train(n_steps=200), 200, 10)
    print(f"spin-boson train, 200 steps: spread 1e-8 vs 1e-10 = {s[1e-8]:.2e}, "
          f"1e-12 vs 1e-10 = {s[1e-12]:.2e}")
    assert s[1e-12] < 1e-8
    assert s[1e-8] < 1e-6


def test_qr_rank_rule_spread_batch_instance():
    inst = workloads.uneven_batch()[1]
    s = _spread(inst, 25, 5)
    print(f"{inst.name}, 25 steps: spread 1e-8 vs 1e-10 = {s[1e-8]:.2e}, "
          f"1e-12 vs 1e-10 = {s[1e-12]:.2e}")
    assert max(s.values()) < 1e-6
