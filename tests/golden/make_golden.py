"""Write the oracle trajectories that the GPU parity tests and bench.py compare with.

Every stored value comes from the FP64 CPU oracle (``oracle/``) run on the seeded
workloads of ``workloads.py``; nothing here touches the GPU library.

    python tests/golden/make_golden.py [spin_boson|exciton|batch|batch200|ps2|pade|tfd|mix|all] [--procs N]

Files (numpy .npz, no pickles):
  spin_boson_train_2000.npz   spin-boson K=3 N=10 train R=8, ps1, 2000 steps,
                              rho_S at every 10th step
  exciton_7site_50.npz        7-site exciton K=28 N=8 binary R=16, ps1, 50 steps,
                              rho_S at every 10th step
  batch512_25.npz             the 512-instance uneven batch (seed 2), ps1, 25 steps,
                              rho_S of every instance at every 5th step; instance i's
                              M_i x M_i matrices are rows offsets[i]:offsets[i+1] of
                              the flattened record arrays
  batch512_200_sample.npz     the same batch over its configured 200 steps, rho_S at
                              every 10th step, for a sample: every 32nd instance, the
                              instances a too-large RK4 step once made diverge
                              (61, 121, 153, 267, 304, 387, 429) and instance 393
                              (the largest trace drift); same record layout, with
                              `ids` naming the sampled instances and `spread` the
                              largest trace distance, over the records, between
                              the oracle at QR rank thresholds 1e-10 and 1e-12:
                              how far the truncated-rank trajectory itself
                              depends on that convention
  pade_structured_500.npz     the paper's Sec. III A 1 structured spin-boson model
                              (Pade, K=4, depth 25, train R=16, dt 0.1 fs), ps1,
                              500 steps (50 fs), rho_S at every 50th step
  tfd_spin_boson_100.npz      the paper's Sec. III A 5 thermofield ML-MCTDH listing
                              (50 star modes of Fock dimension 8, binary tree R=16,
                              1 fs steps), ps1 on the wavefunction, 100 steps, rho_S
                              at every 10th step
  mix_spin_boson_train_100.npz  the spin-boson train under the mixed strategy: ps2
                              (eps 1e-8) until a bond reaches rank 8, then vmf with
                              adaptive dopri5 (rtol 1e-5, atol 1e-7, shift 1e-7);
                              100 steps, rho_S at every 10th step, the number of ps2
                              steps before the switch (`switch`) and the accepted and
                              rejected dopri5 substeps (`accepted`, `rejected`)
  ps2_ternary_cap8_10.npz     structured bath K=24 N=10 on the ternary tree, ps2 with
                              eps 1e-6 and rank cap 8, 10 steps: rho_S at every step
                              and the rank chosen at every split (`ranks`, one row
                              per step in sweep order)
Each file stores the inputs it depends on (time steps, step counts, a digest of
the workload parameters) so that a stale file is detected instead of compared.
"""
import argparse
import hashlib
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def workload_digest(insts):
    """Digest of every input parameter of a list of workload instances."""
    h = hashlib.sha256()
    for inst in insts:
        h.update(np.ascontiguousarray(inst.H).tobytes())
        h.update(np.ascontiguousarray(inst.rho0).tobytes())
        for b in inst.baths:
            h.update(np.ascontiguousarray(b.Q).tobytes())
            h.update(repr((b.T, b.dl, b.bo, b.n_ltc)).encode())
            if getattr(b, "decomposition", "matsubara") != "matsubara":
                h.update(b.decomposition.encode())
        h.update(repr((inst.depth, inst.tree, inst.rank, inst.dt, inst.method, inst.eps,
                       None if inst.drive is None else inst.drive[1:])).encode())
        if getattr(inst, "metric", "abs") != "abs":
            h.update(repr(inst.metric).encode())
    return h.hexdigest()


def tfd_digest(inst):
    """Digest of every input parameter of a thermofield instance."""
    h = hashlib.sha256()
    for a in (inst.H, inst.Q, inst.psi0):
        h.update(np.ascontiguousarray(a).tobytes())
    h.update(repr((inst.lam, inst.w0, inst.eta, inst.T, inst.cutoff, inst.n_modes, inst.dim,
                   inst.n_ary, inst.rank, inst.dt)).encode())
    return h.hexdigest()


def load(fname, insts):
    """The stored oracle trajectories of `fname`, checked against the inputs of
    `insts` (a stale file raises instead of being compared)."""
    with np.load(os.path.join(HERE, fname), allow_pickle=False) as z:
        out = {k: z[k] for k in z.files}
    want = tfd_digest(insts[0]) if hasattr(insts[0], "psi0") else workload_digest(insts)
    if str(out["digest"]) != want:
        raise RuntimeError(f"{fname} was written for other workload inputs: rerun "
                           "tests/golden/make_golden.py")
    return out


def batch_rhos(g, record):
    """Per-instance rho_S matrices of one record of a batch file."""
    off = g["offsets"]
    out = []
    for i in range(len(off) - 1):
        m = int(round(np.sqrt(off[i + 1] - off[i])))
        out.append(g["rho"][record, off[i]:off[i + 1]].reshape(m, m))
    return out


def _single(args):
    name, n_steps, every = args
    import workloads
    from oracle.run import propagate
    inst = {"spin_boson": workloads.spin_boson_train,
            "exciton": workloads.exciton_7site,
            "pade": workloads.structured_spin_boson_pade}[name](n_steps=n_steps)
    steps, rhos, _, _ = propagate(inst, n_steps=n_steps, every=every)
    return name, inst, steps, rhos


BATCH200_IDS = sorted(set(range(0, 512, 32)) | {61, 121, 153, 267, 304, 387, 393, 429})


def _batch_one(args):
    i, n_steps, every = args[:3]
    import workloads
    import oracle.integrators as integ
    from oracle.run import propagate
    from oracle.ttn import trace_distance
    inst = workloads.uneven_batch()[i]
    steps, rhos, _, _ = propagate(inst, n_steps=n_steps, every=every)
    spread = 0.0
    if len(args) > 3 and args[3]:
        old = integ.QR_RANK_TOL
        integ.QR_RANK_TOL = 1e-12
        try:
            _, alt, _, _ = propagate(inst, n_steps=n_steps, every=every)
        finally:
            integ.QR_RANK_TOL = old
        spread = max(trace_distance(a, b) for a, b in zip(rhos, alt))
    return i, steps, rhos, spread


def _ps2(args):
    n_steps, cap = args
    import workloads
    from oracle.run import propagate
    inst = workloads.structured_bath_ternary(n_steps=n_steps)
    steps, rhos, ranks, _ = propagate(inst, n_steps=n_steps, every=1, max_rank=cap)
    return inst, steps, rhos, ranks


def write_ps2(n_steps, cap, fname, pool):
    t0 = time.time()
    inst, steps, rhos, ranks = pool.apply(_ps2, ((n_steps, cap),))
    np.savez_compressed(os.path.join(HERE, fname), steps=steps, rho=rhos,
                        ranks=np.array(ranks, dtype=np.int32), cap=cap, eps=inst.eps,
                        digest=workload_digest([inst]))
    print(f"{fname}: {len(steps)} records, {time.time() - t0:.1f} s", flush=True)


def write_single(name, n_steps, every, fname, pool):
    t0 = time.time()
    _, inst, steps, rhos = pool.apply(_single, ((name, n_steps, every),))
    np.savez_compressed(os.path.join(HERE, fname), steps=steps, rho=rhos, dt=inst.dt,
                        digest=workload_digest([inst]))
    print(f"{fname}: {len(steps)} records, {time.time() - t0:.1f} s", flush=True)


def write_tfd(n_steps, every, fname):
    import workloads
    from oracle.tfd import propagate_tfd
    t0 = time.time()
    inst = workloads.tfd_spin_boson()
    steps, rhos = propagate_tfd(inst, n_steps=n_steps, every=every)
    np.savez_compressed(os.path.join(HERE, fname), steps=steps, rho=rhos, dt=inst.dt,
                        digest=tfd_digest(inst))
    print(f"{fname}: {len(steps)} records, {time.time() - t0:.1f} s", flush=True)


def write_mix(n_steps, every, fname):
    import copy
    import workloads
    from oracle.run import build
    from oracle.ttn import initial_state
    from oracle.vmf import propagate_mix
    t0 = time.time()
    inst = workloads.spin_boson_train_mix(n_steps)
    terms, tree = build(inst)
    steps, rhos, switch, prop = propagate_mix(copy.deepcopy(tree), terms,
                                              initial_state(tree, inst.rho0), inst.dt, n_steps,
                                              inst.eps, inst.rank, every=every)
    np.savez_compressed(os.path.join(HERE, fname), steps=steps, rho=rhos, dt=inst.dt,
                        switch=switch, accepted=prop.ode.accepted, rejected=prop.ode.rejected,
                        digest=workload_digest([inst]))
    print(f"{fname}: {len(steps)} records, switch {switch}, {time.time() - t0:.1f} s", flush=True)


def write_batch(n_steps, every, fname, pool, ids=None, spread=False):
    import workloads
    insts = workloads.uneven_batch()
    ids = list(range(len(insts))) if ids is None else list(ids)
    t0 = time.time()
    res = {}
    # largest instances first, so that the pool's tail is short
    order = sorted(ids, key=lambda i: -insts[i].M * insts[i].K * insts[i].depth * insts[i].rank)
    spreads = {}
    for i, steps, rhos, sp in pool.imap_unordered(_batch_one,
                                                  [(i, n_steps, every, spread) for i in order]):
        res[i] = (steps, rhos)
        spreads[i] = sp
    steps = res[ids[0]][0]
    offsets = np.zeros(len(ids) + 1, dtype=np.int64)
    for j, i in enumerate(ids):
        offsets[j + 1] = offsets[j] + insts[i].M * insts[i].M
    rec = np.zeros((len(steps), int(offsets[-1])), dtype=np.complex128)
    for j, i in enumerate(ids):
        assert np.array_equal(res[i][0], steps)
        rec[:, offsets[j]:offsets[j + 1]] = res[i][1].reshape(len(steps), -1)
    np.savez_compressed(os.path.join(HERE, fname), steps=steps, rho=rec, offsets=offsets,
                        ids=np.array(ids), dt=np.array([x.dt for x in insts]),
                        spread=np.array([spreads[i] for i in ids]),
                        digest=workload_digest(insts))
    print(f"{fname}: {len(insts)} instances x {len(steps)} records, "
          f"{time.time() - t0:.1f} s", flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("what", nargs="?", default="all",
                    choices=["spin_boson", "exciton", "batch", "batch200", "ps2", "pade", "tfd",
                             "mix", "all"])
    ap.add_argument("--procs", type=int, default=os.cpu_count())
    a = ap.parse_args()
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    with Pool(a.procs) as pool:
        if a.what in ("spin_boson", "all"):
            write_single("spin_boson", 2000, 10, "spin_boson_train_2000.npz", pool)
        if a.what in ("exciton", "all"):
            write_single("exciton", 50, 10, "exciton_7site_50.npz", pool)
        if a.what in ("batch", "all"):
            write_batch(25, 5, "batch512_25.npz", pool)
        if a.what in ("batch200", "all"):
            write_batch(200, 10, "batch512_200_sample.npz", pool, ids=BATCH200_IDS, spread=True)
        if a.what in ("pade", "all"):
            write_single("pade", 500, 50, "pade_structured_500.npz", pool)
        if a.what in ("ps2", "all"):
            write_ps2(10, 8, "ps2_ternary_cap8_10.npz", pool)
        if a.what in ("tfd", "all"):
            write_tfd(100, 10, "tfd_spin_boson_100.npz")
        if a.what in ("mix", "all"):
            write_mix(100, 10, "mix_spin_boson_train_100.npz")


if __name__ == "__main__":
    main()
