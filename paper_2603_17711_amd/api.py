"""Thin Python layer over the C ABI: trees, generators, plans and device buffers.

Device memory and streams come from PyTorch (torch.empty on the current HIP
device, torch.cuda.current_stream()); every step of the computation runs in
libtenso.so.
"""
import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BF16, DRIVE_FN, FP32, FP32_3M, FP64, PS1, PS2, VMF, PlanOpts, VmfOpts, c128,
                   check, lib)
from .heom import heom_table


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(C.POINTER(C.c_int32))


def _c128(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a, a.ctypes.data_as(C.POINTER(c128))


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


class Tree:
    def __init__(self, handle):
        self.h = handle

    @classmethod
    def train(cls, M, dims, rank):
        d, dp = _i32(dims)
        h = C.c_void_p()
        check(lib().tenso_tree_train(M, len(dims), dp, rank, C.byref(h)))
        return cls(h)

    @classmethod
    def nary(cls, M, dims, n_ary, rank):
        d, dp = _i32(dims)
        h = C.c_void_p()
        check(lib().tenso_tree_nary(M, len(dims), dp, n_ary, rank, C.byref(h)))
        return cls(h)

    @classmethod
    def from_parents(cls, parent, end_node, end_dim, max_rank, bond_rank=None):
        p, pp = _i32(parent)
        e, ep = _i32(end_node)
        d, dp = _i32(end_dim)
        br = None
        if bond_rank is not None:
            b, br = _i32(bond_rank)
        h = C.c_void_p()
        check(lib().tenso_build_tree(len(parent), pp, len(end_node), ep, dp, max_rank, br,
                                     C.byref(h)))
        return cls(h)

    @property
    def n_nodes(self):
        return check(lib().tenso_tree_n_nodes(self.h))

    def ranks(self):
        out = np.zeros(self.n_nodes, np.int32)
        check(lib().tenso_tree_ranks(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out

    def __del__(self):
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "h", None) and L is not None:  # modules may be torn down at exit
            L.tenso_tree_destroy(self.h)
            self.h = None


class Generator:
    def __init__(self, tree, table):
        coef, slot, nfac, fend, mats = table.arrays()
        self._keep = (coef, slot, nfac, fend, mats)
        h = C.c_void_p()
        check(lib().tenso_build_generator(
            tree.h, len(coef), coef.ctypes.data_as(C.POINTER(c128)),
            slot.ctypes.data_as(C.POINTER(C.c_int32)), nfac.ctypes.data_as(C.POINTER(C.c_int32)),
            fend.ctypes.data_as(C.POINTER(C.c_int32)), mats.ctypes.data_as(C.POINTER(c128)),
            C.byref(h)))
        self.h = h
        self.n_slots = int(slot.max() + 1) if len(slot) and slot.max() >= 0 else 0

    def __del__(self):
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "h", None) and L is not None:  # modules may be torn down at exit
            L.tenso_gen_destroy(self.h)
            self.h = None


class Plan:
    """A compiled propagation problem with its device state and workspace."""

    def __init__(self, tree, gen, precision=FP32, method=PS1, max_rank=0, device="cuda"):
        import torch
        # torch owns the device: initialise it before the library's first HIP call
        torch.cuda.init()
        torch.zeros(1, device=device)
        self.tree, self.gen = tree, gen
        opts = PlanOpts(precision, method, max_rank)
        h = C.c_void_p()
        check(lib().tenso_plan_create(tree.h, gen.h, C.byref(opts), C.byref(h)))
        self.h = h
        sb, wb = C.c_size_t(), C.c_size_t()
        check(lib().tenso_plan_sizes(h, C.byref(sb), C.byref(wb)))
        self.state = torch.zeros(int(sb.value), dtype=torch.uint8, device=device)
        self.ws = torch.zeros(int(wb.value), dtype=torch.uint8, device=device)
        self.n_nodes = tree.n_nodes
        self.M = None

    def shapes(self):
        nl = np.zeros(self.n_nodes, np.int32)
        dims = np.zeros(8 * self.n_nodes, np.int32)
        check(lib().tenso_plan_shapes(self.h, nl.ctypes.data_as(C.POINTER(C.c_int32)),
                                      dims.ctypes.data_as(C.POINTER(C.c_int32))))
        return [tuple(int(x) for x in dims[8 * s:8 * s + nl[s]]) for s in range(self.n_nodes)]

    def init_state(self, rho0):
        r, rp = _c128(rho0)
        self.M = r.shape[0]
        check(lib().tenso_state_init(self.h, rp, C.c_void_p(self.state.data_ptr()), _stream()))

    def import_state(self, cores):
        flat, fp = _c128(np.concatenate([np.asarray(c).reshape(-1) for c in cores]))
        check(lib().tenso_state_import(self.h, fp, C.c_void_p(self.state.data_ptr()), _stream()))

    def export_state(self):
        shapes = self.shapes()
        n = sum(int(np.prod(s)) for s in shapes)
        out = np.zeros(n, np.complex128)
        check(lib().tenso_state_export(self.h, C.c_void_p(self.state.data_ptr()),
                                       out.ctypes.data_as(C.POINTER(c128)), None, _stream()))
        cores, o = [], 0
        for s in shapes:
            k = int(np.prod(s))
            cores.append(out[o:o + k].reshape(s).copy())
            o += k
        return cores

    def apply(self, center, drive=None, noalloc=False):
        """Effective generator at `center` (the state must be canonical toward
        it); drive: one value per slot at the time of interest.  noalloc=True
        calls the variant that allocates nothing (static scratch, no workspace)."""
        import torch
        shape = self.shapes()[center]
        out = torch.zeros(int(np.prod(shape)) * 2, dtype=torch.float64, device=self.state.device)
        dv = None
        if drive is not None:
            d = np.ascontiguousarray(drive, dtype=np.float64)
            dv = d.ctypes.data_as(C.POINTER(C.c_double))
        if noalloc:
            check(lib().tenso_apply_generator_noalloc(self.h, C.c_void_p(self.state.data_ptr()),
                                                      center, dv, C.c_void_p(out.data_ptr()),
                                                      _stream()))
        else:
            check(lib().tenso_apply_generator(self.h, C.c_void_p(self.state.data_ptr()), center, dv,
                                              C.c_void_p(out.data_ptr()),
                                              C.c_void_p(self.ws.data_ptr()), _stream()))
        o = out.cpu().numpy()
        return (o[0::2] + 1j * o[1::2]).reshape(shape)

    def step(self, n_steps, dt, t0=0.0, drive_tab=None):
        ptr = C.c_void_p(drive_tab.data_ptr()) if drive_tab is not None else None
        check(lib().tenso_step_fixed(self.h, C.c_void_p(self.state.data_ptr()), t0, dt, n_steps,
                                     ptr, C.c_void_p(self.ws.data_ptr()), _stream()))

    def set_graph(self, enable):
        """Replay steps from a captured HIP graph (default) or launch eagerly."""
        check(lib().tenso_plan_set_graph(self.h, int(bool(enable))))

    def set_tile_work(self, flops):
        """Flops per apply-kernel tile (default 16e6)."""
        check(lib().tenso_plan_set_tile_work(self.h, float(flops)))

    def step_adaptive(self, n_steps, dt, eps, max_rank, t0=0.0, drive_tab=None):
        ptr = C.c_void_p(drive_tab.data_ptr()) if drive_tab is not None else None
        check(lib().tenso_step_adaptive(self.h, C.c_void_p(self.state.data_ptr()), t0, dt,
                                        n_steps, eps, max_rank, ptr,
                                        C.c_void_p(self.ws.data_ptr()), _stream()))

    @staticmethod
    def _vmf_opts(rtol, atol, reg, fixed_substeps, max_substeps):
        return VmfOpts(float(rtol), float(atol), float(reg), int(fixed_substeps), int(max_substeps))

    @staticmethod
    def _drive_cb(drive):
        """C callback filling f_slots from drive(t) (a sequence of slot values)."""
        if drive is None:
            return DRIVE_FN()

        def cb(t, out, _ctx):
            for k, v in enumerate(drive(t)):
                out[k] = float(v)
        return DRIVE_FN(cb)

    def step_vmf(self, n_steps, dt, t0=0.0, rtol=1e-5, atol=1e-7, reg=1e-7, fixed_substeps=0,
                 max_substeps=100000, drive=None):
        """Direct integration (dopri5); drive: t -> slot values (None if undriven)."""
        o = self._vmf_opts(rtol, atol, reg, fixed_substeps, max_substeps)
        cb = self._drive_cb(drive)
        check(lib().tenso_step_vmf(self.h, C.c_void_p(self.state.data_ptr()), t0, dt, n_steps,
                                   C.byref(o), cb, None, C.c_void_p(self.ws.data_ptr()), _stream()))

    def step_mix(self, n_steps, dt, eps, max_aux_rank, t0=0.0, rtol=1e-5, atol=1e-7, reg=1e-7,
                 fixed_substeps=0, max_substeps=100000, drive=None):
        """ps2 until a bond reaches max_aux_rank, then vmf; returns the number
        of ps2 steps before the switch (-1 while still in ps2)."""
        o = self._vmf_opts(rtol, atol, reg, fixed_substeps, max_substeps)
        cb = self._drive_cb(drive)
        sw = C.c_int32()
        check(lib().tenso_step_mix(self.h, C.c_void_p(self.state.data_ptr()), t0, dt, n_steps,
                                   float(eps), int(max_aux_rank), C.byref(o), cb, None,
                                   C.c_void_p(self.ws.data_ptr()), _stream(), C.byref(sw)))
        return int(sw.value)

    def vmf_derivative(self, reg=1e-7, drive=None):
        """Time derivative of every core (list of arrays, as export_state)."""
        import torch
        out = torch.zeros_like(self.state)
        dv = None
        if drive is not None:
            d = np.ascontiguousarray(drive, dtype=np.float64)
            dv = d.ctypes.data_as(C.POINTER(C.c_double))
        check(lib().tenso_vmf_derivative(self.h, C.c_void_p(self.state.data_ptr()), float(reg), dv,
                                         C.c_void_p(out.data_ptr()),
                                         C.c_void_p(self.ws.data_ptr()), _stream()))
        shapes = self.shapes()
        n = sum(int(np.prod(sh)) for sh in shapes)
        flat = np.zeros(n, np.complex128)
        check(lib().tenso_state_export(self.h, C.c_void_p(out.data_ptr()),
                                       flat.ctypes.data_as(C.POINTER(c128)), None, _stream()))
        res, o = [], 0
        for sh in shapes:
            k = int(np.prod(sh))
            res.append(flat[o:o + k].reshape(sh).copy())
            o += k
        return res

    def set_ps2_truncation(self, atol=0.0, ratio=0.0):
        """ps2 splits keep ceil(ratio * #(sigma > atol)) directions (ratio >= 1);
        ratio = 0 restores the eps rule."""
        check(lib().tenso_plan_set_ps2_truncation(self.h, float(atol), float(ratio)))

    def vmf_stats(self):
        """(accepted, rejected, next proposed substep) of direct integration."""
        a, r, h = C.c_int64(), C.c_int64(), C.c_double()
        check(lib().tenso_vmf_stats(self.h, C.byref(a), C.byref(r), C.byref(h)))
        return int(a.value), int(r.value), float(h.value)

    def rank_log(self, cap=100000):
        out = np.zeros(cap, np.int32)
        n = check(lib().tenso_rank_trajectory(self.h, out.ctypes.data_as(C.POINTER(C.c_int32)), cap))
        return out[:n].tolist()

    def ranks(self):
        out = np.zeros(self.n_nodes, np.int32)
        check(lib().tenso_state_export(self.h, C.c_void_p(self.state.data_ptr()), None,
                                       out.ctypes.data_as(C.POINTER(C.c_int32)), _stream()))
        return out

    def rho(self):
        M = self.M
        out = np.zeros((M, M), np.complex128)
        tr = C.c_double()
        check(lib().tenso_reduced_rho(self.h, C.c_void_p(self.state.data_ptr()),
                                      out.ctypes.data_as(C.POINTER(c128)), C.byref(tr),
                                      C.c_void_p(self.ws.data_ptr()), _stream()))
        return out

    def rho_pure(self):
        """Tr_bath |psi><psi| of a wavefunction state (bra end of dimension 1)."""
        M = self.M
        out = np.zeros((M, M), np.complex128)
        tr = C.c_double()
        check(lib().tenso_reduced_rho_pure(self.h, C.c_void_p(self.state.data_ptr()),
                                           out.ctypes.data_as(C.POINTER(c128)), C.byref(tr),
                                           C.c_void_p(self.ws.data_ptr()), _stream()))
        return out

    def __del__(self):
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "h", None) and L is not None:  # modules may be torn down at exit
            L.tenso_plan_destroy(self.h)
            self.h = None


def svd_truncate(A, iso=0, eps=0.0, max_rank=None):
    """FP64 SVD of a complex matrix on the device by the ps2 split's method
    (tenso_svd_truncate).  A: complex128 array or torch tensor (rows x cols).
    Returns (sigma, vectors, (r', k, r_eps), missed): the p = min(64, rows,
    cols, 2 min(max_rank, rows, cols) + 8) leading singular values, the leading
    singular vectors of the left
    (iso 0, rows x p) or right (iso 1, cols x p) side, the truncation decision
    for (eps, max_rank) and the energy fraction outside the captured subspace."""
    import torch
    t = torch.as_tensor(A).to(device="cuda", dtype=torch.complex128).contiguous()
    rows, cols = t.shape
    mr = int(max_rank if max_rank is not None else min(rows, cols))
    p = min(64, rows, cols, 2 * min(mr, rows, cols) + 8)
    n = rows if iso == 0 else cols
    vec = torch.zeros((n, p), dtype=torch.complex128, device="cuda")
    sig = np.zeros(p)
    dec = np.zeros(3, np.int32)
    missed = C.c_double()
    check(lib().tenso_svd_truncate(C.c_void_p(t.data_ptr()), rows, cols, iso, float(eps),
                                   mr,
                                   sig.ctypes.data_as(C.POINTER(C.c_double)),
                                   C.c_void_p(vec.data_ptr()),
                                   dec.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(missed),
                                   _stream()))
    return sig, vec.cpu().numpy(), tuple(int(x) for x in dec), missed.value


def build_instance(inst, precision=FP32, rank=None, device="cuda", method=None):
    """Tree + generator + plan for a workloads.Instance (ps1, or ps2 when
    inst.method == "ps2": `rank` is then the rank cap; method overrides
    with PS1 / PS2 / VMF)."""
    drive_ops = [] if inst.drive is None else [inst.drive[0]]
    table, dims = heom_table(inst.H, inst.baths, inst.depth, drive_ops,
                             metric=getattr(inst, "metric", "abs"))
    R = inst.rank if rank is None else rank
    if inst.tree == "train":
        tree = Tree.train(inst.M, dims, R)
    else:
        tree = Tree.nary(inst.M, dims, int(inst.tree[4:]), R)
    gen = Generator(tree, table)
    if method is None:
        method = PS2 if inst.method == "ps2" else PS1
    plan = Plan(tree, gen, precision=precision, method=method, max_rank=R, device=device)
    plan.init_state(inst.rho0)
    return plan


def drive_table(inst, n_steps, t0=0.0, device="cuda"):
    """f(t0 + j dt/4), j = 0..4 n_steps, as a [1, 4n+1] device tensor (None if undriven)."""
    import torch
    if inst.drive is None:
        return None
    ts = t0 + np.arange(4 * n_steps + 1) * (inst.dt / 4.0)
    vals = np.array([inst.drive_value(t) for t in ts], dtype=np.float64)
    return torch.tensor(vals.reshape(1, -1), dtype=torch.float64, device=device)


class Batch:
    """Many independent ps1 plans advanced together (tenso_batch_*)."""

    def __init__(self, plans):
        self.plans = list(plans)
        n = len(self.plans)
        hp = (C.c_void_p * n)(*[p.h for p in self.plans])
        hs = (C.c_void_p * n)(*[p.state.data_ptr() for p in self.plans])
        hw = (C.c_void_p * n)(*[p.ws.data_ptr() for p in self.plans])
        h = C.c_void_p()
        check(lib().tenso_batch_create(n, hp, hs, hw, C.byref(h)))
        self.h = h

    def step(self, n_steps, dts, t0s=None, drive_tabs=None):
        n = len(self.plans)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dts, np.float64), (n,)))
        t0 = np.zeros(n) if t0s is None else np.ascontiguousarray(t0s, np.float64)
        tabs = None
        if drive_tabs is not None:
            tabs = (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None)
                                      for t in drive_tabs])
        check(lib().tenso_batch_step(self.h, t0.ctypes.data_as(C.POINTER(C.c_double)),
                                     dt.ctypes.data_as(C.POINTER(C.c_double)), n_steps, tabs,
                                     _stream()))

    def step_record(self, n_steps, dts, every, t0s=None, drive_tabs=None):
        """As step(), recording every instance's rho_S before the first step and
        after every `every` steps (tenso_batch_step_record).  Returns a list of
        records, each a list of per-instance M_i x M_i complex arrays."""
        import torch
        n = len(self.plans)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dts, np.float64), (n,)))
        t0 = np.zeros(n) if t0s is None else np.ascontiguousarray(t0s, np.float64)
        nb = C.c_size_t()
        offs = (C.c_size_t * n)()
        check(lib().tenso_batch_record_bytes(self.h, C.byref(nb), offs))
        n_rec = n_steps // every + 1
        buf = torch.zeros(n_rec * int(nb.value), dtype=torch.uint8,
                          device=self.plans[0].state.device)
        tabs = None
        if drive_tabs is not None:
            tabs = (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None)
                                      for t in drive_tabs])
        check(lib().tenso_batch_step_record(self.h, t0.ctypes.data_as(C.POINTER(C.c_double)),
                                            dt.ctypes.data_as(C.POINTER(C.c_double)), n_steps,
                                            every, tabs, C.c_void_p(buf.data_ptr()), _stream()))
        raw = buf.cpu().numpy()
        out = []
        for j in range(n_rec):
            rec = raw[j * int(nb.value):(j + 1) * int(nb.value)]
            mats = []
            for i, p in enumerate(self.plans):
                a = rec[offs[i]:offs[i] + 16 * p.M * p.M].view(np.complex128)
                mats.append(a.reshape(p.M, p.M).copy())
            out.append(mats)
        return out

    def set_graph(self, enable):
        """Replay batched steps from a captured HIP graph (default) or launch eagerly."""
        check(lib().tenso_batch_set_graph(self.h, int(bool(enable))))

    def status(self):
        """Per instance: True where the last step call found NaN/inf in its state."""
        out = np.zeros(len(self.plans), np.int32)
        check(lib().tenso_batch_status(self.h, out.ctypes.data_as(C.POINTER(C.c_int32))))
        return out.astype(bool)

    def set_parts(self, n_parts):
        """Independent parts of a step (1..4), parallel branches of the step graph."""
        check(lib().tenso_batch_set_parts(self.h, int(n_parts)))

    def autotune(self, dts, trial_steps=2, drive_tabs=None):
        """Pick the fastest apply tile size for this batch (states are restored
        exactly); returns it in flops."""
        import torch
        n = len(self.plans)
        dt = np.ascontiguousarray(np.broadcast_to(np.asarray(dts, np.float64), (n,)))
        nb = C.c_size_t()
        check(lib().tenso_batch_state_bytes(self.h, C.byref(nb)))
        backup = torch.empty(int(nb.value), dtype=torch.uint8, device=self.plans[0].state.device)
        tabs = None
        if drive_tabs is not None:
            tabs = (C.c_void_p * n)(*[(t.data_ptr() if t is not None else None)
                                      for t in drive_tabs])
        out = C.c_double()
        check(lib().tenso_batch_autotune(self.h, dt.ctypes.data_as(C.POINTER(C.c_double)),
                                         int(trial_steps), tabs, C.c_void_p(backup.data_ptr()),
                                         int(nb.value), C.byref(out), _stream()))
        return float(out.value)

    def rho(self):
        outs = [np.zeros((p.M, p.M), np.complex128) for p in self.plans]
        ptrs = (C.POINTER(c128) * len(outs))(*[o.ctypes.data_as(C.POINTER(c128)) for o in outs])
        check(lib().tenso_batch_reduced_rho(self.h, ptrs, _stream()))
        return outs

    def __del__(self):
        L = getattr(_lib, "_lib", None) if _lib is not None else None
        if getattr(self, "h", None) and L is not None:  # modules may be torn down at exit
            L.tenso_batch_destroy(self.h)
            self.h = None
