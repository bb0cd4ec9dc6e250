"""SOP term table of the bexcitonic HEOM for the C ABI (paper Eqs. heom-std,
dissipator, master_lvn).

Per feature k (bath coupling Q, metric factor f_k of Sec. VII D: 'abs'
f_k = sqrt((|c_k|+|cbar_k|)/2), 're' f_k = +-sqrt(|Re c_k + Re cbar_k|/2) with
the sign negative when Im c_k + Im cbar_k > 1e-14, or one complex constant;
a zero factor becomes 1):
  gamma_k n_k ; c_k Q> (x) a+_k/f_k ; -cbar_k Q< (x) a+_k/f_k ;
  -Q> (x) f_k a_k ; +Q< (x) f_k a_k
plus -i H> and +i H< (and -i f(t) Hd>, +i f(t) Hd< per drive slot), where
A> acts on the ket end with A and A< on the bra end with conj(A).
Ends: 0 ket, 1 bra, 2+k feature k.
"""
import numpy as np

from . import bath as _bath


class TermTable:
    """Flat arrays in the layout of tenso_build_generator."""

    def __init__(self):
        self.coef, self.slot, self.nfac, self.fend, self.mats = [], [], [], [], []

    def add(self, coef, factors, slot=-1):
        self.coef.append(complex(coef))
        self.slot.append(int(slot))
        self.nfac.append(len(factors))
        for end, mat in factors:
            self.fend.append(int(end))
            self.mats.append(np.ascontiguousarray(mat, dtype=np.complex128).reshape(-1))

    def arrays(self):
        mats = np.concatenate(self.mats) if self.mats else np.zeros(0, np.complex128)
        return (np.asarray(self.coef, np.complex128), np.asarray(self.slot, np.int32),
                np.asarray(self.nfac, np.int32), np.asarray(self.fend, np.int32), mats)

    def __len__(self):
        return len(self.coef)


_METRIC_EPS = 1e-14


def metric_factor(metric, c, cb):
    """f_k for one feature."""
    if isinstance(metric, str):
        if metric == "abs":
            f = np.sqrt((abs(c) + abs(cb)) / 2.0)
        elif metric == "re":
            f = np.sqrt(abs(c.real + cb.real) / 2.0)
            if c.imag + cb.imag > _METRIC_EPS:
                f = -f
        else:
            raise ValueError(f"unknown metric {metric!r}")
    else:
        f = complex(metric)
        if f == 0:
            raise ValueError("a metric factor must be nonzero")
    return 1.0 if f == 0 else f


def heom_table(H, baths, depth, drive_ops=(), metric="abs"):
    """baths: list of workloads.Bath-like objects (Q, T, dl, bo, n_ltc);
    metric: "abs", "re" or a complex constant (Sec. VII D).
    Returns (TermTable, feature dims)."""
    H = np.asarray(H, dtype=np.complex128)
    tab = TermTable()
    tab.add(-1j, [(0, H)])
    tab.add(1j, [(1, H.conj())])
    dims = []
    k = 0
    for b in baths:
        c, cb, g = _bath.features(b.T, b.dl, b.bo, b.n_ltc,
                                  method=getattr(b, "decomposition", "matsubara"))
        Q = np.asarray(b.Q, dtype=np.complex128)
        for j in range(len(c)):
            N = depth if np.isscalar(depth) else depth[k]
            f = metric_factor(metric, complex(c[j]), complex(cb[j]))
            n = np.arange(N, dtype=float)
            num = np.diag(n).astype(np.complex128)
            up = np.diag(np.sqrt(n[1:]) / f, -1).astype(np.complex128)
            dn = np.diag(np.sqrt(n[1:]) * f, 1).astype(np.complex128)
            e = 2 + k
            tab.add(g[j], [(e, num)])
            tab.add(c[j], [(0, Q), (e, up)])
            tab.add(-cb[j], [(1, Q.conj()), (e, up)])
            tab.add(-1.0, [(0, Q), (e, dn)])
            tab.add(1.0, [(1, Q.conj()), (e, dn)])
            dims.append(N)
            k += 1
    for slot, Hd in enumerate(drive_ops):
        Hd = np.asarray(Hd, dtype=np.complex128)
        tab.add(-1j, [(0, Hd)], slot=slot)
        tab.add(1j, [(1, Hd.conj())], slot=slot)
    return tab, dims
