"""Tree tensor networks for the EDO (paper Sec. II C).

Omega[i, j, n_1..n_K] = Con(A^(0), U^(1), ..., U^(K-1)) (Eq. omega_tensor and
the general-tree equation after it).  The root A^(0) carries the system legs
(i, j); the other cores are semi-unitary (Eq. semiunitary): rows indexed by the
leg toward the root are orthonormal.

Data layout used throughout the oracle
--------------------------------------
* ``parent[s]``: parent node of s (parent[0] = -1, node 0 is the root).
* ``end_node[e]``: node that holds end e (0 = ket, 1 = bra, 2+k = feature k).
* Legs of node s, in order: the bond to its parent (if s is not the root), then
  the ends attached to s in increasing end index, then its child nodes in
  increasing node id.  Core s is a dense complex128 array with one axis per leg.
* ``rank[s]`` (s >= 1) is the dimension of the bond between s and parent[s].

Readings (documented; the paper leaves these open):
* n-ary tree ("treeN"): the root holds ket, bra and one bond to the tree built
  over all features; a list of features becomes a single end if it has one
  element, a node holding them as ends if it has at most n, otherwise a node
  with n children built over contiguous near-equal chunks (larger first).
* Train: root(ket, bra, ->1); node s holds feature s-1 and a bond to s+1; the
  last node holds the last two features (Eq. omega_tensor).
* Ranks are clamped until every core can be semi-unitary: the bond between a
  parent p and child c is at most the product of c's other leg dimensions and
  at most the product of p's other leg dimensions.
* Initial state: root[i, j, 0, ...] = rho_S(0)[i, j]; any other core
  U[a, beta] = delta(a, flat(beta)) (row-major flat index over its non-parent
  legs).  This is rho_S(0) (x) |0..0>, and the rows are orthonormal.

Pins (tests): dense contraction of the initial state equals rho_S (x) vacuum;
the environment-based effective generator equals the gradient of
<Omega, L Omega> with respect to conj(core) computed by dense brute force, for
random tiny trees of every shape and every center (exact to round-off).
"""
import numpy as np


class Tree:
    """Topology + bond ranks (the paper's Frame plus a rank per bond)."""

    def __init__(self, parent, end_node, end_dims, ranks=None, max_rank=None):
        self.parent = list(parent)
        self.n = len(self.parent)
        assert self.parent[0] == -1
        for s in range(1, self.n):
            assert 0 <= self.parent[s] < s, "parents must precede children"
        self.end_node = list(end_node)
        self.end_dims = list(end_dims)
        self.children = [[c for c in range(self.n) if self.parent[c] == s]
                         for s in range(self.n)]
        self.ends = [[e for e in range(len(self.end_node)) if self.end_node[e] == s]
                     for s in range(self.n)]
        assert 0 in self.ends[0] and 1 in self.ends[0], "root holds ket and bra"
        # legs: ('p', parent) / ('e', end) / ('c', child)
        self.legs = []
        for s in range(self.n):
            lg = [] if s == 0 else [('p', self.parent[s])]
            lg += [('e', e) for e in self.ends[s]]
            lg += [('c', c) for c in self.children[s]]
            self.legs.append(lg)
        # subtree ends
        self.sub_ends = [set() for _ in range(self.n)]
        for s in reversed(range(self.n)):
            self.sub_ends[s] |= set(self.ends[s])
            for c in self.children[s]:
                self.sub_ends[s] |= self.sub_ends[c]
        if ranks is None:
            ranks = [0] + [max_rank] * (self.n - 1)
        self.rank = list(ranks)
        self._clamp()

    def leg_dim(self, s, leg):
        kind, x = leg
        if kind == 'p':
            return self.rank[s]
        if kind == 'e':
            return self.end_dims[x]
        return self.rank[x]

    def shape(self, s):
        return tuple(self.leg_dim(s, l) for l in self.legs[s])

    def leg_of_child(self, s, c):
        return self.legs[s].index(('c', c))

    def _clamp(self):
        changed = True
        while changed:
            changed = False
            for c in range(1, self.n):
                p = self.parent[c]
                lo = int(np.prod([self.leg_dim(c, l) for l in self.legs[c][1:]]))
                hi = int(np.prod([self.leg_dim(p, l) for l in self.legs[p]
                                  if l != ('c', c)]))
                r = min(self.rank[c], lo, hi)
                if r != self.rank[c]:
                    self.rank[c] = r
                    changed = True

    def preorder(self, s=0):
        out = [s]
        for c in self.children[s]:
            out += self.preorder(c)
        return out


def train_tree(M, mode_dims, rank):
    """Tensor train (Eq. omega_tensor)."""
    K = len(mode_dims)
    end_dims = [M, M] + list(mode_dims)
    if K <= 1:
        return Tree([-1], [0, 0] + [0] * K, end_dims, max_rank=rank)
    parent = [-1] + list(range(K - 1))
    end_node = [0, 0] + [k + 1 for k in range(K - 1)] + [K - 1]
    return Tree(parent, end_node, end_dims, max_rank=rank)


def nary_tree(M, mode_dims, n_ary, rank):
    """Balanced n-ary tree ("treeN"), preorder node numbering."""
    K = len(mode_dims)
    end_dims = [M, M] + list(mode_dims)
    parent = [-1]
    end_node = [0, 0] + [None] * K

    def chunks(lst, n):
        q, r = divmod(len(lst), n)
        out, i = [], 0
        for j in range(n):
            sz = q + (1 if j < r else 0)
            out.append(lst[i:i + sz])
            i += sz
        return out

    def build(feats, holder):
        if len(feats) == 1:
            end_node[2 + feats[0]] = holder
            return
        me = len(parent)
        parent.append(holder)
        if len(feats) <= n_ary:
            for f in feats:
                end_node[2 + f] = me
        else:
            for ch in chunks(feats, n_ary):
                build(ch, me)

    if K:
        build(list(range(K)), 0)
    return Tree(parent, end_node, end_dims, max_rank=rank)


# --------------------------------------------------------------------------
# state
# --------------------------------------------------------------------------

def initial_state(tree, rho0):
    cores = []
    for s in range(tree.n):
        shp = tree.shape(s)
        C = np.zeros(shp, dtype=np.complex128)
        if s == 0:
            idx = (slice(None), slice(None)) + (0,) * (len(shp) - 2)
            C[idx] = rho0
        else:
            flat = C.reshape(shp[0], -1)
            for a in range(shp[0]):
                flat[a, a] = 1.0
            C = flat.reshape(shp)
        cores.append(C)
    return cores


def contract_dense(tree, cores):
    """Omega[e_0, e_1, ...] by contracting every bond (the Con() operation)."""
    def sub(s):
        # returns tensor with axes: [parent leg (if s>0)] + sorted sub-ends of s
        T = cores[s]
        axes = []  # label of each current axis: ('p',) or ('e', e)
        for leg in tree.legs[s]:
            axes.append(leg if leg[0] != 'c' else leg)
        # contract child tensors one by one
        for c in tree.children[s]:
            Tc, cax = sub(c)  # cax[0] == ('p',)
            i = axes.index(('c', c))
            T = np.tensordot(T, Tc, axes=([i], [0]))
            axes = axes[:i] + axes[i + 1:] + cax[1:]
        return T, axes

    T, axes = sub(0)
    order = [axes.index(('e', e)) for e in range(len(tree.end_dims))]
    return np.transpose(T, order)


def mode_product(T, X, leg):
    """(X x_leg T)[.., a, ..] = sum_a' X[a, a'] T[.., a', ..]."""
    out = np.tensordot(X, T, axes=([1], [leg]))
    return np.moveaxis(out, 0, leg)


def is_isometry_toward(C, leg, tol=1e-10):
    """Rows indexed by `leg` orthonormal over the other legs."""
    Cm = np.moveaxis(C, leg, 0).reshape(C.shape[leg], -1)
    return np.abs(Cm.conj() @ Cm.T - np.eye(Cm.shape[0])).max() < tol


# --------------------------------------------------------------------------
# environments (mean fields) and effective generators
# --------------------------------------------------------------------------

class Envs:
    """Per-term environment matrices.

    down[x][m]: for the subtree under x, seen through the bond (x, parent(x));
        D[a', a] = sum_beta conj(C_x[a', beta]) ((x)_l X_{m,l} C_x)[a, beta]
        with X = child down-envs / end factors.  None = identity (term m has no
        factor in the subtree).
    up[x][m]: for the complement of the subtree of x, computed from the parent
        core p with X = up[p] on p's parent leg and down / factors elsewhere.
    """

    def __init__(self, tree, terms):
        self.tree = tree
        self.terms = terms
        self.down = [[None] * len(terms) for _ in range(tree.n)]
        self.up = [[None] * len(terms) for _ in range(tree.n)]

    def leg_op(self, s, leg, m):
        """X_{m,leg} at node s (None = identity)."""
        kind, x = leg
        if kind == 'p':
            return self.up[s][m]
        if kind == 'e':
            return self.terms[m]['factors'].get(x)
        return self.down[x][m]

    def _sandwich(self, C, open_leg, ops):
        """sum over all legs but open_leg of conj(C) * ((x) ops) C."""
        T = C
        for leg, X in ops:
            T = mode_product(T, X, leg)
        Cm = np.moveaxis(C, open_leg, 0).reshape(C.shape[open_leg], -1)
        Tm = np.moveaxis(T, open_leg, 0).reshape(T.shape[open_leg], -1)
        return Cm.conj() @ Tm.T

    def update_down(self, x, C):
        """Recompute down[x] from core x (an isometry toward its parent)."""
        tr = self.tree
        for m in range(len(self.terms)):
            if not (set(self.terms[m]['factors']) & tr.sub_ends[x]):
                self.down[x][m] = None
                continue
            ops = []
            for i, leg in enumerate(tr.legs[x]):
                if leg[0] == 'p':
                    continue
                X = self.leg_op(x, leg, m)
                if X is not None:
                    ops.append((i, X))
            self.down[x][m] = self._sandwich(C, 0, ops)

    def update_up(self, x, Cp):
        """Recompute up[x] from the parent core (an isometry toward x)."""
        tr = self.tree
        p = tr.parent[x]
        open_leg = tr.leg_of_child(p, x)
        for m in range(len(self.terms)):
            if set(self.terms[m]['factors']) <= tr.sub_ends[x]:
                self.up[x][m] = None
                continue
            ops = []
            for i, leg in enumerate(tr.legs[p]):
                if i == open_leg:
                    continue
                X = self.leg_op(p, leg, m)
                if X is not None:
                    ops.append((i, X))
            self.up[x][m] = self._sandwich(Cp, open_leg, ops)


def apply_node(envs, s, C, drive):
    """Effective generator at center s: sum_m coef_m (x)_l X_{m,l} C."""
    from .sop import term_coef
    tr = envs.tree
    Y = np.zeros_like(C)
    for m, term in enumerate(envs.terms):
        T = C
        for i, leg in enumerate(tr.legs[s]):
            X = envs.leg_op(s, leg, m)
            if X is not None:
                T = mode_product(T, X, i)
        Y += term_coef(term, drive) * T
    return Y


def apply_bond(envs, c, B, drive):
    """Effective generator on the bond matrix between parent(c) and c:
    K(B) = sum_m coef_m U_m[c] B D_m[c]^T."""
    from .sop import term_coef
    Y = np.zeros_like(B)
    for m, term in enumerate(envs.terms):
        T = B
        U, D = envs.up[c][m], envs.down[c][m]
        if U is not None:
            T = U @ T
        if D is not None:
            T = T @ D.T
        Y += term_coef(term, drive) * T
    return Y


def two_site_legs(tree, s, c):
    """Legs of Theta = C_s joined with C_c over their bond:
    s's legs except the one to c, then c's legs except its parent leg."""
    i = tree.leg_of_child(s, c)
    return ([(s, l) for j, l in enumerate(tree.legs[s]) if j != i] +
            [(c, l) for l in tree.legs[c][1:]])


def merge(tree, cores, s, c):
    i = tree.leg_of_child(s, c)
    T = np.tensordot(cores[s], cores[c], axes=([i], [0]))
    return T  # axes: s legs without i, then c legs 1..


def apply_two_site(envs, s, c, Theta, drive):
    """Effective generator on the merged tensor of nodes s and c."""
    from .sop import term_coef
    tr = envs.tree
    legs = two_site_legs(tr, s, c)
    Y = np.zeros_like(Theta)
    for m, term in enumerate(envs.terms):
        T = Theta
        for i, (node, leg) in enumerate(legs):
            X = envs.leg_op(node, leg, m)
            if X is not None:
                T = mode_product(T, X, i)
        Y += term_coef(term, drive) * T
    return Y


# --------------------------------------------------------------------------
# observables
# --------------------------------------------------------------------------

def reduced_rho(tree, cores):
    """rho_S = <0..0|Omega> (Sec. II B), contracted bottom-up; any gauge."""
    def vec(s):
        T = cores[s]
        # contract legs from the last to the first so indices stay valid
        for i in reversed(range(len(tree.legs[s]))):
            kind, x = tree.legs[s][i]
            if kind == 'p':
                continue
            if kind == 'e':
                if s == 0 and x in (0, 1):
                    continue
                T = np.take(T, 0, axis=i)
            else:
                T = np.tensordot(T, vec(x), axes=([i], [0]))
        return T
    return vec(0)


def trace_distance(r1, r2):
    return 0.5 * np.linalg.svd(r1 - r2, compute_uv=False).sum()
