"""Sequential FP64 LoRaSp / GC factorization and solve (oracle; test infrastructure only).

Every function below follows the paper's block-matrix description step by step, one
super node at a time, with NumPy/SciPy dense kernels as the only primitives:

* ``compress``      §3.2 "Compression" (eq. local_compression, compression_sw) and §6
                    "Preserving a vector during compression" (eq. compression_xy,
                    eq. preserve, the U1/U2 construction that follows it).
* ``pivot``         §3.2 "Elimination" (S = U^T A_ss^-1 U) and Appendix A
                    (P_ss := S^-1 U^T A_ss^-1, M_ss := A_ss^-1 - P_ss^T S P_ss).
* ``eliminate_node`` one round of compression, extension (eq. extended) and
                    elimination (eq. extended_rearranged, K = L K2 L^T), producing the
                    blocks of A^(i+1): A_nn - A_ns M_ss A_sn on the neighbours,
                    S^-1 on the new red node, A_ns P_ss^T towards the neighbours and R
                    towards the well-separated nodes.
* ``factor``        Algorithm "Setup": merge sibling red nodes, eliminate every super
                    node of the level, recurse on the parent level, exact root.
* ``apply``         Algorithm "Solve" (forward substitution, restriction, parent
                    solve, prolongation, backward substitution in reverse order).

Readings of points the paper leaves open (each also used by the GPU library, which
implements them separately):

R1  eps is relative and spectral: keep singular values sigma_j > eps * sigma_1(A_sw).
    For GC the kept part of (I - U1 U1^T) A_sw is measured against sigma_1(A_sw)
    itself (§6: ||E|| / ||A_sw|| < eps).
R2  eps == 0 means no truncation: keep min(m - |U1|, |W|) directions, so the
    extension is exact (equivalent-extension lemma, §4).
R4  U1 = orthonormal basis of [phi_s, A_sw phi_w] by modified Gram-Schmidt with one
    re-orthogonalisation; a column is dropped when its remainder is <= 1e-10 of its
    norm. U2 lives in the orthogonal complement of U1 (Householder completion).
R5  A super node with no well-separated block keeps k = 0 (exact elimination, empty
    red node), for both variants. A super node with well-separated blocks keeps at
    least one column (the first unit vector when A_sw is exactly zero). Nodes of size 0
    are dropped from the block pattern.
R7  When k = m (U square and invertible) M_ss is set to exactly zero, the value
    Appendix A gives for that case; otherwise the fill it creates would be rounding
    noise, and compressing noise against a relative threshold is not reproducible.
R6  Neighbour = footprint adjacency in the original graph (§3.1); a red node has the
    footprint of its super node; N(s) / W(s) are the nodes with a block to s that are /
    are not neighbours.
R8  Elimination order inside a level (§3.2 only asks for "a given ordering"): colour
    by colour; each colour is chosen greedily among the remaining super nodes, taking a
    node only if it has no block to a node already in the colour. The pass visits the
    nodes in index order (order="index") or (order="waiting", the default) first the
    nodes with the most partners (nodes with a block to them) still remaining, ties by
    lower index. Inside a colour, nodes are eliminated in index order.
R10 The parent-level super node I is the merge of red nodes 2I and 2I+1 of the level
    below (the two halves of its bisection).
R11 A_nb in the formula for A~~_nn is A_ns A_ss^-1 U, so A~~_nn = A_nn - A_ns M_ss A_sn.
R12 The compressed blocks in Algorithm "Setup" are A_sw and A_ws (as in §3.2).
R13 The red-node right-hand side starts at 0; the forward loop runs in elimination
    order and uses the current right-hand side of each super node.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

from .tree import tree_depth, cluster_leaves, leaf_index, footprint_adjacency, GeometricNeighbours

LORASP = 0
GC = 1          # preserve the given vectors (constant vector by default)
GC_PROJ1 = 2    # approximately preserve them: first-order one-sided projection (Appendix B)

ORTH_DROP_TOL = 1e-10


class NotSPDError(RuntimeError):
    def __init__(self, msg, depth=None, node=None):
        super().__init__(msg)
        self.depth = depth
        self.node = node


# ---------------------------------------------------------------------------
# Compression (§3.2 eq. local_compression; §6 eq. compression_xy / preserve)
# ---------------------------------------------------------------------------
def orth_columns(Z: np.ndarray, tol: float = ORTH_DROP_TOL) -> np.ndarray:
    """Orthonormal basis of the columns of Z, in column order (reading R4)."""
    m = Z.shape[0]
    basis: list[np.ndarray] = []
    for j in range(Z.shape[1]):
        z = Z[:, j]
        nz = np.linalg.norm(z)
        if nz == 0.0 or len(basis) >= m:
            continue
        v = z.copy()
        for _ in range(2):
            for q in basis:
                v -= (q @ v) * q
        nv = np.linalg.norm(v)
        if nv > tol * nz:
            basis.append(v / nv)
    if not basis:
        return np.zeros((m, 0))
    return np.column_stack(basis)


def truncated_left_basis(Z: np.ndarray, eps1: float, margins: list | None = None) -> np.ndarray:
    """Leading left singular vectors of Z with sigma_j > eps1 sigma_1(Z) (Appendix B, first
    step of the first-order one-sided projection); eps1 = 0 gives an orthonormal basis of Z's
    range (reading R4, as GC)."""
    if eps1 == 0.0:
        return orth_columns(Z)
    keep = [j for j in range(Z.shape[1]) if np.linalg.norm(Z[:, j]) > 0.0]
    Z = Z[:, keep]
    if Z.shape[1] == 0:
        return np.zeros((Z.shape[0], 0))
    Uz, sz, _ = np.linalg.svd(Z, full_matrices=False)
    if margins is not None and sz[0] > 0.0:
        margins.append(float(np.min(np.abs(sz / sz[0] - eps1))))
    return Uz[:, :int(np.count_nonzero(sz > eps1 * sz[0]))]


def compress(A_sw: np.ndarray, eps: float, variant: int,
             phi_s: np.ndarray | None = None, phi_w: np.ndarray | None = None,
             margins: list | None = None, eps1: float = 0.0) -> np.ndarray:
    """Orthonormal U (m x k) for the low-rank part of the well-separated block A_sw.

    LoRaSp: U = leading left singular vectors of A_sw with sigma_j > eps * sigma_1.
    GC:     U1 = orth([phi_s, A_sw phi_w]); U2 = leading left singular vectors of
            A_sw projected on the complement of U1, with sigma_j > eps * sigma_1(A_sw);
            U = [U1, U2]. Then A_sw phi_w and phi_s lie in span U (eq. preserve), so
            U U^T A_sw phi_w = A_sw phi_w and R U^T phi_s = A_ws phi_s (eq. compression_xy).

    ``margins``, when given, receives min_j |sigma_j / sigma_1(A_sw) - eps| over the singular
    values the threshold decides on (reading R16: a rank decided within 1e-9 of the
    threshold can flip under rounding, so a parity case must keep clear of it).
    """
    m, wt = A_sw.shape
    sigma1 = np.linalg.svd(A_sw, compute_uv=False)[0] if min(m, wt) > 0 else 0.0
    if variant == LORASP:
        U1 = np.zeros((m, 0))
        Qc = np.eye(m)
    else:
        Z = np.hstack([phi_s.reshape(m, -1), (A_sw @ phi_w).reshape(m, -1)])
        U1 = truncated_left_basis(Z, eps1, margins) if variant == GC_PROJ1 else orth_columns(Z)
        q = U1.shape[1]
        Qc = np.linalg.qr(U1, mode="complete")[0][:, q:] if q > 0 else np.eye(m)
    Bc = Qc.T @ A_sw                                   # (I - U1 U1^T) A_sw in complement coords
    cap = min(Bc.shape[0], wt)
    if cap > 0:
        Ub, sb, _ = np.linalg.svd(Bc, full_matrices=False)
    else:
        Ub, sb = np.zeros((Bc.shape[0], 0)), np.zeros(0)
    if eps == 0.0:
        k2 = cap                                        # R2: no truncation
    else:
        k2 = int(np.count_nonzero(sb[:cap] > eps * sigma1))
        if margins is not None and cap > 0 and sigma1 > 0.0:
            margins.append(float(np.min(np.abs(sb[:cap] / sigma1 - eps))))
    if U1.shape[1] + k2 == 0 and cap > 0:
        k2 = 1                                          # R5: keep at least one direction
        if sigma1 == 0.0:                               # A_sw exactly zero: first unit vector
            return np.eye(m)[:, :1]
    return np.hstack([U1, Qc @ Ub[:, :k2]])


# ---------------------------------------------------------------------------
# Pivot (Appendix A: P_ss, M_ss)
# ---------------------------------------------------------------------------
def pivot(A_ss: np.ndarray, U: np.ndarray):
    """Return (M_ss, P_ss, S, S^-1) for the super-node block A_ss and basis U.

    S = U^T A_ss^-1 U, P_ss = S^-1 U^T A_ss^-1, M_ss = A_ss^-1 - P_ss^T S P_ss.
    Raises NotSPDError when the Cholesky factorisation of A_ss (or of S) fails.
    """
    m = A_ss.shape[0]
    try:
        c = sla.cho_factor(A_ss, lower=True, check_finite=True)
    except np.linalg.LinAlgError as e:
        raise NotSPDError(f"pivot block not positive definite: {e}") from e
    Ainv = sla.cho_solve(c, np.eye(m))
    k = U.shape[1]
    S = U.T @ Ainv @ U
    if k > 0:
        try:
            cs = sla.cho_factor(S, lower=True)
        except np.linalg.LinAlgError as e:
            raise NotSPDError(f"S = U^T A_ss^-1 U not positive definite: {e}") from e
        Sinv = sla.cho_solve(cs, np.eye(k))
    else:
        Sinv = np.zeros((0, 0))
    P = Sinv @ U.T @ Ainv
    if k == m:
        M = np.zeros((m, m))      # U invertible: M_ss vanishes (Appendix A)
    else:
        M = Ainv - P.T @ S @ P
    return M, P, S, Sinv


# ---------------------------------------------------------------------------
# The current block matrix of one level
# ---------------------------------------------------------------------------
@dataclass
class LevelState:
    """Current matrix at depth d: dense blocks between current nodes (both orientations)."""

    d: int
    blocks: dict = field(default_factory=dict)      # (i, j) -> ndarray (|i| x |j|)
    partners: dict = field(default_factory=dict)    # i -> set of j != i with a block
    size: dict = field(default_factory=dict)        # i -> current size
    phi: dict = field(default_factory=dict)         # i -> current preserved vectors (|i| x p)
    state: dict = field(default_factory=dict)       # i -> 'S' (super) or 'R' (red)

    def set_block(self, i, j, B):
        self.blocks[(i, j)] = B
        if i != j:
            self.blocks[(j, i)] = B.T.copy()
            self.partners.setdefault(i, set()).add(j)
            self.partners.setdefault(j, set()).add(i)

    def drop_node(self, i):
        for j in list(self.partners.get(i, ())):
            del self.blocks[(i, j)]
            del self.blocks[(j, i)]
            self.partners[j].discard(i)
        self.partners.pop(i, None)
        self.blocks.pop((i, i), None)


@dataclass
class NodeFactor:
    """What the solve phase needs from one eliminated super node."""

    s: int
    m: int
    k: int
    M: np.ndarray                 # M_ss (m x m)
    P: np.ndarray                 # P_ss (k x m)
    nbrs: list                    # [(n, 'S' or 'R' at elimination time, A_ns)]
    W: list                       # well-separated partners (indices), for inspection
    U: np.ndarray                 # compression basis (m x k)
    Wstate: list = None           # 'S' / 'R' of each well-separated partner at elimination


@dataclass
class LevelFactor:
    d: int
    colours: list                 # list of lists of super nodes
    nodes: dict                   # s -> NodeFactor
    super_size: dict              # s -> m_s (0 for empty)
    child_size: dict              # s -> (k_{2s}, k_{2s+1}) red sizes of depth d+1
    red_size: dict                # s -> k_s

    @property
    def order(self):
        return [s for c in self.colours for s in c]


@dataclass
class Factorization:
    n: int
    L: int
    leaves: list                  # 2^L arrays of original indices
    levels: dict                  # d -> LevelFactor (d = L-1 ... 0)
    eps: float
    variant: int
    root_chol: object = None      # only when L == 0
    margins: list = field(default_factory=list)   # R16 margin of every thresholded compression
    level_eps: dict = field(default_factory=dict)  # d -> compression tolerance used at depth d

    def ranks(self, d):
        return [self.levels[d].red_size.get(s, 0) for s in range(1 << d)]

    @property
    def tie_margin(self) -> float:
        """Smallest |sigma_j / sigma_1 - eps| met by any rank decision (R16); inf if none."""
        return min(self.margins) if self.margins else float("inf")


EPS_SCHEDULES = ("constant", "shrink", "grow")


def level_eps(eps: float, schedule: str, d: int, L: int, n: int, dim: int) -> float:
    """Compression tolerance at depth d (§7.1 "3D cases", Table 3 and the list before it).

    The leaf level of the schedules is the first super-node depth lmax = L - 1.
    constant: eps.  shrink: eps 2^((d - lmax)/3), the paper's adaptive GC choice (eps at the
    leaves, smaller toward the root).  grow: eps h 2^((lmax - d)/3) with h = n^(-1/dim), the
    paper's adaptive LoRaSp choice (small at the leaves, larger toward the root).
    """
    lmax = max(L - 1, 0)
    if schedule == "constant":
        return eps
    if schedule == "shrink":
        return eps * 2.0 ** ((d - lmax) / 3.0)
    if schedule == "grow":
        h = float(n) ** (-1.0 / max(1, dim))
        return eps * h * 2.0 ** ((lmax - d) / 3.0)
    raise ValueError(f"unknown eps schedule {schedule!r}")


def eliminate_node(st: LevelState, s: int, adj: set, eps: float, variant: int,
                   margins: list | None = None, eps1: float = 0.0) -> NodeFactor:
    """Compress, extend and eliminate super node s of the current level state.

    §3.2: N(s) are the current nodes with a block to s that are neighbours of s, W(s)
    the ones that are not. After the step the red node r(s) takes index s with blocks
    A_rr = S^-1, A_nr = A_ns P_ss^T (= L_nb), A_wr = R_w, and A_n1n2 -= A_n1s M_ss A_sn2.
    """
    partners = sorted(st.partners.get(s, ()))
    N = [j for j in partners if (s, j) in adj]
    W = [j for j in partners if (s, j) not in adj]
    A_ss = st.blocks[(s, s)]
    m = A_ss.shape[0]
    if W:
        A_sW = np.hstack([st.blocks[(s, w)] for w in W])
        phi_s = st.phi.get(s)
        phi_W = np.vstack([st.phi[w] for w in W]) if variant != LORASP else None
        U = compress(A_sW, eps, variant, phi_s, phi_W, margins=margins, eps1=eps1)
        RT = U.T @ A_sW                               # R^T = U^T A_sw (eq. compression_sw)
    else:
        A_sW = np.zeros((m, 0))
        U = np.zeros((m, 0))
        RT = np.zeros((0, 0))
    k = U.shape[1]
    try:
        M, P, S, Sinv = pivot(A_ss, U)
    except NotSPDError as e:
        e.node = s
        e.depth = st.d
        raise
    A_Ns = {n: st.blocks[(n, s)].copy() for n in N}

    # Schur complement on the neighbours: A~~_nn = A_nn - A_ns M_ss A_sn
    for a, n1 in enumerate(N):
        T1 = A_Ns[n1] @ M
        for n2 in N[a:]:
            upd = T1 @ A_Ns[n2].T
            old = st.blocks.get((n1, n2))
            if old is None:
                old = np.zeros((st.size[n1], st.size[n2]))
            st.set_block(n1, n2, old - upd)

    # Replace s by its red node r(s)
    phi_s = st.phi.get(s)
    st.drop_node(s)
    st.state[s] = "R"
    st.size[s] = k
    if k > 0:
        st.set_block(s, s, Sinv)                          # A_rr = S^-1
        for n in N:
            st.set_block(n, s, A_Ns[n] @ P.T)          # L_nb = A_ns A_ss^-1 U S^-1
        col = 0
        for w in W:
            width = st.size[w]
            st.set_block(s, w, RT[:, col:col + width])  # block (r, w) = R^T restricted to w
            col += width
        if variant != LORASP:
            st.phi[s] = U.T @ phi_s                     # parent-level preserved vector
    else:
        st.phi.pop(s, None)
    return NodeFactor(s=s, m=m, k=k, M=M, P=P, nbrs=[(n, None, A_Ns[n]) for n in N],
                      W=W, U=U)


def _leaf_blocks(row_ptr, col_idx, values, leaves, leaf_of, n):
    local = np.empty(n, dtype=np.int64)
    for c in leaves:
        local[c] = np.arange(len(c))
    blocks = {}
    rp = np.asarray(row_ptr, dtype=np.int64)
    for u in range(n):
        iu = leaf_of[u]
        for t in range(rp[u], rp[u + 1]):
            v = int(col_idx[t])
            key = (iu, int(leaf_of[v]))
            B = blocks.get(key)
            if B is None:
                B = np.zeros((len(leaves[key[0]]), len(leaves[key[1]])))
                blocks[key] = B
            B[local[u], local[v]] += values[t]
    return blocks


def factor(row_ptr, col_idx, values, coords=None, leaf: int = 16, eps: float = 1e-2,
           variant: int = GC, phi: np.ndarray | None = None,
           eps_schedule: str = "constant", neighbours: str = "footprint",
           eps1: float = 0.0, order: str = "waiting") -> Factorization:
    """Algorithm "Setup": build the hierarchical factorization of the SPD matrix A.

    ``phi`` (n x p) are the vectors GC preserves; default is the constant vector
    (GC-constant). Ignored for LoRaSp. ``eps_schedule`` picks the per-level tolerance
    (see ``level_eps``; dim is the coordinate dimension, 1 without coordinates).
    ``neighbours``: "footprint" (R6, the original graph's adjacency, §3.1) or "geometric"
    (R6g, the distance rule of §7's experiments, ``GeometricNeighbours``).
    ``order``: how each colour's greedy pass visits the remaining nodes (R8): "waiting"
    (most partners still remaining first) or "index".
    ``variant = GC_PROJ1`` approximately preserves ``phi`` (the vectors X of Appendix B, e.g.
    eigenvectors divided by their eigenvalues): U1 keeps the singular directions of
    [X_s, A_sw X_w] above eps1 times the largest, then U2 is chosen as for GC.
    """
    n = len(row_ptr) - 1
    L = tree_depth(n, leaf)
    leaves = cluster_leaves(coords, n, L)
    leaf_of = leaf_index(leaves, n)
    if variant != LORASP:
        phi = np.ones((n, 1)) if phi is None else np.asarray(phi, dtype=np.float64).reshape(n, -1)
    A_leaf = _leaf_blocks(row_ptr, col_idx, values, leaves, leaf_of, n)
    if L == 0:
        A = A_leaf[(0, 0)]
        try:
            c = sla.cho_factor(A, lower=True)
        except np.linalg.LinAlgError as e:
            raise NotSPDError(f"root not positive definite: {e}", depth=0, node=0) from e
        return Factorization(n=n, L=0, leaves=leaves, levels={}, eps=eps, variant=variant,
                             root_chol=c)

    # Red nodes of the leaf level
    red = LevelState(d=L)
    for i, c in enumerate(leaves):
        red.size[i] = len(c)
        red.state[i] = "R"
        if variant != LORASP:
            red.phi[i] = phi[c]
    for (i, j), B in A_leaf.items():
        red.blocks[(i, j)] = B
        if i != j:
            red.partners.setdefault(i, set()).add(j)

    levels = {}
    margins: list = []
    eps_at = {}
    dim = 1 if coords is None else np.asarray(coords).reshape(n, -1).shape[1]
    for d in range(L - 1, -1, -1):
        eps_d = level_eps(eps, eps_schedule, d, L, n, dim)
        eps_at[d] = eps_d
        cur, child_size = _merge(red, d, variant)
        if neighbours == "geometric":
            adj = GeometricNeighbours(coords, leaves, L, d)
        else:
            adj = footprint_adjacency(row_ptr, col_idx, leaf_of, L, d)
        super_size = dict(cur.size)
        remaining = [s for s in range(1 << d) if cur.size[s] > 0]
        colours, nodes = [], {}
        while remaining:
            # R8: the greedy pass in index order, or the nodes with the most partners still
            # waiting first (ties by index)
            if order == "waiting":
                waiting = set(remaining)
                visit = sorted(remaining, key=lambda s: (-len(cur.partners.get(s, set()) & waiting), s))
            else:
                visit = remaining
            colour = []
            for s in visit:
                if all((s, c) not in cur.blocks for c in colour):
                    colour.append(s)
            colour.sort()
            for s in colour:
                before = {j: cur.state[j] for j in cur.partners.get(s, ())}
                nf = eliminate_node(cur, s, adj, eps_d, variant, margins, eps1)
                nf.nbrs = [(nb, before[nb], A) for (nb, _, A) in nf.nbrs]
                nf.Wstate = [before[w] for w in nf.W]
                nodes[s] = nf
            taken = set(colour)
            remaining = [s for s in remaining if s not in taken]
            colours.append(colour)
        levels[d] = LevelFactor(d=d, colours=colours, nodes=nodes, super_size=super_size,
                                child_size=child_size,
                                red_size={s: cur.size[s] for s in range(1 << d)})
        red = cur
    return Factorization(n=n, L=L, leaves=leaves, levels=levels, eps=eps, variant=variant,
                         margins=margins, level_eps=eps_at)


def _merge(red: LevelState, d: int, variant: int):
    """Merge sibling red nodes 2I, 2I+1 of depth d+1 into super nodes I of depth d."""
    cur = LevelState(d=d)
    child_size = {}
    for I in range(1 << d):
        ka, kb = red.size.get(2 * I, 0), red.size.get(2 * I + 1, 0)
        child_size[I] = (ka, kb)
        cur.size[I] = ka + kb
        cur.state[I] = "S"
        if variant != LORASP and ka + kb > 0:
            parts = [red.phi[c] for c in (2 * I, 2 * I + 1) if red.size.get(c, 0) > 0]
            cur.phi[I] = np.vstack(parts)
    keys = set()
    for (i, j) in red.blocks:
        keys.add((i >> 1, j >> 1))
    for (I, J) in keys:
        if (J, I) in cur.blocks and I != J:
            continue
        B = np.zeros((cur.size[I], cur.size[J]))
        ka = child_size[I][0]
        kc = child_size[J][0]
        for a in (0, 1):
            for c in (0, 1):
                blk = red.blocks.get((2 * I + a, 2 * J + c))
                if blk is None:
                    continue
                r0 = 0 if a == 0 else ka
                c0 = 0 if c == 0 else kc
                B[r0:r0 + blk.shape[0], c0:c0 + blk.shape[1]] = blk
        if I == J:
            cur.blocks[(I, I)] = B
        else:
            cur.set_block(I, J, B)
    return cur, child_size


# ---------------------------------------------------------------------------
# Solve (Algorithm "Solve"; §3.3)
# ---------------------------------------------------------------------------
def apply(F: Factorization, r: np.ndarray) -> np.ndarray:
    """z = A_H^{-1} r for one or several right-hand sides (columns of r)."""
    r = np.asarray(r, dtype=np.float64)
    vec = r.ndim == 1
    R = r.reshape(F.n, -1)
    if F.L == 0:
        z = sla.cho_solve(F.root_chol, R[F.leaves[0]])
        out = np.empty_like(R)
        out[F.leaves[0]] = z
        return out.reshape(r.shape)
    rhs = {i: R[c].copy() for i, c in enumerate(F.leaves)}
    x = _solve_depth(F, F.L - 1, rhs, R.shape[1])
    out = np.empty_like(R)
    for i, c in enumerate(F.leaves):
        out[c] = x[i]
    return out.reshape(r.shape) if not vec else out[:, 0]


def _solve_depth(F: Factorization, d: int, child_rhs: dict, nrhs: int) -> dict:
    lev = F.levels[d]
    phi_S, phi_R = {}, {}
    for s in range(1 << d):
        ka, kb = lev.child_size[s]
        if ka + kb > 0:
            parts = [child_rhs[c] for c, kc in ((2 * s, ka), (2 * s + 1, kb)) if kc > 0]
            phi_S[s] = np.vstack(parts)
        phi_R[s] = np.zeros((lev.red_size[s], nrhs))
    # forward substitution, in elimination order: phi_n = r_n - A_ns M_ss r_s
    for s in lev.order:
        nf = lev.nodes[s]
        t = nf.M @ phi_S[s]
        for (nb, st, A_ns) in nf.nbrs:
            if st == "S":
                phi_S[nb] -= A_ns @ t
            else:
                phi_R[nb] -= A_ns @ t
    # restriction: phi_r = phi_r + P_ss phi_s
    for s in lev.order:
        nf = lev.nodes[s]
        phi_R[s] += nf.P @ phi_S[s]
    # parent-level solve
    if d > 0:
        x_R = _solve_depth(F, d - 1, phi_R, nrhs)
    else:
        x_R = {s: np.zeros((0, nrhs)) for s in phi_R}
    # prolongation + backward substitution in reverse order:
    # x_s = P_ss^T psi_r + M_ss (b_s - A_sn x_n)
    x_S = {}
    for s in reversed(lev.order):
        nf = lev.nodes[s]
        acc = phi_S[s].copy()
        for (nb, st, A_ns) in nf.nbrs:
            acc -= A_ns.T @ (x_S[nb] if st == "S" else x_R[nb])
        x_S[s] = nf.M @ acc + nf.P.T @ x_R[s]
    out = {}
    for s in range(1 << d):
        ka, kb = lev.child_size[s]
        xs = x_S.get(s, np.zeros((0, nrhs)))
        out[2 * s] = xs[:ka]
        out[2 * s + 1] = xs[ka:ka + kb]
    return out


def apply_matrix(F: Factorization) -> np.ndarray:
    """Dense A_H^{-1} (brute force, small n only)."""
    return apply(F, np.eye(F.n))
