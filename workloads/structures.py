"""Seeded synthetic structures made of repeated patterns.

A ``Problem`` is the statement of the method's input (the dual split of
section 2, eq. 2): for every pattern its Neumann stiffness K (CSR) and the set
of boundary nodes, for every occurrence the pattern it instantiates, its
rotation O (pattern frame -> global frame, section 4.2) and its loads f, and
the signed Boolean assembly A as a list of multipliers, each joining one node of
one occurrence (sign +1) to one node of another (sign -1), or, for a Dirichlet
condition imposed by a multiplier (Total FETI reading of section 4.1.3), to a
single node.  It also carries the permutation maps used to build multivectors
(section 3.1): index structure, not arithmetic.

Readings taken here (the paper does not define them for 3-D grids):

* multipliers at nodes shared by q > 2 occurrences form a non-redundant chain
  of q-1 links in ascending occurrence id; each Dirichlet node gets one
  multiplier on the lowest-id occurrence that holds it;
* the pattern boundary is the union of the local nodes that carry a multiplier
  in any occurrence of the pattern;
* permutation classes group multipliers with the same (pattern, local node)
  pair at both ends; Pi_k shifts every class cyclically by k positions in
  ascending occurrence order; a multiplier in a class of size one is kept.

Everything random is drawn from ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from . import mesh as M

BASE_SEED = 12086387


@dataclass
class Pattern:
    name: str
    dpn: int
    coords: np.ndarray            # (n_nodes, dim) pattern frame
    K: sp.csr_matrix              # (n, n) full symmetric, Neumann (floating)
    kernel_dim: int               # rigid modes of the free pattern
    bnodes: np.ndarray = None     # sorted local boundary nodes

    @property
    def n_nodes(self) -> int:
        return self.coords.shape[0]

    @property
    def n(self) -> int:
        return self.n_nodes * self.dpn

    @property
    def bdofs(self) -> np.ndarray:
        return (self.bnodes[:, None] * self.dpn + np.arange(self.dpn)[None, :]).ravel().astype(np.int32)

    @property
    def n_b(self) -> int:
        return len(self.bnodes) * self.dpn


@dataclass
class Problem:
    name: str
    dpn: int
    patterns: List[Pattern]
    occ_pattern: np.ndarray       # (n_occ,) int32
    occ_rot: np.ndarray           # (n_occ, 3, 3) pattern frame -> global frame
    occ_gnode: List[np.ndarray]   # per occurrence: local node -> global node
    n_gnodes: int
    dirichlet_gnodes: np.ndarray  # global nodes with u = 0
    mult_occ: np.ndarray          # (N_mn, 2) int32, -1 = no second endpoint
    mult_node: np.ndarray         # (N_mn, 2) int32 local node at each endpoint
    mult_sign: np.ndarray         # (N_mn, 2) int8
    n_rhs: int
    f_local: List[np.ndarray]     # per occurrence (n_p, n_rhs), pattern frame
    perm_node: np.ndarray         # (n_perm, N_mn) int32: (Pi_k z)[mn] = z[perm_node[k, mn]]
    tol: float = 1e-8
    meta: dict = field(default_factory=dict)
    # non-Boolean assembly (section 5: mortar coupling of non-matching meshes): side e of
    # multiplier i couples the local nodes entry_node[k] of occurrence mult_occ[i, e] with weights
    # entry_weight[k], k in [entry_ptr[2i+e], entry_ptr[2i+e+1]); None: the signed Boolean
    # assembly given by mult_node and mult_sign
    entry_ptr: Optional[np.ndarray] = None
    entry_node: Optional[np.ndarray] = None
    entry_weight: Optional[np.ndarray] = None

    @property
    def n_occ(self) -> int:
        return len(self.occ_pattern)

    @property
    def n_mult_nodes(self) -> int:
        return self.mult_occ.shape[0]

    @property
    def n_lambda(self) -> int:
        return self.n_mult_nodes * self.dpn

    @property
    def n_perm(self) -> int:
        return self.perm_node.shape[0]

    @property
    def has_rotation(self) -> bool:
        return not np.allclose(self.occ_rot, np.eye(3)[None], atol=0.0, rtol=0.0)

    def perm_dof(self) -> np.ndarray:
        """(n_perm, N_lambda) dof-level permutation source index."""
        d = self.dpn
        return (self.perm_node[:, :, None] * d + np.arange(d)[None, None, :]).reshape(self.n_perm, -1).astype(np.int32)

    def n_dirichlet_mult(self) -> int:
        return int((self.mult_occ[:, 1] < 0).sum())

    @property
    def weighted(self) -> bool:
        return self.entry_ptr is not None

    def entries(self):
        """(entry_ptr, entry_node, entry_weight) of the assembly; for a Boolean structure, the one
        node and the sign of each side."""
        if self.weighted:
            return self.entry_ptr, self.entry_node, self.entry_weight
        has = (self.mult_occ >= 0).ravel()
        ptr = np.concatenate([[0], np.cumsum(has)]).astype(np.int32)
        return ptr, self.mult_node.ravel()[has].astype(np.int32), self.mult_sign.ravel()[has].astype(float)


# --------------------------------------------------------------------------- multipliers

def chain_multipliers(occ, lnode, gnode, is_dirichlet_g, swap_rule=None):
    """Non-redundant signed Boolean multipliers for copies (occ, lnode) of global nodes.

    Returns (mult_occ, mult_node, mult_sign) at node level, interface links first,
    ordered by (occ_A, occ_B, node_A), then Dirichlet multipliers ordered by (occ, node).
    """
    occ = np.asarray(occ, np.int64)
    lnode = np.asarray(lnode, np.int64)
    gnode = np.asarray(gnode, np.int64)
    order = np.lexsort((occ, gnode))
    o, l, g = occ[order], lnode[order], gnode[order]
    same = g[1:] == g[:-1]
    a = np.nonzero(same)[0]
    oa, la, ob, lb = o[a], l[a], o[a + 1], l[a + 1]
    if swap_rule is not None:
        sw = swap_rule(oa, la, ob, lb)
        oa, ob = np.where(sw, ob, oa), np.where(sw, oa, ob)
        la, lb = np.where(sw, lb, la), np.where(sw, la, lb)
    lo = np.lexsort((la, ob, oa))
    oa, la, ob, lb = oa[lo], la[lo], ob[lo], lb[lo]
    first = np.ones(len(g), bool)
    first[1:] = ~same
    dpos = np.nonzero(first & is_dirichlet_g[g])[0]
    do, dl = o[dpos], l[dpos]
    lo = np.lexsort((dl, do))
    do, dl = do[lo], dl[lo]
    n_i, n_d = len(oa), len(do)
    mult_occ = np.full((n_i + n_d, 2), -1, np.int32)
    mult_node = np.full((n_i + n_d, 2), -1, np.int32)
    mult_sign = np.zeros((n_i + n_d, 2), np.int8)
    mult_occ[:n_i, 0], mult_occ[:n_i, 1] = oa, ob
    mult_node[:n_i, 0], mult_node[:n_i, 1] = la, lb
    mult_sign[:n_i, 0], mult_sign[:n_i, 1] = 1, -1
    mult_occ[n_i:, 0], mult_node[n_i:, 0], mult_sign[n_i:, 0] = do, dl, 1
    return mult_occ, mult_node, mult_sign


def pattern_boundaries(patterns, occ_pattern, mult_occ, mult_node):
    for p, pat in enumerate(patterns):
        sel = []
        for e in range(2):
            ok = mult_occ[:, e] >= 0
            occs = mult_occ[ok, e]
            sel.append(mult_node[ok, e][occ_pattern[occs] == p])
        pat.bnodes = np.unique(np.concatenate(sel)).astype(np.int32)


def permutation_maps(occ_pattern, mult_occ, mult_node, n_perm, product=False):
    """Cyclic shifts within classes of equivalent multipliers (section 3.1 and 4.1 examples).

    product=False: Pi_k shifts every class by k.  product=True (the enriched multivector of the
    two-stand donut, section 4.1.2): the classes are grouped by the pair of patterns they join, each
    group gets its own shift digit, and the rows run over every combination of digits (the first
    group, the one with the largest classes, varying fastest); n_perm None takes them all.
    """
    n = mult_occ.shape[0]
    pa = occ_pattern[mult_occ[:, 0]]
    pb = np.where(mult_occ[:, 1] >= 0, occ_pattern[np.maximum(mult_occ[:, 1], 0)], -1)
    nb = np.where(mult_occ[:, 1] >= 0, mult_node[:, 1], -1)
    keys = np.stack([pa, pb, mult_node[:, 0], nb], axis=1)
    _, cls = np.unique(keys, axis=0, return_inverse=True)
    cls = cls.ravel()
    # members of a class in ascending (occ_A, occ_B) order, multipliers are already sorted so
    order = np.lexsort((np.arange(n), mult_occ[:, 1], mult_occ[:, 0], cls))
    sizes = np.bincount(cls)
    start = np.concatenate([[0], np.cumsum(sizes)[:-1]])
    pos = np.empty(n, np.int64)
    pos[order] = np.arange(n) - start[cls[order]]
    if not product:
        perm = np.empty((n_perm, n), np.int32)
        for k in range(n_perm):
            src_pos = (pos + k) % sizes[cls]
            perm[k] = order[start[cls] + src_pos]
        return perm
    # groups of classes by the pair of patterns they join, largest classes first
    kind_of = {}
    for m_ in range(n):
        kind_of.setdefault(int(cls[m_]), (int(pa[m_]), int(pb[m_])))
    base = {}
    for c_, kd in kind_of.items():
        base[kd] = max(base.get(kd, 1), int(sizes[c_]))
    kinds = sorted(base, key=lambda kd: (-base[kd], kd))
    radix = [base[kd] for kd in kinds]
    total = int(np.prod(radix))
    n_perm = total if n_perm is None else min(n_perm, total)
    kidx = np.array([kinds.index(kind_of[int(c_)]) for c_ in cls], np.int64)
    perm = np.empty((n_perm, n), np.int32)
    for r in range(n_perm):
        digits, q = [], r
        for b in radix:
            digits.append(q % b)
            q //= b
        k = np.asarray(digits, np.int64)[kidx]
        src_pos = (pos + k) % sizes[cls]
        perm[r] = order[start[cls] + src_pos]
    return perm


# --------------------------------------------------------------------------- builders

def _finish(name, dpn, patterns, occ_pattern, occ_rot, occ_gnode, n_gnodes, dirichlet_g,
            f_local, n_rhs, n_perm, tol, meta, swap_rule=None, product_perm=False):
    occ_pattern = np.asarray(occ_pattern, np.int32)
    occ = np.concatenate([np.full(len(g), s) for s, g in enumerate(occ_gnode)])
    ln = np.concatenate([np.arange(len(g)) for g in occ_gnode])
    gn = np.concatenate(occ_gnode)
    isd = np.zeros(n_gnodes, bool)
    isd[dirichlet_g] = True
    mo, mn, ms = chain_multipliers(occ, ln, gn, isd, swap_rule)
    pattern_boundaries(patterns, occ_pattern, mo, mn)
    perm = permutation_maps(occ_pattern, mo, mn, n_perm, product=product_perm)
    return Problem(name=name, dpn=dpn, patterns=patterns, occ_pattern=occ_pattern,
                   occ_rot=np.asarray(occ_rot, float), occ_gnode=[np.asarray(g, np.int64) for g in occ_gnode],
                   n_gnodes=int(n_gnodes), dirichlet_gnodes=np.asarray(dirichlet_g, np.int64),
                   mult_occ=mo, mult_node=mn, mult_sign=ms, n_rhs=n_rhs, f_local=f_local,
                   perm_node=perm, tol=tol, meta=meta)


def grid_structure(name, kind, pat_shape, pat_size, grid, n_rhs=1, n_perm=1, load="normal",
                   dirichlet=(0, 0), traction=None, seed=0, tol=1e-8):
    """Axis-aligned grid of identical box patterns (no rotation).

    kind: 'heat' (2-D quads, 1 dof/node) or 'elast' (3-D bricks, 3 dofs/node).
    dirichlet: (axis, side) of the global face with u = 0, or None.
    load: 'unit_source' (consistent loads of f = 1) or 'normal' (i.i.d. N(0,1) nodal forces
          drawn per occurrence, load case, node, component).
    traction: optional (axis, side, t) uniform traction on a global face, added to every case.
    """
    dim = len(pat_shape)
    mesh = M.GridMesh(pat_shape, pat_size)
    if kind == "heat":
        assert dim == 2
        dpn, kdim = 1, 1
        K = M.assemble(mesh, M.quad_laplace(*mesh.h), 1)
    elif kind == "elast":
        assert dim == 3
        dpn, kdim = 3, 6
        K = M.assemble(mesh, M.hex_elasticity(*mesh.h), 3)
    else:
        raise ValueError(kind)
    pat = Pattern(name=f"{name}-pattern", dpn=dpn, coords=mesh.coords, K=K, kernel_dim=kdim)
    grid = tuple(grid)
    gidx = np.indices(grid[::-1]).reshape(dim, -1)[::-1].T  # occurrence grid index, x fastest
    n_occ = len(gidx)
    gshape = [grid[d] * pat_shape[d] for d in range(dim)]
    gnpa = [s + 1 for s in gshape]
    occ_gnode = []
    for s in range(n_occ):
        lat = mesh.lattice + gidx[s] * np.asarray(pat_shape)
        if dim == 2:
            gid = lat[:, 0] + gnpa[0] * lat[:, 1]
        else:
            gid = lat[:, 0] + gnpa[0] * (lat[:, 1] + gnpa[1] * lat[:, 2])
        occ_gnode.append(gid)
    n_g = int(np.prod(gnpa))
    glat = np.indices(gnpa[::-1]).reshape(dim, -1)[::-1].T
    if dirichlet is not None:
        ax, side = dirichlet
        target = 0 if side == 0 else gshape[ax]
        dir_g = np.nonzero(glat[:, ax] == target)[0]
    else:
        dir_g = np.zeros(0, np.int64)
    n = mesh.n_nodes * dpn
    if load == "unit_source":
        fe = M.quad_unit_source(*mesh.h)
        fp = M.assemble_vector(mesh, fe, dpn)
        f_local = [np.repeat(fp[:, None], n_rhs, axis=1) for _ in range(n_occ)]
    elif load == "normal":
        rng = np.random.Generator(np.random.PCG64(seed))
        draws = rng.standard_normal((n_occ, n_rhs, mesh.n_nodes, dpn))
        f_local = [np.ascontiguousarray(draws[s].reshape(n_rhs, n).T) for s in range(n_occ)]
    else:
        raise ValueError(load)
    if traction is not None:
        ax, side, t = traction
        ft = M.face_traction_load(mesh, ax, side, t)
        for s in range(n_occ):
            if gidx[s, ax] == (grid[ax] - 1 if side == 1 else 0):
                f_local[s] = f_local[s] + ft[:, None]
    rot = np.repeat(np.eye(3)[None], n_occ, axis=0)
    meta = dict(kind=kind, pat_shape=tuple(pat_shape), pat_size=tuple(pat_size), grid=grid,
                grid_index=gidx, global_shape=tuple(gshape), load=load, seed=seed)
    return _finish(name, dpn, [pat], np.zeros(n_occ, np.int32), rot, occ_gnode, n_g, dir_g,
                   f_local, n_rhs, n_perm, tol, meta)


def ring_heat(n_occ=3, pat_shape=(4, 4), stand=False, n_rhs=1, n_perm=None, seed=1, dirichlet_bottom=False,
              stands=None, enriched=False):
    """Periodic ring of unit-square heat patterns (section 3's toy problem, cut open as a strip
    whose last right edge is glued to the first left edge).  Interface (s, s+1) has the right edge
    of s as its '+' side.  stand=True adds one stand pattern (a 1 x 1/2 rectangle) on top of
    occurrence n_occ-1 (section 4.1.1).  stands: ring occurrences that each carry a stand, in the
    order of the stand occurrences (section 4.1.2 puts two stands on ring pieces 2 and 1: stands=
    (1, 0)); every stand has its own nodes apart from its base edge.  enriched=True builds the
    product permutations of the enriched multivector (independent shifts of the ring interfaces
    and of the stand interfaces; n_perm None takes all of them).  dirichlet_bottom fixes the bottom
    edge of occurrence 0;
    dirichlet_bottom="periodic" fixes the bottom-edge nodes off the interfaces of every ring
    occurrence, which keeps the ring truly periodic.
    """
    nx, ny = pat_shape
    mesh = M.GridMesh(pat_shape, (1.0, 1.0))
    K = M.assemble(mesh, M.quad_laplace(*mesh.h), 1)
    pats = [Pattern("ring-pattern", 1, mesh.coords, K, 1)]
    W = n_occ * nx
    occ_gnode = []
    for s in range(n_occ):
        gx = (mesh.lattice[:, 0] + s * nx) % W
        occ_gnode.append(gx + W * mesh.lattice[:, 1])
    occ_pattern = [0] * n_occ
    n_g = W * (ny + 1)
    if stands is None:
        stands = (n_occ - 1,) if stand else ()
    if len(stands):
        smesh = M.GridMesh((nx, max(ny // 2, 1)), (1.0, 0.5))
        Ks = M.assemble(smesh, M.quad_laplace(*smesh.h), 1)
        pats.append(Pattern("stand-pattern", 1, smesh.coords, Ks, 1))
        iy = smesh.lattice[:, 1]
        ix = smesh.lattice[:, 0]
        per_stand = (nx + 1) * smesh.shape[1]
        for j, s_on in enumerate(stands):
            gx = (ix + s_on * nx) % W
            own = n_g + j * per_stand + ix + (nx + 1) * (iy - 1)
            occ_gnode.append(np.where(iy == 0, gx + W * ny, own))
            occ_pattern.append(1)
        n_g = n_g + len(stands) * per_stand
    if dirichlet_bottom == "periodic":
        # the bottom-edge nodes of every ring occurrence off its interfaces (truly periodic)
        gx = np.arange(W)
        dir_g = gx[gx % nx != 0]
    elif dirichlet_bottom:
        dir_g = np.nonzero((np.arange(n_g) < W) & (np.arange(n_g) < nx + 1))[0]
    else:
        dir_g = np.zeros(0, np.int64)
    n_total = len(occ_gnode)
    rng = np.random.Generator(np.random.PCG64(seed))
    f_local = [rng.standard_normal((len(g), n_rhs)) for g in occ_gnode]
    rot = np.repeat(np.eye(3)[None], n_total, axis=0)

    def swap(oa, la, ob, lb):
        # make the right edge of the ring occurrence the '+' side of a ring interface
        ring = (oa < n_occ) & (ob < n_occ)
        return ring & (la % (nx + 1) == 0) & (lb % (nx + 1) == nx)

    meta = dict(kind="heat", ring=n_occ, stand=bool(len(stands)), stands=tuple(stands), grid=(n_occ,),
                pat_shape=pat_shape)
    if n_perm is None and not enriched:
        n_perm = n_occ
    return _finish(f"ring{n_occ}{'-stand' * len(stands)}", 1, pats, occ_pattern, rot, occ_gnode,
                   n_g, dir_g, f_local, n_rhs, n_perm, 1e-10, meta, swap_rule=swap, product_perm=enriched)


def mirror_row_heat(n_occ=2, pat_shape=(4, 4), reaction=0.1, n_rhs=1, seed=2):
    """A row of heat patterns with a reaction term (K + reaction * I: no floating occurrence),
    every other occurrence the mirror image of the first about its shared edge, so that
    neighbours meet on the same local edge: the right edges of 0 and 1, the left edges of 1 and
    2, and so on.  With two occurrences the pattern boundary is one edge; with a pattern one
    element wide and three or more occurrences every node is a boundary node.  No Dirichlet
    condition (the reaction term makes every occurrence non-singular).
    """
    nx, ny = pat_shape
    mesh = M.GridMesh(pat_shape, (1.0, 1.0))
    K = (M.assemble(mesh, M.quad_laplace(*mesh.h), 1) + reaction * sp.identity(mesh.n_nodes)).tocsr()
    K.sort_indices()
    pats = [Pattern("mirror-pattern", 1, mesh.coords, K, 0)]
    W = n_occ * nx + 1
    occ_gnode = []
    for s in range(n_occ):
        ix = mesh.lattice[:, 0]
        gx = s * nx + (nx - ix if s % 2 else ix)
        occ_gnode.append(gx + W * mesh.lattice[:, 1])
    n_g = W * (ny + 1)
    rng = np.random.Generator(np.random.PCG64(seed))
    f_local = [rng.standard_normal((mesh.n_nodes, n_rhs)) for _ in range(n_occ)]
    rot = np.repeat(np.eye(3)[None], n_occ, axis=0)
    meta = dict(kind="heat", grid=(n_occ,), pat_shape=pat_shape, reaction=reaction)
    return _finish(f"mirror-row{n_occ}", 1, pats, [0] * n_occ, rot, occ_gnode, n_g, np.zeros(0, np.int64),
                   f_local, n_rhs, 1, 1e-10, meta)


def random_spd_ring(n_occ=5, n_if=40, n_rhs=1, n_perm=None, seed=4, shift=0.005):
    """Academic ring of a pattern whose stiffness is a random dense symmetric positive definite
    matrix on its interface dofs only (so its Schur complement is that matrix): the first n_if
    dofs face the previous occurrence, the last n_if the next one, and occurrence n_occ-1 closes
    the ring on occurrence 0.  K = M M^T / n + shift I with M i.i.d. N(0, 1); no occurrence floats
    and there is no Dirichlet condition.  Loads i.i.d. N(0, 1) per occurrence (non-periodic).
    Interface (s, s+1) has the last n_if dofs of s as its '+' side, so the multipliers form one
    cyclic class per dof and Pi_k shifts the ring by k occurrences.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    n = 2 * n_if
    Mr = rng.standard_normal((n, n))
    Kd = Mr @ Mr.T / n + shift * np.eye(n)
    Kd = 0.5 * (Kd + Kd.T)
    K = sp.csr_matrix(Kd)
    K.sort_indices()
    pats = [Pattern("random-spd-pattern", 1, np.zeros((n, 2)), K, 0)]
    occ_gnode = []
    for s_ in range(n_occ):
        left = s_ * n_if + np.arange(n_if)
        right = ((s_ + 1) % n_occ) * n_if + np.arange(n_if)
        occ_gnode.append(np.concatenate([left, right]))
    f_local = [rng.standard_normal((n, n_rhs)) for _ in range(n_occ)]
    rot = np.repeat(np.eye(3)[None], n_occ, axis=0)

    def swap(oa, la, ob, lb):
        # the '+' side of every interface is the right half of the lower occurrence in ring order
        return la < n_if

    meta = dict(kind="random-spd", ring=n_occ, n_if=n_if, shift=shift, seed=seed)
    return _finish(f"random-spd-ring{n_occ}", 1, pats, [0] * n_occ, rot, occ_gnode, n_occ * n_if,
                   np.zeros(0, np.int64), f_local, n_rhs, n_perm if n_perm is not None else n_occ, 1e-10, meta,
                   swap_rule=swap)


def rot_z(angle: float) -> np.ndarray:
    c, s = np.cos(angle), np.sin(angle)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def ring_elast(n_occ=3, pat_shape=(2, 3, 2), r_in=1.0, r_out=1.5, height=0.5, n_rhs=1, n_perm=None, seed=3,
               tol=1e-8, clamp=True):
    """Closed ring of n_occ identical annular-sector bricks (elasticity), occurrence s rotated by
    2 pi s / n_occ about z (section 4.2: rotations in the assembly; section 4.3: the ring of
    rotated occurrences).  pat_shape = (radial, circumferential, axial) elements; the sector spans
    [0, 2 pi / n_occ].  The bottom face of occurrence 0 is clamped (clamp=True), nothing
    (False), or, with clamp="periodic", the bottom-face nodes off the interfaces of every
    occurrence (a truly periodic structure).  Interface (s, s+1) has the
    far face of s as its '+' side; loads are i.i.d. N(0,1) nodal forces in the pattern frame.
    """
    nr_, nt, nz = pat_shape
    mesh = M.GridMesh(pat_shape, (1.0, 1.0, 1.0))
    lat = mesh.lattice
    ang = 2 * np.pi / n_occ
    r = r_in + (r_out - r_in) * lat[:, 0] / nr_
    th = ang * lat[:, 1] / nt
    zc = height * lat[:, 2] / nz
    coords = np.stack([r * np.cos(th), r * np.sin(th), zc], axis=1)
    K = M.assemble_general(mesh.elements(), coords, 3)
    pat = Pattern("sector-pattern", 3, coords, K, 6)
    rots = np.stack([rot_z(ang * s) for s in range(n_occ)])
    # global nodes by coinciding coordinates
    allc = np.concatenate([coords @ rots[s].T for s in range(n_occ)])
    key = np.round(allc / (1e-6 * r_out)).astype(np.int64)
    _, gid = np.unique(key, axis=0, return_inverse=True)
    gid = gid.ravel()
    occ_gnode = [gid[s * mesh.n_nodes:(s + 1) * mesh.n_nodes] for s in range(n_occ)]
    n_g = int(gid.max()) + 1
    bottom0 = occ_gnode[0][lat[:, 2] == 0] if clamp else np.zeros(0, np.int64)
    if clamp == "periodic":
        # the bottom-face nodes of every occurrence that lie on no interface: the same local nodes
        # in every occurrence, so the structure stays truly periodic under the ring shifts
        inner_bottom = (lat[:, 2] == 0) & (lat[:, 1] > 0) & (lat[:, 1] < nt)
        bottom0 = np.concatenate([occ_gnode[s][inner_bottom] for s in range(n_occ)])
    rng = np.random.Generator(np.random.PCG64(seed))
    f_local = [rng.standard_normal((mesh.n_nodes * 3, n_rhs)) for _ in range(n_occ)]
    far = lat[:, 1] == nt

    def swap(oa, la, ob, lb):
        # the far face (theta = 2 pi / n_occ) of the lower occurrence is the '+' side
        return (~far[la]) & far[lb]

    meta = dict(kind="elast", ring=n_occ, rotated=True, pat_shape=pat_shape, grid=(n_occ,))
    return _finish(f"ring-elast{n_occ}", 3, [pat], np.zeros(n_occ, np.int32), rots, occ_gnode, n_g, bottom0,
                   f_local, n_rhs, n_perm if n_perm is not None else n_occ, tol, meta, swap_rule=swap)


def uneven_three(plate=(24, 8, 2), sector=(6, 16, 4), base=16, n_sectors=16, plates_per_sector=3,
                 n_rhs=1, n_perm=8, seed=0, tol=1e-8):
    """Three elasticity patterns of uneven size joined by algebraic glue (node lists and frame
    rotations, not one geometric mesh):

    * ring sectors (pattern 1; shape = (radial, circumferential, axial) elements) spanning
      2 pi / n_sectors, occurrence s rotated by 2 pi s / n_sectors about z, closed into a ring
      through their end faces (these do coincide geometrically);
    * a base block (pattern 2; base^3 elements) whose top face, over the sector's bottom-face
      node grid (circumferential x radial), is glued to the bottom face of sector 0; the base's
      bottom face is clamped;
    * thin plates (pattern 0; shape = (length, width, thickness) elements), plate q rotated by
      2 pi q / (n_sectors plates_per_sector) about z, glued by a 5 x 3 node patch of their root
      face (x = 0; width nodes 2..6, all thickness nodes) to patch q % plates_per_sector of the
      outer face of sector q // plates_per_sector (circumferential nodes 1 + 5w .. 5 + 5w, axial
      nodes 1..3).

    Occurrences: sectors first, then plates, then the base.  Loads are i.i.d. N(0,1) nodal forces
    in each occurrence's frame.
    """
    nr_, nt, nz = sector
    assert nr_ >= 1 and nt >= 5 * plates_per_sector + 1 and nz >= 4 and plate[1] >= 7 and plate[2] == 2
    assert base >= nt and base >= nr_
    # ---- patterns
    pm = M.GridMesh(plate, (plate[0] / 8.0, plate[1] / 8.0, plate[2] / 8.0))
    Kp = M.assemble(pm, M.hex_elasticity(*pm.h), 3)
    sm = M.GridMesh(sector, (1.0, 1.0, 1.0))
    lat = sm.lattice
    ang = 2 * np.pi / n_sectors
    r_in, r_out, height = 2.0, 3.0, 0.5
    r = r_in + (r_out - r_in) * lat[:, 0] / nr_
    th = ang * lat[:, 1] / nt
    zc = height * lat[:, 2] / nz
    scoords = np.stack([r * np.cos(th), r * np.sin(th), zc], axis=1)
    Ks = M.assemble_general(sm.elements(), scoords, 3)
    bm = M.GridMesh((base,) * 3, (2.0,) * 3)
    Kb = M.assemble(bm, M.hex_elasticity(*bm.h), 3)
    pats = [Pattern("plate-pattern", 3, pm.coords, Kp, 6), Pattern("sector-pattern", 3, scoords, Ks, 6),
            Pattern("base-pattern", 3, bm.coords, Kb, 6)]
    n_plates = n_sectors * plates_per_sector
    # ---- sectors: global nodes by coinciding coordinates
    srot = np.stack([rot_z(ang * s) for s in range(n_sectors)])
    allc = np.concatenate([scoords @ srot[s].T for s in range(n_sectors)])
    key = np.round(allc / (1e-6 * r_out)).astype(np.int64)
    _, gid = np.unique(key, axis=0, return_inverse=True)
    gid = gid.ravel()
    occ_gnode = [gid[s * sm.n_nodes:(s + 1) * sm.n_nodes].astype(np.int64) for s in range(n_sectors)]
    n_g = int(gid.max()) + 1
    sec_node = lambda ir, it, iz: sm.node_id(np.stack([ir, it, iz], axis=-1))
    # ---- plates
    prot = np.stack([rot_z(2 * np.pi * q / n_plates) for q in range(n_plates)])
    jj, kk = np.meshgrid(np.arange(2, 7), np.arange(3), indexing="ij")
    root = pm.node_id(np.stack([np.zeros_like(jj), jj, kk], axis=-1)).ravel()
    for q in range(n_plates):
        g = n_g + np.arange(pm.n_nodes, dtype=np.int64)
        n_g += pm.n_nodes
        sidx, w = divmod(q, plates_per_sector)
        target = sec_node(np.full_like(jj, nr_), 1 + 5 * w + (jj - 2), 1 + kk).ravel()
        g[root] = occ_gnode[sidx][target]
        occ_gnode.append(g)
    # ---- base: top-face patch over the sector's (circumferential x radial) bottom node grid
    g = n_g + np.arange(bm.n_nodes, dtype=np.int64)
    n_g += bm.n_nodes
    ti, ri = np.meshgrid(np.arange(nt + 1), np.arange(nr_ + 1), indexing="ij")
    top = bm.node_id(np.stack([ti, ri, np.full_like(ti, base)], axis=-1)).ravel()
    g[top] = occ_gnode[0][sec_node(ri, ti, np.zeros_like(ti)).ravel()]
    occ_gnode.append(g)
    dir_g = g[bm.face_nodes(2, 0)]
    # compact the global numbering
    used, inv = np.unique(np.concatenate(occ_gnode), return_inverse=True)
    off = np.cumsum([0] + [len(x) for x in occ_gnode])
    occ_gnode = [inv[off[i]:off[i + 1]].astype(np.int64) for i in range(len(off) - 1)]
    dir_g = np.searchsorted(used, dir_g)
    n_g = len(used)
    occ_pattern = [1] * n_sectors + [0] * n_plates + [2]
    rots = np.concatenate([srot, prot, np.eye(3)[None]])
    rng = np.random.Generator(np.random.PCG64(seed))
    f_local = [rng.standard_normal((len(x) * 3, n_rhs)) for x in occ_gnode]
    far = lat[:, 1] == nt

    def swap(oa, la, ob, lb):
        # ring interfaces: the far end face of the lower sector is the '+' side
        ring = (oa < n_sectors) & (ob < n_sectors)
        out = np.zeros(len(oa), bool)
        out[ring] = (~far[la[ring]]) & far[lb[ring]]
        return out

    meta = dict(kind="elast", uneven=True, rotated=True, plate=tuple(plate), sector=tuple(sector), base=base,
                n_sectors=n_sectors, plates_per_sector=plates_per_sector, seed=seed)
    return _finish(f"uneven-plate{n_plates}-sector{n_sectors}-base{base}", 3, pats, occ_pattern, rots, occ_gnode,
                   n_g, dir_g, f_local, n_rhs, n_perm, tol, meta, swap_rule=swap)


# --------------------------------------------------------------------------- named configurations

# --------------------------------------------------------------------------- non-matching meshes

def mortar_weights_1d(xs: np.ndarray, xm: np.ndarray) -> np.ndarray:
    """Coupling weights of two non-matching piecewise-linear meshes of one segment, by the mortar
    method with dual Lagrange multipliers (Wohlmuth's biorthogonal basis).

    The multipliers live on the non-mortar side (nodes xs); row i of the result W gives
    u_s(x_i) = sum_l W[i, l] u_m(xm_l), W = D^{-1} M with D_ii = int phi_i (phi: the non-mortar hat
    functions) and M_il = int psi_i chi_l, where psi_i = 2 phi_i - phi_j on each non-mortar element
    [x_i, x_j] (the dual basis: int psi_i phi_k = delta_ik D_kk) and chi_l are the mortar-side hats.
    The products are integrated exactly (two Gauss points per piece between consecutive breakpoints
    of both meshes).  Rows sum to one and linear functions are reproduced exactly.
    """
    xs = np.asarray(xs, float)
    xm = np.asarray(xm, float)
    ns, nm = len(xs), len(xm)
    D = np.zeros(ns)
    Mw = np.zeros((ns, nm))
    br = np.unique(np.concatenate([xs, xm]))
    g = np.array([-1.0, 1.0]) / np.sqrt(3.0)

    def hats(x, nodes):
        # values of every hat function of a 1-D mesh at the points x
        v = np.zeros((len(x), len(nodes)))
        e = np.clip(np.searchsorted(nodes, x, side="right") - 1, 0, len(nodes) - 2)
        t_ = (x - nodes[e]) / (nodes[e + 1] - nodes[e])
        v[np.arange(len(x)), e] = 1.0 - t_
        v[np.arange(len(x)), e + 1] = t_
        return v, e

    for a, b in zip(br[:-1], br[1:]):
        x = 0.5 * (a + b) + 0.5 * (b - a) * g
        w = np.full(2, 0.5 * (b - a))
        phi, e = hats(x, xs)
        chi, _ = hats(x, xm)
        # dual basis on the non-mortar element holding each point
        psi = np.zeros_like(phi)
        for q in range(len(x)):
            i, j = e[q], e[q] + 1
            psi[q, i] = 2.0 * phi[q, i] - phi[q, j]
            psi[q, j] = 2.0 * phi[q, j] - phi[q, i]
        D += w @ phi
        Mw += (psi * w[:, None]).T @ chi
    return Mw / D[:, None]


def mortar_row(kind="heat", shapes=((8, 8), (6, 6)), n_occ=4, n_rhs=1, load="normal", seed=61, n_perm=None,
               tol=1e-10):
    """A row of unit boxes meshed alternately by two patterns whose shared faces do not match:
    occurrence s is [s, s+1] x [0, 1]^(d-1) with pattern s % 2.  kind 'heat' (2-D quads, one dof
    per node) or 'elast' (3-D bricks, E = 1, nu = 0.3, three dofs per node).  The interface between
    s and s+1 carries one multiplier (per dof of a node) for each node of the x = 0 face of s+1 (the
    non-mortar side), coupled to the x = 1 face of s by mortar_weights_1d (in 3-D the tensor
    product of the weights along y and z, exact for these structured faces): the non-Boolean
    assembly of section 5.  u = 0 on the x = 0 face of occurrence 0 (Total FETI Dirichlet
    multipliers).  load: 'normal' (i.i.d. N(0,1) nodal loads) or, for heat, 'flux' (no source, unit
    outward flux on the right edge of the last occurrence: the exact solution is u = x, which the
    mortar coupling reproduces).
    """
    pats, meshes = [], []
    dim = len(shapes[0])
    for k, shp in enumerate(shapes):
        mesh = M.GridMesh(shp, (1.0,) * dim)
        if kind == "heat":
            assert dim == 2
            dpn, kdim = 1, 1
            K = M.assemble(mesh, M.quad_laplace(*mesh.h), 1)
        else:
            assert dim == 3
            dpn, kdim = 3, 6
            K = M.assemble(mesh, M.hex_elasticity(*mesh.h), 3)
        pats.append(Pattern(f"mortar-{kind}-pattern{k}", dpn, mesh.coords, K, kdim))
        meshes.append(mesh)
    occ_pattern = np.array([s % len(shapes) for s in range(n_occ)], np.int32)

    def face(s, side):
        # nodes of the x = side face of occurrence s, ordered by (z, y), and the 1-D coordinates
        m = meshes[occ_pattern[s]]
        nodes = m.face_nodes(0, side)
        c = m.coords[nodes]
        order = np.lexsort(tuple(c[:, d] for d in range(1, dim)))
        axes = [np.unique(c[:, d]) for d in range(1, dim)]
        return nodes[order], axes

    def face_weights(ys_axes, ym_axes):
        Wt = np.ones((1, 1))
        for a_s, a_m in zip(ys_axes, ym_axes):    # y fastest, z slowest
            Wt = np.kron(mortar_weights_1d(a_s, a_m), Wt)
        return Wt

    mo, mn, ms, ptr, en, ew = [], [], [], [0], [], []
    for s in range(n_occ - 1):
        sn, ax_s = face(s + 1, 0)   # non-mortar: x = 0 face of s + 1
        mnodes, ax_m = face(s, 1)   # mortar: x = 1 face of s
        Wt = face_weights(ax_s, ax_m)
        for i in range(len(sn)):
            nz = np.nonzero(np.abs(Wt[i]) > 1e-14)[0]
            ref = nz[np.argmax(np.abs(Wt[i, nz]))]
            mo.append((s + 1, s))
            mn.append((sn[i], mnodes[ref]))
            ms.append((1, -1))
            en.append(sn[i])
            ew.append(1.0)
            ptr.append(len(en))
            en.extend(mnodes[nz])
            ew.extend(-Wt[i, nz])
            ptr.append(len(en))
    dn, _ = face(0, 0)
    for n_ in dn:
        mo.append((0, -1))
        mn.append((n_, -1))
        ms.append((1, 0))
        en.append(n_)
        ew.append(1.0)
        ptr.append(len(en))
        ptr.append(len(en))
    mo = np.asarray(mo, np.int32)
    mn = np.asarray(mn, np.int32)
    ms = np.asarray(ms, np.int8)
    ptr = np.asarray(ptr, np.int32)
    en = np.asarray(en, np.int32)
    ew = np.asarray(ew, float)
    # pattern boundary: every local node that any assembly entry names
    occ_of_entry = np.repeat(mo.ravel(), np.diff(ptr))
    for p, pat in enumerate(pats):
        sel = (occ_of_entry >= 0) & (occ_pattern[np.maximum(occ_of_entry, 0)] == p)
        pat.bnodes = np.unique(en[sel]).astype(np.int32)
    perm = permutation_maps(occ_pattern, mo, mn, n_occ if n_perm is None else n_perm)
    # no global mesh: every occurrence keeps its own nodes (the meshes do not match)
    occ_gnode, off = [], 0
    for s in range(n_occ):
        nn = meshes[occ_pattern[s]].n_nodes
        occ_gnode.append(off + np.arange(nn))
        off += nn
    rng = np.random.Generator(np.random.PCG64(seed))
    f_local = []
    for s in range(n_occ):
        m = meshes[occ_pattern[s]]
        if load == "normal":
            draws = rng.standard_normal((n_rhs, m.n_nodes, dpn))
            f_local.append(np.ascontiguousarray(draws.reshape(n_rhs, -1).T))
        elif load == "flux" and kind == "heat":
            f = np.zeros((m.n_nodes, n_rhs))
            if s == n_occ - 1:
                nodes, (y,) = face(s, 1)
                h = np.diff(y)
                f[nodes, :] = (np.concatenate([h, [0.0]]) / 2 + np.concatenate([[0.0], h]) / 2)[:, None]
            f_local.append(f)
        else:
            raise ValueError(load)
    rot = np.repeat(np.eye(3)[None], n_occ, axis=0)
    meta = dict(kind=kind, mortar=True, shapes=tuple(map(tuple, shapes)), grid=(n_occ,), load=load)
    return Problem(name=f"mortar-{kind}-row{n_occ}", dpn=dpn, patterns=pats, occ_pattern=occ_pattern,
                   occ_rot=rot, occ_gnode=occ_gnode, n_gnodes=off, dirichlet_gnodes=np.zeros(0, np.int64),
                   mult_occ=mo, mult_node=mn, mult_sign=ms, n_rhs=n_rhs, f_local=f_local, perm_node=perm, tol=tol,
                   meta=meta, entry_ptr=ptr, entry_node=en, entry_weight=ew)


def config(i: int, small: bool = False) -> Problem:
    """The five benchmark configurations, 0-based (seed 12086387 + i).

    0: 2-D heat, 16x16 Q1 square pattern, 1x4 row, f = 1, u = 0 on the left edge.
    1: 3-D elasticity, 12^3 brick pattern, 4x4x4 grid, clamped x = 0, N(0,1) nodal forces.
    2: same with 8 load cases.
    3: uneven three-pattern batch: 24x8x2 plates x 48 (rotated by 7.5 deg steps), 16x6x4 ring
       sectors x 16 (22.5 deg steps), one 16^3 base block clamped at the bottom (uneven_three).
    4: 20^3 brick pattern, 8x8x8 grid, 16 load cases plus traction (1,0,0) on x = 1.
    """
    seed = BASE_SEED + i
    if i == 0:
        return grid_structure("heat-row-16x16x4", "heat", (16, 16), (1.0, 1.0), (4, 1), n_rhs=1, n_perm=3,
                              load="unit_source", dirichlet=(0, 0), seed=seed, tol=1e-10)
    if i == 1:
        return grid_structure("elast-12cube-4x4x4", "elast", (12, 12, 12), (0.25,) * 3, (4, 4, 4), n_rhs=1,
                              n_perm=8, dirichlet=(0, 0), seed=seed)
    if i == 2:
        return grid_structure("elast-12cube-4x4x4-8rhs", "elast", (12, 12, 12), (0.25,) * 3, (4, 4, 4), n_rhs=8,
                              n_perm=1, dirichlet=(0, 0), seed=seed)
    if i == 3:
        return uneven_three(seed=seed)
    if i == 4:
        return grid_structure("elast-20cube-8x8x8-16rhs", "elast", (20, 20, 20), (0.125,) * 3, (8, 8, 8),
                              n_rhs=16, n_perm=1, dirichlet=(0, 0), traction=(0, 1, (1.0, 0.0, 0.0)), seed=seed)
    raise NotImplementedError(f"configuration {i}")


def small_elast(pat=(3, 3, 3), grid=(2, 2, 2), n_rhs=1, n_perm=1, seed=7, traction=None):
    side = 1.0 / max(grid)
    return grid_structure(f"elast-{pat[0]}cube-{'x'.join(map(str, grid))}", "elast", pat, (side,) * 3, grid,
                          n_rhs=n_rhs, n_perm=n_perm, dirichlet=(0, 0), traction=traction, seed=seed)


def small_heat(pat=(4, 4), grid=(3, 2), n_rhs=1, n_perm=1, seed=5, load="normal"):
    return grid_structure(f"heat-{pat[0]}sq-{'x'.join(map(str, grid))}", "heat", pat, (1.0, 1.0), grid,
                          n_rhs=n_rhs, n_perm=n_perm, load=load, dirichlet=(0, 0), seed=seed, tol=1e-10)
