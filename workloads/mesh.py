"""Finite-element discretisation used to build the synthetic inputs.

This module produces the *inputs* of the repeated-pattern FETI method: the
Neumann stiffness matrix K of a pattern and its nodal loads.  It holds none of
the method's own arithmetic (no condensation, no interface operator, no
solver); both the CPU oracle and the GPU library receive what it builds.

Elements (the paper's test problems are thermal and elastic, section 3.4 and
section 4.2; its matrices came from an external mesher and are not available):

* Q1 bilinear quadrilateral for the scalar heat equation, conductivity k,
  integrated with 2x2 Gauss points.  On a square it is the classical
  [4,-1,-2,-1]/6 stencil.
* Q1 trilinear hexahedron for isotropic linear elasticity (E, nu), integrated
  with 2x2x2 Gauss points.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_G = 1.0 / np.sqrt(3.0)
_GAUSS = (-_G, _G)

# reference-node signs, counter-clockwise for the quad, bottom then top face
# for the hexahedron
QUAD_NODES = np.array([(-1, -1), (1, -1), (1, 1), (-1, 1)], dtype=float)
HEX_NODES = np.array([(-1, -1, -1), (1, -1, -1), (1, 1, -1), (-1, 1, -1),
                      (-1, -1, 1), (1, -1, 1), (1, 1, 1), (-1, 1, 1)], dtype=float)


def quad_laplace(hx: float, hy: float, k: float = 1.0) -> np.ndarray:
    """4x4 conductivity matrix of an axis-aligned hx*hy bilinear element."""
    Ke = np.zeros((4, 4))
    det = hx * hy / 4.0
    for xi in _GAUSS:
        for eta in _GAUSS:
            dxi = QUAD_NODES[:, 0] * (1 + eta * QUAD_NODES[:, 1]) / 4.0
            deta = QUAD_NODES[:, 1] * (1 + xi * QUAD_NODES[:, 0]) / 4.0
            B = np.vstack([dxi * 2.0 / hx, deta * 2.0 / hy])
            Ke += k * B.T @ B * det
    return Ke


def quad_unit_source(hx: float, hy: float) -> np.ndarray:
    """Consistent nodal load of a unit volumetric source on one quad."""
    return np.full(4, hx * hy / 4.0)


def lame(E: float, nu: float):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    return lam, mu


def hex_elasticity(hx: float, hy: float, hz: float, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """24x24 stiffness of an axis-aligned trilinear brick, dofs node-major (x,y,z)."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    Ke = np.zeros((24, 24))
    det = hx * hy * hz / 8.0
    s = HEX_NODES
    for a in _GAUSS:
        for b in _GAUSS:
            for c in _GAUSS:
                dNa = s[:, 0] * (1 + b * s[:, 1]) * (1 + c * s[:, 2]) / 8.0
                dNb = s[:, 1] * (1 + a * s[:, 0]) * (1 + c * s[:, 2]) / 8.0
                dNc = s[:, 2] * (1 + a * s[:, 0]) * (1 + b * s[:, 1]) / 8.0
                dx, dy, dz = dNa * 2.0 / hx, dNb * 2.0 / hy, dNc * 2.0 / hz
                B = np.zeros((6, 24))
                B[0, 0::3] = dx
                B[1, 1::3] = dy
                B[2, 2::3] = dz
                B[3, 1::3] = dz
                B[3, 2::3] = dy
                B[4, 0::3] = dz
                B[4, 2::3] = dx
                B[5, 0::3] = dy
                B[5, 1::3] = dx
                Ke += B.T @ D @ B * det
    return Ke


class GridMesh:
    """Structured box mesh of quads (2-D) or bricks (3-D).

    Node (ix, iy[, iz]) has id ix + (nx+1)*(iy + (ny+1)*iz).
    """

    def __init__(self, shape, size, origin=None):
        self.shape = tuple(int(v) for v in shape)
        self.dim = len(self.shape)
        self.size = tuple(float(v) for v in size)
        self.h = tuple(self.size[d] / self.shape[d] for d in range(self.dim))
        self.origin = np.zeros(self.dim) if origin is None else np.asarray(origin, float)
        npd = [s + 1 for s in self.shape]
        self.nodes_per_axis = tuple(npd)
        self.n_nodes = int(np.prod(npd))
        idx = np.indices(npd[::-1]).reshape(self.dim, -1)[::-1].T  # (n_nodes, dim), x fastest
        self.lattice = idx.astype(np.int64)
        self.coords = self.origin + idx * np.asarray(self.h)

    def node_id(self, ijk):
        ijk = np.asarray(ijk, dtype=np.int64)
        npd = self.nodes_per_axis
        if self.dim == 2:
            return ijk[..., 0] + npd[0] * ijk[..., 1]
        return ijk[..., 0] + npd[0] * (ijk[..., 1] + npd[1] * ijk[..., 2])

    def elements(self) -> np.ndarray:
        """(n_elem, 4|8) node ids in the reference-node order above."""
        ne = self.shape
        e = np.indices(ne[::-1]).reshape(self.dim, -1)[::-1].T
        corners = QUAD_NODES if self.dim == 2 else HEX_NODES
        off = ((corners + 1) / 2).astype(np.int64)
        return self.node_id(e[:, None, :] + off[None, :, :])

    def face_nodes(self, axis: int, side: int) -> np.ndarray:
        """Nodes on the face lattice[axis] == 0 (side 0) or == shape[axis] (side 1)."""
        target = 0 if side == 0 else self.shape[axis]
        return np.nonzero(self.lattice[:, axis] == target)[0]

    def surface_nodes(self) -> np.ndarray:
        m = np.zeros(self.n_nodes, bool)
        for d in range(self.dim):
            m |= (self.lattice[:, d] == 0) | (self.lattice[:, d] == self.shape[d])
        return np.nonzero(m)[0]


def assemble(mesh: GridMesh, Ke: np.ndarray, dpn: int) -> sp.csr_matrix:
    """Assemble one element matrix (identical for all cells) over the grid, full symmetric CSR."""
    el = mesh.elements()
    nen = el.shape[1]
    dofs = (el[:, :, None] * dpn + np.arange(dpn)[None, None, :]).reshape(len(el), nen * dpn)
    rows = np.repeat(dofs, nen * dpn, axis=1).ravel()
    cols = np.tile(dofs, (1, nen * dpn)).ravel()
    vals = np.tile(Ke.ravel(), len(el))
    n = mesh.n_nodes * dpn
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    K.indptr = K.indptr.astype(np.int32)
    K.indices = K.indices.astype(np.int32)
    return K


def assemble_vector(mesh: GridMesh, fe: np.ndarray, dpn: int) -> np.ndarray:
    el = mesh.elements()
    nen = el.shape[1]
    dofs = (el[:, :, None] * dpn + np.arange(dpn)[None, None, :]).reshape(len(el), nen * dpn)
    f = np.zeros(mesh.n_nodes * dpn)
    np.add.at(f, dofs.ravel(), np.tile(fe.ravel(), len(el)))
    return f


def face_traction_load(mesh: GridMesh, axis: int, side: int, t) -> np.ndarray:
    """Consistent nodal load of a uniform traction t on one face of a brick mesh."""
    t = np.asarray(t, float)
    dpn = len(t)
    f = np.zeros((mesh.n_nodes, dpn))
    tang = [d for d in range(mesh.dim) if d != axis]
    area = np.prod([mesh.h[d] for d in tang])
    target = 0 if side == 0 else mesh.shape[axis]
    # face cells: lattice cells on that face
    ranges = [range(mesh.shape[d]) for d in tang]
    for a in ranges[0]:
        for b in ranges[1]:
            for da in (0, 1):
                for db in (0, 1):
                    ijk = [0] * 3
                    ijk[axis] = target
                    ijk[tang[0]] = a + da
                    ijk[tang[1]] = b + db
                    f[mesh.node_id(ijk)] += t * area / 4.0
    return f.ravel()


def hex_elasticity_general(X: np.ndarray, E: float = 1.0, nu: float = 0.3) -> np.ndarray:
    """24x24 stiffness of a trilinear brick with arbitrary corner coordinates X (8,3)."""
    lam, mu = lame(E, nu)
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[np.arange(3), np.arange(3)] += 2 * mu
    D[3, 3] = D[4, 4] = D[5, 5] = mu
    s = HEX_NODES
    Ke = np.zeros((24, 24))
    for a in _GAUSS:
        for b in _GAUSS:
            for c in _GAUSS:
                dN = np.vstack([s[:, 0] * (1 + b * s[:, 1]) * (1 + c * s[:, 2]),
                                s[:, 1] * (1 + a * s[:, 0]) * (1 + c * s[:, 2]),
                                s[:, 2] * (1 + a * s[:, 0]) * (1 + b * s[:, 1])]) / 8.0
                J = dN @ X                      # J[i, j] = d x_j / d xi_i
                dX = np.linalg.solve(J, dN)      # d N / d x_j, (3, 8)
                B = np.zeros((6, 24))
                B[0, 0::3] = dX[0]
                B[1, 1::3] = dX[1]
                B[2, 2::3] = dX[2]
                B[3, 1::3] = dX[2]
                B[3, 2::3] = dX[1]
                B[4, 0::3] = dX[2]
                B[4, 2::3] = dX[0]
                B[5, 0::3] = dX[1]
                B[5, 1::3] = dX[0]
                Ke += B.T @ D @ B * np.linalg.det(J)
    return Ke


def assemble_general(elements: np.ndarray, coords: np.ndarray, dpn: int, E=1.0, nu=0.3) -> sp.csr_matrix:
    """Assemble brick elements with their own geometry (mapped meshes)."""
    nen = elements.shape[1]
    rows, cols, vals = [], [], []
    for el in elements:
        Ke = hex_elasticity_general(coords[el], E, nu)
        d = (el[:, None] * dpn + np.arange(dpn)[None, :]).ravel()
        rows.append(np.repeat(d, nen * dpn))
        cols.append(np.tile(d, nen * dpn))
        vals.append(Ke.ravel())
    n = coords.shape[0] * dpn
    K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    K.indptr = K.indptr.astype(np.int32)
    K.indices = K.indices.astype(np.int32)
    return K
