"""Plain FP64 CPU oracle of repeated-pattern FETI.  TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this module.  It shares no code with the GPU library: it reads the
problem statement produced by ``workloads`` and follows the paper (Gosselet,
Rixen, Rey, "A domain decomposition strategy to efficiently solve structures
containing repeated patterns") step by step, with NumPy/SciPy primitives
(sparse LU, dense eigendecomposition, dense inverse, matrix products).

Every function names the passage it follows.  Readings where the paper is
silent are marked READING.

Parity status of each function (what pins it, see tests/test_oracle_*.py):
* pattern condensation, kernel, pseudo-inverse: pinned (dense Schur, pinv,
  analytic rigid modes, S S+ S = S);
* assembly operators, F, G, Q, lambda_0: pinned (continuity of rigid motions,
  antisymmetry, dense F, projector identities);
* lumped and Dirichlet preconditioners: pinned (exact inverse on a mirror-image pair,
  lumped = Dirichlet without interior dofs, multiplicity scaling away from cross-points,
  spectrum of the preconditioned operator bounded below by 1, K_bb - S >= 0 ordering,
  unchanged solutions);
* lumped or Dirichlet preconditioner inside Q, Q^T and lambda_0 (coarse=...): pinned
  (Q Q = Q, G^T Q = 0, Q^T the transpose, G^T lambda_0 = e, solutions equal to the global
  solve, and a swapped-sides mutation);
* periodic shortcut of the multivector product: pinned (same iterates as the full products on
  truly periodic rings, commutation of F, Q and the preconditioner with the permutations, and a
  non-periodic negative control);
* classical and block solvers, recovery: pinned against a brute-force global
  solve assembled from the global node numbering, and the closed-form 1-D
  solution of the heat row;
* non-Boolean (mortar) assembly of non-matching meshes: pinned (the coupling weights
  reproduce linear fields, B u = 0 for every linear field cut into the occurrences, the
  solution equals the dense saddle-point solve of the constrained problem and the exact
  linear solution of the flux problem, and matching meshes give the Boolean result);
* iteration counts against the paper's tables: parity unpinned (the paper's
  matrices are not reproduced); its academic study (random dense SPD pattern,
  five and nine repetitions, Dirichlet preconditioner) is checked qualitatively.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

KERNEL_TAU = 1e-10      # READING: eigenvalues below tau * lambda_max(S) span the kernel
ETA_DROP = 1e-12        # READING: eigenvalues of eta below this * (energy of the block before
                        # orthogonalisation) are dropped (section 3.3)


# =========================================================================== pattern level

class PatternOracle:
    """One pattern: S, its kernel Z, the pseudo-inverse S+ (section 2, definitions after eq. 3).

    S = K_bb - K_bi K_ii^{-1} K_ib is the local Schur complement.  For a floating
    pattern S is singular; Z is an orthonormal basis of its kernel and
    S+ = (S + Z Z^T)^{-1} - Z Z^T is the Moore-Penrose pseudo-inverse (READING:
    the paper only asks K K+ y = y on range K; this choice is canonical because
    Z Z^T does not depend on the basis).
    """

    def __init__(self, K: sp.csr_matrix, bdofs: np.ndarray, expected_kernel: int | None = None,
                 tau: float = KERNEL_TAU):
        n = K.shape[0]
        self.n = n
        self.b = np.asarray(bdofs, np.int64)
        mask = np.ones(n, bool)
        mask[self.b] = False
        self.i = np.nonzero(mask)[0]
        K = K.tocsc()
        self.K = K
        self.Kii = K[self.i][:, self.i].tocsc()
        self.Kib = K[self.i][:, self.b].toarray()
        self.Kbb = K[self.b][:, self.b].toarray()
        self.lu = spla.splu(self.Kii)
        self.X = self.lu.solve(self.Kib)                 # K_ii^{-1} K_ib
        S = self.Kbb - self.Kib.T @ self.X
        self.S = 0.5 * (S + S.T)
        self.Z = kernel_basis(self.S, tau)
        if expected_kernel is not None and self.Z.shape[1] != expected_kernel:
            raise ValueError(f"kernel dimension {self.Z.shape[1]} != {expected_kernel}")
        self.Splus = pseudo_inverse(self.S, self.Z)
        # N = [-K_ii^{-1} K_ib Z ; Z] in the pattern's dof order (kernel of K, section 2)
        N = np.zeros((n, self.Z.shape[1]))
        N[self.i] = -self.X @ self.Z
        N[self.b] = self.Z
        self.N = N

    @property
    def k(self) -> int:
        return self.Z.shape[1]

    @property
    def n_b(self) -> int:
        return len(self.b)

    def condensed_load(self, f: np.ndarray) -> np.ndarray:
        """g = f_b - K_bi K_ii^{-1} f_i (the load seen by the boundary, section 2)."""
        return f[self.b] - self.Kib.T @ self.lu.solve(np.ascontiguousarray(f[self.i]))

    def interior(self, f: np.ndarray, u_b: np.ndarray) -> np.ndarray:
        """u_i = K_ii^{-1} (f_i - K_ib u_b): the interior rows of K u = f - t^T lambda_b."""
        return self.lu.solve(np.ascontiguousarray(f[self.i] - self.Kib @ u_b))


def kernel_basis(S: np.ndarray, tau: float = KERNEL_TAU) -> np.ndarray:
    """Orthonormal basis of the numerical kernel of a symmetric PSD matrix (section 2: N)."""
    w, V = np.linalg.eigh(S)
    lmax = max(abs(w[-1]), abs(w[0]))
    keep = np.abs(w) < tau * lmax
    return np.ascontiguousarray(V[:, keep])


def pseudo_inverse(S: np.ndarray, Z: np.ndarray) -> np.ndarray:
    """S+ = (S + Z Z^T)^{-1} - Z Z^T (Moore-Penrose when Z spans ker S)."""
    P = Z @ Z.T
    Sp = np.linalg.inv(S + P) - P
    return 0.5 * (Sp + Sp.T)


# =========================================================================== interface level

class FetiOracle:
    """The dual interface problem (eq. 3) of a Problem.

    F = sum_s A^(s) S+ A^(s)T, G = [.. A^(s) t N^(s) ..], d = sum_s A^(s) t K+ f^(s),
    e^T = [.. f^(s)T N^(s) ..] (section 2).  With the identity in place of F~^{-1} in the
    projector (READING), Q = I - G (G^T G)^{-1} G^T and lambda_0 = G (G^T G)^{-1} e
    (section 2, projector and initialisation).  The solvers take the identity, lumped or
    Dirichlet preconditioner (section 2) for z = Q F~^{-1} r.  For elasticity A^(s) carries the
    occurrence rotation O^(s) (section 4.2): A^(s)T takes global-frame interface
    values to the pattern frame.
    """

    def __init__(self, problem, patterns: list | None = None, coarse: str | None = None):
        """coarse: None for the identity in the projector, or "lumped" / "dirichlet" for that
        preconditioner as F~^{-1} in Q and lambda_0 (section 2)."""
        pb = problem
        self.pb = pb
        self.dpn = dpn = pb.dpn
        if patterns is None:
            patterns = [PatternOracle(p.K, p.bdofs, p.kernel_dim) for p in pb.patterns]
        self.pats = patterns
        self.n_lambda = pb.n_lambda
        # boundary position of every local node, per pattern
        self.bpos = []
        for p in pb.patterns:
            pos = np.full(p.n_nodes, -1, np.int64)
            pos[p.bnodes] = np.arange(len(p.bnodes))
            self.bpos.append(pos)
        self.A = [self._assembly(s) for s in range(pb.n_occ)]
        cols = []
        self.coarse_off = np.zeros(pb.n_occ + 1, np.int64)
        for s in range(pb.n_occ):
            Zs = self.pats[pb.occ_pattern[s]].Z
            cols.append(sp.csr_matrix(self.A[s] @ Zs))
            self.coarse_off[s + 1] = self.coarse_off[s] + Zs.shape[1]
        self.G = sp.hstack(cols).tocsr() if cols else sp.csr_matrix((self.n_lambda, 0))
        self.GtG = (self.G.T @ self.G).toarray()
        self._GtG_cho = None
        self._AAt = self._AAt_lu = None
        self.coarse = coarse
        self._MG = self._H_cho = None

    # -- signed Boolean assembly (eq. 2) ------------------------------------------------
    def _assembly(self, s: int) -> sp.csr_matrix:
        """A^(s): N_lambda x n_b(s); (A v)[l] = sign * O^(s) v[node] at every endpoint on s.

        A non-Boolean structure (mortar coupling of non-matching meshes, section 5) gives each
        side of a multiplier several local nodes with real weights: (A v)[l] = sum_k w_k O^(s)
        v[node_k] over the entries of the side on s."""
        pb, dpn = self.pb, self.dpn
        p = pb.occ_pattern[s]
        nb = self.pats[p].n_b
        O = pb.occ_rot[s][:dpn, :dpn] if dpn > 1 else np.ones((1, 1))
        rows, cols, vals = [], [], []
        if getattr(pb, "entry_ptr", None) is not None:
            ptr, node, wgt = pb.entry_ptr, pb.entry_node, pb.entry_weight
            for e in range(2):
                sel = np.nonzero(pb.mult_occ[:, e] == s)[0]
                for m_ in sel:
                    for k in range(ptr[2 * m_ + e], ptr[2 * m_ + e + 1]):
                        bp = self.bpos[p][node[k]]
                        assert bp >= 0
                        for c in range(dpn):
                            for c2 in range(dpn):
                                if O[c, c2] != 0.0:
                                    rows.append([m_ * dpn + c])
                                    cols.append([bp * dpn + c2])
                                    vals.append([wgt[k] * O[c, c2]])
            if not rows:
                return sp.csr_matrix((self.n_lambda, nb))
            return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                                 shape=(self.n_lambda, nb))
        for e in range(2):
            sel = np.nonzero(pb.mult_occ[:, e] == s)[0]
            if len(sel) == 0:
                continue
            bp = self.bpos[p][pb.mult_node[sel, e]]
            assert np.all(bp >= 0)
            sg = pb.mult_sign[sel, e].astype(float)
            for c in range(dpn):
                for c2 in range(dpn):
                    if O[c, c2] == 0.0:
                        continue
                    rows.append(sel * dpn + c)
                    cols.append(bp * dpn + c2)
                    vals.append(sg * O[c, c2])
        if not rows:
            return sp.csr_matrix((self.n_lambda, nb))
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(self.n_lambda, nb))

    # -- operators ----------------------------------------------------------------------
    def F(self, X: np.ndarray) -> np.ndarray:
        """F X = sum_s A^(s) S+ A^(s)T X (section 2; section 3.2 computes all occurrences as S+ W)."""
        X = np.asarray(X, float)
        vec = X.ndim == 1
        X2 = X[:, None] if vec else X
        Y = np.zeros_like(X2)
        for s in range(self.pb.n_occ):
            Sp = self.pats[self.pb.occ_pattern[s]].Splus
            Y += self.A[s] @ (Sp @ (self.A[s].T @ X2))
        return Y[:, 0] if vec else Y

    def Gt(self, X):
        return self.G.T @ X

    def coarse_solve(self, c):
        """(G^T G)^{-1} c by a Cholesky factor computed on first use (G^T G is singular for a
        structure with no Dirichlet condition at all; such structures never reach this)."""
        if self.GtG.size == 0:
            return c
        if self._GtG_cho is None:
            self._GtG_cho = sla.cho_factor(self.GtG)
        return sla.cho_solve(self._GtG_cho, c)

    def _coarse_M(self):
        """F~^{-1} G and the Cholesky factor of G^T F~^{-1} G (section 2, projector with a
        preconditioner), formed once."""
        if self._MG is None:
            Gd = self.G.toarray()
            self._MG = self.precondition(Gd, self.coarse)
            H = Gd.T @ self._MG
            self._H_cho = sla.cho_factor(0.5 * (H + H.T))
        return self._MG, self._H_cho

    def Q(self, X: np.ndarray) -> np.ndarray:
        """Q X = X - F~^{-1} G (G^T F~^{-1} G)^{-1} G^T X (section 2); with the identity in place
        of F~^{-1} (the default) Q = I - G (G^T G)^{-1} G^T = Q^T."""
        if self.G.shape[1] == 0:
            return np.array(X, float)
        if self.coarse is None:
            return X - self.G @ self.coarse_solve(self.G.T @ X)
        MG, H = self._coarse_M()
        return X - MG @ sla.cho_solve(H, self.G.T @ X)

    def Qt(self, X: np.ndarray) -> np.ndarray:
        """Q^T X = X - G (G^T F~^{-1} G)^{-1} (F~^{-1} G)^T X (F~^{-1} symmetric); Q itself for the
        identity."""
        if self.G.shape[1] == 0 or self.coarse is None:
            return self.Q(X)
        MG, H = self._coarse_M()
        return X - self.G @ sla.cho_solve(H, MG.T @ X)

    # -- preconditioners (section 2) -------------------------------------------------------
    def assembly_gram(self) -> sp.csc_matrix:
        """A A^T = sum_s A^(s) A^(s)T, the Gram matrix of the signed Boolean assembly (eq. 2)."""
        if self._AAt is None:
            M = sp.csr_matrix((self.n_lambda, self.n_lambda))
            for As in self.A:
                M = M + As @ As.T
            self._AAt = M.tocsc()
            self._AAt_lu = spla.splu(self._AAt)
        return self._AAt

    def scale(self, X: np.ndarray) -> np.ndarray:
        """The scaling of the preconditioners (section 2), applied to a lambda block: (A A^T)^{-1} X.

        READING: the paper takes diagonal scalings beta^(s) whose sum over the subdomains is the
        identity.  Its condition, sum_s beta^(s) A^(s) A^(s)T = I wherever no two multipliers
        share a local dof, is taken in the form that also holds at cross-points joined by a
        chain of non-redundant multipliers: beta^(s) A^(s) -> (A A^T)^{-1} A^(s), the same for
        every s.  Away from cross-points A A^T is diagonal (2 on an interface multiplier, 1 on a
        Dirichlet one), which gives the multiplicity scaling 1/2 and 1.  At a cross-point the
        chain links share dofs and A A^T couples them; a diagonal 1/2 there makes the
        preconditioned operator far worse conditioned than no preconditioner at all.
        """
        self.assembly_gram()
        X = np.asarray(X, float)
        return self._AAt_lu.solve(np.ascontiguousarray(X))

    def local_precond_matrix(self, p: int, kind: str) -> np.ndarray:
        """The pattern matrix of a preconditioner: S (Dirichlet) or K_bb (lumped), section 2."""
        if kind == "dirichlet":
            return self.pats[p].S
        if kind == "lumped":
            return self.pats[p].Kbb
        raise ValueError(kind)

    def precondition(self, X: np.ndarray, kind: str | None) -> np.ndarray:
        """F~^{-1} X = sum_s beta A^(s) M A^(s)T beta X with beta = (A A^T)^{-1} (see scale),
        M = S of the pattern (Dirichlet) or its K_bb (lumped), or X itself for the identity
        preconditioner (kind None); section 2.

        READING: M is the pattern's matrix over the whole pattern boundary (the union of the
        dofs carrying a multiplier in any occurrence), shared by every occurrence; A^(s)T gives
        zero on the boundary dofs of s that carry no multiplier, so there they act as fixed.
        """
        X = np.asarray(X, float)
        if kind is None:
            return X.copy()
        vec = X.ndim == 1
        X2 = X[:, None] if vec else X
        T = self.scale(X2)
        Y = np.zeros_like(X2)
        for s in range(self.pb.n_occ):
            Mloc = self.local_precond_matrix(self.pb.occ_pattern[s], kind)
            Y += self.A[s] @ (Mloc @ (self.A[s].T @ T))
        Y = self.scale(Y)
        return Y[:, 0] if vec else Y

    # -- right-hand sides ---------------------------------------------------------------
    def loads(self, f_local=None):
        """Condensed loads g^(s), d = sum A S+ g, e = [Z^T g^(s)] (eq. 3 right-hand side)."""
        pb = self.pb
        f_local = pb.f_local if f_local is None else f_local
        g = []
        for s in range(pb.n_occ):
            P = self.pats[pb.occ_pattern[s]]
            g.append(P.condensed_load(f_local[s]))
        nr = g[0].shape[1]
        d = np.zeros((self.n_lambda, nr))
        e = np.zeros((self.G.shape[1], nr))
        for s in range(pb.n_occ):
            P = self.pats[pb.occ_pattern[s]]
            d += self.A[s] @ (P.Splus @ g[s])
            e[self.coarse_off[s]:self.coarse_off[s + 1]] = P.Z.T @ g[s]
        return g, d, e

    def lambda0(self, e, lam00=None):
        """lambda_0 = F~^{-1} G (G^T F~^{-1} G)^{-1} e + Q lambda_00 (Table 1, initialisation); F~^{-1} = I
        by default."""
        if not self.G.shape[1]:
            l0 = np.zeros((self.n_lambda, e.shape[1]))
        elif self.coarse is None:
            l0 = self.G @ self.coarse_solve(e)
        else:
            MG, H = self._coarse_M()
            l0 = MG @ sla.cho_solve(H, e)
        if lam00 is not None:
            l0 = l0 + self.Q(lam00)
        return l0

    def residual(self, lam, d):
        """r = Q^T (d - F lambda) (Table 1, initial residual)."""
        return self.Qt(d - self.F(lam))

    def permute(self, z: np.ndarray) -> np.ndarray:
        """Multivector [Pi_0 z, .., Pi_{np-1} z] for every column of z (section 3.1, eq. for w~).

        Columns are ordered (load case, permutation): column l*np + k = Pi_k z_l.  With rotated
        occurrences the permuted values are carried into the frame of their new place (section 4.2):
        READING: the value taken from multiplier m' for multiplier m is O^(a(m)) O^(a(m'))^T z[m'],
        a(.) the occurrence of the first endpoint, so the field seen from the pattern frame is moved.
        """
        pb = self.pb
        Pn = pb.perm_node
        nr, dpn, nm = z.shape[1], pb.dpn, pb.n_mult_nodes
        np_ = Pn.shape[0]
        out = np.empty((z.shape[0], nr * np_))
        zn = z.reshape(nm, dpn, nr)
        rotate = dpn == 3 and pb.has_rotation
        for k in range(np_):
            src = Pn[k]
            moved = zn[src]                                    # (nm, dpn, nr)
            if rotate:
                Ot = pb.occ_rot[pb.mult_occ[:, 0]]             # frame of the target's first endpoint
                Os = pb.occ_rot[pb.mult_occ[src, 0]]           # frame of the source's first endpoint
                Rk = np.einsum("mab,mcb->mac", Ot, Os)         # O_t O_s^T
                moved = np.einsum("mab,mbr->mar", Rk, moved)
            for l in range(nr):
                out[:, l * np_ + k] = moved[:, :, l].reshape(-1)
        return out

    # -- solvers (Table 1) ----------------------------------------------------------------
    def solve_classical(self, d, e, tol, max_it=2000, lam00=None, record=None, precond=None):
        """Projected conjugate gradient for each load case on its own (FETI-mrhs, section 3.4).

        The left column of Table 1 is its right column with one direction per iteration and no
        permutation, so each load case runs solve_block below on its own column, with the identity
        permutation and the short recurrence (the new direction made F-orthogonal to the previous
        one only).  Stopping per load case: ||r|| / ||r_0|| <= tol.

        record: optional list receiving lambda after every iteration (first load case).
        precond: None (identity), "lumped" or "dirichlet": z = Q F~^{-1} r (section 2).  READING: the
        projector keeps the identity in place of F~^{-1} whatever the preconditioner (the paper
        allows any of them there) unless the oracle was built with coarse=..., which puts that
        preconditioner in Q, Q^T and lambda_0 (then the residual and the products take Q^T, the
        directions Q).
        """
        nr = d.shape[1]
        lam = np.zeros((self.n_lambda, nr))
        its, hist = [], []
        for c in range(nr):
            rec = [] if (record is not None and c == 0) else None
            l00 = None if lam00 is None else lam00[:, c:c + 1]
            lc, st = self.solve_block(d[:, c:c + 1], e[:, c:c + 1], tol, max_it, lam00=l00, full_reorth=False,
                                      record=rec, precond=precond, permute=False)
            lam[:, c] = lc[:, 0]
            its.append(st["iterations"])
            hist.append(st["history"])
            if rec is not None:
                record.extend(x[:, 0] for x in rec)
        return lam, dict(iterations=its, history=hist)

    def solve_block(self, d, e, tol, max_it=2000, lam00=None, full_reorth=True, record=None, precond=None,
                    periodic=False, permute=True):
        """Multivector projected CG, Table 1 right column.

        permute=False takes the identity in place of the structure's permutations (one direction per
        column of z: the classical method for a single column).

        precond: as in solve_classical; the permutations act on z = Q F~^{-1} r.
        periodic: the shortcut of truly periodic structures (section 3.1, after Table 1): when F,
        Q and F~^{-1} commute with every permutation, Q F of the multivector [Pi_k z] is the
        multivector of the single product Q F z, [Pi_k Q F z], and the orthogonalisation against
        the stored blocks acts on P with the coefficients it applies to W (F W_i = P_i), so each
        iteration needs one product on n_rhs columns.  READING: the permuted product is
        re-projected like the permuted direction.

        full_reorth=True: every new block is F-orthogonalised against all stored blocks and
        F-normalised, W <- W eta^{-1/2}, P <- P eta^{-1/2} with eta = P^T W (section 3.3);
        eigenvalues of eta below ETA_DROP * e are dropped (pseudo-inverse, section 3.3).
        READING of the scale e: the largest F-energy z^T F z of a column of the block before
        the orthogonalisation (with F-orthonormal stored blocks it is |P_i^T z|^2 summed over
        the stored blocks plus the diagonal of eta), and at least the largest eigenvalue of
        eta; a direction is dropped when almost none of its energy is new, which also ends
        the iteration once the stored blocks span the whole space.
        full_reorth=False: the short recurrence of Table 1 (beta against the previous block),
        with a pseudo-inverse of W^T P.
        Stopping (READING): max over load cases of ||r_c|| / ||r0_c|| <= tol.
        """
        lam = self.lambda0(e, lam00)
        r = self.Qt(d - self.F(lam))
        r0 = np.linalg.norm(r, axis=0)
        r0[r0 == 0] = 1.0
        perm = self.permute if permute else (lambda x: x)
        periodic = periodic and permute
        z = self.Q(self.precondition(r, precond))
        Zb = self.Q(perm(z))          # READING: re-project permuted directions
        Pz = self.Qt(perm(self.Qt(self.F(z)))) if periodic else None
        Ws, Ps = [], []
        W_prev = P_prev = None
        hist = [1.0]
        drops = 0
        j = 0
        while np.max(np.linalg.norm(r, axis=0) / r0) > tol and j < max_it:
            if full_reorth:
                e_pre = np.zeros(Zb.shape[1])
                for Wi, Pi in zip(Ws, Ps):
                    B = Pi.T @ Zb
                    e_pre += (B * B).sum(axis=0)
                    Zb = Zb - Wi @ B
                    if periodic:
                        Pz = Pz - Pi @ B
                Pb = Pz if periodic else self.Qt(self.F(Zb))
                eta = Zb.T @ Pb
                eta = 0.5 * (eta + eta.T)
                ev, V = np.linalg.eigh(eta)
                e_pre += np.diag(eta)
                keep = ev > ETA_DROP * max(ev.max(), e_pre.max(), 0.0)
                drops += int((~keep).sum())
                if not keep.any():
                    break
                T = V[:, keep] / np.sqrt(ev[keep])[None, :]
                W = Zb @ T
                P = Pb @ T
                alpha = W.T @ r
                lam = lam + W @ alpha
                r = r - P @ alpha
                Ws.append(W)
                Ps.append(P)
            else:
                if W_prev is None:
                    W = Zb
                    P = Pz if periodic else None
                else:
                    beta = -np.linalg.pinv(WtP) @ (P_prev.T @ Zb)
                    W = Zb + W_prev @ beta
                    P = Pz + P_prev @ beta if periodic else None
                if P is None:
                    P = self.Qt(self.F(W))
                WtP = W.T @ P
                WtP = 0.5 * (WtP + WtP.T)
                alpha = np.linalg.pinv(WtP) @ (W.T @ r)
                lam = lam + W @ alpha
                r = r - P @ alpha
                W_prev, P_prev = W, P
            j += 1
            hist.append(float(np.max(np.linalg.norm(r, axis=0) / r0)))
            if record is not None:
                record.append(lam.copy())
            z = self.Q(self.precondition(r, precond))
            Zb = self.Q(perm(z))
            if periodic:
                Pz = self.Qt(perm(self.Qt(self.F(z))))
        return lam, dict(iterations=j, history=hist, rank_drops=drops)

    # -- recovery -------------------------------------------------------------------------
    def recover(self, lam, d, g, f_local=None):
        """Local displacements from lambda (eq. 2 with the kernel term).

        READING of the coarse unknown's sign: eq. 2 gives u^(s) = K+(f - t^T A^T lambda) + N alpha_s
        with F lambda - G alpha = d, so alpha = (G^T G)^{-1} G^T (F lambda - d) and the paper's
        g = -alpha.  Boundary: u_b = S+ (g^(s) - A^(s)T lambda) + Z alpha_s; interior:
        u_i = K_ii^{-1} (f_i - K_ib u_b).
        """
        pb = self.pb
        f_local = pb.f_local if f_local is None else f_local
        alpha = self.coarse_solve(self.G.T @ (self.F(lam) - d)) if self.G.shape[1] else None
        u = []
        for s in range(pb.n_occ):
            P = self.pats[pb.occ_pattern[s]]
            ub = P.Splus @ (g[s] - self.A[s].T @ lam)
            if alpha is not None and P.k:
                ub = ub + P.Z @ alpha[self.coarse_off[s]:self.coarse_off[s + 1]]
            us = np.zeros((P.n, lam.shape[1]))
            us[P.b] = ub
            us[P.i] = P.interior(f_local[s], ub)
            u.append(us)
        return u

    def solve(self, method="block", tol=None, max_it=2000, full_reorth=True, precond=None, periodic=False):
        tol = self.pb.tol if tol is None else tol
        g, d, e = self.loads()
        if method == "classical":
            lam, st = self.solve_classical(d, e, tol, max_it, precond=precond)
        else:
            lam, st = self.solve_block(d, e, tol, max_it, full_reorth=full_reorth, precond=precond,
                                       periodic=periodic)
        u = self.recover(lam, d, g)
        return lam, u, st


# =========================================================================== brute force

def global_solve(problem):
    """Assembled global problem K u = f (eq. 1) with u = 0 on the Dirichlet nodes.

    The global matrix is assembled from the global node numbering (occurrence
    stiffness rotated to the global frame), independently of the multipliers.
    Returns u per occurrence (pattern frame) and the global vector.
    """
    pb = problem
    if getattr(pb, "meta", {}).get("mortar"):
        raise ValueError("global_solve: the occurrences of a mortar structure share no mesh; use constrained_solve")
    dpn = pb.dpn
    n = pb.n_gnodes * dpn
    rows, cols, vals = [], [], []
    f = np.zeros((n, pb.n_rhs))
    for s in range(pb.n_occ):
        pat = pb.patterns[pb.occ_pattern[s]]
        O = pb.occ_rot[s][:dpn, :dpn] if dpn > 1 else np.ones((1, 1))
        R = sp.kron(sp.identity(pat.n_nodes), sp.csr_matrix(O)).tocsr()
        Kg = (R @ pat.K @ R.T).tocoo()
        gd = (pb.occ_gnode[s][:, None] * dpn + np.arange(dpn)[None, :]).ravel()
        rows.append(gd[Kg.row])
        cols.append(gd[Kg.col])
        vals.append(Kg.data)
        np.add.at(f, gd, R @ pb.f_local[s])
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    fixed = np.zeros(n, bool)
    for c in range(dpn):
        fixed[pb.dirichlet_gnodes * dpn + c] = True
    free = np.nonzero(~fixed)[0]
    Kf = K[free][:, free].tocsc()
    ug = np.zeros((n, pb.n_rhs))
    if len(free) <= 3000:
        ug[free] = sla.cho_solve(sla.cho_factor(Kf.toarray()), f[free])
    else:
        ug[free] = spla.splu(Kf).solve(f[free])
    u = []
    for s in range(pb.n_occ):
        pat = pb.patterns[pb.occ_pattern[s]]
        O = pb.occ_rot[s][:dpn, :dpn] if dpn > 1 else np.ones((1, 1))
        R = sp.kron(sp.identity(pat.n_nodes), sp.csr_matrix(O)).tocsr()
        gd = (pb.occ_gnode[s][:, None] * dpn + np.arange(dpn)[None, :]).ravel()
        u.append(R.T @ ug[gd])
    return u, ug, K, f


def constrained_solve(problem, oracle: FetiOracle | None = None):
    """The constrained global problem behind eq. 2, solved directly: minimise the energy
    sum_s (u_s^T K_s u_s / 2 - f_s^T u_s) subject to B u = 0, B = [.. A^(s) t^(s) ..], by the dense
    saddle-point system [K B^T; B 0] [u; lambda] = [f; 0] (K block diagonal, floating blocks
    included).  For structures without a global mesh (non-matching, mortar-coupled occurrences)
    this is the brute-force reference; on conforming meshes it equals global_solve.  Tiny sizes only.
    Returns u per occurrence (pattern frame) and lambda."""
    pb = problem
    o = FetiOracle(pb) if oracle is None else oracle
    ns = [pb.patterns[p].n for p in pb.occ_pattern]
    off = np.concatenate([[0], np.cumsum(ns)])
    n = int(off[-1])
    nl = pb.n_lambda
    Kd = np.zeros((n + nl, n + nl))
    rhs = np.zeros((n + nl, pb.n_rhs))
    for s in range(pb.n_occ):
        pat = pb.patterns[pb.occ_pattern[s]]
        P = o.pats[pb.occ_pattern[s]]
        Kd[off[s]:off[s + 1], off[s]:off[s + 1]] = pat.K.toarray()
        Bs = np.zeros((nl, ns[s]))
        Bs[:, P.b] = o.A[s].toarray()
        Kd[n:, off[s]:off[s + 1]] = Bs
        Kd[off[s]:off[s + 1], n:] = Bs.T
        rhs[off[s]:off[s + 1]] = pb.f_local[s]
    x = np.linalg.solve(Kd, rhs)
    return [x[off[s]:off[s + 1]] for s in range(pb.n_occ)], x[n:]


def multipliers_from_displacements(oracle: FetiOracle, u):
    """lambda solving B^T lambda = f - K u occurrence by occurrence (rows of eq. 2).

    With non-redundant multipliers B = [A^(s) t^(s)] has full row rank, so lambda is the
    unique least-squares solution.
    """
    pb = oracle.pb
    blocks_B, blocks_r = [], []
    for s in range(pb.n_occ):
        P = oracle.pats[pb.occ_pattern[s]]
        res = pb.f_local[s] - pb.patterns[pb.occ_pattern[s]].K @ u[s]
        blocks_B.append(oracle.A[s])
        blocks_r.append(res[P.b])
    B = sp.hstack(blocks_B).tocsr()          # N_lambda x sum n_b
    r = np.vstack(blocks_r)
    BBt = (B @ B.T).tocsc()
    return spla.splu(BBt).solve(np.asarray(B @ r))
