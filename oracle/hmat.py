"""Parametric H^2-matrix: offline stage, online stage, MVM (oracle; test infrastructure only).

Paper passages followed:
* Sec. 3.2 "Cluster Basis": factor matrices [U_{s,k}]_{ij} = l_j^{(B_{s,k})}(x_{s,i,k}),
  U_s = U_{s,d} (face-splitting) ... U_{s,1}.
* Sec. 3.4.1 "Transfer Matrices" and the lemma of App. "Transfer Matrices":
  E_{s'} = E_{s',d} (x) ... (x) E_{s',1}.  Reading: the printed entry formula has
  its indices swapped relative to the lemma Gamma_{s'} U_s = U_{s'} E_{s'}; the
  lemma's orientation is used, [E_{s',k}]_{j,i} = l_i^{(B_{s,k})}(eta_j^{(B_{s',k})})
  (row = child node, column = parent polynomial).
* App. "PTTK Method": far tensor
  [M_b]_{i,k,j} = kappa(eta_i^{(B_s)}, eta_j^{(B_t)}; eta_k^{(B_theta)}), and the
  coupling C_b(theta) = L_b H_b(theta) R_b^T (Sec. 4.2, eq. "ff_h2_approx").
* Sec. 4.3 "Near-Field Approximations": [A_b]_{(ij), k} = kappa(x_{s,i}, x_{t,j}; eta_k),
  e = i + (j-1) n_s, D_b(theta) = reshape(a_b(theta), [n_s, n_t]) (MATLAB order).
* Alg. "Offline Stage: Parametric H^2-matrix", Alg. "Online Stage", Alg. PTTK online.
* Alg. "H^2-matrix MVM" with FastForward and FastBackward; the coupling step of
  Alg. "Modified H^2-Matrix MVM" in its explicit form y_hat_s += C_b x_hat_t.
* Sec. 5.2: for a stationary kernel M_b depends only on the level and the box
  offset, so one tensor per translation class is compressed (``dedup=True``);
  ``dedup=False`` compresses every far block separately, as the algorithm is
  written.
* Sec. 6 "Error Calculation": sampled-row relative error against the exact kernel.
* Def. "Parametric H-matrix", App. PTTK offline phase 3 and Alg. "H-matrix MVM" with the
  parametric far-field substitution: the H-matrix variant (``h_far_factors``,
  ``instantiate_h``, ``matvec_h``), sharing the near field and the far tensors.

Compression is the truncated HOSVD of ``oracle.tucker`` (see there for the reading
of the tolerance), or with ``compress="tt"`` TT-cross followed by TT-rounding
(``oracle.tt``; Sec. 2.1), whose cores are converted exactly into the same form
(spatial factors L, R, U_e and a parameter core with identity parameter factors).
TT-cross is not symmetric in the mode order, so in that mode a far class whose
offset is lexicographically below its negative takes the transposed factors of its
mirror class, and a near block (s, t) with s > t the transpose of block (t, s).  The nugget of a regularised system is not part of kappa; it
is added in the MVM as nugget * x.
"""

import numpy as np

from . import cheb
from . import tree as tr
from . import tt as ttm
from . import tucker


class PH2:
    """Offline data of a parametric H^2-matrix, with compression done lazily per tensor."""

    def __init__(self, X, *, l_max, eta2, kernel, theta_lo, theta_hi, p_s, p_theta, tol,
                 box=(0.0, 1.0), dedup=True, compress="tucker"):
        self.X = np.asarray(X, dtype=np.float64)
        self.n, self.d = self.X.shape
        self.kernel = kernel
        self.theta_lo = np.atleast_1d(np.asarray(theta_lo, dtype=np.float64))
        self.theta_hi = np.atleast_1d(np.asarray(theta_hi, dtype=np.float64))
        self.d_theta = self.theta_lo.shape[0]
        self.p_s = int(p_s)
        self.p_theta = int(p_theta)
        self.P = self.p_s ** self.d
        self.tol = float(tol)
        self.dedup = dedup
        if compress not in ("tucker", "tt"):
            raise ValueError("compress must be 'tucker' or 'tt'")
        self.compress = compress
        self.tt_evals = 0         # distinct tensor entries evaluated by TT-cross
        self._far_tt = {}         # raw TT cores per compressed far key
        # offline stage, first line: cluster tree and block cluster tree
        self.tree = tr.build_cluster_tree(self.X, box[0], box[1], l_max)
        self.near, self.far = tr.build_block_tree(self.tree, eta2)
        self.classes, self.block_class = tr.translation_classes(self.tree, self.far)
        self.class_rep = {}
        for i, c in enumerate(self.block_class):
            self.class_rep.setdefault(c, i)      # first far block of each class
        self.theta_nodes = [cheb.chebyshev_nodes(self.theta_lo[k], self.theta_hi[k], self.p_theta)
                            for k in range(self.d_theta)]
        self._far = {}
        self._near = {}
        self._E = {}
        self._U = {}

    # ---------------------------------------------------------------- bases
    def cluster_basis(self, s):
        """U_s = U_{s,d} (face-splitting) ... U_{s,1}, rows in the node's point order (Sec. 3.2)."""
        if s not in self._U:
            t = self.tree
            self._U[s] = cheb.tensor_lagrange(t.lo[s], t.hi[s], self.p_s, self.X[t.idx[s]])
        return self._U[s]

    def transfer_factors(self, child):
        """Per-axis factors [E_{s',k}]_{j,i} = l_i^{(B_s,k)}(eta_j^{(B_s',k)}) (lemma orientation)."""
        t = self.tree
        par = t.parent[child]
        out = []
        for k in range(self.d):
            parent_nodes = cheb.chebyshev_nodes(t.lo[par][k], t.hi[par][k], self.p_s)
            child_nodes = cheb.chebyshev_nodes(t.lo[child][k], t.hi[child][k], self.p_s)
            out.append(cheb.lagrange(parent_nodes, child_nodes))   # [j, i]
        return out

    def transfer(self, child):
        """E_{s'} = E_{s',d} (x) ... (x) E_{s',1} as an explicit P x P matrix."""
        if child not in self._E:
            f = self.transfer_factors(child)
            E = f[0]
            for k in range(1, self.d):
                E = np.kron(f[k], E)
            self._E[child] = E
        return self._E[child]

    # ---------------------------------------------------------------- tensors
    def theta_grid(self):
        """All parameter interpolation nodes eta_k^{(B_theta)}, shape (p,)*d_theta + (d_theta,)."""
        mesh = np.meshgrid(*self.theta_nodes, indexing="ij")
        return np.stack(mesh, axis=-1)

    def far_tensor_of_block(self, bi):
        """[M_b]_{i,k_1..,j} = kappa(eta_i^{(B_s)}, eta_j^{(B_t)}; eta_k), i and j flattened little-endian."""
        s, u = self.far[bi]
        t = self.tree
        ns = cheb.tensor_nodes(t.lo[s], t.hi[s], self.p_s)     # (P, d)
        nt = cheb.tensor_nodes(t.lo[u], t.hi[u], self.p_s)
        th = self.theta_grid()                                  # (p,..,dθ)
        sh_theta = th.shape[:-1]
        x = ns.reshape((self.P,) + (1,) * self.d_theta + (1, self.d))
        y = nt.reshape((1,) + (1,) * self.d_theta + (self.P, self.d))
        thb = th.reshape((1,) + sh_theta + (1, self.d_theta))
        return self.kernel(x, y, thb)                           # (P, p.., P)

    def near_tensor(self, s, u):
        """[A_b]_{e,k} = kappa(x_{s,i}, x_{t,j}; eta_k), e = i + j n_s (column-major pairs)."""
        t = self.tree
        Xs = self.X[t.idx[s]]
        Xt = self.X[t.idx[u]]
        ns, nt = len(Xs), len(Xt)
        # pair (i, j) at flat position j * ns + i
        x = np.broadcast_to(Xs[None, :, :], (nt, ns, self.d)).reshape(ns * nt, self.d)
        y = np.broadcast_to(Xt[:, None, :], (nt, ns, self.d)).reshape(ns * nt, self.d)
        th = self.theta_grid()
        sh_theta = th.shape[:-1]
        xb = x.reshape((ns * nt,) + (1,) * self.d_theta + (self.d,))
        yb = y.reshape((ns * nt,) + (1,) * self.d_theta + (self.d,))
        thb = th.reshape((1,) + sh_theta + (self.d_theta,))
        return self.kernel(xb, yb, thb)                         # (N_e, p..)

    # ---------------------------------------------------------------- compression
    def far_key(self, bi):
        return self.block_class[bi] if self.dedup else bi

    def far_factors(self, key):
        """Compressed far tensor of a class (dedup) or of a far block: (core, [L, Θ_1.., R]).
        T-HOSVD, or TT-cross + TT-rounding converted to the same form (``compress="tt"``)."""
        if key not in self._far:
            if self.compress == "tt":
                mk = self._mirror_key(key)
                if mk is not None:
                    core, facs = self.far_factors(mk)
                    # M_mirror[i, k, j] = M[j, k, i]: swap the spatial factors and core modes
                    self._far[key] = (np.moveaxis(np.moveaxis(core, 0, -1), -2, 0), [facs[-1]] + facs[1:-1] + [facs[0]])
                else:
                    cores = self._tt_far(key)
                    self._far[key] = ttm.far_factors(cores, self.d, self.d_theta)
            else:
                bi = self.class_rep[key] if self.dedup else key
                core, facs, _ = tucker.thosvd(self.far_tensor_of_block(bi), self.tol)
                self._far[key] = (core, facs)
        return self._far[key]

    def _mirror_key(self, key):
        """TT mode: the class whose factors this one transposes (its offset is below its
        negative and that class exists), else None."""
        if not self.dedup:
            return None
        lev, o = self.classes[key]
        neg = tuple(-c for c in o)
        if tuple(o) < neg and (lev, neg) in self._class_index():
            return self._class_index()[(lev, neg)]
        return None

    def _class_index(self):
        if not hasattr(self, "_cidx"):
            self._cidx = {k: i for i, k in enumerate(self.classes)}
        return self._cidx

    def _tt_far(self, key):
        """TT-cross + TT-rounding of the far tensor of ``key`` with modes
        (i_1..i_d, k_1..k_dθ, j_1..j_d) (Sec. 2.1; App. PTTK review)."""
        if key not in self._far_tt:
            bi = self.class_rep[key] if self.dedup else key
            M = self.far_tensor_of_block(bi)                    # (P, p.., P), nodes little-endian
            p, d, dth = self.p_s, self.d, self.d_theta
            Mm = M.reshape((p,) * d + M.shape[1:1 + dth] + (p,) * d, order="F")
            dims = list(Mm.shape)
            cores, ev = ttm.tt_compress(lambda idx: Mm[tuple(idx.T)], dims, self.tol)
            self.tt_evals += ev
            self._far_tt[key] = cores
        return self._far_tt[key]

    def far_tt_cores(self, key):
        """Raw TT cores of a far key that is compressed itself (not a mirror)."""
        return self._tt_far(key)

    def near_factors(self, bi):
        """Compressed near tensor A_b of near block bi: (core, [U_e, Θ_1..])."""
        if bi not in self._near:
            s, u = self.near[bi]
            A = self.near_tensor(s, u)
            if self.compress == "tt":
                cores, ev = ttm.tt_compress(lambda idx: A[tuple(idx.T)], list(A.shape), self.tol)
                self.tt_evals += ev
                self._near[bi] = ttm.near_factors(cores, self.d_theta)
            else:
                core, facs, _ = tucker.thosvd(A, self.tol)
                self._near[bi] = (core, facs)
        return self._near[bi]

    def _near_index(self):
        if not hasattr(self, "_nidx"):
            self._nidx = {tuple(b): i for i, b in enumerate(self.near)}
        return self._nidx

    # ---------------------------------------------------------------- online stage
    def theta_vectors(self, theta, deriv_dim=None):
        theta = np.atleast_1d(np.asarray(theta, dtype=np.float64))
        if np.any(theta < self.theta_lo) or np.any(theta > self.theta_hi):
            raise ValueError("theta outside the parameter box")
        return cheb.parametric_vectors(theta, self.theta_lo, self.theta_hi, self.p_theta, deriv_dim)

    def coupling(self, key, vs):
        """C_b(theta) = L_b H_b(theta) R_b^T with H_b = core contracted with Θ_i^T v_i (Alg. PTTK online)."""
        core, facs = self.far_factors(key)
        H = core
        for i in range(self.d_theta):
            w = facs[1 + i].T @ vs[i]
            H = np.tensordot(H, w, axes=([1], [0]))             # contract the next θ mode
        return facs[0] @ H @ facs[-1].T

    def near_block(self, bi, vs):
        """D_b(theta) = reshape(U_e c_b, [n_s, n_t]) column-major, c_b = core x_θ (Θ_i^T v_i) (Sec. 4.3)."""
        s, u = self.near[bi]
        if self.compress == "tt" and s > u:
            return self.near_block(self._near_index()[(u, s)], vs).T
        core, facs = self.near_factors(bi)
        c = core
        for i in range(self.d_theta):
            w = facs[1 + i].T @ vs[i]
            c = np.tensordot(c, w, axes=([1], [0]))
        a = facs[0] @ c
        s, u = self.near[bi]
        ns, nt = len(self.tree.idx[s]), len(self.tree.idx[u])
        return a.reshape(nt, ns).T                               # MATLAB reshape

    def instantiate(self, theta, deriv_dim=None, near_blocks=None, far_keys=None):
        """Alg. "Online Stage": D_b for near blocks, C for far classes/blocks.

        With ``deriv_dim = i`` the parametric vector v_i is replaced by v_i', which
        instantiates the partial derivative d K~ / d theta_i exactly (multilinearity).
        """
        vs = self.theta_vectors(theta, deriv_dim)
        if near_blocks is None:
            near_blocks = range(len(self.near))
        if far_keys is None:
            far_keys = range(len(self.classes)) if self.dedup else range(len(self.far))
        D = {bi: self.near_block(bi, vs) for bi in near_blocks}
        C = {k: self.coupling(k, vs) for k in far_keys}
        return {"D": D, "C": C}

    # ---------------------------------------------------------------- parametric H-matrix
    def h_far_factors(self, bi):
        """Far block b = (s, t) in the parametric H-matrix format (Def. "Parametric H-matrix";
        App. PTTK, offline phase 3): S_b = U_s L_b and T_b = U_t R_b, with U_s and U_t the
        Chebyshev bases of the block's own clusters evaluated at their points (not through
        transfer matrices) and L_b, R_b the outer factors of the block's compressed far tensor."""
        if not hasattr(self, "_hST"):
            self._hST = {}
        if bi not in self._hST:
            s, u = self.far[bi]
            core, facs = self.far_factors(self.far_key(bi))
            self._hST[bi] = (self._tree_order_basis(s) @ facs[0], self._tree_order_basis(u) @ facs[-1])
        return self._hST[bi]

    def _tree_order_basis(self, s):
        """U_s evaluated at the points of cluster s in tree order (rows begin_s .. end_s - 1 of the
        permuted vector; for an inner cluster the concatenation of its children's ranges)."""
        t = self.tree
        return cheb.tensor_lagrange(t.lo[s], t.hi[s], self.p_s, self.X[t.perm[t.begin[s]:t.end[s]]])

    def h_core(self, key, vs):
        """H_b(theta): the far core contracted with Θ_i^T v_i(theta_i) (Alg. PTTK online)."""
        core, facs = self.far_factors(key)
        H = core
        for i in range(self.d_theta):
            H = np.tensordot(H, facs[1 + i].T @ vs[i], axes=([1], [0]))
        return H

    def instantiate_h(self, theta, deriv_dim=None):
        """Alg. "Online Stage" for the parametric H-matrix: D_b for near blocks, H_b for far keys."""
        vs = self.theta_vectors(theta, deriv_dim)
        keys = range(len(self.classes)) if self.dedup else range(len(self.far))
        return {"D": {bi: self.near_block(bi, vs) for bi in range(len(self.near))},
                "H": {k: self.h_core(k, vs) for k in keys}}

    def matvec_h(self, inst, x, nugget=0.0):
        """Alg. "H-matrix MVM" with the parametric far field (Sec. "MVM", parametric H-matrices):
        y_s += S_b (H_b(theta) (T_b^T x_t)) for every far block, y_s += D_b x_t for every near
        block; y = (K~(theta) + nugget I) x, x of shape (n, R) in original order."""
        t = self.tree
        x = np.asarray(x, dtype=np.float64)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        xt = x[t.perm]
        yt = np.zeros_like(xt)
        for bi, (s, u) in enumerate(self.far):
            S, T = self.h_far_factors(bi)
            yt[t.begin[s]:t.end[s]] += S @ (inst["H"][self.far_key(bi)] @ (T.T @ xt[t.begin[u]:t.end[u]]))
        for bi, (s, u) in enumerate(self.near):
            yt[t.begin[s]:t.end[s]] += inst["D"][bi] @ xt[t.begin[u]:t.end[u]]
        y = np.empty_like(x)
        y[t.perm] = yt
        y += nugget * x
        return y[:, 0] if squeeze else y

    # ---------------------------------------------------------------- MVM
    def _upward(self, xt):
        """FastForward: leaves x_hat = U^T x; inner nodes x_hat = sum E_{s'}^T x_hat_{s'}."""
        t = self.tree
        xh = {}
        for s in reversed(range(t.n_nodes)):                   # children before parents
            if not t.children[s]:
                xh[s] = self.cluster_basis(s).T @ xt[t.begin[s]:t.end[s]]
            else:
                acc = np.zeros((self.P, xt.shape[1]))
                for c in t.children[s]:
                    acc += self.transfer(c).T @ xh[c]
                xh[s] = acc
        return xh

    def matvec(self, inst, x, nugget=0.0):
        """Alg. "H^2-matrix MVM": y = (K~(theta) + nugget I) x, x of shape (n, R) in original order."""
        t = self.tree
        x = np.asarray(x, dtype=np.float64)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        xt = x[t.perm]
        xh = self._upward(xt)
        yh = {s: np.zeros((self.P, x.shape[1])) for s in range(t.n_nodes)}
        for bi, (s, u) in enumerate(self.far):
            yh[s] += inst["C"][self.far_key(bi)] @ xh[u]
        yt = np.zeros_like(xt)
        for bi, (s, u) in enumerate(self.near):
            yt[t.begin[s]:t.end[s]] += inst["D"][bi] @ xt[t.begin[u]:t.end[u]]
        for s in range(t.n_nodes):                              # FastBackward, parents first
            if t.children[s]:
                for c in t.children[s]:
                    yh[c] += self.transfer(c) @ yh[s]
            else:
                yt[t.begin[s]:t.end[s]] += self.cluster_basis(s) @ yh[s]
        y = np.empty_like(x)
        y[t.perm] = yt
        y += nugget * x
        return y[:, 0] if squeeze else y

    def blocks_for_rows(self, rows):
        """Near blocks and far keys that touch the given original row indices."""
        t = self.tree
        inv = np.empty(self.n, dtype=np.int64)
        inv[t.perm] = np.arange(self.n)
        pos = inv[np.asarray(rows)]
        leaves = sorted({lf for lf in t.leaves for p_ in pos if t.begin[lf] <= p_ < t.end[lf]})
        anc = set()
        for lf in leaves:
            s = lf
            while s >= 0:
                anc.add(s)
                s = t.parent[s]
        near = [bi for bi, (s, _) in enumerate(self.near) if s in anc]
        far = sorted({self.far_key(bi) for bi, (s, _) in enumerate(self.far) if s in anc})
        return near, far, anc, pos

    def matvec_rows(self, theta, x, rows, deriv_dim=None, nugget=0.0):
        """[(K~(theta) + nugget I) x]_rows, compressing only the tensors those rows need.

        Same algorithm as ``matvec`` restricted to the rows: full upward pass, the
        coupling and near-field products of the blocks in the rows' leaf-to-root
        paths, and the downward pass along those paths.
        """
        near, far, _, _ = self.blocks_for_rows(rows)
        inst = self.instantiate(theta, deriv_dim, near_blocks=near, far_keys=far)
        return self.matvec_rows_inst(inst, x, rows, nugget)

    def matvec_rows_inst(self, inst, x, rows, nugget=0.0):
        """``matvec`` restricted to the given rows, with an instance holding (at least) the
        near blocks and far keys of those rows' leaf-to-root paths."""
        t = self.tree
        x = np.asarray(x, dtype=np.float64)
        squeeze = x.ndim == 1
        if squeeze:
            x = x[:, None]
        near, _, anc, pos = self.blocks_for_rows(rows)
        xt = x[t.perm]
        xh = self._upward(xt)
        yh = {s: np.zeros((self.P, x.shape[1])) for s in anc}
        for bi, (s, u) in enumerate(self.far):
            if s in anc:
                yh[s] += inst["C"][self.far_key(bi)] @ xh[u]
        yt = np.zeros_like(xt)
        for bi in near:
            s, u = self.near[bi]
            yt[t.begin[s]:t.end[s]] += inst["D"][bi] @ xt[t.begin[u]:t.end[u]]
        for s in sorted(anc):
            if t.children[s]:
                for c in t.children[s]:
                    if c in anc:
                        yh[c] += self.transfer(c) @ yh[s]
            else:
                yt[t.begin[s]:t.end[s]] += self.cluster_basis(s) @ yh[s]
        out = yt[pos] + nugget * x[np.asarray(rows)]
        return out[:, 0] if squeeze else out

    # ---------------------------------------------------------------- dense forms
    def dense(self, inst):
        """Dense K~ assembled block by block: D_b, and U_s C_b U_t^T with U_s of Sec. 3.2."""
        t = self.tree
        K = np.zeros((self.n, self.n))
        for bi, (s, u) in enumerate(self.near):
            K[np.ix_(t.idx[s], t.idx[u])] = inst["D"][bi]
        for bi, (s, u) in enumerate(self.far):
            K[np.ix_(t.idx[s], t.idx[u])] = (self.cluster_basis(s) @ inst["C"][self.far_key(bi)]
                                             @ self.cluster_basis(u).T)
        return K

    def plain_dense(self, theta):
        """Untruncated interpolant, no tree algebra and no SVD (Sec. 2.2 eqs. int_of_kappa_1/3).

        Near pairs: psi(x, y; theta) = sum_k kappa(x, y; eta_k) Lambda_k(theta).
        Far pairs: phi(x, y; theta) = sum_{i,k,j} kappa(eta_i, eta_j; eta_k)
                   Lambda_i(x) Lambda_k(theta) Lambda_j(y).
        """
        t = self.tree
        vs = self.theta_vectors(theta)
        lam = vs[0]
        for k in range(1, self.d_theta):
            lam = np.multiply.outer(lam, vs[k])                 # Λ_k(θ) on the θ grid
        K = np.zeros((self.n, self.n))
        for s, u in self.near:
            A = self.near_tensor(s, u)                          # (N_e, p..)
            a = np.tensordot(A, lam, axes=(list(range(1, 1 + self.d_theta)),
                                           list(range(self.d_theta))))
            K[np.ix_(t.idx[s], t.idx[u])] = a.reshape(len(t.idx[u]), len(t.idx[s])).T
        for bi, (s, u) in enumerate(self.far):
            M = self.far_tensor_of_block(bi)
            MF = np.tensordot(M, lam, axes=(list(range(1, 1 + self.d_theta)),
                                            list(range(self.d_theta))))
            Ls = cheb.tensor_lagrange(t.lo[s], t.hi[s], self.p_s, self.X[t.idx[s]])
            Lt = cheb.tensor_lagrange(t.lo[u], t.hi[u], self.p_s, self.X[t.idx[u]])
            K[np.ix_(t.idx[s], t.idx[u])] = Ls @ MF @ Lt.T
        return K

    def exact_dense(self, theta):
        """K(X, X; theta) by direct kernel evaluation."""
        th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
        return self.kernel(self.X[:, None, :], self.X[None, :, :], th)


def exact_rows(X, kernel, theta, rows, x):
    """[K(X, X; theta) x]_rows by direct evaluation (Sec. 6 "Error Calculation")."""
    X = np.asarray(X, dtype=np.float64)
    th = np.atleast_1d(np.asarray(theta, dtype=np.float64))
    Kr = kernel(X[np.asarray(rows)][:, None, :], X[None, :, :], th)
    return Kr @ x


def sampled_error(model, thetas, x, rows):
    """Sec. 6 "Error Calculation": mean over theta of ||[Kx]_J - [K~x]_J|| / ||[Kx]_J||."""
    errs = []
    for th in thetas:
        ex = exact_rows(model.X, model.kernel, th, rows, x)
        ap = model.matvec_rows(th, x, rows)
        errs.append(np.linalg.norm(ex - ap) / np.linalg.norm(ex))
    return float(np.mean(errs))
