"""Dense one-site TDVP sweep of the super-MPS |rho>> (oracle; test
infrastructure only).

Paper sections followed:
* SM Sec. II.A (Choi map): the site tensor A[a, sigma, sigma', b] is a
  super-MPS tensor with s = (sigma, sigma'); H acts on sigma only (H (x) 1).
* SM Fig. optimalB(c,d): rank-3 environments L_i, R_i, the one-site
  effective Hamiltonian H^(1) A = L.A.W.R and the bond one H^(0) S = L.S.R.
* SM Sec. II.E (splitting): dA/dbeta = -H^(1) A and dS/dbeta = +H^(0) S are
  integrated one after the other; A <- exp(-tau H^(1)) A,
  S <- exp(+tau H^(0)) S.  A left-to-right sweep followed by the
  right-to-left one is the symmetric (second-order) integrator.
* SM Sec. II.F steps 1-7: site exponential, QR A = A^L S, backward bond
  exponential, absorb S into the next site, move on; mirrored with LQ.
* SM Sec. II.H: Lanczos exponential exp(tH) b = ||b|| sum_i c_i q_i, c the
  first column of exp(tT), T the Krylov tridiagonal matrix; the contraction
  order L.A, then W, then R (SM Fig. Lanczos).
* Bilayer observables (SM Sec. II.A): ||rho(beta)||_F^2 = Z(2 beta),
  E = <<rho|H (x) 1|rho>> / <<rho|rho>>.

Readings where the paper is silent (stated once here):
* One call of ``sweep`` advances beta by dbeta: left-to-right with
  tau = dbeta/2, then right-to-left with tau = dbeta/2; the two exponentials
  at the last site are merged into one with 2*tau (same generator).
* The state is kept as e^Lambda times a normalised mixed-canonical MPS: after
  every local exponential the tensor is normalised and ln of its norm is
  added to Lambda, so Lambda = ln ||rho||_F.
* Krylov: fixed dimension K, full reorthogonalisation (two classical
  Gram-Schmidt passes), lucky breakdown when beta_j <= tol * ||H q_j||,
  exp(tT) from the eigen-decomposition of T.
* QR / LQ with non-negative diagonal of the triangular factor.
"""
import numpy as np


# ---------------------------------------------------------------- contractions
def heff1(L, W, R, A):
    """H^(1) A (SM Fig. optimalB(c)): out[x,so,sp,y] =
    sum L[x,a,al] A[al,si,sp,be] W[a,so,si,b] R[y,b,be], contracted in the
    order of SM Fig. Lanczos: L.A, then W, then R."""
    T1 = np.tensordot(L, A, axes=([2], [0]))              # x a si sp be
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 2]))       # x sp be so b
    out = np.tensordot(T2, R, axes=([2, 4], [2, 1]))      # x sp so y
    return out.transpose(0, 2, 1, 3)


def heff2(L, W1, W2, R, C):
    """Two-site generator H^(2) C of the 2-TDVP flow (SM Sec. 2-TDVP in the
    initial stage, Eq. S-2TDVP) on C_i = A_i^L A_{i+1}:
    out[x,so1,sp1,so2,sp2,y] = sum L[x,a,al] C[al,si1,sp1,si2,sp2,be]
    W1[a,so1,si1,b] W2[b,so2,si2,c] R[y,c,be], contracted as L.C, then W1,
    then W2, then R."""
    T1 = np.tensordot(L, C, axes=([2], [0]))              # x a si1 sp1 si2 sp2 be
    T2 = np.tensordot(T1, W1, axes=([1, 2], [0, 2]))      # x sp1 si2 sp2 be so1 b
    T3 = np.tensordot(T2, W2, axes=([6, 2], [0, 2]))      # x sp1 sp2 be so1 so2 c
    out = np.tensordot(T3, R, axes=([3, 6], [2, 1]))      # x sp1 sp2 so1 so2 y
    return out.transpose(0, 3, 1, 4, 2, 5)


def heff0(L, R, S):
    """H^(0) S (SM Fig. optimalB(d)): out[x,y] = sum L[x,a,al] S[al,be] R[y,a,be]."""
    T = np.tensordot(L, S, axes=([2], [0]))               # x a be
    return np.tensordot(T, R, axes=([1, 2], [1, 2]))      # x y


def env_left(L, A, W):
    """L_{i+1}[y',b,y] = sum conj(A)[x',so,sp,y'] L[x',a,x] A[x,si,sp,y] W[a,so,si,b]."""
    T1 = np.tensordot(L, A, axes=([2], [0]))              # x' a si sp y
    T2 = np.tensordot(T1, W, axes=([1, 2], [0, 2]))       # x' sp y so b
    return np.tensordot(A.conj(), T2, axes=([0, 1, 2], [0, 3, 1])).transpose(0, 2, 1)


def env_right(R, A, W):
    """R_{i}[x',a,x] = sum conj(A)[x',so,sp,y'] W[a,so,si,b] A[x,si,sp,y] R[y',b,y]."""
    T1 = np.tensordot(A, R, axes=([3], [2]))              # x si sp y' b
    T2 = np.tensordot(T1, W, axes=([1, 4], [2, 3]))       # x sp y' a so
    return np.tensordot(A.conj(), T2, axes=([1, 2, 3], [4, 1, 2])).transpose(0, 2, 1)


# ---------------------------------------------------------------- Lanczos exp
def lanczos_expm(apply, v, t, K, tol=1e-13):
    """exp(t H) v for symmetric H given by ``apply`` (SM Sec. II.H).

    Returns (result, info) with info = dict(k=Krylov size used,
    err=beta_K |[exp(tT)]_{K,1}| a-posteriori estimate)."""
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return np.zeros_like(v), dict(k=0, err=0.0)
    Q = [v / nv]
    alpha, beta = [], []
    for j in range(K):
        w = apply(Q[j])
        hn = np.linalg.norm(w)
        a = float(np.vdot(Q[j], w))
        w = w - a * Q[j]
        if j > 0:
            w = w - beta[j - 1] * Q[j - 1]
        for _ in range(2):
            c = [float(np.vdot(q, w)) for q in Q]
            for ci, q in zip(c, Q):
                w = w - ci * q
        alpha.append(a)
        b = np.linalg.norm(w)
        beta.append(b)
        if b <= tol * hn or j == K - 1:
            break
        Q.append(w / b)
    k = len(alpha)
    T = np.diag(alpha) + np.diag(beta[:k - 1], 1) + np.diag(beta[:k - 1], -1)
    lam, V = np.linalg.eigh(T)
    c = V @ (np.exp(t * lam) * V[0, :])
    out = np.zeros_like(v)
    for ci, q in zip(c, Q):
        out = out + ci * q
    err = beta[k - 1] * abs(c[k - 1]) if k == K else 0.0
    return nv * out, dict(k=k, err=err)


# ---------------------------------------------------------------- gauge moves
def qr_pos(M):
    """M = Q R with Q having orthonormal columns and diag(R) >= 0."""
    Q, R = np.linalg.qr(M, mode="reduced")
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return Q * s[None, :], R * s[:, None]


def lq_pos(M):
    """M = L Q with Q having orthonormal rows and diag(L) >= 0."""
    Q, R = qr_pos(M.T)
    return R.T, Q.T


def qr_pos_blocked(M, row_q, col_q):
    """QR of a charge-conserving matrix, one charge block at a time.

    M[r, c] vanishes unless row_q[r] == col_q[c]; after permuting rows and
    columns by charge the matrix is block diagonal, and its QR is the QR of
    each block (Q stays charge conserving exactly)."""
    Q = np.zeros_like(M)
    R = np.zeros((M.shape[1], M.shape[1]))
    for q in sorted(set(col_q)):
        cols = [c for c, qc in enumerate(col_q) if qc == q]
        rows = [r for r, qr in enumerate(row_q) if qr == q]
        if not rows:
            raise ValueError("column sector without rows")
        qb, rb = qr_pos(M[np.ix_(rows, cols)])
        if qb.shape[1] < len(cols):
            raise ValueError("sector with more columns than rows")
        Q[np.ix_(rows, cols)] = qb
        R[np.ix_(cols, cols)] = rb
    return Q, R


def lq_pos_blocked(M, row_q, col_q):
    Q, R = qr_pos_blocked(M.T, col_q, row_q)
    return R.T, Q.T


# ---------------------------------------------------------------- the state
class State:
    """e^Lambda times a mixed-canonical super-MPS with the centre at ``centre``."""

    def __init__(self, A, Ws, beta, lam=0.0):
        self.A = [a.copy() for a in A]
        self.W = Ws
        self.N = len(A)
        self.beta = float(beta)
        self.lam = float(lam)
        self.centre = None
        self.Lenv = [None] * (self.N + 1)
        self.Renv = [None] * (self.N + 1)
        self.max_krylov_err = 0.0
        self.layouts = None          # charge layouts of the bonds (symmetric runs)
        self.mode = "u1u1"           # their block structure (charges.project)

    def dims(self):
        return [self.A[0].shape[0]] + [a.shape[3] for a in self.A]

    def _qr(self, k):
        """A_k reshaped (D_k 16) x D_{k+1} = Q R (blockwise when charges are known)."""
        Dl, _, _, Dr = self.A[k].shape
        M = self.A[k].reshape(Dl * 16, Dr)
        if self.layouts is None:
            return qr_pos(M)
        from .charges import s_charges
        ql, qr = self.layouts[k].charges, self.layouts[k + 1].charges
        row_q = [(a[0] + c[0], a[1] + c[1]) for a in ql for c in s_charges(self.mode)]
        return qr_pos_blocked(M, row_q, qr)

    def _lq(self, k):
        """A_k reshaped D_k x (16 D_{k+1}) = L Q (blockwise when charges are known)."""
        Dl, _, _, Dr = self.A[k].shape
        M = self.A[k].reshape(Dl, 16 * Dr)
        if self.layouts is None:
            return lq_pos(M)
        from .charges import s_charges
        ql, qr = self.layouts[k].charges, self.layouts[k + 1].charges
        col_q = [(b[0] - c[0], b[1] - c[1]) for c in s_charges(self.mode) for b in qr]
        return lq_pos_blocked(M, ql, col_q)

    def canonicalise(self):
        """Right-canonicalise by LQ from site N-1 down to 1, centre at site 0,
        normalise the centre into Lambda, build every right environment."""
        N = self.N
        for k in range(N - 1, 0, -1):
            Dl, _, _, Dr = self.A[k].shape
            Lm, Q = self._lq(k)
            self.A[k] = Q.reshape(Q.shape[0], 4, 4, Dr)
            self.A[k - 1] = np.tensordot(self.A[k - 1], Lm, axes=([3], [0]))
        nrm = np.linalg.norm(self.A[0])
        self.A[0] /= nrm
        self.lam += np.log(nrm)
        self.centre = 0
        self.Lenv[0] = np.ones((1, 1, 1))
        self.Renv[N] = np.ones((1, 1, 1))
        for k in range(N - 1, 0, -1):
            self.Renv[k] = env_right(self.Renv[k + 1], self.A[k], self.W[k])

    def _normalise(self, X):
        nrm = np.linalg.norm(X)
        self.lam += np.log(nrm)
        return X / nrm

    def _site_exp(self, k, t, K, tol):
        L, R, W = self.Lenv[k], self.Renv[k + 1], self.W[k]
        out, info = lanczos_expm(lambda x: heff1(L, W, R, x), self.A[k], t, K, tol)
        self.max_krylov_err = max(self.max_krylov_err, info["err"])
        self.A[k] = self._normalise(out)

    def _bond_exp(self, k, S, t, K, tol):
        L, R = self.Lenv[k], self.Renv[k]
        out, info = lanczos_expm(lambda x: heff0(L, R, x), S, t, K, tol)
        self.max_krylov_err = max(self.max_krylov_err, info["err"])
        return self._normalise(out)

    def sweep(self, dbeta, K=8, tol=1e-13):
        """One symmetric 1-TDVP step beta -> beta + dbeta (SM Sec. II.F)."""
        assert self.centre == 0
        N, tau = self.N, 0.5 * dbeta
        for k in range(N - 1):                      # left to right
            self._site_exp(k, -tau, K, tol)
            Dl, _, _, Dr = self.A[k].shape
            Q, S = self._qr(k)
            self.A[k] = Q.reshape(Dl, 4, 4, Q.shape[1])
            self.Lenv[k + 1] = env_left(self.Lenv[k], self.A[k], self.W[k])
            S = self._bond_exp(k + 1, S, +tau, K, tol)
            self.A[k + 1] = np.tensordot(S, self.A[k + 1], axes=([1], [0]))
        self._site_exp(N - 1, -2.0 * tau, K, tol)   # merged turn
        for k in range(N - 1, 0, -1):               # right to left
            Dl, _, _, Dr = self.A[k].shape
            Lm, Q = self._lq(k)
            self.A[k] = Q.reshape(Q.shape[0], 4, 4, Dr)
            self.Renv[k] = env_right(self.Renv[k + 1], self.A[k], self.W[k])
            Lm = self._bond_exp(k, Lm, +tau, K, tol)
            self.A[k - 1] = np.tensordot(self.A[k - 1], Lm, axes=([3], [0]))
            self._site_exp(k - 1, -tau, K, tol)
        self.beta += dbeta

    # ------------------------------------------------------------ 2-TDVP
    def _pair_exp(self, k, t, K, tol):
        """C = A_k A_{k+1} <- exp(t H^(2)) C (normalised into Lambda)."""
        C = np.tensordot(self.A[k], self.A[k + 1], axes=([3], [0]))     # x so1 si1 so2 si2 y
        L, R = self.Lenv[k], self.Renv[k + 2]
        W1, W2 = self.W[k], self.W[k + 1]
        out, info = lanczos_expm(lambda x: heff2(L, W1, W2, R, x), C, t, K, tol)
        self.max_krylov_err = max(self.max_krylov_err, info["err"])
        return self._normalise(out)

    @staticmethod
    def _split(C, D_max, cutoff, left_orth):
        """SVD of C reshaped (D_k 16) x (16 D_{k+2}), truncated to the largest
        singular values: at most D_max of them, each above cutoff x the
        largest.  left_orth: (U, S V^+), else (U S, V^+)."""
        Dl, Dr = C.shape[0], C.shape[5]
        U, s, Vh = np.linalg.svd(C.reshape(Dl * 16, 16 * Dr), full_matrices=False)
        r = int(np.sum(s > cutoff * s[0])) if cutoff > 0 else len(s)
        r = max(1, min(r, D_max))
        U, s, Vh = U[:, :r], s[:r], Vh[:r]
        if left_orth:
            return U.reshape(Dl, 4, 4, r), (s[:, None] * Vh).reshape(r, 4, 4, Dr)
        return (U * s).reshape(Dl, 4, 4, r), Vh.reshape(r, 4, 4, Dr)

    def sweep2(self, dbeta, D_max, cutoff=0.0, K=8, tol=1e-13):
        """One symmetric 2-TDVP step beta -> beta + dbeta (SM Sec. "2-TDVP in
        the initial stage", Eq. S-2TDVP): left to right over the pairs
        (k, k+1), C_k <- exp(-tau H^(2)) C_k, an SVD split that grows or
        truncates the bond (at most D_max states, each above cutoff x the
        largest singular value), then the backward one-site step
        A_{k+1} <- exp(+tau H^(1)) A_{k+1}; the two exponentials of the last
        pair merged into one with 2 tau; right to left mirrored.  Bond
        dimensions change: the state carries no charge layouts here."""
        assert self.centre == 0 and self.layouts is None
        N, tau = self.N, 0.5 * dbeta
        for k in range(N - 2):                       # left to right
            C = self._pair_exp(k, -tau, K, tol)
            self.A[k], self.A[k + 1] = self._split(C, D_max, cutoff, True)
            self.Lenv[k + 1] = env_left(self.Lenv[k], self.A[k], self.W[k])
            self._site_exp(k + 1, +tau, K, tol)
        for k in range(N - 2, -1, -1):               # right to left, merged turn first
            C = self._pair_exp(k, -2.0 * tau if k == N - 2 else -tau, K, tol)
            self.A[k], self.A[k + 1] = self._split(C, D_max, cutoff, False)
            self.Renv[k + 1] = env_right(self.Renv[k + 2], self.A[k + 1], self.W[k + 1])
            if k > 0:
                self._site_exp(k, +tau, K, tol)
        self.beta += dbeta

    # ------------------------------------------------------------ observables
    def energy(self):
        """<<rho|H (x) 1|rho>>/<<rho|rho>> from the normalised centre (site 0)."""
        k = self.centre
        A = self.A[k]
        HA = heff1(self.Lenv[k], self.W[k], self.Renv[k + 1], A)
        return float(np.vdot(A, HA)) / float(np.vdot(A, A))

    def expectation(self, Ws):
        """<<rho|O (x) 1|rho>> / <<rho|rho>> for an operator O given as an MPO
        (boundary bonds of dimension 1), e.g. a sum of on-site operators:
        right environments of O down to bond 1, then O^(1) at the centre."""
        assert self.centre == 0
        R = np.ones((1, 1, 1))
        for k in range(self.N - 1, 0, -1):
            R = env_right(R, self.A[k], Ws[k])
        A = self.A[0]
        OA = heff1(np.ones((1, 1, 1)), Ws[0], R, A)
        return float(np.vdot(A, OA)) / float(np.vdot(A, A))

    def super_expectation(self, Ws):
        """<<rho|X|rho>> / <<rho|rho>> for a super-operator X given as an MPO
        with 16 x 16 local matrices W[a, s_out, s_in, b] (s = 4 sigma +
        sigma', boundary bonds of dimension 1) that may act on the ancilla
        index too: the site tensors are read as A[x, s, y] and the same right
        environments and centre apply are taken with s in place of sigma."""
        assert self.centre == 0
        R = np.ones((1, 1, 1))
        for k in range(self.N - 1, 0, -1):
            A = self.A[k].reshape(self.A[k].shape[0], 16, self.A[k].shape[3])
            T1 = np.tensordot(A, R, axes=([2], [2]))                      # x si y' b
            T2 = np.tensordot(T1, Ws[k], axes=([1, 3], [2, 3]))            # x y' a so
            R = np.tensordot(A.conj(), T2, axes=([1, 2], [3, 1])).transpose(0, 2, 1)
        A = self.A[0].reshape(self.A[0].shape[0], 16, self.A[0].shape[3])
        T1 = np.tensordot(np.ones((1, 1, 1)), A, axes=([2], [0]))         # x a si be
        T2 = np.tensordot(T1, Ws[0], axes=([1, 2], [0, 2]))                # x be so b
        XA = np.tensordot(T2, R, axes=([1, 3], [2, 1]))                     # x so y
        return float(np.vdot(A, XA)) / float(np.vdot(A, A))

    def ln_trace(self):
        """ln Tr rho(beta): contract every site with delta(sigma, sigma')."""
        v = np.ones(1)
        for a in self.A:
            v = v @ np.einsum("xssy->xy", a)
        return self.lam + np.log(v[0])

    def swap_overlap(self):
        """<<rho|P|rho>> / <<rho|rho>> with P the exchange of sigma and sigma'
        on every site (P|rho>> = |rho^T>>, the Choi map of SM Sec. II.A), by
        transfer matrices E'[y, y'] = sum E[x, x'] A[x, s, s', y] A[x', s', s, y']."""
        E = np.ones((1, 1))
        N2 = np.ones((1, 1))
        for a in self.A:
            T = np.tensordot(E, a, axes=([0], [0]))                  # x' so sp y
            E = np.tensordot(T, a, axes=([0, 1, 2], [0, 2, 1]))      # y y'
            T = np.tensordot(N2, a, axes=([0], [0]))
            N2 = np.tensordot(T, a, axes=([0, 1, 2], [0, 1, 2]))
        return float(E[0, 0]) / float(N2[0, 0])

    def herm_defect(self):
        """||rho - rho^T||_F / ||rho||_F = sqrt(2 - 2 <<rho|P|rho>>/<<rho|rho>>)
        (rho real: rho^T = rho^dagger); zero for the exact state."""
        return float(np.sqrt(max(0.0, 2.0 - 2.0 * self.swap_overlap())))

    def observables(self):
        """Bilayer values at the physical inverse temperature 2*beta."""
        N = self.N
        lnZ = 2.0 * self.lam
        bp = 2.0 * self.beta
        E = self.energy()
        return dict(beta=self.beta, beta_phys=bp, lnZ=lnZ, f=-lnZ / (N * bp),
                    E=E, e=E / N, lnZ_single=self.ln_trace())


# ---------------------------------------------------------------- start state
def initial_state(mpo_model, beta0, D, symmetric, pad_eps=0.0, seed=0, sector_cap=0, taylor_order=1, mode="u1u1"):
    """rho0 = 1 - beta0 H (main text, noninteracting-benchmark paragraph), or
    for taylor_order > 1 the SETTN start sum_{n <= order} (-beta0 H)^n / n!
    (SM I.E, ``oracle.mpo.settn_rho0``), padded to bond D as described in
    ``oracle.charges``, right-canonicalised, centre normalised into Lambda;
    beta = beta0."""
    from . import charges
    from . import mpo as _mpo
    N = mpo_model.N
    if taylor_order == 1:
        A0 = mpo_model.rho0_tensors(beta0)
        rho0_q = [mpo_model.bond_charges(k) for k in range(N)]
    else:
        A0, rho0_q = _mpo.settn_rho0(mpo_model, beta0, taylor_order)
        rho0_q = list(rho0_q)
    rho0_q.append([(0, 0)])            # bond N of rho0 after the boundary vector
    layouts = charges.bond_layouts(rho0_q, N, D, symmetric, sector_cap, mode)
    A = charges.padded_rho0(A0, layouts, symmetric, pad_eps, seed, mode)
    st = State(A, mpo_model.mpo_for_env(), beta0)
    if symmetric:
        st.layouts = layouts
        st.mode = mode
    st.canonicalise()
    return st
