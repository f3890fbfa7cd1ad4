"""Block-sparse form of the one-site TDVP sweep (oracle; TEST INFRASTRUCTURE
ONLY: nothing in the product imports, links or calls it).

The same method as ``oracle.tdvp`` (SM Sec. II.F steps 1-7, the splitting of
SM Sec. II.E, the Lanczos exponential of SM Sec. II.H, the contraction order
L.A, then W, then R of SM Fig. Lanczos, the bilayer observables of SM
Sec. II.A), with every tensor stored by U(1)charge x U(1)spin blocks so that
the workload's bond dimensions (D = 2000 and more) fit in memory and time.

Symmetric tensors as block-shifted matrices.  A charge q = (n_up, n_dn)
labels every bond sector.  With s = 4 sigma + sigma' and
Delta(s) = q(sigma) - q(sigma'):
* the site tensor A[x, s, y] is 16 matrices A^s[x, y], each non-zero only
  between a left sector q and the right sector q + Delta(s): one dense block
  per (q, s);
* a left environment L[x', a, x] is one matrix L^a[x', x] per MPO state a,
  non-zero only for q(x') = q(x) + qH(a); a right environment R[y', b, y] is
  R^b[y', y] with q(y') = q(y) + qH(b) (bra index first, MPO state charge
  qH; both follow from the MPO conserving qH(b) = qH(a) + q(sigma_o) -
  q(sigma_i));
* a bond matrix S is block diagonal.
Each contraction of ``oracle.tdvp`` becomes, per MPO state and super index,
a product of such matrices, done one charge block at a time with a plain
matmul; sums over MPO states and super indices are taken in the order the
dense contraction states them.  Nothing is fused or reordered beyond that:
    H^(1) A:  T1^{a,s} = L^a A^s;
              T2^{b,(so,sp)} = sum_{a,si} W[a,so,si,b] T1^{a,(si,sp)};
              out^{s} = sum_b T2^{b,s} (R^b)^T,
    H^(0) S:  out = sum_a (L^a S) (R^a)^T,
    L_{k+1}^b = sum_s (A^s)^T T2^{b,s}            (T2 of L_k and A_k),
    R_k^a     = sum_s A^s (Y2^{a,s})^T, with Y1^{b,s} = A^s (R^b)^T and
                Y2^{a,(so,sp)} = sum_{b,si} W[a,so,si,b] Y1^{b,(si,sp)}.
QR (left-to-right) stacks, for every right sector q, the blocks A^s of all
(left sector, s) that end in q, and factors that stack; LQ (right-to-left)
concatenates, for every left sector, the blocks A^s that start there.  With
a non-negative triangular diagonal both factorisations are unique, and the
order in which blocks are stacked only permutes the rows of Q, so they equal
the dense oracle's blockwise QR.

The vectors of a Lanczos exponential are the blocks laid end to end (one
flat float64 array), handed to ``oracle.tdvp.lanczos_expm`` unchanged.

The start (rho0 = 1 - beta0 H from the MPO of ``oracle.mpo``, the sector
dimensions and the seeded padding of ``oracle.charges``) is built blockwise,
entry for entry the tensor ``oracle.tdvp.initial_state`` builds densely, and
canonicalised the same way.  Block structure "u1u1" only (both charges).
"""
import numpy as np

from . import charges as _ch
from . import tdvp as _td

S_CHARGES = _ch.S_CHARGES
# the super indices with sigma = sigma' (the single-layer trace)
DIAG_S = (0, 5, 10, 15)


def qadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def qsub(a, b):
    return (a[0] - b[0], a[1] - b[1])


class Bond:
    """Sectors of one bond: charge -> (offset in the dense index order, dim).
    The dense order is sectors sorted by charge (``oracle.charges``)."""

    def __init__(self, layout):
        self.layout = layout
        self.sec = {}
        pos = 0
        for q in sorted(set(layout.charges)):
            d = sum(1 for c in layout.charges if c == q)
            self.sec[q] = (pos, d)
            pos += d
        self.dim = pos
        assert [q for q in sorted(self.sec) for _ in range(self.sec[q][1])] == list(layout.charges)

    def d(self, q):
        return self.sec[q][1]

    def off(self, q):
        return self.sec[q][0]


class SiteLayout:
    """Blocks (q, s) of a site tensor between bonds bl and br, laid end to end
    in the order q (sorted), then s."""

    def __init__(self, bl, br):
        self.blocks = []        # (q, s, qr, dl, dr, offset)
        pos = 0
        for q in sorted(bl.sec):
            for s in range(16):
                qr = qadd(q, S_CHARGES[s])
                if qr not in br.sec:
                    continue
                dl, dr = bl.d(q), br.d(qr)
                self.blocks.append((q, s, qr, dl, dr, pos))
                pos += dl * dr
        self.size = pos
        self.index = {(b[0], b[1]): i for i, b in enumerate(self.blocks)}

    def views(self, v):
        """{s: {q: block}} of a flat vector (views, no copies)."""
        out = {s: {} for s in range(16)}
        for (q, s, qr, dl, dr, off) in self.blocks:
            out[s][q] = v[off:off + dl * dr].reshape(dl, dr)
        return out

    def flatten(self, A):
        """Flat vector of a {s: {q: block}} tensor (absent blocks are zero)."""
        v = np.zeros(self.size)
        for (q, s, qr, dl, dr, off) in self.blocks:
            b = A[s].get(q)
            if b is not None:
                v[off:off + dl * dr] = b.reshape(-1)
        return v


# ---------------------------------------------------------------- contractions
def _w_terms(W):
    """Non-zero entries of an MPO tensor W[a, so, si, b], grouped by (b, so):
    {(b, so): [(a, si, w), ...]} in increasing (a, si)."""
    terms = {}
    DHl, _, _, DHr = W.shape
    for b in range(DHr):
        for so in range(4):
            lst = [(a, si, float(W[a, so, si, b])) for a in range(DHl) for si in range(4)
                   if W[a, so, si, b] != 0.0]
            if lst:
                terms[(b, so)] = lst
    return terms


def _w_terms_right(W):
    """The same entries grouped by (a, so) for the right environment:
    {(a, so): [(b, si, w), ...]} in increasing (b, si)."""
    terms = {}
    DHl, _, _, DHr = W.shape
    for a in range(DHl):
        for so in range(4):
            lst = [(b, si, float(W[a, so, si, b])) for b in range(DHr) for si in range(4)
                   if W[a, so, si, b] != 0.0]
            if lst:
                terms[(a, so)] = lst
    return terms


def _l_times_a(L, qHl, A):
    """T1^{a,s} = L^a A^s (SM Fig. Lanczos, first contraction), blocks keyed
    by the bra sector q' of L."""
    T1 = {}
    for a, La in enumerate(L):
        for s in range(16):
            As = A[s]
            blk = {}
            for qp, Lb in La.items():
                q = qsub(qp, qHl[a])             # ket sector of L^a's block
                Ab = As.get(q)
                if Ab is not None:
                    blk[qp] = Lb @ Ab
            if blk:
                T1[(a, s)] = blk
    return T1


def _w_stage(T1, terms):
    """T2^{b,(so,sp)} = sum_{a,si} W[a,so,si,b] T1^{a,(si,sp)}."""
    T2 = {}
    for (b, so), lst in terms.items():
        for sp in range(4):
            acc = {}
            for (a, si, w) in lst:
                src = T1.get((a, 4 * si + sp))
                if src is None:
                    continue
                for qp, blk in src.items():
                    if qp in acc:
                        acc[qp] = acc[qp] + w * blk
                    else:
                        acc[qp] = w * blk
            if acc:
                T2[(b, 4 * so + sp)] = acc
    return T2


def heff1(L, qHl, W, R, qHr, A):
    """H^(1) A in blocks: out^s = sum_b T2^{b,s} (R^b)^T (contraction order of
    SM Fig. Lanczos: L.A, then W, then R).  A: {s: {q: block}}; returns the
    same structure (blocks keyed by the left sector q)."""
    T1 = _l_times_a(L, qHl, A)
    T2 = _w_stage(T1, _w_terms(W))
    out = {s: {} for s in range(16)}
    for (b, s), blk in T2.items():
        Rb = R[b]
        o = out[s]
        for q, X in blk.items():
            # X: rows in the left sector q, columns in the ket sector
            # qy = q + Delta(s) - qH(b) of R^b; R^b's block of bra sector
            # q + Delta(s) maps to that ket sector
            qr = qadd(q, S_CHARGES[s])
            Rblk = Rb.get(qr)
            if Rblk is None:
                continue
            y = X @ Rblk.T
            if q in o:
                o[q] = o[q] + y
            else:
                o[q] = y
    return out


def heff0(L, R, qH, S):
    """H^(0) S = sum_a (L^a S) (R^a)^T on one bond (SM Fig. optimalB(d)); S
    and the result are block diagonal {q: block}."""
    out = {}
    for a, La in enumerate(L):
        Ra = R[a]
        for qp, Lb in La.items():
            q = qsub(qp, qH[a])
            Sb = S.get(q)
            Rb = Ra.get(qp)
            if Sb is None or Rb is None:
                continue
            y = (Lb @ Sb) @ Rb.T
            if qp in out:
                out[qp] = out[qp] + y
            else:
                out[qp] = y
    return out


def env_left(L, qHl, A, W, DHr):
    """L_{k+1}^b = sum_s (A^s)^T T2^{b,s}, T2 the W stage of L_k A_k."""
    T1 = _l_times_a(L, qHl, A)
    T2 = _w_stage(T1, _w_terms(W))
    Ln = [dict() for _ in range(DHr)]
    for (b, s), blk in T2.items():
        for q, X in blk.items():
            Ab = A[s].get(q)
            if Ab is None:
                continue
            qy = qadd(q, S_CHARGES[s])          # bra sector y' of the new environment
            y = Ab.T @ X
            if qy in Ln[b]:
                Ln[b][qy] = Ln[b][qy] + y
            else:
                Ln[b][qy] = y
    return Ln


def env_right(R, qHr, A, W, qHl):
    """R_k^a = sum_s A^s (Y2^{a,s})^T with Y1^{b,s} = A^s (R^b)^T and
    Y2^{a,(so,sp)} = sum_{b,si} W[a,so,si,b] Y1^{b,(si,sp)} (the order of
    ``oracle.tdvp.env_right``: A.R, then W, then conj(A)).  qHr: charges of
    the MPO states of R_{k+1}; qHl: those of the new environment."""
    Y1 = {}
    for b, Rb in enumerate(R):
        for s in range(16):
            blk = {}
            for q, Ab in A[s].items():
                qr = qadd(q, S_CHARGES[s])       # right sector of A^s's block = ket sector of R^b
                Rblk = Rb.get(qadd(qr, qHr[b]))  # R^b's block of that ket sector (keyed by bra)
                if Rblk is not None:
                    blk[q] = Ab @ Rblk.T
            if blk:
                Y1[(b, s)] = blk
    Y2 = {}
    for (a, so), lst in _w_terms_right(W).items():
        for sp in range(4):
            acc = {}
            for (b, si, w) in lst:
                src = Y1.get((b, 4 * si + sp))
                if src is None:
                    continue
                for q, blk in src.items():
                    if q in acc:
                        acc[q] = acc[q] + w * blk
                    else:
                        acc[q] = w * blk
            if acc:
                Y2[(a, 4 * so + sp)] = acc
    Rn = [dict() for _ in range(len(qHl))]
    for (a, s), blk in Y2.items():
        for q, X in blk.items():
            # X: rows x in the ket sector q, columns y'; A^s's block of bra
            # sector q' = q + qH(a) shares those columns
            qp = qadd(q, qHl[a])
            Ab = A[s].get(qp)
            if Ab is None:
                continue
            y = Ab @ X.T
            if qp in Rn[a]:
                Rn[a][qp] = Rn[a][qp] + y
            else:
                Rn[a][qp] = y
    return Rn


# ---------------------------------------------------------------- gauge moves
def qr_site(A, br):
    """A reshaped (D_l 16) x D_r = Q S per right sector (SM Sec. II.F step 2):
    for every right sector q, the blocks A^s of all (left sector, s) ending
    in q are stacked and factored with a non-negative diagonal.  Returns
    (Q as {s: {q: block}}, S as {q: block})."""
    Q = {s: {} for s in range(16)}
    S = {}
    for qr in sorted(br.sec):
        parts = [(s, q) for s in range(16) for q in A[s] if qadd(q, S_CHARGES[s]) == qr]
        if not parts:
            raise ValueError("right sector without rows")
        M = np.vstack([A[s][q] for (s, q) in parts])
        if M.shape[0] < M.shape[1]:
            raise ValueError("sector with more columns than rows")
        Qm, Rm = _td.qr_pos(M)
        r = 0
        for (s, q) in parts:
            n = A[s][q].shape[0]
            Q[s][q] = Qm[r:r + n]
            r += n
        S[qr] = Rm
    return Q, S


def lq_site(A, bl):
    """A reshaped D_l x (16 D_r) = L Q per left sector (right-to-left move):
    for every left sector q the blocks A^s starting there are concatenated
    and factored with a non-negative diagonal.  Returns (L as {q: block},
    Q as {s: {q: block}})."""
    Q = {s: {} for s in range(16)}
    Lm = {}
    for q in sorted(bl.sec):
        parts = [s for s in range(16) if q in A[s]]
        if not parts:
            raise ValueError("left sector without columns")
        M = np.hstack([A[s][q] for s in parts])
        if M.shape[1] < M.shape[0]:
            raise ValueError("sector with more rows than columns")
        Lq, Qm = _td.lq_pos(M)
        c = 0
        for s in parts:
            n = A[s][q].shape[1]
            Q[s][q] = Qm[:, c:c + n]
            c += n
        Lm[q] = Lq
    return Lm, Q


def absorb_left(S, A):
    """S A^s for a block-diagonal S on the left bond."""
    return {s: {q: S[q] @ blk for q, blk in A[s].items()} for s in range(16)}


def absorb_right(A, S):
    """A^s S for a block-diagonal S on the right bond."""
    return {s: {q: blk @ S[qadd(q, S_CHARGES[s])] for q, blk in A[s].items()} for s in range(16)}


def _bond_flat(bond):
    """Layout of a block-diagonal bond matrix laid end to end: [(q, d, off)]."""
    out, pos = [], 0
    for q in sorted(bond.sec):
        d = bond.d(q)
        out.append((q, d, pos))
        pos += d * d
    return out, pos


# ---------------------------------------------------------------- the state
class BlockState:
    """e^Lambda times a mixed-canonical block-sparse super-MPS (centre at 0
    between sweeps), with the environments of ``oracle.tdvp.State``."""

    def __init__(self, bonds, A, Ws, qH, beta, lam=0.0):
        self.N = len(A)
        self.bonds = bonds                    # Bond per bond 0..N
        self.A = A                            # {s: {q: block}} per site
        self.W = Ws                           # MPO tensors with 1-dim boundary bonds
        self.qH = qH                          # MPO state charges per bond 0..N
        self.beta = float(beta)
        self.lam = float(lam)
        self.layout = [SiteLayout(bonds[k], bonds[k + 1]) for k in range(self.N)]
        self.Lenv = [None] * (self.N + 1)
        self.Renv = [None] * (self.N + 1)
        self.max_krylov_err = 0.0
        self.centre = None

    # ------------------------------------------------------------ pieces
    def _normalise_flat(self, v):
        nrm = np.linalg.norm(v)
        self.lam += np.log(nrm)
        return v / nrm

    def _site_exp(self, k, t, K, tol):
        lay = self.layout[k]
        L, R, W = self.Lenv[k], self.Renv[k + 1], self.W[k]
        qHl, qHr = self.qH[k], self.qH[k + 1]

        def apply(x):
            return lay.flatten(heff1(L, qHl, W, R, qHr, lay.views(x)))

        out, info = _td.lanczos_expm(apply, lay.flatten(self.A[k]), t, K, tol)
        self.max_krylov_err = max(self.max_krylov_err, info["err"])
        self.A[k] = lay.views(self._normalise_flat(out))

    def _bond_exp(self, k, S, t, K, tol):
        lay, size = _bond_flat(self.bonds[k])
        L, R, qH = self.Lenv[k], self.Renv[k], self.qH[k]

        def views(v):
            return {q: v[off:off + d * d].reshape(d, d) for (q, d, off) in lay}

        def flatten(X):
            v = np.zeros(size)
            for (q, d, off) in lay:
                if q in X:
                    v[off:off + d * d] = X[q].reshape(-1)
            return v

        out, info = _td.lanczos_expm(lambda x: flatten(heff0(L, R, qH, views(x))), flatten(S), t, K, tol)
        self.max_krylov_err = max(self.max_krylov_err, info["err"])
        return views(self._normalise_flat(out))

    def _env_left(self, k):
        self.Lenv[k + 1] = env_left(self.Lenv[k], self.qH[k], self.A[k], self.W[k], len(self.qH[k + 1]))

    def _env_right(self, k):
        self.Renv[k] = env_right(self.Renv[k + 1], self.qH[k + 1], self.A[k], self.W[k], self.qH[k])

    def canonicalise(self):
        """Right-canonicalise by LQ from site N-1 down to 1, centre at site 0,
        normalise the centre into Lambda, build every right environment (the
        steps of ``oracle.tdvp.State.canonicalise``)."""
        N = self.N
        for k in range(N - 1, 0, -1):
            Lm, Q = lq_site(self.A[k], self.bonds[k])
            self.A[k] = Q
            self.A[k - 1] = absorb_right(self.A[k - 1], Lm)
        v = self.layout[0].flatten(self.A[0])
        self.A[0] = self.layout[0].views(self._normalise_flat(v))
        self.centre = 0
        self.Lenv[0] = [{(0, 0): np.ones((1, 1))}]
        self.Renv[N] = [{(0, 0): np.ones((1, 1))}]
        for k in range(N - 1, 0, -1):
            self._env_right(k)

    def sweep(self, dbeta, K=8, tol=1e-13):
        """One symmetric 1-TDVP step beta -> beta + dbeta (SM Sec. II.F), the
        step sequence of ``oracle.tdvp.State.sweep``."""
        assert self.centre == 0
        N, tau = self.N, 0.5 * dbeta
        for k in range(N - 1):                      # left to right
            self.site_step_lr(k, tau, K, tol)
        self._site_exp(N - 1, -2.0 * tau, K, tol)   # merged turn
        for k in range(N - 1, 0, -1):               # right to left
            Lm, Q = lq_site(self.A[k], self.bonds[k])
            self.A[k] = Q
            self._env_right(k)
            Lm = self._bond_exp(k, Lm, +tau, K, tol)
            self.A[k - 1] = absorb_right(self.A[k - 1], Lm)
            self._site_exp(k - 1, -tau, K, tol)
        self.beta += dbeta

    def site_step_lr(self, k, tau, K=8, tol=1e-13):
        """The left-to-right step at site k < N-1: site exponential, QR, left
        environment, backward bond exponential, absorb into site k+1."""
        self._site_exp(k, -tau, K, tol)
        Q, S = qr_site(self.A[k], self.bonds[k + 1])
        self.A[k] = Q
        self._env_left(k)
        S = self._bond_exp(k + 1, S, +tau, K, tol)
        self.A[k + 1] = absorb_left(S, self.A[k + 1])

    # ------------------------------------------------------------ observables
    def energy(self):
        """<<rho|H (x) 1|rho>> / <<rho|rho>> from the normalised centre (site 0)."""
        lay = self.layout[0]
        A = self.A[0]
        HA = heff1(self.Lenv[0], self.qH[0], self.W[0], self.Renv[1], self.qH[1], A)
        v, hv = lay.flatten(A), lay.flatten(HA)
        return float(np.dot(v, hv)) / float(np.dot(v, v))

    def ln_trace(self):
        """ln Tr rho(beta): transfer matrices with delta(sigma, sigma') (the
        super indices with Delta = 0 keep the sector)."""
        v = {(0, 0): np.ones((1, 1))}
        for A in self.A:
            nv = {}
            for s in DIAG_S:
                for q, blk in A[s].items():
                    if q not in v:
                        continue
                    y = v[q] @ blk
                    nv[q] = nv[q] + y if q in nv else y
            v = nv
        return self.lam + np.log(v[(0, 0)][0, 0])

    def swap_overlap(self):
        """<<rho|P|rho>> / <<rho|rho>> (``oracle.tdvp.State.swap_overlap``) in
        blocks: P maps s = 4 sigma + sigma' to 4 sigma' + sigma and negates its
        charge, so the transfer matrix E pairs a left sector q with -q:
        E'[q + Delta(s)] = sum_{s, q} (A^s[q])^T E[q] A^{P(s)}[-q]."""
        neg = lambda q: (-q[0], -q[1])
        E = {(0, 0): np.ones((1, 1))}
        N2 = {(0, 0): np.ones((1, 1))}
        for A in self.A:
            nE, nN = {}, {}
            for s in range(16):
                ps = 4 * (s % 4) + s // 4
                for q, blk in A[s].items():
                    qy = qadd(q, S_CHARGES[s])
                    if q in E and neg(q) in A[ps]:
                        y = blk.T @ E[q] @ A[ps][neg(q)]
                        nE[qy] = nE[qy] + y if qy in nE else y
                    if q in N2:
                        y = blk.T @ N2[q] @ blk
                        nN[qy] = nN[qy] + y if qy in nN else y
            E, N2 = nE, nN
        return float(E[(0, 0)][0, 0]) / float(N2[(0, 0)][0, 0])

    def herm_defect(self):
        """||rho - rho^T||_F / ||rho||_F = sqrt(2 - 2 <<rho|P|rho>>/<<rho|rho>>)."""
        return float(np.sqrt(max(0.0, 2.0 - 2.0 * self.swap_overlap())))

    def observables(self):
        """Bilayer values at the physical inverse temperature 2*beta (the
        definitions of ``oracle.tdvp.State.observables``)."""
        N = self.N
        lnZ = 2.0 * self.lam
        bp = 2.0 * self.beta
        E = self.energy()
        return dict(beta=self.beta, beta_phys=bp, lnZ=lnZ, f=-lnZ / (N * bp),
                    E=E, e=E / N, lnZ_single=self.ln_trace())

    def to_dense(self, k):
        """Site tensor k as a dense [D_k, 4, 4, D_{k+1}] array (sectors in the
        dense index order of ``oracle.charges``)."""
        bl, br = self.bonds[k], self.bonds[k + 1]
        out = np.zeros((bl.dim, 16, br.dim))
        for s in range(16):
            for q, blk in self.A[k][s].items():
                qr = qadd(q, S_CHARGES[s])
                out[bl.off(q):bl.off(q) + blk.shape[0], s, br.off(qr):br.off(qr) + blk.shape[1]] = blk
        return out.reshape(bl.dim, 4, 4, br.dim)


# ---------------------------------------------------------------- start state
def initial_state(mpo_model, beta0, D, pad_eps=0.0, seed=0, sector_cap=0):
    """rho0 = 1 - beta0 H padded to bond D with U(1)xU(1) sectors, entry for
    entry the tensors of ``oracle.tdvp.initial_state(..., symmetric=True)``
    built blockwise: the rho0 states of each sector first, padding entries
    (charge-allowed, left or right index a padding state) set to pad_eps
    (2u - 1) with u the SplitMix64 draw of ``oracle.charges.noise_uniform``
    at flat = (x 16 + s) D_{k+1} + y; then right-canonicalised with the
    centre normalised into Lambda."""
    N = mpo_model.N
    A0 = mpo_model.rho0_tensors(beta0)
    rho0_q = [mpo_model.bond_charges(k) for k in range(N)] + [[(0, 0)]]
    layouts = _ch.bond_layouts(rho0_q, N, D, True, sector_cap, "u1u1")
    bonds = [Bond(lay) for lay in layouts]
    A = []
    for k in range(N):
        bl, br = bonds[k], bonds[k + 1]
        Ll, Lr = layouts[k], layouts[k + 1]
        Dr = br.dim
        a16 = A0[k].reshape(A0[k].shape[0], 16, A0[k].shape[3])
        site = {s: {} for s in range(16)}
        for q in sorted(bl.sec):
            for s in range(16):
                qr = qadd(q, S_CHARGES[s])
                if qr not in br.sec:
                    continue
                x = np.arange(bl.off(q), bl.off(q) + bl.d(q))
                y = np.arange(br.off(qr), br.off(qr) + br.d(qr))
                blk = np.zeros((len(x), len(y)))
                if pad_eps != 0.0:
                    X, Y = np.meshgrid(x, y, indexing="ij")
                    mask = Ll.is_pad[X] | Lr.is_pad[Y]
                    flat = (X * 16 + s) * Dr + Y
                    blk[mask] = pad_eps * _ch.noise_uniform(seed, k, flat[mask])
                site[s][q] = blk
        # rho0 entries (left and right rho0 states, never padding)
        for i, xi in enumerate(Ll.rho0_index):
            q = Ll.charges[xi]
            for s in range(16):
                qr = qadd(q, S_CHARGES[s])
                if qr not in br.sec:
                    continue
                for j, yj in enumerate(Lr.rho0_index):
                    v = a16[i, s, j]
                    if v == 0.0:
                        continue
                    if Lr.charges[yj] != qr:
                        raise ValueError("rho0 breaks charge conservation")
                    site[s][q][xi - bl.off(q), yj - br.off(qr)] = v
        A.append(site)
    Ws = mpo_model.mpo_for_env()
    qH = [mpo_model.bond_charges(k) for k in range(N)] + [[(0, 0)]]
    st = BlockState(bonds, A, Ws, qH, beta0)
    st.canonicalise()
    return st
