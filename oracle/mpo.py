"""Finite-state-machine MPO of the Hubbard Hamiltonian and the super-MPS of
rho0 = 1 - beta0*H (oracle; test infrastructure only).

Paper: Eq. (3); the MPO of H with a small bond D_H is only cited (main text,
noninteracting-benchmark paragraph); the Choi map of SM Sec. II.A turns an MPO
tensor W[a, sigma, sigma', b] into a super-MPS tensor with the combined index
s = (sigma, sigma').

Fermion signs (Jordan-Wigner along the snake, mode order up before down):
c_{i,s} = (prod_{j<i} P_j) c^loc_{i,s} with the site parity P = (-1)^{n}, so
for i < j
    c+_{i s} c_{j s} = (c+_s P)_i  (prod_{i<k<j} P_k)  (c_s)_j
    c+_{j s} c_{i s} = (P c_s)_i   (prod_{i<k<j} P_k)  (c+_s)_j .

Bond states (a convention shared by every builder of this MPO, so that a
padded rho0 is the same tensor everywhere).  With ks = N // 2:
    bond 0: [start];  bond N: [start, done];
    bond k, 0 < k <= ks (source-indexed):
        [start] + [src(i, type) for i in pending_src(k) ascending, type] + [done]
    bond k, ks < k < N (destination-indexed):
        [start] + [dst(j, type) for j in pending_dst(k) ascending, type] + [done]
type runs over (c+_up P, c+_dn P, P c_up, P c_dn); pending_src(k) = sites
i < k with a neighbour j >= k, pending_dst(k) = sites j >= k with a
neighbour i < k.  A source channel carries the left operator of site i and
propagates with P; a destination channel carries the sum over sources i of
-t times their left operators and is closed at j by the right operator.  The
switch site ks maps src(i) to dst(j) with -t P for each neighbour j > ks of
i.  Indexing by source on the left half and by destination on the right half
keeps every bond inside the maximal charge sectors near both chain ends (a
source-indexed right edge is not minimal on 2D lattices).
W[a, so, si, b] acts as the operator sum_{so,si} |so><si| on the ket.
"""
import numpy as np

from . import lattice

# local basis {0, up, down, updown}, |updown> = c+_up c+_dn |0>
CDAG_UP = np.zeros((4, 4)); CDAG_UP[1, 0] = 1.0; CDAG_UP[3, 2] = 1.0
CDAG_DN = np.zeros((4, 4)); CDAG_DN[2, 0] = 1.0; CDAG_DN[3, 1] = -1.0
C_UP = CDAG_UP.T.copy()
C_DN = CDAG_DN.T.copy()
PAR = np.diag([1.0, -1.0, -1.0, 1.0])
N_UP = np.diag([0.0, 1.0, 0.0, 1.0])
N_DN = np.diag([0.0, 0.0, 1.0, 1.0])
ID4 = np.eye(4)

# channel types: (left operator at the source site, right operator at the partner)
CHANNELS = (
    (CDAG_UP @ PAR, C_UP),
    (CDAG_DN @ PAR, C_DN),
    (PAR @ C_UP, CDAG_UP),
    (PAR @ C_DN, CDAG_DN),
)
# pairing-field channels (main text, d-wave pairing paragraph): for i < j,
# a_i b_j = (a P)_i (prod P) b_j; the four terms of
# c_i,dn c_j,up - c_i,up c_j,dn - c+_i,dn c+_j,up + c+_i,up c+_j,dn
PAIR_CHANNELS = (
    (C_DN @ PAR, C_UP, 1.0),
    (C_UP @ PAR, C_DN, -1.0),
    (CDAG_DN @ PAR, CDAG_UP, -1.0),
    (CDAG_UP @ PAR, CDAG_DN, 1.0),
)
# U(1)xU(1) charge carried by a channel: q(b) = q(a) + q(so) - q(si)
CHANNEL_CHARGE = ((1, 0), (0, 1), (-1, 0), (0, -1), (0, -1), (-1, 0), (0, 1), (1, 0))


def channel_ops(ty):
    """(left operator, right operator, sign) of channel type ty: 0..3 hopping
    (sign 1, amplitude -t), 4..7 pairing (amplitude -hp s_ij / (2 sqrt 2))."""
    if ty < 4:
        return CHANNELS[ty][0], CHANNELS[ty][1], 1.0
    return PAIR_CHANNELS[ty - 4]


def local_charge(sigma):
    """(n_up, n_dn) of a local basis state."""
    return (sigma & 1, sigma >> 1)


class HubbardMPO:
    """W tensors of Eq. (3) with the bond-state convention above."""

    def __init__(self, W, L, geometry, t=1.0, U=8.0, mu=0.0, tp=0.0, hp=0.0):
        self.N = N = W * L
        self.t, self.U, self.mu, self.tp, self.hp = float(t), float(U), float(mu), float(tp), float(hp)
        # hopping amplitude per coupled pair (i < j): t on bonds, tp on the
        # diagonal neighbours of SM Eq. S1 when tp != 0
        self.amp = {b: self.t for b in lattice.nn_bonds(W, L, geometry)}
        if self.tp != 0.0:
            self.amp.update({b: self.tp for b in lattice.nnn_bonds(W, L, geometry)})
        # pairing field -hp Delta_tot on the bonds (d-wave form factor s_ij)
        self.ntypes = 8 if self.hp != 0.0 else 4
        self.pamp = {}
        if self.hp != 0.0:
            order = lattice.snake_order(W, L)
            for (i, j) in lattice.nn_bonds(W, L, geometry):
                s = 1.0 if order[i][0] != order[j][0] else -1.0
                self.pamp[(i, j)] = -self.hp * s / (2.0 * np.sqrt(2.0))
        self.partners = [set() for _ in range(N)]
        for (i, j) in list(self.amp) + list(self.pamp):
            self.partners[i].add(j)
        # bond states: list of labels per bond k = 0..N
        self.ks = ks = N // 2
        self.states = []
        for k in range(N + 1):
            if k == 0:
                self.states.append(["start"])
                continue
            if k == N:
                self.states.append(["start", "done"])
                continue
            lab = ["start"]
            if k <= ks:
                pend = [i for i in range(k) if any(j >= k for j in self.partners[i])]
                lab += [("src", i, ty) for i in pend for ty in range(self.ntypes)]
            else:
                pend = [j for j in range(k, N) if any(i < k for i in self.neighbours(j))]
                lab += [("dst", j, ty) for j in pend for ty in range(self.ntypes)]
            lab.append("done")
            self.states.append(lab)
        self.W = [self._site(k) for k in range(N)]

    def neighbours(self, j):
        return [i for i in range(self.N) if j in self.partners[i] or i in self.partners[j]]

    def charge(self, label):
        if label in ("start", "done"):
            return (0, 0)
        return CHANNEL_CHARGE[label[2]]

    def bond_charges(self, k):
        return [self.charge(lab) for lab in self.states[k]]

    def coef(self, i, j, ty):
        """Amplitude of channel type ty between i < j (times the channel's sign)."""
        if ty < 4:
            return -self.amp.get((i, j), 0.0)
        return self.pamp.get((i, j), 0.0) * PAIR_CHANNELS[ty - 4][2]

    def _site(self, k):
        left, right = self.states[k], self.states[k + 1]
        ri = {lab: n for n, lab in enumerate(right)}
        Wk = np.zeros((len(left), 4, 4, len(right)))
        onsite = self.U * (N_UP @ N_DN) - self.mu * (N_UP + N_DN)
        later = sorted(j for j in self.partners[k])          # neighbours j > k
        for a, lab in enumerate(left):
            if lab == "start":
                Wk[a, :, :, ri["start"]] += ID4
                if "done" in ri:
                    Wk[a, :, :, ri["done"]] += onsite
                for ty in range(self.ntypes):
                    left = channel_ops(ty)[0]
                    if ("src", k, ty) in ri:
                        Wk[a, :, :, ri[("src", k, ty)]] += left
                    for j in later:
                        if ("dst", j, ty) in ri:
                            Wk[a, :, :, ri[("dst", j, ty)]] += self.coef(k, j, ty) * left
            elif lab == "done":
                Wk[a, :, :, ri["done"]] += ID4
            elif lab[0] == "src":
                _, i, ty = lab
                if lab in ri:
                    Wk[a, :, :, ri[lab]] += PAR
                for j in sorted(self.partners[i]):
                    if j > k and ("dst", j, ty) in ri:
                        Wk[a, :, :, ri[("dst", j, ty)]] += self.coef(i, j, ty) * PAR
                if k in self.partners[i]:
                    Wk[a, :, :, ri["done"]] += self.coef(i, k, ty) * channel_ops(ty)[1]
            else:
                _, j, ty = lab
                if j == k:
                    Wk[a, :, :, ri["done"]] += channel_ops(ty)[1]
                else:
                    Wk[a, :, :, ri[lab]] += PAR
        return Wk

    def h_boundary_right(self):
        """Right boundary vector selecting 'done' (the MPO of H)."""
        return np.array([0.0, 1.0])

    def mpo_for_env(self):
        """W tensors with both boundary bonds of dimension 1 (for environments)."""
        Ws = [w.copy() for w in self.W]
        Ws[-1] = np.tensordot(Ws[-1], self.h_boundary_right(), axes=([3], [0]))[..., None]
        return Ws

    def rho0_tensors(self, beta0):
        """Super-MPS tensors A[a, so, si, b] of rho0 = 1 - beta0 H (Choi map)."""
        As = [w.copy() for w in self.W]
        r = np.array([1.0, -beta0])
        As[-1] = np.tensordot(As[-1], r, axes=([3], [0]))[..., None]
        return As


def local_sum_mpo(N, op_diag):
    """MPO of sum_i op_i for a diagonal on-site operator (entries on the basis
    {0, up, down, updown}): channels start (identity so far) and done (op
    placed), boundary bonds of dimension 1 (start on the left, done on the
    right)."""
    op = np.diag(np.asarray(op_diag, dtype=float))
    one = np.eye(4)
    W = np.zeros((2, 4, 4, 2))
    W[0, :, :, 0] = one
    W[0, :, :, 1] = op
    W[1, :, :, 1] = one
    Ws = [W.copy() for _ in range(N)]
    Ws[0] = Ws[0][:1]
    Ws[-1] = Ws[-1][..., 1:]
    return Ws


def mpo_to_dense(Ws):
    """Contract an MPO (boundary bonds of dimension 1) to a 4^N x 4^N matrix."""
    M = Ws[0][0]                      # (so, si, b)
    M = M.transpose(2, 0, 1)          # (b, so, si)
    for Wk in Ws[1:]:
        # M[b, O, I], Wk[b, so, si, c] -> M[c, (O so), (I si)]
        T = np.tensordot(M, Wk, axes=([0], [0]))       # (O, I, so, si, c)
        T = T.transpose(4, 0, 2, 1, 3)                  # (c, O, so, I, si)
        c, O, so, I, si = T.shape
        M = T.reshape(c, O * so, I * si)
    assert M.shape[0] == 1
    return M[0]


SZ = np.diag([0.0, 0.5, -0.5, 0.0])
SP = CDAG_UP @ C_DN          # S+ = c+_up c_dn on one site: |up><dn|
SM = SP.T.copy()
# spin channels: (left operator, right operator, coefficient); all bosonic
SPIN_CHANNELS = ((SZ, SZ, 1.0), (SP, SM, 0.5), (SM, SP, 0.5))


def spin_pair_mpo(N, pairs):
    """MPO of sum over pairs (i < j) of S_i . S_j (boundary bonds of dimension
    1): channels start, src(i, type) for every site i < k that has a partner
    j >= k (type over Sz, S+, S-), and done."""
    later = [sorted(j for (i2, j) in pairs if i2 == i) for i in range(N)]
    def states(k):
        st = [("start",)]
        for i in range(k):
            if later[i] and later[i][-1] >= k:
                st += [("src", i, ty) for ty in range(3)]
        return st + [("done",)]
    bonds = [states(k) for k in range(N + 1)]
    Ws = []
    for k in range(N):
        L, R = bonds[k], bonds[k + 1]
        col = {s: b for b, s in enumerate(R)}
        W = np.zeros((len(L), 4, 4, len(R)))
        for a, s in enumerate(L):
            if s[0] == "start":
                W[a, :, :, col[("start",)]] += ID4
                for ty, (lop, _, _) in enumerate(SPIN_CHANNELS):
                    if ("src", k, ty) in col:
                        W[a, :, :, col[("src", k, ty)]] += lop
            elif s[0] == "done":
                W[a, :, :, col[("done",)]] += ID4
            else:
                _, i, ty = s
                _, rop, cf = SPIN_CHANNELS[ty]
                if ("src", i, ty) in col:
                    W[a, :, :, col[("src", i, ty)]] += ID4
                if k in later[i]:
                    W[a, :, :, col[("done",)]] += cf * rop
        Ws.append(W)
    Ws[0] = Ws[0][:1]
    Ws[-1] = Ws[-1][..., -1:]
    return Ws


def green_mpo(W, L, k):
    """Super-operator MPO (tensors W[a, s_out, s_in, b], s = 4 sigma + sigma',
    16 x 16 local matrices, boundary bonds of dimension 1) of
        X(k) = sum_s sum_{r, r'} cos(k.(r - r')) c+_{r s} (x) (c_{r' s})^T ,
    so that <<rho|X|rho>> = sum_{r r'} cos(k.(r - r')) Tr[rho c+_r rho c_r']
    = N Tr[rho c+_k rho c_k] (main text, Fermi-surface paragraph; the Choi map
    of SM Sec. II.A sends A rho B to (A (x) B^T)|rho>>).

    With the Jordan-Wigner strings, c+_r = (prod_{q<r} P_q) CDAG_r and
    (c_r')^T = (prod_{q<r'} P_q) CDAG_r' (P diagonal, C^T = CDAG), so X is a
    sum of products of local (ket op) (x) (ancilla op).  cos(k.(r - r')) =
    cos(k.r) cos(k.r') + sin(k.r) sin(k.r') splits every pair into two
    separable terms.  Bond states: start (nothing placed yet: P (x) P),
    (ket, spin, cos|sin) (ket operator placed: 1 (x) P until the ancilla one),
    (anc, spin, cos|sin) (ancilla operator placed: P (x) 1), done (1 (x) 1);
    a site that holds both operators goes from start to done directly."""
    N = W * L
    ph = [k[0] * x + k[1] * y for (x, y) in lattice.snake_order(W, L)]
    mid = [("ket", sp, f) for sp in (0, 1) for f in (0, 1)] + [("anc", sp, f) for sp in (0, 1) for f in (0, 1)]
    bonds = [["start"]] + [["start"] + mid + ["done"] for _ in range(N - 1)] + [["done"]]
    cdag = (CDAG_UP, CDAG_DN)
    Ws = []
    for q in range(N):
        Lb, Rb = bonds[q], bonds[q + 1]
        col = {s: b for b, s in enumerate(Rb)}
        trig = (np.cos(ph[q]), np.sin(ph[q]))
        Wq = np.zeros((len(Lb), 16, 16, len(Rb)))

        def put(a, lab, ket, anc, c):
            if lab in col:
                Wq[a, :, :, col[lab]] += c * np.kron(ket, anc)

        for a, s in enumerate(Lb):
            if s == "start":
                put(a, "start", PAR, PAR, 1.0)
                for sp in (0, 1):
                    for f in (0, 1):
                        put(a, ("ket", sp, f), cdag[sp], PAR, trig[f])
                        put(a, ("anc", sp, f), PAR, cdag[sp], trig[f])
                    put(a, "done", cdag[sp], cdag[sp], 1.0)
            elif s == "done":
                put(a, "done", ID4, ID4, 1.0)
            else:
                side, sp, f = s
                if side == "ket":
                    put(a, s, ID4, PAR, 1.0)
                    put(a, "done", ID4, cdag[sp], trig[f])
                else:
                    put(a, s, PAR, ID4, 1.0)
                    put(a, "done", cdag[sp], ID4, trig[f])
        Ws.append(Wq)
    return Ws


SETTN_TOL = 1e-8      # a column is dependent if its residual is <= SETTN_TOL x its norm


def _mgs_keep(M, tol_rel):
    """Ordered modified Gram-Schmidt (two passes) over the columns of M:
    returns (Q, R) with M = Q R and Q's columns orthonormal.  A column whose
    residual norm is <= tol_rel x its own norm is a linear dependency: it is
    dropped and its coefficients go to R.  Columns are taken in their order,
    so the result is deterministic.  A residual within a factor 10 of the
    threshold raises (the decision would depend on rounding)."""
    m, n = M.shape
    Q = []
    R = np.zeros((n, n))
    for j in range(n):
        v = M[:, j].copy()
        n0 = np.linalg.norm(v)
        coef = np.zeros(len(Q))
        for _ in range(2):
            for i, q in enumerate(Q):
                c = q @ v
                coef[i] += c
                v -= c * q
        nv = np.linalg.norm(v)
        R[:len(Q), j] = coef
        if n0 == 0.0:
            continue
        if 0.1 * tol_rel * n0 < nv <= 10.0 * tol_rel * n0:
            raise ValueError("SETTN reduction: a residual is too close to the threshold")
        if nv > tol_rel * n0:
            Q.append(v / nv)
            R[len(Q) - 1, j] = nv
    r = len(Q)
    Qm = np.array(Q).T if r else np.zeros((m, 0))
    return Qm, R[:r, :]


def settn_rho0(model, beta0, order, tol_rel=SETTN_TOL):
    """SETTN start (SM I.E): super-MPS tensors of
        rho0 = sum_{n <= order} (-beta0 H)^n / n!
    and the charge of every bond state (bonds 0..N-1; bond N has one state of
    charge 0 after the boundary vector).

    H^order as the product MPO of ``order`` copies of H's MPO (bond states are
    tuples of H's states, charge the sum); at the right end every factor is in
    'start' (identity) or 'done' (H), so a tuple with k factors done stands for
    H^k, and the boundary vector puts (-beta0)^k / k! / C(order, k) on it.
    order = 1 is 1 - beta0 H.  The product bond is then reduced exactly (to
    linearly independent states): left to right, the columns of each site's
    left unfolding of one charge are orthonormalised by ordered modified
    Gram-Schmidt (dependent columns, residual <= tol_rel x their own norm,
    are dropped) and the coefficients move into the next site; then right to
    left over the rows of the right unfoldings.  A column counts as dependent
    when its residual is below SETTN_TOL of its norm: the reduction is exact
    up to directions of relative weight 1e-8 (in practice the dependent
    residuals are at rounding level and the kept ones far above); a decision
    inside the guard band raises instead of resting on rounding."""
    from math import comb, factorial
    N = model.N
    W = model.W
    charges = [model.bond_charges(k) for k in range(N + 1)]
    total = 0
    for k in range(N):
        dl, dr = len(charges[k]) ** order, len(charges[k + 1]) ** order
        total += dl * 16 * dr
        if dl > 8192 or dr > 8192 or dl * 16 * dr > 2 ** 26:
            raise ValueError("SETTN start: the product MPO is too large for this order")
    if total > 2 ** 28:
        raise ValueError("SETTN start: the product MPO is too large for this order")
    A, Q = [], []
    for k in range(N):
        P, qL, qR = W[k], list(charges[k]), list(charges[k + 1])
        for _ in range(order - 1):
            a, _, _, b = P.shape
            c, _, _, d = W[k].shape
            P = np.einsum("AotB,atib->AaoiBb", P, W[k]).reshape(a * c, 4, 4, b * d)
            qL = [(x[0] + y[0], x[1] + y[1]) for x in qL for y in charges[k]]
            qR = [(x[0] + y[0], x[1] + y[1]) for x in qR for y in charges[k + 1]]
        A.append(P)
        Q.append(qL)
        if k == N - 1:
            Q.append(qR)
    # boundary vector over the last bond's tuples of (start = 0, done = 1)
    nR = len(charges[N])
    r = np.zeros(nR ** order)
    for idx in range(nR ** order):
        digits = [(idx // nR ** (order - 1 - i)) % nR for i in range(order)]
        kdone = sum(digits)
        r[idx] = (-beta0) ** kdone / factorial(kdone) / comb(order, kdone)
    A[-1] = np.tensordot(A[-1], r, axes=([3], [0]))[..., None]
    Q[N] = [(0, 0)]
    if order == 1:
        return A, Q[:N]
    # exact reduction, left to right
    for k in range(N - 1):
        a, _, _, b = A[k].shape
        M = A[k].reshape(a * 16, b)
        cols, coefs, newq = [], [], []
        for q in sorted(set(Q[k + 1])):
            J = [j for j in range(b) if Q[k + 1][j] == q]
            Qm, R = _mgs_keep(M[:, J], tol_rel)
            if Qm.shape[1] == 0:
                continue
            cols.append(Qm)
            T = np.zeros((Qm.shape[1], b))
            T[:, J] = R
            coefs.append(T)
            newq += [q] * Qm.shape[1]
        A[k] = np.concatenate(cols, axis=1).reshape(a, 4, 4, -1)
        C = np.concatenate(coefs, axis=0)
        A[k + 1] = np.tensordot(C, A[k + 1], axes=([1], [0]))
        Q[k + 1] = newq
    # right to left over the rows
    for k in range(N - 1, 0, -1):
        a, _, _, b = A[k].shape
        M = A[k].reshape(a, 16 * b).T
        rows, coefs, newq = [], [], []
        for q in sorted(set(Q[k])):
            J = [j for j in range(a) if Q[k][j] == q]
            Qm, R = _mgs_keep(M[:, J], tol_rel)
            if Qm.shape[1] == 0:
                continue
            rows.append(Qm.T)
            T = np.zeros((Qm.shape[1], a))
            T[:, J] = R
            coefs.append(T)
            newq += [q] * Qm.shape[1]
        A[k] = np.concatenate(rows, axis=0).reshape(-1, 4, 4, b)
        C = np.concatenate(coefs, axis=0)           # A_old = C^T A_new
        A[k - 1] = np.tensordot(A[k - 1], C.T, axes=([3], [0]))
        Q[k] = newq
    return A, Q[:N]
