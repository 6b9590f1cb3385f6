"""Block adaptive cross approximation, Algorithm 2, with 3x3 entries (oracle only).

Paper reference: Sec. 3.2. An admissible block G (c x q entries, each a 3x3
matrix) is approximated by a sum of rank-one cross terms G ~ C Q =
sum_k c_k q_k^T (Eq. (8)). At step k the column c_k is the residual column
j_k; the row pivot i_k maximises the entry magnitude over rows not yet used;
c_k is right-multiplied by the inverse of its pivot entry; q_k^T is the
residual row i_k; the next column pivot j_{k+1} maximises the magnitude of
q_k over columns not yet used (Eq. (9)). With nu = ||c_k q_k^T||_F and
lambda = ||C Q||_F the iteration stops when nu <= zeta lambda (Eq. (10)),
lambda^2 being updated incrementally (Algorithm 2).

Readings where the paper is silent or inconsistent (listed in the design notes):
  * entry magnitude for pivoting: the squared Frobenius norm of the 3x3 entry
    as Algorithm 2 writes it (pivot="frobenius", the default); the text around
    Eq. (9) instead calls |.| the determinant, which is available as
    pivot="determinant" (|det| of the entry). The determinant rule never picks
    a nearly singular 3x3 pivot, which keeps c_k = a P^-1 bounded; the
    single-precision forms use it. The stopping guards use Frobenius norms
    under both rules;
  * the initial column is j_1 = floor(q/2) (the paper draws it at random);
  * argmax ties go to the lowest local index;
  * the stopping test is nu^2 <= zeta^2 lambda^2, taken after the term is
    appended (Algorithm 2 order);
  * nu^2 and lambda^2 are exact block Frobenius norms through 3x3 Gram
    matrices: with A_mk = sum_i c_m(i)^T c_k(i) and B_km = sum_j q_k(j) q_m(j)^T,
    nu^2 = tr(A_kk B_kk) and <c_m q_m^T, c_k q_k^T>_F = tr(A_mk B_km);
  * the rank is capped at l_max; a block that reaches l_max without passing the
    test is evaluated densely instead (a counted fallback). Reaching
    min(c, q) terms interpolates every row or column and counts as converged;
  * guards: a residual column whose largest entry has ||a||^2 <= 1e-30 lambda^2
    ends the iteration as converged without a new term; a pivot entry with
    |det P| <= s ||P||_F^3 ends it with a dense fallback, s = 1e-14 under the
    Frobenius rule (a singularity guard only: Algorithm 2 screens pivots by
    size, not by conditioning) and s = 1e-8 under the determinant rule. For a
    3x3 matrix |det P| = s1 s2 s3 <= s1^2 s3, so the 2-norm condition number
    obeys s1 / s3 <= ||P||_F^3 / |det P|. The determinant rule takes the best
    conditioned entry of the column it can find; when even that one has a
    condition number above 1e8 the column holds no usable pivot, and inverting
    it would carry FP64 rounding into c_k = a P^-1 beyond 1e-8 relative. On
    the 6N grid, whose coupling entries are singular, such pivots follow a
    step that grew the residual 1e4-fold, and the block's result then depends
    on the rounding of the inverse at the 1e-6 level.
"""
from __future__ import annotations

import numpy as np

TINY = 1e-30
SING = 1e-14       # Frobenius rule
SING_DET = 1e-8    # determinant rule


class ACAResult:
    def __init__(self, C, Q, piv_i, piv_j, converged, nu2, lam2):
        self.C = C            # [l, c, 3, 3]
        self.Q = Q            # [l, q, 3, 3]
        self.piv_i = piv_i    # [l] local row pivots
        self.piv_j = piv_j    # [l] local column pivots (j_1 .. j_l)
        self.converged = converged
        self.nu2 = nu2        # per step
        self.lam2 = lam2      # per step (after the update)

    @property
    def rank(self):
        return len(self.piv_i)


def aca_block(kern, Xt, Xs, eps: float, l_max: int, piv_j1: int | None = None,
              pivot: str = "frobenius") -> ACAResult:
    """Algorithm 2 on the block G(i, j) = K(Xt[i] - Xs[j])."""
    Xt = np.asarray(Xt, dtype=np.float64)
    Xs = np.asarray(Xs, dtype=np.float64)
    return aca_entries(lambda j: kern(Xt - Xs[j]), lambda i: kern(Xt[i] - Xs),
                       Xt.shape[0], Xs.shape[0], eps, l_max, piv_j1, pivot)


def _magnitude(E, pivot):
    if pivot == "frobenius":
        return np.sum(E * E, axis=(1, 2))
    return np.abs(np.linalg.det(E))


def aca_entries(col, row, c: int, q: int, eps: float, l_max: int,
                piv_j1: int | None = None, pivot: str = "frobenius") -> ACAResult:
    """Algorithm 2 on a c x q block given by col(j) -> [c,3,3], row(i) -> [q,3,3]."""
    assert pivot in ("frobenius", "determinant")
    Cs, Qs, I, J, nus, lams = [], [], [], [], [], []
    used_i = np.zeros(c, dtype=bool)
    used_j = np.zeros(q, dtype=bool)
    lam2 = 0.0
    j = q // 2 if piv_j1 is None else int(piv_j1)
    kmax = min(c, q, l_max)
    converged = False
    for k in range(kmax):
        used_j[j] = True
        # residual column j_k
        a = np.array(col(j), dtype=np.float64)             # [c, 3, 3]
        for m in range(k):
            a = a - Cs[m] @ Qs[m][j]
        # row pivot
        nrm = np.sum(a * a, axis=(1, 2))
        if np.max(np.where(used_i, -1.0, nrm)) <= TINY * lam2:
            converged = True
            break
        ik = int(np.argmax(np.where(used_i, -1.0, _magnitude(a, pivot))))
        P = a[ik]
        fro = np.sqrt(np.sum(P * P))
        if abs(np.linalg.det(P)) <= (SING_DET if pivot == "determinant" else SING) * fro ** 3:
            break
        # normalise by the pivot entry
        ck = a @ np.linalg.inv(P)
        # residual row i_k
        b = np.array(row(ik), dtype=np.float64)            # [q, 3, 3]
        for m in range(k):
            b = b - Cs[m][ik] @ Qs[m]
        qk = b
        used_i[ik] = True
        # next column pivot
        nq = np.where(used_j, -1.0, _magnitude(qk, pivot))
        jn = int(np.argmax(nq))
        # nu^2 and lambda^2 via 3x3 Gram matrices
        Akk = np.einsum("iab,iac->bc", ck, ck)
        Bkk = np.einsum("jab,jcb->ac", qk, qk)
        nu2 = float(np.trace(Akk @ Bkk))
        cross = 0.0
        for m in range(k):
            Amk = np.einsum("iab,iac->bc", Cs[m], ck)     # sum_i c_m(i)^T c_k(i)
            Bkm = np.einsum("jab,jcb->ac", qk, Qs[m])     # sum_j q_k(j) q_m(j)^T
            cross += float(np.trace(Amk @ Bkm))
        lam2 = lam2 + nu2 + 2.0 * cross
        # append the term
        Cs.append(ck)
        Qs.append(qk)
        I.append(ik)
        J.append(j)
        nus.append(nu2)
        lams.append(lam2)
        # stopping test
        if nu2 <= eps * eps * lam2:
            converged = True
            break
        if k + 1 == min(c, q):
            converged = True
            break
        j = jn
    C = np.asarray(Cs).reshape(-1, c, 3, 3)
    Q = np.asarray(Qs).reshape(-1, q, 3, 3)
    return ACAResult(C, Q, np.asarray(I, dtype=np.int64), np.asarray(J, dtype=np.int64),
                     converged, np.asarray(nus), np.asarray(lams))


def lowrank_apply(res: ACAResult, Fs):
    """C (Q F): t_k = sum_j q_k(j) F_j, then u_i = sum_k c_k(i) t_k (Sec. 3, the
    low-rank product applied right to left)."""
    Fs = np.asarray(Fs, dtype=np.float64)
    if res.rank == 0:
        return np.zeros((res.C.shape[1], 3))
    t = np.einsum("kjab,jb->ka", res.Q, Fs)
    return np.einsum("kiab,kb->ia", res.C, t)


def lowrank_dense(res: ACAResult):
    """The materialised approximation C Q as [c, q, 3, 3]."""
    return np.einsum("kiab,kjbc->ijac", res.C, res.Q)
