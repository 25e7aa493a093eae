"""Independent checkers used by the tests (no oracle or library code).

Graph distances come from scipy's csgraph BFS, dense products from numpy,
and the constrained energy minimum from a dense KKT solve.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse import csgraph

from paper_1607_02489_amd.synth import CSR


def graph_of(M: CSR) -> sp.csr_matrix:
    """Undirected unweighted graph of a matrix's off-diagonal structure."""
    A = sp.csr_matrix((np.ones(M.nnz), M.col, M.rowptr), shape=(M.nrows, M.ncols))
    A = A + A.T
    A.setdiag(0)
    A.eliminate_zeros()
    A.data[:] = 1.0
    return A


def hop_dist(G: sp.csr_matrix, sources, limit=None) -> np.ndarray:
    """Hop distances from each source (rows) to every vertex (inf if none)."""
    d = csgraph.shortest_path(G, method="D", unweighted=True, indices=np.asarray(sources))
    return np.atleast_2d(d)


def dense(m: CSR) -> np.ndarray:
    out = np.zeros((m.nrows, m.ncols))
    rows = np.repeat(np.arange(m.nrows), np.diff(m.rowptr))
    out[rows, m.col] = m.val if m.val is not None else 1.0
    return out


def kkt_emin(M: np.ndarray, N: CSR, cidx: np.ndarray, W: np.ndarray, Wc: np.ndarray):
    """Dense solve of min trace(P^T M P) s.t. P on pattern N, C rows fixed to
    injection, P Wc = W on the other rows.  Returns P's values on N."""
    n = N.nrows
    rows = np.repeat(np.arange(n), np.diff(N.rowptr))
    cols = N.col
    free = cidx[rows] < 0
    fixed_val = np.where(free, 0.0, 1.0)
    fi = np.nonzero(free)[0]
    nf = fi.size
    # energy sum_j P_j^T M P_j couples entries (i,j),(k,j) of the same column
    H = np.zeros((nf, nf))
    b = np.zeros(nf)
    bycol = {}
    for e in range(N.nnz):
        bycol.setdefault(cols[e], []).append(e)
    pos = -np.ones(N.nnz, dtype=np.int64)
    pos[fi] = np.arange(nf)
    for j, ents in bycol.items():
        for e in ents:
            for f in ents:
                mik = M[rows[e], rows[f]]
                if mik == 0.0:
                    continue
                if free[e] and free[f]:
                    H[pos[e], pos[f]] += mik
                elif free[e] and not free[f]:
                    b[pos[e]] += mik * fixed_val[f]
    frows = sorted(set(rows[fi].tolist()))
    Cm = np.zeros((len(frows), nf))
    w = np.zeros(len(frows))
    for r, i in enumerate(frows):
        for e in range(N.rowptr[i], N.rowptr[i + 1]):
            Cm[r, pos[e]] = Wc[cols[e]]
        w[r] = W[i]
    K = np.block([[2 * H, Cm.T], [Cm, np.zeros((len(frows), len(frows)))]])
    rhs = np.concatenate([-2 * b, w])
    sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
    vals = fixed_val.copy()
    vals[fi] = sol[:nf]
    return vals


def relfro(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def emin_quadratic(M: np.ndarray, N: CSR, cidx: np.ndarray, Wc: np.ndarray):
    """The EMIN problem of eq. (min_problem) as a quadratic over the vector of
    P's pattern entries: energy(p) = p^T H p with H[(i,j),(k,j)] = M[i,k]
    (entries of the same column couple through M), and the orthogonal
    projector Pi onto the feasible update directions: entries of C rows held
    at zero, and on every F row the component along w_i = W_c restricted to
    the row's pattern removed (so P W_c is unchanged)."""
    n = N.nrows
    rows = np.repeat(np.arange(n), np.diff(N.rowptr))
    cols = np.asarray(N.col)
    same_col = cols[:, None] == cols[None, :]
    H = np.where(same_col, M[rows][:, rows], 0.0)   # M need not be symmetric
    nnz = N.nnz
    Pi = np.eye(nnz)
    for i in range(n):
        a, b = int(N.rowptr[i]), int(N.rowptr[i + 1])
        if a == b:
            continue
        if cidx[i] >= 0:
            Pi[a:b, :] = 0.0
            Pi[:, a:b] = 0.0
            continue
        w = np.zeros(nnz)
        w[a:b] = Wc[cols[a:b]]
        ww = w @ w
        if ww > 0.0:
            Pi -= np.outer(w, w) / ww
    return H, Pi


def krylov_emin_iterate(M: np.ndarray, N: CSR, cidx: np.ndarray, W: np.ndarray, Wc: np.ndarray,
                        k: int) -> np.ndarray:
    """The k-th iterate of conjugate gradients on eq. (min_problem), by its
    characterisation rather than its recurrence: the minimiser of p^T H p over
    p0 + K_k(Pi H Pi, r0), where p0 is the row-normalised binary start (C rows
    by injection), r0 = -Pi H p0 the projected negative gradient, and K_k the
    Krylov space of dimension k (orthonormal basis by twice-repeated
    Gram-Schmidt).  Dense numpy; tiny problems only."""
    n = N.nrows
    rows = np.repeat(np.arange(n), np.diff(N.rowptr))
    cols = np.asarray(N.col)
    H, Pi = emin_quadratic(M, N, cidx, Wc)
    p0 = np.zeros(N.nnz)
    for i in range(n):
        a, b = int(N.rowptr[i]), int(N.rowptr[i + 1])
        if cidx[i] >= 0:
            p0[a:b] = 1.0
            continue
        g = float(np.sum(Wc[cols[a:b]] ** 2))
        if g > 0.0:
            p0[a:b] = W[i] * Wc[cols[a:b]] / g
    A = Pi @ H @ Pi
    r = -(Pi @ (H @ p0))
    basis = []
    v = r.copy()
    for _ in range(k):
        for _rep in range(2):
            for q in basis:
                v = v - (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= 1e-14 * max(np.linalg.norm(r), 1e-300):
            break
        q = v / nv
        basis.append(q)
        v = A @ q
    if not basis:
        return p0
    K = np.stack(basis, 1)
    y = np.linalg.solve(K.T @ H @ K, -(K.T @ (H @ p0)))
    del rows
    return p0 + K @ y


def gmres_krylov_iterate(K: np.ndarray, N: CSR, cidx: np.ndarray, W: np.ndarray, Wc: np.ndarray,
                         k: int) -> np.ndarray:
    """k-th iterate of GMRES on the constrained problem, by its
    characterisation: with Kmask the masked operator over P's pattern entries
    ((i,j),(l,j) -> K[i,l]) and Pi the projector of emin_quadratic, the
    minimiser of ||Pi Kmask p|| over p0 + K_k(Pi Kmask Pi, r0), r0 = -Pi Kmask
    p0 (dense least squares over an orthonormal Krylov basis)."""
    n = N.nrows
    rows = np.repeat(np.arange(n), np.diff(N.rowptr))
    cols = np.asarray(N.col)
    Km, Pi = emin_quadratic(K, N, cidx, Wc)   # Km = K restricted to same-column entries
    p0 = np.zeros(N.nnz)
    for i in range(n):
        a, b = int(N.rowptr[i]), int(N.rowptr[i + 1])
        if cidx[i] >= 0:
            p0[a:b] = 1.0
            continue
        g = float(np.sum(Wc[cols[a:b]] ** 2))
        if g > 0.0:
            p0[a:b] = W[i] * Wc[cols[a:b]] / g
    A = Pi @ Km
    r = -(A @ p0)
    basis = []
    v = r.copy()
    for _ in range(k):
        for _rep in range(2):
            for q in basis:
                v = v - (q @ v) * q
        nv = np.linalg.norm(v)
        if nv <= 1e-14 * max(np.linalg.norm(r), 1e-300):
            break
        q = v / nv
        basis.append(q)
        v = A @ (Pi @ q)
    if not basis:
        return p0
    Q = np.stack(basis, 1)
    y = np.linalg.lstsq(A @ Q, r, rcond=None)[0]
    del rows
    return p0 + Q @ y
