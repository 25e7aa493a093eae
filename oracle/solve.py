"""Oracle of the solve phase: Braess-Sarazin relaxation, the multigrid
V-cycle it smooths, and GMRES preconditioned by that V-cycle (sec. 5.2,
eq. (bs); sec. 6: five Gauss-Seidel sweeps on the Schur complement,
relaxation parameter 0.666, GMRES to a relative residual of 1e-6).

Test infrastructure only: plain FP64 numpy/scipy, slow and direct, shared
with nothing on the GPU path.  Only tests/, the smoke check and bench.py's
CPU baseline use it.

A system on level l is the saddle-point operator
    [ I_d (x) A   B^T ]
    [ B           0   ]
on vectors x = (u, p), u component-blocked (d blocks of n_v), p of n_p.
"""
import numpy as np
import scipy.sparse as sp

from paper_1607_02489_amd.synth import CSR


def to_scipy(M: CSR) -> sp.csr_matrix:
    return sp.csr_matrix((M.val, M.col, M.rowptr), shape=(M.nrows, M.ncols))


class LevelOps:
    """Operators of one level: scalar velocity block A (n_v x n_v), divergence
    block B (n_p x d*n_v); P (n_v x n_vc) and Pp (n_p x n_pc) to the next
    coarser level (None on the coarsest)."""

    def __init__(self, dim, A: CSR, B: CSR, P: CSR = None, Pp: CSR = None):
        self.dim = dim
        self.A = to_scipy(A)
        self.B = to_scipy(B)
        self.P = to_scipy(P) if P is not None else None
        self.Pp = to_scipy(Pp) if Pp is not None else None
        self.nv = self.A.shape[0]
        self.np_ = self.B.shape[0]
        self.n = dim * self.nv + self.np_

    def apply(self, x):
        """y = [I (x) A, B^T; B, 0] x."""
        d, nv = self.dim, self.nv
        u, p = x[:d * nv], x[d * nv:]
        yu = np.concatenate([self.A @ u[c * nv:(c + 1) * nv] for c in range(d)]) + self.B.T @ p
        return np.concatenate([yu, self.B @ u])

    def restrict(self, r):
        """(P^T r_u per component, Pp^T r_p): R = P^T."""
        d, nv = self.dim, self.nv
        u, p = r[:d * nv], r[d * nv:]
        return np.concatenate([self.P.T @ u[c * nv:(c + 1) * nv] for c in range(d)]
                              + [self.Pp.T @ p])

    def prolong(self, xc):
        """(P u_c per component, Pp p_c)."""
        d = self.dim
        nvc = self.P.shape[1]
        u, p = xc[:d * nvc], xc[d * nvc:]
        return np.concatenate([self.P @ u[c * nvc:(c + 1) * nvc] for c in range(d)]
                              + [self.Pp @ p])


def bs_diagonal(A) -> np.ndarray:
    """sec. 5.2: D with d_ii = sum_j |a_ij| (the choice the paper found
    faster than diag(A))."""
    return np.asarray(abs(A).sum(axis=1)).ravel()


def safe_inverse(d) -> np.ndarray:
    """1 / d, and 0 where d = 0 (a velocity row with no entries, which the
    relaxation then leaves unchanged)."""
    out = np.zeros_like(d)
    nz = d != 0.0
    out[nz] = 1.0 / d[nz]
    return out


def schur(B, dinv_u) -> sp.csr_matrix:
    """sec. 5.2: the explicitly formed Schur complement S = B D^-1 B^T (D on
    every velocity component)."""
    return (B @ sp.diags(dinv_u) @ B.T).tocsr()


def gauss_seidel(S, b, x, sweeps: int):
    """Forward Gauss-Seidel in the natural order: each row i takes
    x_i = (b_i - sum_{j != i} s_ij x_j) / s_ii with the newest x_j."""
    x = np.array(x, dtype=np.float64, copy=True)
    rp, col, val = S.indptr, S.indices, S.data
    for _ in range(sweeps):
        for i in range(S.shape[0]):
            a, e = rp[i], rp[i + 1]
            s = b[i]
            dii = 0.0
            for t in range(a, e):
                j = col[t]
                if j == i:
                    dii = val[t]
                else:
                    s -= val[t] * x[j]
            x[i] = s / dii if dii != 0.0 else 0.0   # (a pressure with no coupling stays 0)
    return x


class BraessSarazin:
    """One level's Braess-Sarazin relaxation, eq. (bs):
        x <- x + [D/omega, B^T; B, 0]^-1 (f - K x).
    The block solve: r = f - K x; S dp = B D^-1 r_u - r_p / omega (S = B D^-1
    B^T, gs_sweeps Gauss-Seidel sweeps from dp = 0); du = omega D^-1 (r_u -
    B^T dp)."""

    def __init__(self, L: LevelOps, omega=0.666, gs_sweeps=5):
        self.L = L
        self.omega = omega
        self.sweeps = gs_sweeps
        self.dinv = safe_inverse(bs_diagonal(L.A))
        self.dinv_u = np.tile(self.dinv, L.dim)
        self.S = schur(L.B, self.dinv_u)

    def step(self, x, f):
        L, w = self.L, self.omega
        nu = L.dim * L.nv
        r = f - L.apply(x)
        ru, rpv = r[:nu], r[nu:]
        rhs = L.B @ (self.dinv_u * ru) - rpv / w
        dp = gauss_seidel(self.S, rhs, np.zeros(L.np_), self.sweeps)
        du = w * self.dinv_u * (ru - L.B.T @ dp)
        return x + np.concatenate([du, dp])


def vcycle(levels, smoothers, f, nu=2, coarse_steps=10, l=0, coarse_solve=None):
    """V-cycle from x = 0 on level l: nu Braess-Sarazin steps before and after
    the coarse correction x += P V_{l+1}(R (f - K x)); on the coarsest level
    coarse_steps Braess-Sarazin steps (or coarse_solve(f) when given)."""
    L = levels[l]
    x = np.zeros(L.n)
    if l == len(levels) - 1:
        if coarse_solve is not None:
            return coarse_solve(f)
        for _ in range(coarse_steps):
            x = smoothers[l].step(x, f)
        return x
    for _ in range(nu):
        x = smoothers[l].step(x, f)
    r = f - L.apply(x)
    xc = vcycle(levels, smoothers, L.restrict(r), nu, coarse_steps, l + 1, coarse_solve)
    x = x + L.prolong(xc)
    for _ in range(nu):
        x = smoothers[l].step(x, f)
    return x


def gmres(apply_A, apply_M, f, rtol=1e-6, maxit=200):
    """Right-preconditioned GMRES from x = 0 (no restart): Arnoldi by modified
    Gram-Schmidt on A M, Givens rotations on the Hessenberg matrix, stop when
    the residual norm is at most rtol ||f||; x = M (V y).  Returns (x,
    iterations, residual norms per iteration)."""
    n = f.shape[0]
    beta = np.linalg.norm(f)
    if beta == 0.0:
        return np.zeros(n), 0, [0.0]
    V = [f / beta]
    H = np.zeros((maxit + 1, maxit))
    cs, sn = np.zeros(maxit), np.zeros(maxit)
    g = np.zeros(maxit + 1)
    g[0] = beta
    hist = [beta]
    k = 0
    for j in range(maxit):
        w = apply_A(apply_M(V[j]))
        for i in range(j + 1):
            H[i, j] = np.dot(V[i], w)
            w = w - H[i, j] * V[i]
        H[j + 1, j] = np.linalg.norm(w)
        for i in range(j):
            a, b = H[i, j], H[i + 1, j]
            H[i, j] = cs[i] * a + sn[i] * b
            H[i + 1, j] = -sn[i] * a + cs[i] * b
        a, b = H[j, j], H[j + 1, j]
        r = np.hypot(a, b)
        cs[j], sn[j] = a / r, b / r
        H[j, j], H[j + 1, j] = r, 0.0
        g[j + 1] = -sn[j] * g[j]
        g[j] = cs[j] * g[j]
        k = j + 1
        hist.append(abs(g[j + 1]))
        if abs(g[j + 1]) <= rtol * beta or not (np.linalg.norm(w) > 0.0):
            break
        V.append(w / np.linalg.norm(w))
    y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
    z = np.zeros(n)
    for i in range(k):
        z += y[i] * V[i]
    return apply_M(z), k, hist


def levels_from_oracle(sys_, hier):
    """LevelOps of a hierarchy from oracle.hierarchy: level l's operators
    (level 0: the input system) and its transfers."""
    Ls, cur = [], sys_
    for lev in hier[0]:
        Ls.append(LevelOps(cur.dim, cur.Ahat, cur.Bdiv, lev.Pv, lev.Pp))
        cur = lev.coarse_system()
    Ls.append(LevelOps(cur.dim, cur.Ahat, cur.Bdiv))
    return Ls
