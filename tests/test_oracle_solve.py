"""Pins of the solve-phase oracle (oracle/solve.py) against the mathematics:
dense triangular and block solves, the Galerkin coarse operator, linearity of
the V-cycle, and GMRES's Krylov least-squares property.  CPU only."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import oracle as O
from oracle import solve as S
from paper_1607_02489_amd import synth


def _dense_K(L):
    d, nv = L.dim, L.nv
    A = L.A.toarray()
    B = L.B.toarray()
    K = np.zeros((L.n, L.n))
    for c in range(d):
        K[c * nv:(c + 1) * nv, c * nv:(c + 1) * nv] = A
    K[:d * nv, d * nv:] = B.T
    K[d * nv:, :d * nv] = B
    return K


def _dense_P(L):
    d, nv = L.dim, L.nv
    P, Pp = L.P.toarray(), L.Pp.toarray()
    nvc, npc = P.shape[1], Pp.shape[1]
    Pf = np.zeros((L.n, d * nvc + npc))
    for c in range(d):
        Pf[c * nv:(c + 1) * nv, c * nvc:(c + 1) * nvc] = P
    Pf[d * nv:, d * nvc:] = Pp
    return Pf


def _levels(n=16, jitter=0.1, seed=1, nlev=3, iters=1):
    s = synth.make_system(2, n, jitter=jitter, seed=seed)
    return s, S.levels_from_oracle(s, O.hierarchy(s, nlev, iters=iters))


def test_gauss_seidel_sweep_is_the_triangular_solve():
    """One forward sweep: x1 = (L + D)^-1 (b - U x0) with S = L + D + U."""
    rng = np.random.default_rng(0)
    _, Ls = _levels(8)
    bs = S.BraessSarazin(Ls[0])
    Sd = bs.S.toarray()
    b = rng.standard_normal(Sd.shape[0])
    x0 = rng.standard_normal(Sd.shape[0])
    x1 = S.gauss_seidel(bs.S, b, x0, 1)
    want = sla.solve_triangular(np.tril(Sd), b - np.triu(Sd, 1) @ x0, lower=True)
    assert np.abs(x1 - want).max() <= 1e-12 * np.abs(want).max()
    x2 = S.gauss_seidel(bs.S, b, x0, 2)
    want2 = sla.solve_triangular(np.tril(Sd), b - np.triu(Sd, 1) @ want, lower=True)
    assert np.abs(x2 - want2).max() <= 1e-12 * np.abs(want2).max()


def test_bs_step_with_exact_schur_solve_is_the_block_solve():
    """eq. (bs): with the Schur system solved to convergence, one step adds the
    solution of [D/omega, B^T; B, 0] delta = f - K x.  The system is singular
    (B^T 1 = 0 in the enclosed cavity); delta_u and B^T delta_p are unique."""
    rng = np.random.default_rng(1)
    _, Ls = _levels(4, nlev=1)
    L = Ls[0]
    bs = S.BraessSarazin(L, omega=0.666, gs_sweeps=3000)
    x = rng.standard_normal(L.n)
    f = rng.standard_normal(L.n)
    nu = L.dim * L.nv
    f[nu:] -= f[nu:].mean()                      # a consistent pressure residual
    x[nu:] -= x[nu:].mean()
    got = bs.step(x, f) - x
    K = _dense_K(L)
    M = K.copy()
    M[:nu, :nu] = np.diag(np.tile(S.bs_diagonal(L.A), L.dim) / 0.666)
    r = f - K @ x
    want = np.linalg.lstsq(M, r, rcond=None)[0]
    Bt = L.B.T.toarray()
    assert np.abs(got[:nu] - want[:nu]).max() <= 1e-9 * np.abs(want[:nu]).max()
    assert np.abs(Bt @ (got[nu:] - want[nu:])).max() <= 1e-9 * np.abs(Bt @ want[nu:]).max()


def test_galerkin_coarse_operator_and_two_grid_correction():
    """The coarse level's saddle-point operator is P^T K P with
    P = blockdiag(I_d (x) P_v, P_p) (R = P^T); with no smoothing and an exact
    coarse solve the V-cycle is the two-grid correction P K_c^+ P^T f."""
    rng = np.random.default_rng(2)
    _, Ls = _levels(8, nlev=2)
    K0, Kc = _dense_K(Ls[0]), _dense_K(Ls[1])
    Pf = _dense_P(Ls[0])
    assert np.abs(Kc - Pf.T @ K0 @ Pf).max() <= 1e-12 * np.abs(Kc).max()
    f = rng.standard_normal(Ls[0].n)
    sm = [S.BraessSarazin(L) for L in Ls]
    pinv = np.linalg.pinv(Kc)
    got = S.vcycle(Ls, sm, f, nu=0, coarse_solve=lambda fc: pinv @ fc)
    want = Pf @ (pinv @ (Pf.T @ f))
    assert np.abs(got - want).max() <= 1e-10 * np.abs(want).max()


def test_vcycle_is_linear():
    """A fixed number of steps from zero: the V-cycle is a linear map."""
    rng = np.random.default_rng(3)
    _, Ls = _levels(8, nlev=3)
    sm = [S.BraessSarazin(L) for L in Ls]
    f, g = rng.standard_normal(Ls[0].n), rng.standard_normal(Ls[0].n)
    a, b = 0.7, -1.3
    lhs = S.vcycle(Ls, sm, a * f + b * g, nu=2, coarse_steps=4)
    rhs = a * S.vcycle(Ls, sm, f, nu=2, coarse_steps=4) + b * S.vcycle(Ls, sm, g, nu=2,
                                                                        coarse_steps=4)
    assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(rhs).max()


def test_gmres_iterate_minimises_residual_over_krylov_space():
    """k steps of GMRES (identity preconditioner) give the x in
    K_k(A, f) = span(f, A f, ..., A^(k-1) f) minimising ||f - A x||; with the
    exact inverse as preconditioner one step solves the system."""
    rng = np.random.default_rng(4)
    n = 30
    A = np.eye(n) * 4 + rng.standard_normal((n, n))
    f = rng.standard_normal(n)
    for k in (1, 3, 7):
        x, its, _ = S.gmres(lambda v: A @ v, lambda v: v, f, rtol=0.0, maxit=k)
        Kb = np.column_stack([np.linalg.matrix_power(A, i) @ f for i in range(k)])
        Q, _ = np.linalg.qr(Kb)
        y = np.linalg.lstsq(A @ Q, f, rcond=None)[0]
        assert its == k
        assert np.abs(x - Q @ y).max() <= 1e-9 * np.abs(Q @ y).max()
    Ai = np.linalg.inv(A)
    x, its, _ = S.gmres(lambda v: A @ v, lambda v: Ai @ v, f, rtol=1e-10, maxit=5)
    assert its == 1 and np.abs(A @ x - f).max() <= 1e-10 * np.abs(f).max()


def test_vcycle_gmres_converges_on_a_small_cavity():
    """GMRES with the Braess-Sarazin V-cycle reaches 1e-6 on a 16x16 cavity
    (sec. 6.1's setting: BS(2,2), five Gauss-Seidel sweeps, omega = 0.666),
    and the true residual meets the tolerance."""
    rng = np.random.default_rng(5)
    s, Ls = _levels(16, nlev=3)
    sm = [S.BraessSarazin(L) for L in Ls]
    xs = rng.standard_normal(Ls[0].n)
    f = Ls[0].apply(xs)
    x, its, hist = S.gmres(Ls[0].apply, lambda v: S.vcycle(Ls, sm, v, nu=2, coarse_steps=10), f,
                           rtol=1e-6, maxit=60)
    assert its <= 40
    assert np.linalg.norm(f - Ls[0].apply(x)) <= 1.01e-6 * np.linalg.norm(f)
