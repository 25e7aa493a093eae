"""GPU tests of the solve phase (sec. 5.2, sec. 6) through the C ABI against
the oracle in oracle/solve.py: one Braess-Sarazin step on given operators,
the V-cycle on the same operators and on the oracle's own hierarchy, GMRES
iteration counts, and the iteration trend on the Stokes cavities of
Table 1."""
import numpy as np
import pytest

from oracle import oracle as O
from oracle import solve as S
from paper_1607_02489_amd import synth
from paper_1607_02489_amd.synth import CSR
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _csr(t):
    return CSR(t[0], t[1], t[2], t[3], t[4])


def _gpu_levels(sys_, hier):
    """Oracle LevelOps on the GPU hierarchy's own operators and transfers."""
    Ls, A, B = [], sys_.Ahat, sys_.Bdiv
    for l in range(hier.ntransfers()):
        c = hier.level_csr(l)
        Ls.append(S.LevelOps(sys_.dim, A, B, _csr(c["Pv"]), _csr(c["Pp"])))
        A, B = _csr(c["Ac"]), _csr(c["Bc"])
    Ls.append(S.LevelOps(sys_.dim, A, B))
    return Ls


def _setup(n, jitter=0.0, seed=0, nlevels=6, min_dofs=205, iters=1):
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, n, jitter=jitter, seed=seed)
    d = E.DeviceSystem.upload(s)
    h = E.NativeHierarchy(d, E.params(iters=iters), nlevels, min_dofs=min_dofs)
    torch.cuda.synchronize()
    sv = E.Solver(d, h)
    return s, d, h, sv


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()


def test_bs_step_matches_oracle_on_every_level():
    """One Braess-Sarazin step (D = row sums of |A|, explicit Schur
    complement, five Gauss-Seidel sweeps, omega = 0.666) from a random x with
    a random f, on every level of a 2-D jittered cavity hierarchy, equals the
    oracle's step on the same operators to 1e-12."""
    import torch
    s, d, h, sv = _setup(24, jitter=0.1, seed=4, min_dofs=100)
    Ls = _gpu_levels(s, h)
    rng = np.random.default_rng(0)
    for l, L in enumerate(Ls):
        n, glev = sv.info(l)
        assert n == L.n
        x0, f = rng.standard_normal(L.n), rng.standard_normal(L.n)
        x = _t(x0)
        sv.bs_step(l, x, _t(f))
        torch.cuda.synchronize()
        want = S.BraessSarazin(L).step(x0, f)
        err = np.abs(x.cpu().numpy() - want).max() / np.abs(want).max()
        say(f"[gpu] BS step level {l}: n={L.n}, GS levels {glev}, err {err:.2e}")
        assert err <= 1e-12
    sv.close()
    h.close()


def test_vcycle_matches_oracle():
    """The V-cycle (BS(2,2), 10 BS steps on the coarsest level) on the GPU's
    hierarchy equals the oracle's V-cycle on the same operators to 1e-11, and
    the oracle's V-cycle on its own hierarchy (P and RAP within 1e-10) to
    1e-8."""
    import torch
    s, d, h, sv = _setup(32, jitter=0.1, seed=5)
    Ls = _gpu_levels(s, h)
    sm = [S.BraessSarazin(L) for L in Ls]
    rng = np.random.default_rng(1)
    f = rng.standard_normal(Ls[0].n)
    x = torch.zeros(Ls[0].n, dtype=torch.float64, device="cuda")
    sv.vcycle(_t(f), x)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    want = S.vcycle(Ls, sm, f, nu=2, coarse_steps=10)
    e1 = np.abs(got - want).max() / np.abs(want).max()
    Lo = S.levels_from_oracle(s, O.hierarchy(s, 6, iters=1, min_dofs=205))
    assert [L.n for L in Lo] == [L.n for L in Ls]
    want2 = S.vcycle(Lo, [S.BraessSarazin(L) for L in Lo], f, nu=2, coarse_steps=10)
    e2 = np.abs(got - want2).max() / np.abs(want2).max()
    say(f"[gpu] V-cycle: levels {[L.n for L in Ls]}, vs same operators {e1:.2e}, vs oracle "
        f"hierarchy {e2:.2e}")
    assert e1 <= 1e-11 and e2 <= 1e-8
    sv.close()
    h.close()


@pytest.mark.parametrize("n", [16, 32])
def test_gmres_iterations_match_oracle(n):
    """GMRES preconditioned by the V-cycle to 1e-6 (sec. 6) on a cavity with
    a consistent right-hand side f = K x*: the GPU takes the oracle's number
    of iterations (within one) and its solution meets the tolerance."""
    import torch
    s, d, h, sv = _setup(n)
    Lo = S.levels_from_oracle(s, O.hierarchy(s, 6, iters=1, min_dofs=205))
    rng = np.random.default_rng(n)
    f = Lo[0].apply(rng.standard_normal(Lo[0].n))
    x = torch.zeros(Lo[0].n, dtype=torch.float64, device="cuda")
    its, rel = sv.gmres(_t(f), x, rtol=1e-6, maxit=100)
    torch.cuda.synchronize()
    sm = [S.BraessSarazin(L) for L in Lo]
    _, oits, _ = S.gmres(Lo[0].apply, lambda v: S.vcycle(Lo, sm, v, nu=2, coarse_steps=10), f,
                         rtol=1e-6, maxit=100)
    res = np.linalg.norm(f - Lo[0].apply(x.cpu().numpy())) / np.linalg.norm(f)
    say(f"[gpu] GMRES {n}x{n}: gpu {its} its (estimate {rel:.2e}, true {res:.2e}), oracle {oits}")
    assert abs(its - oits) <= 1 and res <= 1.01e-6
    sv.close()
    h.close()


def test_table1_iteration_trend():
    """Stokes cavities of Table 1 (659 to 37,507 dofs; one EMIN step, tau1 =
    0.06, BS(2,2), levels until the coarsest has fewer than 205 dofs): the
    number of levels is Table 1's l_max or one more (tests/golden/
    table1_dofs.json), and the GMRES iteration count grows slowly with the
    mesh (at most twice the smallest mesh's, at most 40).  The paper's counts
    are for its lid-driven right-hand side; here f = K x* for a random x*."""
    import json
    import pathlib
    import torch
    g = json.loads((pathlib.Path(__file__).parent / "golden" / "table1_dofs.json").read_text())
    counts = {}
    for n in (8, 16, 32, 64):
        s, d, h, sv = _setup(n)
        nlev = h.ntransfers() + 1
        rng = np.random.default_rng(7)
        f = _t(S.LevelOps(2, s.Ahat, s.Bdiv).apply(rng.standard_normal(s.dofs)))
        x = torch.zeros_like(f)
        its, rel = sv.gmres(f, x, rtol=1e-6, maxit=100)
        counts[n] = its
        lm = g["elements_per_side_to_l_max"][str(n)]
        say(f"[gpu] Table 1 cavity {n}x{n} ({s.dofs} dofs): {nlev} levels (paper {lm}), {its} "
            f"GMRES its (paper {g['elements_per_side_to_bs_iterations'][str(n)]})")
        assert nlev in (lm, lm + 1)
        sv.close()
        h.close()
    assert max(counts.values()) <= 40 and counts[64] <= 2 * counts[8]
