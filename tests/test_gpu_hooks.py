"""GPU tests of the two test-hook entry points and of the numeric phase's
failure reports, through the C ABI, against the oracle and closed forms.

emin_pattern_with_cpoints skips Alg. 3 (the coarse pressures are given), so
sec. 4.2's perfect-coarsening closed form runs on the device;
emin_setup_with_pattern runs EMIN (sec. 4.3) on a given operator and
pattern, so the 1-D linear-interpolation closed form and the INFEASIBLE and
BREAKDOWN reports run on the device.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import oracle as O
from paper_1607_02489_amd import synth
from paper_1607_02489_amd.synth import CSR
from tests.gpu_util import compare_level, gpu_level, say
from tests.helpers import dense, relfro

pytestmark = pytest.mark.gpu


def _t(a, dt):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)


@pytest.mark.parametrize("n", [16, 64])
def test_pattern_with_cpoints_perfect_coarsening(n):
    """sec. 4.2: with perfect distance-4 coarse pressures on a uniform mesh
    (the spacing-4 lattice) every target location is a pressure vertex, so
    C-bar is the spacing-2 lattice and the coarse level is Q2-Q1 on the 4h
    mesh, 2(n/2+1)^2 + (n/4+1)^2 dofs.  The whole level (S sets, C-bar, C^(v),
    patterns, P, RAP) also matches the oracle's level with the same given
    C^(p)."""
    import torch
    s = synth.make_system(2, n)
    m = n + 1
    ij = np.stack(np.meshgrid(np.arange(m), np.arange(m), indexing="xy"), -1).reshape(-1, 2)
    is_c = (ij[:, 0] % 4 == 0) & (ij[:, 1] % 4 == 0)
    cp = _t(np.nonzero(is_c)[0].astype(np.int32), torch.int32)
    say(f"[gpu] pattern with given C points, uniform {n}x{n}: dofs={s.dofs}")
    g = gpu_level(s, iters=5, cpoints=cp)
    assert np.array_equal(g["cbar"], (ij[:, 0] % 2 == 0) & (ij[:, 1] % 2 == 0))
    z = g["sizes"]
    assert z["n_cp_alg3"] == int(is_c.sum()) and z["n_cp_extra"] == 0
    assert 2 * z["n_vc"] + z["n_pc"] == 2 * (n // 2 + 1) ** 2 + (n // 4 + 1) ** 2
    compare_level(g, O.level(s, iters=5, cpoints=is_c))


def test_pattern_with_cpoints_jittered_matches_oracle():
    """Given C^(p) on a jittered Oseen mesh (the oracle's own Alg. 3 choice
    plus every seventh other pressure, so every vertex stays within distance
    3 of a C point while the S sets, mid-points and patterns differ from a
    plain run): the level matches the oracle's level with that C^(p)."""
    import torch
    s = synth.make_system(2, 24, jitter=0.1, nu=0.01, wind="stream", seed=3)
    L0 = O.level(s, iters=1)
    is_c = L0.is_cp | (np.arange(s.n_p) % 7 == 3)
    L = O.level(s, iters=5, cpoints=is_c)
    assert L.n_mid != L0.n_mid or not np.array_equal(L.cbar, L0.cbar)
    say(f"[gpu] pattern with given C points, jittered Oseen 24: dofs={s.dofs}")
    g = gpu_level(s, iters=5, cpoints=_t(np.nonzero(is_c)[0].astype(np.int32), torch.int32))
    compare_level(g, L)


def test_pattern_with_cpoints_rejects_bad_lists():
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 8)
    d = E.DeviceSystem.upload(s)
    for bad in ([4, 2], [0, 0], [0, s.n_p]):
        with pytest.raises(E.EminError) as ei:
            E.Pattern(d, E.params(), cpoints=_t(np.array(bad, np.int32), torch.int32))
        assert ei.value.status == 3          # ERR_PATTERN


def _chain(n):
    main = 2.0 * np.ones(n)
    main[0] = main[-1] = 1.0
    return CSR.from_scipy(sp.diags([-np.ones(n - 1), main, -np.ones(n - 1)], [-1, 0, 1]).tocsr())


def _run_hook(M: CSR, N: CSR, cid, W, Wc, iters, mixed=False):
    import torch
    from paper_1607_02489_amd import emin as E
    Md = (M.nrows, M.nnz, _t(M.rowptr, torch.int64), _t(M.col, torch.int32),
          _t(M.val, torch.float64))
    Nd = (N.nnz, _t(N.rowptr, torch.int64), _t(N.col, torch.int32))
    P = torch.empty(max(N.nnz, 1), dtype=torch.float64, device="cuda")
    rep = E.new_report()
    E.setup_with_pattern(Md, Nd, N.ncols, _t(cid, torch.int32), _t(W, torch.float64),
                         _t(Wc, torch.float64), iters, P, mixed=mixed, energy=True, report=rep)
    r = E.sync_report(rep, raise_on_error=False)
    return P.cpu().numpy()[:N.nnz], r


@pytest.mark.parametrize("n", [17, 257, 4097])
def test_setup_with_pattern_1d_hats(n):
    """sec. 4.3: for the 1-D Laplacian with C every 4th node and
    distance-3 patterns the constrained energy minimiser is piecewise-linear
    interpolation (hat functions), reached here in one CG step; the device
    result equals the hats to 1e-12 (and so does the oracle's)."""
    M = _chain(n)
    cv = np.arange(n) % 4 == 0
    is_cv, N, ne = O.velocity_pattern(M, np.zeros(n, bool), cv)
    assert ne == 0
    cid = -np.ones(n, dtype=np.int32)
    cid[is_cv] = np.arange(is_cv.sum())
    nc = int(is_cv.sum())
    say(f"[gpu] setup_with_pattern 1-D hats n={n}")
    Pv, r = _run_hook(M, N, cid, np.ones(n), np.ones(nc), 5)
    assert r.status == 0 and r.its_v == 1
    x = np.arange(n)
    hats = np.maximum(0.0, 1.0 - np.abs(x[:, None] - x[None, cv]) / 4.0)
    P = dense(CSR(N.nrows, N.ncols, N.rowptr, N.col, Pv))
    assert np.abs(P - hats).max() <= 1e-12


def test_setup_with_pattern_matches_oracle_emin():
    """The hook on a real level's velocity block (operator, pattern, C rows
    and modes from the oracle's level) equals the oracle's EMIN to 1e-10,
    with the same energy trace; in mixed precision to 1e-5."""
    s = synth.make_system(2, 20, jitter=0.1, nu=0.02, wind="stream", seed=4)
    L = O.level(s, iters=0)
    Wv = (~L.dir).astype(np.float64)
    cid = -np.ones(s.n_v, dtype=np.int32)
    cid[L.is_cv] = np.arange(L.is_cv.sum())
    Wvc = Wv[L.is_cv]
    ref = O.emin(L.Mv, L.Pv, cid, Wv, Wvc, 7)
    Pv, r = _run_hook(L.Mv, L.Pv, cid, Wv, Wvc, 7)
    assert r.status == 0 and r.its_v == ref.its
    assert relfro(Pv, ref.P.val) <= 1e-10
    assert relfro(np.array(r.energy_v[:8]), ref.energy) <= 1e-10
    Pm, rm = _run_hook(L.Mv, L.Pv, cid, Wv, Wvc, 7, mixed=True)
    assert rm.status == 0 and relfro(Pm, ref.P.val) <= 1e-5


def test_numeric_failure_reports():
    """Device-side failures land in the report: INFEASIBLE for an F row with
    an empty pattern and W_i = 1, BREAKDOWN for a negative definite operator
    (<Z, M Z> <= 0 while <R, R> > 0) -- the same codes the oracle returns on
    the same inputs."""
    n = 5
    cid = np.array([0, -1, -1, -1, 1], dtype=np.int32)
    N = CSR(n, 2, np.array([0, 1, 3, 5, 7, 8], dtype=np.int64),
            np.array([0, 0, 1, 0, 1, 0, 1, 1], dtype=np.int32), None)
    lap = sp.diags([-np.ones(n - 1), 3 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1])
    neg = CSR.from_scipy(-lap.tocsr())
    o = O.emin(neg, N, cid, np.ones(n), np.ones(2), 3, raise_on_error=False)
    _, r = _run_hook(neg, N, cid, np.ones(n), np.ones(2), 3)
    assert o.status == 6 and r.status == 6          # ERR_BREAKDOWN
    N2 = CSR(n, 2, np.array([0, 1, 1, 3, 5, 6], dtype=np.int64),
             np.array([0, 0, 1, 0, 1, 1], dtype=np.int32), None)
    I = CSR.from_scipy(sp.identity(n, format="csr"))
    o = O.emin(I, N2, cid, np.ones(n), np.ones(2), 3, raise_on_error=False)
    _, r = _run_hook(I, N2, cid, np.ones(n), np.ones(2), 3)
    assert o.status == 5 and r.status == 5          # ERR_INFEASIBLE


def test_value_validation():
    """EMIN_FLAG_VALIDATE: a NaN in the velocity block's values is reported
    as ERR_VALUE by emin_pattern (and by the hook for its operator); without
    the flag the inputs are not inspected."""
    import torch
    from paper_1607_02489_amd import emin as E
    s = synth.make_system(2, 6)
    v = s.Ahat.val.copy()
    v[17] = np.nan
    bad = synth.System(2, CSR(s.Ahat.nrows, s.Ahat.ncols, s.Ahat.rowptr, s.Ahat.col, v),
                       s.Bdiv, s.xv, s.p2v)
    with pytest.raises(E.EminError) as ei:
        E.Pattern(E.DeviceSystem.upload(bad), E.params(validate=True))
    assert ei.value.status == 4                      # ERR_VALUE
    M = _chain(9)
    Mv = M.val.copy()
    Mv[3] = np.inf
    Mbad = CSR(M.nrows, M.ncols, M.rowptr, M.col, Mv)
    cv = np.arange(9) % 4 == 0
    is_cv, N, _ = O.velocity_pattern(M, np.zeros(9, bool), cv)
    cid = -np.ones(9, dtype=np.int32)
    cid[is_cv] = np.arange(is_cv.sum())
    Md = (9, Mbad.nnz, _t(Mbad.rowptr, torch.int64), _t(Mbad.col, torch.int32),
          _t(Mbad.val, torch.float64))
    Nd = (N.nnz, _t(N.rowptr, torch.int64), _t(N.col, torch.int32))
    P = torch.empty(N.nnz, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EminError) as ei:
        E.setup_with_pattern(Md, Nd, N.ncols, _t(cid, torch.int32), _t(np.ones(9), torch.float64),
                             _t(np.ones(int(is_cv.sum())), torch.float64), 3, P, validate=True)
    assert ei.value.status == 4
