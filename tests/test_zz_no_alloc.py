"""The allocation-free entry point emin_setup_with_pattern_noalloc, through
the C ABI: two calls in a row (the second on a smaller problem, so the shared
scratch array holds the first call's contents) each equal
emin_setup_with_pattern on the same inputs bit for bit, with the same report;
a problem beyond the scratch bound is refused before any work."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1607_02489_amd import synth
from tests.gpu_util import say

pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    import torch
    s = synth.make_system(2, n, jitter=0.1, nu=0.02, wind="stream", seed=seed)
    L = O.level(s, iters=0)
    Wv = (~L.dir).astype(np.float64)
    cid = -np.ones(s.n_v, dtype=np.int32)
    cid[L.is_cv] = np.arange(L.is_cv.sum())
    t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dt)
    M, N = L.Mv, L.Pv
    Md = (M.nrows, M.nnz, t(M.rowptr, torch.int64), t(M.col, torch.int32), t(M.val, torch.float64))
    Nd = (N.nnz, t(N.rowptr, torch.int64), t(N.col, torch.int32))
    return (Md, Nd, N.ncols, t(cid, torch.int32), t(Wv, torch.float64),
            t(Wv[L.is_cv], torch.float64)), N.nnz


def _run(args, nnz, noalloc, mixed=False):
    import torch
    from paper_1607_02489_amd import emin as E
    P = torch.full((max(nnz, 1),), np.nan, dtype=torch.float64, device="cuda")
    rep = E.new_report()
    E.setup_with_pattern(*args, 5, P, mixed=mixed, energy=True, report=rep, noalloc=noalloc)
    r = E.sync_report(rep, raise_on_error=False)
    return P.cpu().numpy()[:nnz], r


@pytest.mark.parametrize("mixed", [False, True])
def test_noalloc_equals_allocating_entry_point_twice(mixed):
    for n, seed in ((40, 3), (17, 5)):
        args, nnz = _inputs(n, seed)
        say(f"[gpu] no-alloc setup n={n} mixed={mixed}: pattern nnz={nnz}")
        a, ra = _run(args, nnz, noalloc=False, mixed=mixed)
        b, rb = _run(args, nnz, noalloc=True, mixed=mixed)
        assert ra.status == rb.status == 0
        assert np.array_equal(a, b)
        assert ra.its_v == rb.its_v
        assert np.array_equal(np.array(ra.energy_v[:6]), np.array(rb.energy_v[:6]))
        assert np.array_equal(np.array(ra.rho_v[:6]), np.array(rb.rho_v[:6]))


def test_noalloc_rejects_beyond_scratch():
    import torch
    from paper_1607_02489_amd import emin as E
    n = 2_000_000
    z64 = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    z32 = torch.zeros(n, dtype=torch.int32, device="cuda")
    zf = torch.zeros(n, dtype=torch.float64, device="cuda")
    Md = (n, 0, z64, z32, zf)
    Nd = (0, z64, z32)
    with pytest.raises(E.EminError) as ei:
        E.setup_with_pattern(Md, Nd, 0, z32, zf, zf, 2, zf, noalloc=True)
    assert ei.value.status == 10      # EMIN_ERR_CAPACITY
