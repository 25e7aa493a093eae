"""Why a fresh mixed-precision hierarchy can differ from the FP64 one at a
coarse level, shown on the CPU with the oracle (no GPU).

The mixed form runs the Galerkin product in FP32.  The next level's drop
filter (eq. (e:filtering)) then decides on FP32-accumulated values: an entry
whose coupling ratio lies within ~1e-7 of tau1 can be kept by one precision
and dropped by the other, and one such flip changes that level's energy
operator and so its P far more than the rounding itself.  Rounding alone does
not amplify: with the drop masks unchanged, the level-1 P moves by about the
size of the perturbation.  Hence the mixed numeric phases run on the patterns
and drop masks of the FP64 pass.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_1607_02489_amd import synth
from paper_1607_02489_amd.synth import CSR, System
from tests.helpers import relfro

KW = dict(tau1_v=0.038, tau1_p=0.04)


def _fp32_rap(s, L0):
    """Level-0 Galerkin product with FP32 operands and FP32 accumulation
    (scipy's float32 sparse products), on the oracle's coarse patterns."""
    A = s.Ahat.to_scipy().astype(np.float32)
    B = s.Bdiv.to_scipy().astype(np.float32)
    Pv = L0.Pv.to_scipy().astype(np.float32)
    Pp = L0.Pp.to_scipy().astype(np.float32)
    Ac = (Pv.T @ (A @ Pv)).tocsr()
    X = sp.kron(sp.identity(s.dim, dtype=np.float32), Pv).tocsr()
    Bc = (Pp.T @ (B @ X)).tocsr()

    def on(ref, m):
        rows = np.repeat(np.arange(ref.nrows), np.diff(ref.rowptr))
        v = np.asarray(m[rows, ref.col]).ravel().astype(np.float64)
        return CSR(ref.nrows, ref.ncols, ref.rowptr, ref.col, v)

    return on(L0.Ac, Ac), on(L0.Bc, Bc)


def _levels(O, n):
    s = synth.stokes3d(n)
    L0 = O.level(s, iters=5, **KW)
    c = L0.coarse_system()
    Ac32, Bc32 = _fp32_rap(s, L0)
    c32 = System(c.dim, Ac32, Bc32, c.xv, c.p2v)
    return c, c32, O.level(c, iters=5, **KW), O.level(c32, iters=5, **KW)


def test_fp32_rap_without_flips_does_not_amplify(oracle_lib):
    """3-D Stokes 24^3: the FP32 Galerkin product perturbs the level-1
    operator by ~1e-7; no drop decision flips, and the level-1 P moves by
    less than 1e-6 (no amplification by the CG)."""
    c, c32, L1, L1m = _levels(oracle_lib, 24)
    pert = relfro(c32.Ahat.val, c.Ahat.val)
    assert 1e-8 < pert < 1e-6
    assert np.array_equal(L1.keep_v, L1m.keep_v) and np.array_equal(L1.keep_p, L1m.keep_p)
    assert np.array_equal(L1.Pv.col, L1m.Pv.col)
    assert relfro(L1m.Pv.val, L1.Pv.val) < 10 * pert
    assert relfro(L1m.Pp.val, L1.Pp.val) < 10 * relfro(c32.Bdiv.val, c.Bdiv.val)


@pytest.mark.slow
def test_fp32_rap_flips_a_drop_decision_at_48(oracle_lib):
    """3-D Stokes 48^3 (the benchmark's size): the same FP32 product flips a
    level-1 velocity drop decision, the velocity pattern is unchanged, and the
    level-1 P moves by more than 1e-5 -- three orders of magnitude above the
    perturbation of its input."""
    c, c32, L1, L1m = _levels(oracle_lib, 48)
    pert = relfro(c32.Ahat.val, c.Ahat.val)
    assert pert < 1e-6
    assert int((L1.keep_v != L1m.keep_v).sum()) >= 1
    assert np.array_equal(L1.Pv.col, L1m.Pv.col)
    assert relfro(L1m.Pv.val, L1.Pv.val) > 1e-5
