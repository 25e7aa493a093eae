"""Pins of the synthetic Q2-Q1 input generator.

Table 1 of the paper fixes the dof counts of the uniform Q2-Q1 square
meshes; the 1-D quadratic element matrices fix the interior coupling ratios
of the velocity block and of B B^T on an unjittered mesh.
"""
import json
import pathlib

import numpy as np
import pytest

from paper_1607_02489_amd import synth
from tests.helpers import dense

GOLDEN = pathlib.Path(__file__).parent / "golden"
TABLE1 = {int(k): v for k, v in
          json.loads((GOLDEN / "table1_dofs.json").read_text())["elements_per_side_to_dofs"].items()}


@pytest.mark.parametrize("n", sorted(TABLE1))
def test_table1_dof_counts(n):
    # Table 1 (Stokes lid-driven cavity): the Dofs column
    dofs = TABLE1[n]
    assert synth.table1_dofs(n) == dofs
    if n <= 32:
        s = synth.make_system(2, n)
        assert s.dofs == dofs
        assert s.n_v == (2 * n + 1) ** 2 and s.n_p == (n + 1) ** 2


def test_3d_counts():
    s = synth.make_system(3, 3)
    assert s.n_v == 7 ** 3 and s.n_p == 4 ** 3
    assert s.Bdiv.ncols == 3 * s.n_v


def _ratio(A, p, q):
    return abs(A[p, q]) / np.sqrt(A[p, p] * A[q, q])


def test_q2_laplacian_coupling_ratios():
    # tensor products of K1 = (1/3h)[7 -8 1; -8 16 -8; 1 -8 7] and
    # M1 = (h/30)[4 2 -1; 2 16 2; -1 2 4] give these interior ratios
    s = synth.make_system(2, 8)
    A = dense(s.Ahat)
    m = 17
    ix = lambda i, j: i + m * j
    assert _ratio(A, ix(8, 8), ix(9, 8)) == pytest.approx(0.1282056, abs=1e-6)   # vertex-edge
    assert _ratio(A, ix(8, 8), ix(10, 8)) == pytest.approx(3 / 112, abs=1e-12)   # vertex-vertex
    assert _ratio(A, ix(8, 8), ix(9, 9)) == pytest.approx(0.0944911, abs=1e-6)   # vertex-centre
    assert _ratio(A, ix(9, 8), ix(9, 9)) == pytest.approx(0.2261335, abs=1e-6)   # edge-centre
    assert _ratio(A, ix(9, 8), ix(8, 9)) == pytest.approx(1 / 11, abs=1e-12)     # edge-edge
    assert A[ix(9, 8), ix(9, 10)] == 0.0                                         # parallel edges


def test_bbt_ratios_and_25_point():
    s = synth.make_system(2, 8)
    B = s.Bdiv.to_scipy()
    Z = (B @ B.T).toarray()
    mp = 9
    c = 4 + mp * 4
    r = lambda dx, dy: abs(Z[c, c + dx + mp * dy]) / np.sqrt(Z[c, c] * Z[c + dx + mp * dy, c + dx + mp * dy])
    assert r(1, 0) == pytest.approx(0.0686275, abs=1e-6)
    assert r(1, 1) == pytest.approx(0.1568627, abs=1e-6)
    assert r(2, 0) == pytest.approx(0.0147059, abs=1e-6)
    # sec. 4.1: interior stencils of B B^T reach two cells out (25-point
    # box); on a uniform mesh the four (+-2,+-2) corners vanish (21 nonzeros)
    row = (B @ B.T).tocsr()[c]
    assert row.nnz == 21
    offs = {(int(j) % mp - 4, int(j) // mp - 4) for j in row.indices}
    assert offs == {(a, b) for a in range(-2, 3) for b in range(-2, 3)} - {(2, 2), (2, -2), (-2, 2), (-2, -2)}


def test_dirichlet_elimination():
    s = synth.make_system(2, 4)
    A = dense(s.Ahat)
    m = 9
    for i in range(m):            # bottom row of the lattice: boundary nodes
        assert A[i, i] == 1.0
        assert np.count_nonzero(A[i]) == 1 and np.count_nonzero(A[:, i]) == 1
    # all-Dirichlet cavity: B^T 1 = 0 (discrete divergence of a constant pressure)
    B = dense(s.Bdiv)
    assert np.abs(B.sum(axis=0)).max() < 1e-14


def test_seeded_and_symmetric():
    a = synth.stokes2d_small(0)
    b = synth.stokes2d_small(0)
    assert np.array_equal(a.xv, b.xv) and np.array_equal(a.Ahat.val, b.Ahat.val)
    A = dense(a.Ahat)
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    o = synth.make_system(2, 8, nu=0.01, wind="stream", seed=2)
    Ao = dense(o.Ahat)
    assert np.abs(Ao - Ao.T).max() > 1e-6          # convection is non-symmetric
    assert o.p2v.dtype == np.int32 and o.p2v.max() < o.n_v
