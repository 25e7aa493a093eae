"""Seeded synthetic Q2-Q1 (Taylor-Hood) Stokes / Oseen systems.

This module is the input generator shared by the GPU path, the CPU oracle,
the tests and the benchmark.  It holds none of the AMG method's arithmetic:
it only assembles the fine-level finite-element matrices that the method
takes as input (paper section 2: the blocked saddle system with identical
velocity component blocks, the Q2-Q1 element pair, and the Picard/Oseen
operator nu*A_S + K).

Layout of a generated system (all arrays numpy, C-contiguous):

* ``Ahat``  scalar velocity block, CSR over the ``n_v`` velocity nodes
  (rowptr int64[n_v+1], col int32 sorted unique, val float64).  The full
  velocity block is ``I_d (x) Ahat``.
* ``Bdiv``  divergence block, CSR of shape ``n_p x d*n_v``; the column of
  component ``c`` of node ``k`` is ``c*n_v + k`` (component-blocked).
* ``xv``    velocity node coordinates, float64[n_v, d].
* ``p2v``   int32[n_p]: the velocity node co-located with each pressure.

Orderings: velocity nodes lexicographic on the (2n+1)^d lattice, x fastest;
pressures lexicographic on the (n+1)^d vertex lattice.  Dirichlet velocity
nodes are eliminated the usual way: identity row, zeroed row and column of
``Ahat``, zeroed columns of ``Bdiv``.  Entries that vanish in exact
arithmetic (|v| <= 1e-14 max|row|) are pruned so stored structure equals the
numeric support.

Random draws use numpy's PCG64 (``numpy.random.default_rng(seed)``) in a
fixed order: vertex jitter first (all interior vertices, lexicographic, one
uniform draw per coordinate, coordinates interleaved), then the wind modes.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# ---------------------------------------------------------------------------
# reference-element bases
# ---------------------------------------------------------------------------
_GP = np.array([-math.sqrt(0.6), 0.0, math.sqrt(0.6)])
_GW = np.array([5.0 / 9.0, 8.0 / 9.0, 5.0 / 9.0])


def _q2_1d(s):
    """Quadratic Lagrange basis on nodes -1, 0, 1 and derivatives."""
    s = np.asarray(s, dtype=np.float64)
    v = np.stack([0.5 * s * (s - 1.0), 1.0 - s * s, 0.5 * s * (s + 1.0)], -1)
    d = np.stack([s - 0.5, -2.0 * s, s + 0.5], -1)
    return v, d


def _q1_1d(s):
    s = np.asarray(s, dtype=np.float64)
    v = np.stack([0.5 * (1.0 - s), 0.5 * (1.0 + s)], -1)
    d = np.stack([-0.5 * np.ones_like(s), 0.5 * np.ones_like(s)], -1)
    return v, d


def _tensor_basis(dim, fn, pts):
    """Values/gradients of a tensor-product basis at tensor-product points.

    Returns (val[nq, nb], grad[nq, nb, dim]) with both the basis index and
    the point index lexicographic, first coordinate fastest.
    """
    v1, d1 = fn(pts)                       # [np1, nb1]
    np1, nb1 = v1.shape
    if dim == 2:
        # point (p0, p1) -> q = p0 + np1*p1 ; basis (a, b) -> a + nb1*b
        V = np.einsum("xa,yb->yxba", v1, v1).reshape(np1 * np1, nb1 * nb1)
        Gx = np.einsum("xa,yb->yxba", d1, v1).reshape(np1 * np1, nb1 * nb1)
        Gy = np.einsum("xa,yb->yxba", v1, d1).reshape(np1 * np1, nb1 * nb1)
        G = np.stack([Gx, Gy], -1)
    else:
        V = np.einsum("xa,yb,zc->zyxcba", v1, v1, v1).reshape(np1 ** 3, nb1 ** 3)
        Gx = np.einsum("xa,yb,zc->zyxcba", d1, v1, v1).reshape(np1 ** 3, nb1 ** 3)
        Gy = np.einsum("xa,yb,zc->zyxcba", v1, d1, v1).reshape(np1 ** 3, nb1 ** 3)
        Gz = np.einsum("xa,yb,zc->zyxcba", v1, v1, d1).reshape(np1 ** 3, nb1 ** 3)
        G = np.stack([Gx, Gy, Gz], -1)
    return V, G


def _quad_weights(dim):
    if dim == 2:
        return np.einsum("x,y->yx", _GW, _GW).reshape(-1)
    return np.einsum("x,y,z->zyx", _GW, _GW, _GW).reshape(-1)


# ---------------------------------------------------------------------------
# system container
# ---------------------------------------------------------------------------
@dataclass
class CSR:
    nrows: int
    ncols: int
    rowptr: np.ndarray   # int64
    col: np.ndarray      # int32
    val: np.ndarray      # float64

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    @staticmethod
    def from_scipy(m) -> "CSR":
        m = m.tocsr()
        m.sort_indices()
        return CSR(m.shape[0], m.shape[1], m.indptr.astype(np.int64),
                   m.indices.astype(np.int32), m.data.astype(np.float64))

    def to_scipy(self):
        return sp.csr_matrix((self.val, self.col, self.rowptr),
                             shape=(self.nrows, self.ncols))


@dataclass
class System:
    dim: int
    Ahat: CSR
    Bdiv: CSR
    xv: np.ndarray
    p2v: np.ndarray
    meta: dict = field(default_factory=dict)

    @property
    def n_v(self) -> int:
        return self.Ahat.nrows

    @property
    def n_p(self) -> int:
        return self.Bdiv.nrows

    @property
    def dofs(self) -> int:
        return self.dim * self.n_v + self.n_p


# ---------------------------------------------------------------------------
# mesh
# ---------------------------------------------------------------------------
def _vertices(dim, n, jitter, rng):
    h = 1.0 / n
    g = np.arange(n + 1, dtype=np.float64) * h
    if dim == 2:
        Y, X = np.meshgrid(g, g, indexing="ij")
        V = np.stack([X.reshape(-1), Y.reshape(-1)], -1)
        ij = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), indexing="ij"), -1).reshape(-1, 2)[:, ::-1]
    else:
        Z, Y, X = np.meshgrid(g, g, g, indexing="ij")
        V = np.stack([X.reshape(-1), Y.reshape(-1), Z.reshape(-1)], -1)
        ij = np.stack(np.meshgrid(np.arange(n + 1), np.arange(n + 1), np.arange(n + 1),
                                  indexing="ij"), -1).reshape(-1, 3)[:, ::-1]
    interior = np.all((ij > 0) & (ij < n), axis=1)
    if jitter > 0.0:
        nint = int(interior.sum())
        d = rng.uniform(-jitter * h, jitter * h, size=(nint, dim))
        V[interior] += d
    return V


def _element_tables(dim, n):
    """Global velocity-node and pressure indices of every element."""
    nv1 = 2 * n + 1
    npd = n + 1
    e = np.arange(n)
    if dim == 2:
        ey, ex = np.meshgrid(e, e, indexing="ij")
        ex = ex.reshape(-1); ey = ey.reshape(-1)
        a = np.arange(3)
        lb, la = np.meshgrid(a, a, indexing="ij")
        la = la.reshape(-1); lb = lb.reshape(-1)
        vnodes = (2 * ex[:, None] + la[None]) + nv1 * (2 * ey[:, None] + lb[None])
        a = np.arange(2)
        lb, la = np.meshgrid(a, a, indexing="ij")
        la = la.reshape(-1); lb = lb.reshape(-1)
        pnodes = (ex[:, None] + la[None]) + npd * (ey[:, None] + lb[None])
    else:
        ez, ey, ex = np.meshgrid(e, e, e, indexing="ij")
        ex = ex.reshape(-1); ey = ey.reshape(-1); ez = ez.reshape(-1)
        a = np.arange(3)
        lc, lb, la = np.meshgrid(a, a, a, indexing="ij")
        la = la.reshape(-1); lb = lb.reshape(-1); lc = lc.reshape(-1)
        vnodes = ((2 * ex[:, None] + la[None]) + nv1 * (2 * ey[:, None] + lb[None])
                  + nv1 * nv1 * (2 * ez[:, None] + lc[None]))
        a = np.arange(2)
        lc, lb, la = np.meshgrid(a, a, a, indexing="ij")
        la = la.reshape(-1); lb = lb.reshape(-1); lc = lc.reshape(-1)
        pnodes = ((ex[:, None] + la[None]) + npd * (ey[:, None] + lb[None])
                  + npd * npd * (ez[:, None] + lc[None]))
    return vnodes.astype(np.int64), pnodes.astype(np.int64)


def _velocity_coords(dim, n, V, pnodes_vertices):
    """Q2 node coordinates: images of the reference nodes under each
    element's (bi/tri)linear map.  Shared nodes get identical coordinates
    because the shared edge/face is mapped by the same vertices."""
    s = np.array([-1.0, 0.0, 1.0])
    l1, _ = _q1_1d(s)                                      # [3, 2]
    if dim == 2:
        Lm = np.einsum("xa,yb->yxba", l1, l1).reshape(9, 4)
    else:
        Lm = np.einsum("xa,yb,zc->zyxcba", l1, l1, l1).reshape(27, 8)
    return np.einsum("qc,ecd->eqd", Lm, V[pnodes_vertices])


# ---------------------------------------------------------------------------
# assembly
# ---------------------------------------------------------------------------
def _assemble(dim, n, V, nu, wind_fn, chunk=4096, split=False, mass=False):
    nv1 = 2 * n + 1
    n_v = nv1 ** dim
    n_p = (n + 1) ** dim
    vnodes, pnodes = _element_tables(dim, n)
    ne = vnodes.shape[0]
    nbv = 3 ** dim
    nbp = 2 ** dim

    Vq, Gq = _tensor_basis(dim, _q2_1d, _GP)     # [nq, 9|27], [nq, nb, d]
    Pq, _ = _tensor_basis(dim, _q1_1d, _GP)      # [nq, 4|8]
    _, Gg = _tensor_basis(dim, _q1_1d, _GP)      # geometry gradients [nq, nbp, d]
    wq = _quad_weights(dim)

    xv = np.zeros((n_v, dim))
    rowsA, colsA, valsA, valsK = [], [], [], []
    rowsB, colsB, valsB = [], [], []
    valsMv, rowsMp, colsMp, valsMp = [], [], [], []
    for e0 in range(0, ne, chunk):
        e1 = min(ne, e0 + chunk)
        vn = vnodes[e0:e1]
        pn = pnodes[e0:e1]
        Xc = V[pn]                                             # [E, nbp, d]
        xv[vn.reshape(-1)] = _velocity_coords(dim, n, V, pn).reshape(-1, dim)
        J = np.einsum("qad,eak->eqkd", Gg, Xc, optimize=True)  # dx_k/ds_d
        detJ = np.linalg.det(J)
        Jinv = np.linalg.inv(J)                                # ds/dx : [e,q,d,k]
        # physical gradients [E,nq,nbv,d] as batched matmuls over (e,q)
        gphys = np.matmul(Gq[None], Jinv)
        wdet = wq[None, :] * np.abs(detJ)                      # [E,nq]
        E_ = gphys.shape[0]
        nq = gphys.shape[1]
        # Ke_ij = sum_{q,k} w_q |J| g_qik g_qjk  ->  (E, nbv, nq*d) @ (E, nq*d, nbv)
        gw = gphys * wdet[:, :, None, None]
        Gt = gw.transpose(0, 2, 1, 3).reshape(E_, nbv, nq * dim)
        Gm = gphys.transpose(0, 1, 3, 2).reshape(E_, nq * dim, nbv)
        Ke = nu * np.matmul(Gt, Gm)
        Kc = None
        if wind_fn is not None:
            xn = xv[vn]                                        # node coords [E,nbv,d]
            Wn = wind_fn(xn)                                   # nodal wind [E,nbv,d]
            wqv = np.matmul(Vq[None], Wn)                      # wind at qp [E,nq,d]
            adv = np.matmul(gphys, wqv[:, :, :, None])[..., 0]  # w . grad(phi_j) [E,nq,nbv]
            # Ke_ij += sum_q w_q |J| phi_i(q) adv_qj
            Kc = np.matmul((Vq[None] * wdet[:, :, None]).transpose(0, 2, 1), adv)
            if not split:
                Ke = Ke + Kc
        rowsA.append(np.repeat(vn, nbv, axis=1).reshape(-1))
        colsA.append(np.tile(vn, (1, nbv)).reshape(-1))
        valsA.append(Ke.reshape(-1))
        if mass:
            # element mass matrices: sum_q w_q |J| phi_i(q) phi_j(q) (Q2 velocity,
            # scalar) and psi_k(q) psi_l(q) (Q1 pressure)
            Vw = (Vq[None] * wdet[:, :, None]).transpose(0, 2, 1)      # [E,nbv,nq]
            valsMv.append(np.matmul(Vw, np.broadcast_to(Vq[None], (E_,) + Vq.shape)).reshape(-1))
            Pw_ = (Pq[None] * wdet[:, :, None]).transpose(0, 2, 1)     # [E,nbp,nq]
            valsMp.append(np.matmul(Pw_, np.broadcast_to(Pq[None], (E_,) + Pq.shape)).reshape(-1))
            rowsMp.append(np.repeat(pn, nbp, axis=1).reshape(-1))
            colsMp.append(np.tile(pn, (1, nbp)).reshape(-1))
        if split:
            valsK.append((Kc if Kc is not None else np.zeros_like(Ke)).reshape(-1))
        # b_{c,k,i} = int psi_k dphi_i/dx_c  ->  (E, nbp, nq) @ (E, nq, nbv) per c
        Pw = (Pq[None] * wdet[:, :, None]).transpose(0, 2, 1)  # [E,nbp,nq]
        for c in range(dim):
            Bc = np.matmul(Pw, gphys[:, :, :, c])               # [E,nbp,nbv]
            rowsB.append(np.repeat(pn, nbv, axis=1).reshape(-1))
            colsB.append((np.tile(vn, (1, nbp)) + c * n_v).reshape(-1))
            valsB.append(Bc.reshape(-1))
    A = sp.coo_matrix((np.concatenate(valsA), (np.concatenate(rowsA), np.concatenate(colsA))),
                      shape=(n_v, n_v)).tocsr()
    B = sp.coo_matrix((np.concatenate(valsB), (np.concatenate(rowsB), np.concatenate(colsB))),
                      shape=(n_p, dim * n_v)).tocsr()
    A.sum_duplicates(); B.sum_duplicates()
    if mass:
        Mv = sp.coo_matrix((np.concatenate(valsMv), (np.concatenate(rowsA), np.concatenate(colsA))),
                           shape=(n_v, n_v)).tocsr()
        Mp = sp.coo_matrix((np.concatenate(valsMp), (np.concatenate(rowsMp),
                                                      np.concatenate(colsMp))),
                           shape=(n_p, n_p)).tocsr()
        Mv.sum_duplicates(); Mp.sum_duplicates()
        return A, B, xv, (Mv, Mp)
    if split:
        # same COO indices -> same CSR structure, convection values aligned
        K = sp.coo_matrix((np.concatenate(valsK), (np.concatenate(rowsA), np.concatenate(colsA))),
                          shape=(n_v, n_v)).tocsr()
        K.sum_duplicates()
        A.sort_indices(); K.sort_indices()
        assert np.array_equal(A.indptr, K.indptr) and np.array_equal(A.indices, K.indices)
        return A, B, xv, K
    return A, B, xv


def _prune(m, rel=1e-14):
    m = m.tocsr()
    m.sort_indices()
    rmax = np.zeros(m.shape[0])
    absd = np.abs(m.data)
    rows = np.repeat(np.arange(m.shape[0]), np.diff(m.indptr))
    np.maximum.at(rmax, rows, absd)
    keep = absd > rel * rmax[rows]
    m.data = np.where(keep, m.data, 0.0)
    m.eliminate_zeros()
    return m


def _apply_dirichlet(A, B, dmask, dim):
    n_v = A.shape[0]
    keep = sp.diags((~dmask).astype(np.float64))
    A = keep @ A @ keep + sp.diags(dmask.astype(np.float64))
    keepB = sp.diags(np.tile((~dmask).astype(np.float64), dim))
    B = B @ keepB
    return A.tocsr(), B.tocsr()


def _lattice_index(dim, m):
    """Per-node integer lattice coordinates of an m^dim lattice (x fastest)."""
    a = np.arange(m)
    if dim == 2:
        J, I = np.meshgrid(a, a, indexing="ij")
        return np.stack([I.reshape(-1), J.reshape(-1)], -1)
    K, J, I = np.meshgrid(a, a, a, indexing="ij")
    return np.stack([I.reshape(-1), J.reshape(-1), K.reshape(-1)], -1)


def stream_wind_2d(rng, modes=16, kmax=4):
    """Divergence-free wind u = (dpsi/dy, -dpsi/dx) from a random stream
    function psi = sum_m a_m sin(k_m pi x) sin(l_m pi y); u.n = 0 on the
    unit square boundary.  Returned callable maps coords[..., 2] -> wind."""
    a = rng.standard_normal(modes)
    k = rng.integers(1, kmax + 1, size=modes)
    l = rng.integers(1, kmax + 1, size=modes)

    def raw(x):
        X = x[..., 0][..., None]; Y = x[..., 1][..., None]
        u = np.sum(a * np.sin(k * np.pi * X) * (l * np.pi) * np.cos(l * np.pi * Y), -1)
        v = -np.sum(a * (k * np.pi) * np.cos(k * np.pi * X) * np.sin(l * np.pi * Y), -1)
        return np.stack([u, v], -1)

    return raw


def stream_wind_3d(rng, modes=16, kmax=4):
    """Divergence-free 3-D wind u = curl(psi), psi a random vector potential
    built from products of sines (vanishing normal flux on the unit cube)."""
    a = rng.standard_normal((modes, 3))
    kk = rng.integers(1, kmax + 1, size=(modes, 3))

    def raw(x):
        X = x[..., 0][..., None]; Y = x[..., 1][..., None]; Z = x[..., 2][..., None]
        kx, ky, kz = (kk[:, 0] * np.pi, kk[:, 1] * np.pi, kk[:, 2] * np.pi)
        s = lambda k, t: np.sin(k * t)
        c = lambda k, t: np.cos(k * t)
        # psi_i = a_i * sin(kx X) sin(ky Y) sin(kz Z)
        S = s(kx, X) * s(ky, Y) * s(kz, Z)
        dX = kx * c(kx, X) * s(ky, Y) * s(kz, Z)
        dY = ky * s(kx, X) * c(ky, Y) * s(kz, Z)
        dZ = kz * s(kx, X) * s(ky, Y) * c(kz, Z)
        del S
        u = np.sum(a[:, 2] * dY - a[:, 1] * dZ, -1)
        v = np.sum(a[:, 0] * dZ - a[:, 2] * dX, -1)
        w = np.sum(a[:, 1] * dX - a[:, 0] * dY, -1)
        return np.stack([u, v, w], -1)

    return raw


def _scaled(raw, dim, n):
    """Scale a raw wind so that max |u| over the uniform velocity lattice is 1."""
    m = 2 * n + 1
    pts = _lattice_index(dim, m).astype(np.float64) / (m - 1)
    mx = float(np.max(np.linalg.norm(raw(pts), axis=-1)))
    s = 1.0 / mx if mx > 0 else 0.0
    return lambda x: s * raw(x)


def make_system(dim: int, n: int, *, jitter: float = 0.0, seed: int = 0,
                nu: float = 1.0, wind: str | None = None, wind_seed: int | None = None,
                domain: str = "cavity", mass: bool = False) -> System:
    """Assemble a Q2-Q1 Stokes (wind=None) or Oseen system on the unit
    square/cube with n elements per side.

    domain='cavity': Dirichlet velocity on the whole boundary (lid-driven
    cavity; only the Dirichlet set matters for the operator).
    domain='channel': Dirichlet at inflow x=0 and on the side walls, natural
    outflow at x=1.
    wind: None (Stokes), 'stream' (seeded divergence-free Fourier field),
    'channel' (Poiseuille profile plus a seeded divergence-free field).
    """
    rng = np.random.default_rng(seed)
    V = _vertices(dim, n, jitter, rng)
    wind_fn = None
    if wind is not None:
        wrng = np.random.default_rng(seed if wind_seed is None else wind_seed)
        if wind == "stream":
            raw = stream_wind_2d(wrng) if dim == 2 else stream_wind_3d(wrng)
            wind_fn = _scaled(raw, dim, n)
        elif wind == "channel":
            pert = stream_wind_3d(wrng) if dim == 3 else stream_wind_2d(wrng)

            def raw(x, pert=pert):
                out = 0.25 * pert(x)
                if dim == 3:
                    prof = 16.0 * x[..., 1] * (1 - x[..., 1]) * x[..., 2] * (1 - x[..., 2])
                else:
                    prof = 4.0 * x[..., 1] * (1 - x[..., 1])
                out[..., 0] += prof
                return out
            wind_fn = _scaled(raw, dim, n)
        else:
            raise ValueError(f"unknown wind {wind!r}")
    if mass:
        A, B, xv, (Mv, Mp) = _assemble(dim, n, V, nu, wind_fn, mass=True)
    else:
        A, B, xv = _assemble(dim, n, V, nu, wind_fn)
    m = 2 * n + 1
    lat = _lattice_index(dim, m)
    if domain == "cavity":
        dmask = np.any((lat == 0) | (lat == m - 1), axis=1)
    elif domain == "channel":
        side = np.any((lat[:, 1:] == 0) | (lat[:, 1:] == m - 1), axis=1)
        dmask = side | (lat[:, 0] == 0)
    else:
        raise ValueError(domain)
    A, B = _apply_dirichlet(A, B, dmask, dim)
    A = _prune(A)
    B = _prune(B)
    plat = _lattice_index(dim, n + 1)
    if dim == 2:
        p2v = 2 * plat[:, 0] + m * (2 * plat[:, 1])
    else:
        p2v = 2 * plat[:, 0] + m * (2 * plat[:, 1]) + m * m * (2 * plat[:, 2])
    meta = dict(n=n, jitter=jitter, seed=seed, nu=nu, wind=wind, wind_seed=wind_seed,
                domain=domain, dirichlet=int(dmask.sum()))
    if mass:
        # the velocity mass matrix on the space without the Dirichlet nodes
        # (eliminated like the velocity block: zero row and column, unit
        # diagonal), the pressure mass matrix as assembled
        keep = sp.diags((~dmask).astype(np.float64))
        Mv = _prune(keep @ Mv @ keep + sp.diags(dmask.astype(np.float64)))
        meta["Mv"] = CSR.from_scipy(Mv)
        meta["Mp"] = CSR.from_scipy(_prune(Mp))
    return System(dim, CSR.from_scipy(A), CSR.from_scipy(B), np.ascontiguousarray(xv),
                  p2v.astype(np.int32), meta=meta)


def make_split_system(dim: int, n: int, *, jitter: float = 0.0, seed: int = 0,
                      wind: str = "channel", wind_seed: int | None = None,
                      domain: str = "channel") -> System:
    """An Oseen system whose velocity block is kept as two value arrays on one
    structure: the Laplacian part A_S and the convection part K, so that
    nu*A_S + K can be formed for any viscosity without re-assembly.  Ahat
    holds A_S + K; meta['S_val'] and meta['K_val'] hold the parts."""
    rng = np.random.default_rng(seed)
    V = _vertices(dim, n, jitter, rng)
    wrng = np.random.default_rng(seed if wind_seed is None else wind_seed)
    pert = stream_wind_3d(wrng) if dim == 3 else stream_wind_2d(wrng)
    if wind == "channel":
        def raw(x, pert=pert):
            out = 0.25 * pert(x)
            if dim == 3:
                prof = 16.0 * x[..., 1] * (1 - x[..., 1]) * x[..., 2] * (1 - x[..., 2])
            else:
                prof = 4.0 * x[..., 1] * (1 - x[..., 1])
            out[..., 0] += prof
            return out
    elif wind == "stream":
        raw = pert
    else:
        raise ValueError(wind)
    A, B, xv, K = _assemble(dim, n, V, 1.0, _scaled(raw, dim, n), split=True)
    m = 2 * n + 1
    lat = _lattice_index(dim, m)
    if domain == "cavity":
        dmask = np.any((lat == 0) | (lat == m - 1), axis=1)
    else:
        side = np.any((lat[:, 1:] == 0) | (lat[:, 1:] == m - 1), axis=1)
        dmask = side | (lat[:, 0] == 0)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    elim = dmask[rows] | dmask[cols]
    diag = rows == cols
    Sv = np.where(elim, 0.0, A.data)
    Kv = np.where(elim, 0.0, K.data)
    Sv = np.where(elim & diag, 1.0, Sv)
    # joint pruning keeps one structure for both parts
    mag = np.abs(Sv) + np.abs(Kv)
    rmax = np.zeros(A.shape[0])
    np.maximum.at(rmax, rows, mag)
    keep = mag > 1e-14 * rmax[rows]
    rp = np.concatenate([[0], np.cumsum(np.bincount(rows[keep], minlength=A.shape[0]))])
    Ahat = CSR(A.shape[0], A.shape[1], rp.astype(np.int64), cols[keep].astype(np.int32),
               (Sv + Kv)[keep])
    keepB = sp.diags(np.tile((~dmask).astype(np.float64), dim))
    Bd = _prune((B @ keepB).tocsr())
    plat = _lattice_index(dim, n + 1)
    if dim == 2:
        p2v = 2 * plat[:, 0] + m * (2 * plat[:, 1])
    else:
        p2v = 2 * plat[:, 0] + m * (2 * plat[:, 1]) + m * m * (2 * plat[:, 2])
    return System(dim, Ahat, CSR.from_scipy(Bd), np.ascontiguousarray(xv), p2v.astype(np.int32),
                  meta=dict(n=n, seed=seed, wind=wind, domain=domain, S_val=Sv[keep],
                            K_val=Kv[keep], dirichlet=int(dmask.sum())))


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def stokes2d_small(seed: int = 0) -> System:
    """2-D Stokes lid cavity, 8x8 elements, jitter +-0.1h: 578 u + 81 p."""
    return make_system(2, 8, jitter=0.1, seed=seed, nu=1.0)


def oseen2d(n: int = 256, re: float = 100.0, seed: int = 2) -> System:
    """2-D Oseen cavity, Re = 1/nu with |wind|max = 1 on the unit square."""
    return make_system(2, n, jitter=0.0, seed=seed, nu=1.0 / re, wind="stream")


def stokes3d(n: int = 48, seed: int = 3, jitter: float = 0.05) -> System:
    """3-D Stokes cube cavity, jitter +-0.05h: 3(2n+1)^3 u + (n+1)^3 p."""
    return make_system(3, n, jitter=jitter, seed=seed, nu=1.0)


def table1_dofs(n: int) -> int:
    """Q2-Q1 dof count of an n x n square mesh: 2(2n+1)^2 + (n+1)^2."""
    return 2 * (2 * n + 1) ** 2 + (n + 1) ** 2
