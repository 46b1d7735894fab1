"""Seeded synthetic inputs: finite-difference diffusion matrices on regular grids.

This module builds the workload family of the paper's numerical section (§7):
-div(alpha grad u) = f on [0,1]^d with u = 0 on the boundary, discretised by the
second-order central five-point (2D) or seven-point (3D) stencil, plus the
right-hand sides. It holds none of the solver's arithmetic; the CPU oracle and the
GPU library both consume what it produces as plain arrays.

Conventions (stated here once, used by every generator):

* Unknowns are the N^d interior grid nodes, numbered with the x index fastest:
  ``idx = i0 + N*i1 + N*N*i2``.
* No 1/h^2 scaling: the constant-coefficient operator has diagonal 2d and
  off-diagonals -1, the textbook stencil.
* Variable coefficients are given per unknown (cell value a_i). The coupling across
  the face between unknowns i and j along axis t is c_t * 2 a_i a_j / (a_i + a_j)
  (harmonic mean); a face on the Dirichlet boundary contributes c_t * a_i to the
  diagonal. With a == 1 and c == 1 this is exactly the constant stencil.
* CSR arrays: ``row_ptr`` int64 (n+1), ``col_idx`` int32 sorted within each row,
  ``values`` float64. Coordinates are the integer grid positions as float64 (n x d).
* Right-hand sides are ``uniform(-1, 1)`` from ``numpy.random.default_rng(seed)``,
  shaped (n, nrhs) and returned column-major (Fortran order).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """A sparse SPD system A x = b in CSR form with grid coordinates."""

    n: int
    row_ptr: np.ndarray          # int64, n+1
    col_idx: np.ndarray          # int32, nnz
    values: np.ndarray           # float64, nnz
    coords: np.ndarray           # float64, n x dim
    dim: int
    grid: tuple
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.values, self.col_idx.astype(np.int64), self.row_ptr),
                             shape=(self.n, self.n))

    def dense(self) -> np.ndarray:
        return self.to_scipy().toarray()


def _grid_coords(N: int, dim: int) -> np.ndarray:
    axes = [np.arange(N, dtype=np.float64)] * dim
    mesh = np.meshgrid(*axes, indexing="ij")
    # idx = i0 + N*i1 + N^2*i2: i0 varies fastest -> reverse the 'ij' flattening
    cols = [m.transpose(tuple(range(dim))[::-1]).reshape(-1) for m in mesh]
    return np.stack(cols, axis=1)


def diffusion(N: int, dim: int, cell: np.ndarray | None = None,
              axis_scale=(1.0, 1.0, 1.0), name: str = "") -> Problem:
    """Assemble the 5/7-point FD diffusion matrix on an N^dim interior grid.

    ``cell`` holds one positive coefficient per unknown (None = constant 1);
    ``axis_scale`` multiplies the couplings along each axis (anisotropy).
    """
    if dim not in (1, 2, 3):
        raise ValueError("dim must be 1, 2 or 3")
    n = N ** dim
    a = np.ones(n) if cell is None else np.asarray(cell, dtype=np.float64).reshape(n)
    if np.any(a <= 0):
        raise ValueError("coefficients must be positive")
    idx = np.arange(n, dtype=np.int64)
    # per-axis grid index of each unknown
    pos = [(idx // (N ** t)) % N for t in range(dim)]
    diag = np.zeros(n)
    rows, cols, vals = [], [], []
    for t in range(dim):
        c = float(axis_scale[t])
        stride = N ** t
        for step in (-1, +1):
            nb_pos = pos[t] + step
            inside = (nb_pos >= 0) & (nb_pos < N)
            i = idx[inside]
            j = i + step * stride
            face = c * 2.0 * a[i] * a[j] / (a[i] + a[j])
            rows.append(i)
            cols.append(j)
            vals.append(-face)
            np.add.at(diag, i, face)
            ib = idx[~inside]
            np.add.at(diag, ib, c * a[ib])
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    r = np.concatenate(rows)
    cidx = np.concatenate(cols)
    v = np.concatenate(vals)
    order = np.lexsort((cidx, r))
    r, cidx, v = r[order], cidx[order], v[order]
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, r + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Problem(n=n, row_ptr=row_ptr, col_idx=cidx.astype(np.int32), values=v,
                   coords=_grid_coords(N, dim), dim=dim, grid=(N,) * dim,
                   name=name or f"fd{dim}d_N{N}")


def poisson(N: int, dim: int) -> Problem:
    """Constant-coefficient Poisson (alpha = 1), §7.1 of the paper."""
    return diffusion(N, dim, None, name=f"poisson{dim}d_N{N}")


def lognormal_field(N: int, dim: int, sigma: float, seed: int) -> np.ndarray:
    """a_i = exp(sigma * z_i), z_i iid N(0,1), one value per unknown, no correlation."""
    rng = np.random.default_rng(seed)
    return np.exp(sigma * rng.standard_normal(N ** dim))


def lognormal(N: int, dim: int, sigma: float, seed: int, axis_scale=(1.0, 1.0, 1.0)) -> Problem:
    p = diffusion(N, dim, lognormal_field(N, dim, sigma, seed), axis_scale=axis_scale,
                  name=f"lognormal{dim}d_N{N}_s{sigma:g}")
    p.meta.update(sigma=sigma, seed=seed, axis_scale=tuple(axis_scale))
    return p


def piecewise_inclusion(N: int, low: float = 1e-5) -> Problem:
    """2D coefficient `low` inside [1/4,3/4]^2 and 1 elsewhere (§7.2, first case).

    Node (i0, i1) sits at x = ((i0+1)/(N+1), (i1+1)/(N+1)).
    """
    h = 1.0 / (N + 1)
    x = (np.arange(N) + 1) * h
    inside = (x >= 0.25) & (x <= 0.75)
    a = np.where(inside[None, :] & inside[:, None], low, 1.0).reshape(-1)  # [i1, i0]
    return diffusion(N, 2, a, name=f"inclusion2d_N{N}")


def uniform_random(N: int, dim: int, seed: int) -> Problem:
    """Coefficients iid U(0,1] per unknown (§7.2, second case; zero excluded)."""
    rng = np.random.default_rng(seed)
    a = 1.0 - rng.random(N ** dim)  # (0, 1]
    return diffusion(N, dim, a, name=f"urandom{dim}d_N{N}")


def chain(n: int) -> Problem:
    """1D three-point Laplacian (tridiagonal) with coordinates 0..n-1."""
    return diffusion(n, 1, None, name=f"chain_n{n}")


def rhs(n: int, nrhs: int, seed: int) -> np.ndarray:
    """b ~ U(-1,1), (n, nrhs), column-major."""
    rng = np.random.default_rng(seed)
    return np.asfortranarray(rng.uniform(-1.0, 1.0, size=(n, nrhs)))


def poisson_eigenvalues(N: int, dim: int) -> np.ndarray:
    """Closed-form spectrum of the constant stencil: sum_t (2 - 2 cos(j_t pi/(N+1)))."""
    lam1 = 2.0 - 2.0 * np.cos(np.arange(1, N + 1) * np.pi / (N + 1))
    out = lam1
    for _ in range(dim - 1):
        out = (out[:, None] + lam1[None, :]).reshape(-1)
    return np.sort(out)


def poisson_smallest_eigenvector(N: int, dim: int) -> np.ndarray:
    """Product of sin(pi (i_t+1)/(N+1)) over axes, unit 2-norm, in unknown order."""
    s = np.sin(np.pi * (np.arange(N) + 1) / (N + 1))
    v = s
    for _ in range(dim - 1):
        v = (s[:, None] * v[None, :]).reshape(-1)  # slower axis outermost
    return v / np.linalg.norm(v)


# ---------------------------------------------------------------------------
# The named workloads. Seeds: coefficient seed 1000+c, right-hand side 2000+c.
# ---------------------------------------------------------------------------
WORKLOADS = {
    "c1_poisson2d_32": dict(kind="poisson", N=32, dim=2, leaf=16, eps=1e-2, seed=1),
    "c2_lognormal2d_256": dict(kind="lognormal", N=256, dim=2, sigma=2.0, leaf=16, eps=1e-2, seed=2),
    "c3_poisson3d_64": dict(kind="poisson", N=64, dim=3, leaf=64, eps=1e-2, seed=3),
    "c5_aniso3d_128": dict(kind="lognormal", N=128, dim=3, sigma=3.0, leaf=64, eps=1e-2,
                           axis_scale=(1.0, 1e-2, 1e-4), seed=5),
}


def workload(name: str) -> tuple[Problem, dict]:
    w = dict(WORKLOADS[name])
    if w["kind"] == "poisson":
        p = poisson(w["N"], w["dim"])
    else:
        p = lognormal(w["N"], w["dim"], w["sigma"], 1000 + w["seed"],
                      axis_scale=w.get("axis_scale", (1.0, 1.0, 1.0)))
    return p, w


# ---------------------------------------------------------------------------------------
# Serving stream: a sequence of independent SPD systems of mixed sizes
# ---------------------------------------------------------------------------------------
def serving_stream(count: int, seed: int = 4, rate: float | None = None) -> list[dict]:
    """Request specifications for a stream of `count` systems (generated lazily by
    `serving_problem`): half 2-D 5-point on N^2 with N ~ U{64..256}, half 3-D 7-point on N^3
    with N ~ U{16..48}, lognormal cell coefficients (sigma = 1), leaf 16 (2-D) / 64 (3-D),
    eps 1e-2, 1..8 right-hand sides. Arrival times follow a Poisson process of `rate`
    requests per second (all at t = 0 when rate is None). Seeds come from one SeedSequence."""
    ss = np.random.SeedSequence(seed)
    kids = ss.spawn(count + 1)
    top = np.random.default_rng(kids[0])
    t = 0.0
    out = []
    for i in range(count):
        if rate is not None and i > 0:
            t += top.exponential(1.0 / rate)
        dim = 2 if top.random() < 0.5 else 3
        N = int(top.integers(64, 257)) if dim == 2 else int(top.integers(16, 49))
        out.append(dict(rid=i, dim=dim, N=N, sigma=1.0, leaf=16 if dim == 2 else 64, eps=1e-2,
                        nrhs=int(top.integers(1, 9)), seed=int(kids[i + 1].generate_state(1)[0]),
                        arrival=t))
    return out


def serving_problem(spec: dict) -> tuple[Problem, np.ndarray]:
    """Matrix and right-hand sides (n x nrhs, Fortran order, U(-1, 1)) of one request."""
    p = lognormal(spec["N"], spec["dim"], spec["sigma"], spec["seed"] % (2 ** 31))
    b = rhs(p.n, spec["nrhs"], (spec["seed"] + 1) % (2 ** 31))
    return p, b
