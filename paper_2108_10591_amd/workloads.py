"""Seeded synthetic inputs for the pipelined BiCGSafe solvers.

This module builds sparse matrices (CSR, FP64 values, int32 column indices,
int64 row pointers) and right-hand sides.  It holds none of the solver's
arithmetic: it is shared by the CPU oracle's tests and by the GPU path so
that both see bit-identical inputs.

The paper's experiments (Section 5) use SuiteSparse matrices that are not
available here; the generators below produce synthetic matrices of the same
classes (3D fluid-dynamics stencils with ~7 nonzeros per row, and uneven
rows with ~27 nonzeros per row) and keep the paper's protocol: the exact
solution is the all-ones vector (``b = A * 1``), ``x0 = 0``, FP64.

Discretisation used for the convection-diffusion families (the paper has no
PDE of its own): vertex-centred finite differences on the unit square/cube
with ``N`` interior nodes per dimension, ``h = 1/(N+1)``, homogeneous
Dirichlet boundaries (neighbours outside the domain are dropped), rows scaled
by ``h^2``.  Diffusion uses the harmonic mean of the two node coefficients on
each face (the node's own coefficient on a boundary face); convection is
first-order upwind.  Node order is lexicographic with x fastest, and columns
are ascending within each row.
"""
from __future__ import annotations

import dataclasses
import functools
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "CSR", "convection_diffusion", "cd2d", "cd3d", "rand_band", "rhs_ones",
    "identity", "diag_distinct", "skew_blocks", "small_nonsym", "random_csr",
    "workload", "WORKLOADS",
]


@dataclasses.dataclass
class CSR:
    """A square sparse matrix in CSR form plus its right-hand side."""
    n: int
    rowptr: np.ndarray  # int64[n+1]
    col: np.ndarray     # int32[nnz]
    val: np.ndarray     # float64[nnz]
    b: np.ndarray | None = None  # float64[n]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self):
        import scipy.sparse as sp
        return sp.csr_matrix((self.val, self.col, self.rowptr), shape=(self.n, self.n))

    def to_dense(self) -> np.ndarray:
        d = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        np.add.at(d, (rows, self.col.astype(np.int64)), self.val)
        return d


def rhs_ones(rowptr: np.ndarray, val: np.ndarray) -> np.ndarray:
    """``b = A * 1``: the FP64 row sums of ``A`` (so the exact solution is all ones)."""
    n = len(rowptr) - 1
    b = np.zeros(n)
    nz = np.diff(rowptr) > 0
    if val.size:
        b[nz] = np.add.reduceat(val, rowptr[:-1][nz])
    return b


def _from_dense_rows(cols: np.ndarray, vals: np.ndarray, mask: np.ndarray, name: str) -> CSR:
    counts = mask.sum(axis=1)
    rowptr = np.zeros(cols.shape[0] + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    col = cols[mask].astype(np.int32)
    val = vals[mask].astype(np.float64)
    return CSR(cols.shape[0], rowptr, col, val, rhs_ones(rowptr, val), name)


def convection_diffusion(N: int, velocity, kfield: np.ndarray | None = None, name: str = "") -> CSR:
    """Upwind convection-diffusion operator on an ``N^d`` grid (d = len(velocity)).

    ``kfield`` holds the diffusion coefficient per node, shaped ``(N,)*d``
    with the x axis last (fastest); ``None`` means constant 1.
    """
    d = len(velocity)
    n = N ** d
    h = 1.0 / (N + 1)
    shape = (N,) * d
    k = np.ones(shape) if kfield is None else np.asarray(kfield, dtype=np.float64).reshape(shape)
    # axis a of the numpy array holds grid direction (d-1-a); direction 0 (x) is fastest
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    # slots: -e_{d-1} .. -e_0, diag, +e_0 .. +e_{d-1}: ascending column offsets
    nslot = 2 * d + 1
    cols = np.zeros((n, nslot), dtype=np.int64)
    vals = np.zeros((n, nslot))
    mask = np.zeros((n, nslot), dtype=bool)
    diag = np.zeros(shape)
    cols[:, d] = idx.ravel()
    mask[:, d] = True
    for direction in range(d):
        ax = d - 1 - direction
        stride = N ** direction
        vd = float(velocity[direction])
        for sgn in (-1, +1):
            slot = d + sgn * (direction + 1)
            # neighbour Q = P + sgn * e_direction, and whether it is inside
            kq = np.roll(k, -sgn, axis=ax)
            pos = np.arange(N).reshape([-1 if a == ax else 1 for a in range(d)])
            inside = (pos + sgn >= 0) & (pos + sgn < N)
            inside = np.broadcast_to(inside, shape)
            kf = np.where(inside, 2.0 * k * kq / (k + kq), k)
            diag += kf
            off = -kf
            upstream = (vd > 0 and sgn < 0) or (vd < 0 and sgn > 0)
            if upstream:
                off = off - h * abs(vd)
            cols[:, slot] = (idx + sgn * stride).ravel()
            vals[:, slot] = np.where(inside, off, 0.0).ravel()
            mask[:, slot] = inside.ravel()
        diag += h * abs(vd)
    vals[:, d] = diag.ravel()
    return _from_dense_rows(cols, vals, mask, name or f"cd{d}d_{N}")


def _convection_diffusion_2d_many(N: int, vx: np.ndarray, vy: np.ndarray, kfields: np.ndarray):
    """convection_diffusion(N, (vx[j], vy[j]), kfields[j]) for every j at once: the same
    per-entry arithmetic in the same order, vectorised over the problems, which share
    the sparsity pattern.  Returns (rowptr, col, values[m, nnz])."""
    m = len(vx)
    d, n = 2, N * N
    h = 1.0 / (N + 1)
    k = np.asarray(kfields, dtype=np.float64).reshape(m, N, N)
    idx = np.arange(n, dtype=np.int64).reshape(N, N)
    nslot = 2 * d + 1
    cols = np.zeros((n, nslot), dtype=np.int64)
    vals = np.zeros((m, n, nslot))
    mask = np.zeros((n, nslot), dtype=bool)
    diag = np.zeros((m, N, N))
    cols[:, d] = idx.ravel()
    mask[:, d] = True
    for direction, vel in enumerate((np.asarray(vx, np.float64), np.asarray(vy, np.float64))):
        ax = d - 1 - direction
        stride = N ** direction
        speed = (h * np.abs(vel))[:, None, None]
        for sgn in (-1, +1):
            slot = d + sgn * (direction + 1)
            kq = np.roll(k, -sgn, axis=ax + 1)
            pos = np.arange(N).reshape([-1 if a == ax else 1 for a in range(d)])
            inside = np.broadcast_to((pos + sgn >= 0) & (pos + sgn < N), (N, N))
            kf = np.where(inside, 2.0 * k * kq / (k + kq), k)
            diag += kf
            off = -kf
            upstream = ((vel > 0) & (sgn < 0)) | ((vel < 0) & (sgn > 0))
            off = np.where(upstream[:, None, None], off - speed, off)
            cols[:, slot] = (idx + sgn * stride).ravel()
            vals[:, :, slot] = np.where(inside, off, 0.0).reshape(m, n)
            mask[:, slot] = inside.ravel()
        diag += speed
    vals[:, :, d] = diag.reshape(m, n)
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    return rowptr, cols[mask].astype(np.int32), vals[:, mask]


def cd2d(N: int = 64, beta: float = 10.0, kfield=None) -> CSR:
    """2D 5-point upwind convection-diffusion, convection (beta, beta)."""
    return convection_diffusion(N, (beta, beta), kfield, name=f"cd2d_{N}")


def cd3d(N: int = 128, beta: float = 20.0, seed: int = 2108) -> CSR:
    """3D 7-point upwind convection-diffusion, convection (1,1,1)*beta, diffusion exp(N(0,1)) per node."""
    rng = np.random.default_rng(seed)
    k = np.exp(rng.standard_normal((N, N, N)))
    return convection_diffusion(N, (beta, beta, beta), k, name=f"cd3d_{N}")


def rand_band(n: int = 1_000_000, seed: int = 10591, gamma: float = 1.37629, lmin: int = 3,
              lmax: int = 200, band: int = 5000, diag_factor: float = 1.1) -> CSR:
    """Random nonsymmetric CSR with uneven rows.

    Row lengths (diagonal included) follow p(L) ~ L^-gamma on [lmin, lmax]
    (gamma = 1.37629 gives mean 27 on [3, 200]), capped by the columns the band
    holds; off-diagonal columns are drawn
    uniformly without replacement within +-band of the diagonal; off-diagonal
    values are U(-1, 1) and the diagonal is diag_factor times the row's
    absolute off-diagonal sum.
    """
    rng = np.random.default_rng(seed)
    lengths = np.arange(lmin, lmax + 1)
    p = lengths.astype(np.float64) ** -gamma
    p /= p.sum()
    L = rng.choice(lengths, size=n, p=p)
    # a row cannot hold more off-diagonal entries than its band has columns
    r = np.arange(n, dtype=np.int64)
    cand = np.minimum(n - 1, r + band) - np.maximum(0, r - band)
    m = np.minimum(L - 1, cand).astype(np.int64)
    rows = np.repeat(r, m)
    lo = np.maximum(0, rows - band)
    hi = np.minimum(n - 1, rows + band)
    width = hi - lo  # candidates excluding the diagonal
    c = lo + rng.integers(0, width)
    c += c >= rows
    # redraw duplicated (row, col) pairs until every row's columns are distinct
    while True:
        key = rows * n + c
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(ks.size, dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        redo = order[dup]
        cr = lo[redo] + rng.integers(0, width[redo])
        cr += cr >= rows[redo]
        c[redo] = cr
    rows = rows[order]
    c = c[order]
    off = rng.uniform(-1.0, 1.0, size=c.size)
    absum = np.zeros(n)
    np.add.at(absum, rows, np.abs(off))
    allrows = np.concatenate([rows, np.arange(n, dtype=np.int64)])
    allcols = np.concatenate([c, np.arange(n, dtype=np.int64)])
    allvals = np.concatenate([off, diag_factor * absum])
    order = np.argsort(allrows * n + allcols, kind="stable")
    col = allcols[order].astype(np.int32)
    val = allvals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(m + 1, out=rowptr[1:])
    return CSR(n, rowptr, col, val, rhs_ones(rowptr, val), f"rand_band_{n}")


# ----------------------------------------------------------------------------
# Small matrices with known structure (for closed-form and special-case checks)
# ----------------------------------------------------------------------------

def _from_dense(a: np.ndarray, name: str, b: np.ndarray | None = None) -> CSR:
    n = a.shape[0]
    mask = a != 0.0
    counts = mask.sum(axis=1)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    cols = np.nonzero(mask)[1].astype(np.int32)
    val = a[mask].astype(np.float64)
    bb = rhs_ones(rowptr, val) if b is None else np.asarray(b, dtype=np.float64)
    return CSR(n, rowptr, cols, val, bb, name)


def identity(n: int, seed: int = 0) -> CSR:
    """A = I with a random right-hand side."""
    rng = np.random.default_rng(seed)
    return _from_dense(np.eye(n), f"eye_{n}", rng.uniform(0.5, 1.5, n))


def diag_distinct(n: int, eigs, seed: int = 0) -> CSR:
    """Diagonal A whose entries take exactly the distinct values ``eigs``, each at least once."""
    rng = np.random.default_rng(seed)
    eigs = np.asarray(eigs, dtype=np.float64)
    lam = np.concatenate([eigs, rng.choice(eigs, size=n - len(eigs))])
    lam = lam[rng.permutation(n)]
    return _from_dense(np.diag(lam), f"diag{len(eigs)}_{n}", lam * rng.uniform(0.5, 1.5, n))


def skew_blocks(n: int, seed: int = 0) -> CSR:
    """Block-diagonal skew-symmetric matrix of 2x2 blocks [[0, c], [-c, 0]] with integer c and b.

    With integer entries every product is exact, so ``(r, A r)`` is exactly zero.
    """
    assert n % 2 == 0
    rng = np.random.default_rng(seed)
    a = np.zeros((n, n))
    for k in range(0, n, 2):
        c = float(rng.integers(1, 5))
        a[k, k + 1] = c
        a[k + 1, k] = -c
    return _from_dense(a, f"skew_{n}", rng.integers(1, 5, n).astype(np.float64))


def small_nonsym(n: int, seed: int, density: float = 0.3, dominance: float = 1.5) -> CSR:
    """Random sparse nonsymmetric matrix, diagonally dominant by ``dominance``; b = A*1."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(-1.0, 1.0, (n, n)) * (rng.random((n, n)) < density)
    np.fill_diagonal(a, 0.0)
    np.fill_diagonal(a, dominance * np.abs(a).sum(axis=1) + 1.0)
    return _from_dense(a, f"nonsym_{n}_{seed}")


def random_csr(n: int, seed: int, lengths=None, unsorted: bool = False, duplicates: bool = False) -> CSR:
    """Random CSR with a given row-length multiset, for SpMV checks.

    ``lengths`` may contain zeros (empty rows) and long rows.  Columns are
    uniform over [0, n); with ``unsorted`` the columns of each row are
    shuffled, and with ``duplicates`` some (row, col) pairs repeat.
    """
    rng = np.random.default_rng(seed)
    if lengths is None:
        lengths = rng.integers(0, 40, n)
    lengths = np.asarray(lengths, dtype=np.int64)
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(lengths, out=rowptr[1:])
    nnz = int(rowptr[-1])
    col = rng.integers(0, n, nnz).astype(np.int32)
    if not duplicates:
        # distinct sorted columns per row (a row longer than n necessarily repeats some)
        for i in np.nonzero(lengths)[0]:
            s, e = rowptr[i], rowptr[i + 1]
            m = int(e - s)
            col[s:e] = np.sort(rng.choice(n, size=m, replace=m > n))
    if unsorted:
        for i in np.nonzero(lengths)[0]:
            s, e = rowptr[i], rowptr[i + 1]
            col[s:e] = col[s:e][rng.permutation(int(e - s))]
    val = rng.uniform(-1.0, 1.0, nnz)
    return CSR(n, rowptr, col, val, rhs_ones(rowptr, val), f"random_{n}_{seed}")


# ----------------------------------------------------------------------------
# Batches of independent systems
# ----------------------------------------------------------------------------

@dataclasses.dataclass
class Batch:
    """Independent systems A_k x_k = b_k, solved together."""
    systems: list
    name: str = ""

    @property
    def nsys(self) -> int:
        return len(self.systems)

    def sys_ptr(self) -> np.ndarray:
        """int64[nsys+1]: first row of each system in the concatenation."""
        p = np.zeros(self.nsys + 1, dtype=np.int64)
        np.cumsum([A.n for A in self.systems], out=p[1:])
        return p

    def concat(self) -> CSR:
        """The block-diagonal matrix of all systems (global column indices) and the
        concatenated right-hand sides."""
        ptr = self.sys_ptr()
        rowptr = [np.zeros(1, dtype=np.int64)]
        off = 0
        for A in self.systems:
            rowptr.append(A.rowptr[1:] + off)
            off += A.nnz
        col = np.concatenate([A.col.astype(np.int64) + ptr[k] for k, A in enumerate(self.systems)])
        return CSR(int(ptr[-1]), np.concatenate(rowptr), col.astype(np.int32),
                   np.concatenate([A.val for A in self.systems]),
                   np.concatenate([A.b for A in self.systems]), self.name)


def cd2d_batch(nsys: int = 512, seed: int = 3, nmin: int = 32, nmax: int = 256,
               beta_max: float = 50.0, sigma: float = 0.5) -> Batch:
    """``nsys`` 2D upwind convection-diffusion systems: grid side N uniform in
    [nmin, nmax], convection (beta, beta) with beta ~ U(0, beta_max), diffusion
    exp(N(0, sigma^2)) per node; b = A*1 for each."""
    rng = np.random.default_rng(seed)
    systems = []
    for k in range(nsys):
        N = int(rng.integers(nmin, nmax + 1))
        beta = float(rng.uniform(0.0, beta_max))
        kf = np.exp(sigma * rng.standard_normal((N, N)))
        A = convection_diffusion(N, (beta, beta), kf, name=f"cd2d_{N}_{k}")
        systems.append(A)
    return Batch(systems, f"cd2d_batch_{nsys}")


def grf(count: int, N: int, corr_len: float, rng) -> np.ndarray:
    """``count`` Gaussian random fields on the N x N interior nodes of the unit
    square (spacing 1/(N+1)): zero mean, unit variance, covariance
    exp(-d^2 / (2 corr_len^2)).  White noise filtered with the square root of
    that covariance's spectral density, exp(-2 pi^2 corr_len^2 |f|^2), on a
    periodic grid twice as large, of which one quarter is kept (so that the
    wrap-around does not couple opposite edges)."""
    M = 2 * N
    f = np.fft.fftfreq(M, d=1.0 / (N + 1))
    FX, FY = np.meshgrid(f, f, indexing="ij")
    dens = np.exp(-2.0 * np.pi ** 2 * corr_len ** 2 * (FX ** 2 + FY ** 2))
    amp = np.sqrt(dens)
    out = np.empty((count, N, N))
    # the noise is drawn in chunk order; the transforms of the chunks are independent
    # and run on threads (numpy's FFT releases the interpreter lock): the same values
    # as one after another
    chunks = []
    for c0 in range(0, count, 128):
        m = min(128, count - c0)
        chunks.append((c0, m, rng.standard_normal((m, M, M))))

    def filtered(chunk):
        c0, m, z = chunk
        out[c0:c0 + m] = np.fft.ifft2(np.fft.fft2(z) * amp).real[:, :N, :N]

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        list(ex.map(filtered, chunks))
    return out / np.sqrt(dens.sum() / M ** 2)


def _threads() -> int:
    """Worker threads for the generators: the CPUs this process may use, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def varcoef_problems(count: int, N: int = 128, seed: int = 0, corr_len: float = 0.1,
                     vmax: float = 30.0):
    """Variable-coefficient 2D convection-diffusion problems for the learned
    initial guess: diffusion exp(g) with g a unit-variance Gaussian random field
    of correlation length ``corr_len``, convection v = U(0, vmax) (cos t, sin t)
    with t ~ U(0, 2 pi), unit source (b = h^2 per row, the rows being scaled by
    h^2).  Returns the Batch and the network input per problem,
    float32[count, N, N, 3] = (g, v_x / vmax, v_y / vmax) at every node."""
    rng = np.random.default_rng(seed)
    g = grf(count, N, corr_len, rng)
    speed = rng.uniform(0.0, vmax, count)
    theta = rng.uniform(0.0, 2.0 * np.pi, count)
    vx, vy = speed * np.cos(theta), speed * np.sin(theta)
    h2 = 1.0 / (N + 1) ** 2

    def assemble(c0):  # chunks of problems, independent of each other, on threads
        m = min(64, count - c0)
        rowptr, col, vals = _convection_diffusion_2d_many(N, vx[c0:c0 + m], vy[c0:c0 + m],
                                                         np.exp(g[c0:c0 + m]))
        return [CSR(N * N, rowptr, col, vals[j], np.full(N * N, h2), f"varcoef_{N}_{c0 + j}")
                for j in range(m)]

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        systems = [A for part in ex.map(assemble, range(0, count, 64)) for A in part]
    feats = np.empty((count, N, N, 3), dtype=np.float32)
    feats[..., 0] = g
    feats[..., 1] = (vx / vmax)[:, None, None]
    feats[..., 2] = (vy / vmax)[:, None, None]
    return Batch(systems, f"varcoef_{N}_{count}_{seed}"), feats


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

WORKLOADS = {
    # 2D 64x64, convection (10, 10), diffusion 1, tol 1e-10
    "cd2d_64": dict(tol=1e-10, make=lambda: cd2d(64, 10.0)),
    # 3D 128^3, convection (20, 20, 20), diffusion exp(N(0,1)) seed 2108, tol 1e-8
    "cd3d_128": dict(tol=1e-8, make=lambda: cd3d(128, 20.0, 2108)),
    # random power-law rows in [3, 200] (mean 27), band +-5000, n = 1M, seed 10591, tol 1e-10
    "rand_band_1m": dict(tol=1e-10, make=lambda: rand_band(1_000_000, 10591)),
}


BATCHES = {
    # 512 systems, N ~ U[32, 256], beta ~ U(0, 50), diffusion exp(N(0, 0.5^2)), tol 1e-8
    "cd2d_batch_512": dict(tol=1e-8, make=lambda: cd2d_batch(512, 3)),
}


@functools.lru_cache(maxsize=2)
def batch(name: str) -> Batch:
    """Build (and cache per process) one of the named batches."""
    return BATCHES[name]["make"]()


@functools.lru_cache(maxsize=4)
def workload(name: str) -> CSR:
    """Build (and cache per process) one of the named workloads."""
    return WORKLOADS[name]["make"]()
