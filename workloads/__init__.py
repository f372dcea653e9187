"""Seeded synthetic inputs for tagged uniform-BLR compression.

This module only *draws* inputs: point clouds on (jittered) grids with their
box tessellation, the Gaussian tagging matrix ``T`` and the per-box Gaussian
test blocks ``G`` / ``H`` (Alg. 2, the draws before the sketch), the planted
exact-rank uniform-BLR test matrix, and the standard workload descriptions.
It contains none of the compression method's arithmetic, so that both the
CPU oracle and the HIP library can consume the same arrays without sharing
code.

Random streams are counter-based (numpy's Philox4x32-10 bit generator,
Salmon et al., SC'11) keyed by ``(seed, stream)``; every array is therefore
reproducible on any host from its seed alone.

Layouts: ``pts`` is ``(N, d)`` C-order; ``T`` is ``(b, ell)`` and ``G``/``H``
are ``(N, r)``, both Fortran (column-major) order, which is the layout the
C ABI expects.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# Philox sub-stream ids (one per kind of random draw).
STREAM_T = 0
STREAM_G = 1
STREAM_H = 2
STREAM_SYNTH_A = 3
STREAM_JITTER = 4
STREAM_ARRIVALS = 5
STREAM_POWER = 6
STREAM_JOBS = 7
STREAM_GAMMA_U = 8
STREAM_GAMMA_V = 9


def rng(seed: int, stream: int) -> np.random.Generator:
    """Counter-based generator keyed by (seed, stream)."""
    key = np.array([int(seed) & 0xFFFFFFFFFFFFFFFF, int(stream)], dtype=np.uint64)
    return np.random.Generator(np.random.Philox(key=key))


def gaussian_colmajor(seed: int, stream: int, nrows: int, ncols: int) -> np.ndarray:
    """nrows x ncols iid N(0,1), column-major; column c holds draws c*nrows..(c+1)*nrows-1."""
    g = rng(seed, stream).standard_normal((ncols, nrows))
    return np.asfortranarray(g.T)


@dataclass
class Geometry:
    """Points in [0,1]^d ordered box-major, plus the box lattice.

    box ``i`` owns rows ``box_ptr[i]:box_ptr[i+1]``; its lattice coordinate is
    ``lattice[i]`` and its id is ``bx + Bx*(by + By*bz)`` (x fastest).
    """
    dim: int
    pts: np.ndarray          # (N, dim) float64
    box_ptr: np.ndarray      # (b+1,) int64
    lattice: np.ndarray      # (b, dim) int32
    boxes_per_axis: tuple
    pts_per_box_axis: tuple

    @property
    def n(self) -> int:
        return int(self.box_ptr[-1])

    @property
    def nboxes(self) -> int:
        return len(self.box_ptr) - 1

    def box_sizes(self) -> np.ndarray:
        return np.diff(self.box_ptr)


def grid_geometry(dim: int, boxes_per_axis, pts_per_box_axis, jitter: float = 0.0,
                  seed: int = 0) -> Geometry:
    """Cell-centred grid with ``boxes_per_axis[t] * pts_per_box_axis[t]`` points on axis t.

    Point coordinate on axis t is ``(g + 1/2) / n_t`` for grid index g, plus an
    optional uniform jitter of ``+-jitter * h_t`` (``jitter < 1/2`` keeps every
    point inside its cell).  Inside a box points are ordered lexicographically
    with x fastest.
    """
    B = tuple(int(v) for v in (boxes_per_axis if np.ndim(boxes_per_axis) else [boxes_per_axis] * dim))
    q = tuple(int(v) for v in (pts_per_box_axis if np.ndim(pts_per_box_axis) else [pts_per_box_axis] * dim))
    assert len(B) == dim and len(q) == dim
    n_axis = [B[t] * q[t] for t in range(dim)]
    nb = int(np.prod(B))
    m = int(np.prod(q))
    lattice = np.zeros((nb, dim), dtype=np.int32)
    for i in range(nb):
        rem = i
        for t in range(dim):
            lattice[i, t] = rem % B[t]
            rem //= B[t]
    # local offsets inside a box, x fastest
    local = np.zeros((m, dim), dtype=np.int64)
    for a in range(m):
        rem = a
        for t in range(dim):
            local[a, t] = rem % q[t]
            rem //= q[t]
    gidx = (lattice[:, None, :].astype(np.int64) * np.array(q)[None, None, :]) + local[None, :, :]
    gidx = gidx.reshape(nb * m, dim)
    h = np.array([1.0 / n_axis[t] for t in range(dim)])
    pts = (gidx + 0.5) * h[None, :]
    if jitter:
        u = rng(seed, STREAM_JITTER).uniform(-1.0, 1.0, size=pts.shape)
        pts = pts + jitter * u * h[None, :]
    box_ptr = np.arange(nb + 1, dtype=np.int64) * m
    return Geometry(dim, np.ascontiguousarray(pts), box_ptr, lattice, B, q)


def tag_matrix(seed: int, nboxes: int, ell: int) -> np.ndarray:
    """Gaussian tagging matrix T (b x ell), column-major (Alg. 2, line forming T)."""
    return gaussian_colmajor(seed, STREAM_T, nboxes, ell)


def gaussian_test_blocks(seed: int, n: int, r: int):
    """The stacked per-box Gaussian blocks G = [G_1; ...; G_b] and H (each N x r)."""
    return gaussian_colmajor(seed, STREAM_G, n, r), gaussian_colmajor(seed, STREAM_H, n, r)


def refinement_gammas(seed: int, nboxes: int, r_lo: int, r: int):
    """Per-box r_lo x r Gaussian mixing blocks (b x r_lo x r each) for the refinement
    sketch of the mixed-precision mode: (gamma_u, gamma_v), C-ordered, so that the flat
    device layout holds entry (a, c) of block l at (l*r_lo + a)*r + c."""
    gu = gaussian_colmajor(seed, STREAM_GAMMA_U, nboxes * r_lo, r)
    gv = gaussian_colmajor(seed, STREAM_GAMMA_V, nboxes * r_lo, r)
    return (np.ascontiguousarray(gu.reshape(nboxes, r_lo, r)),
            np.ascontiguousarray(gv.reshape(nboxes, r_lo, r)))


def planted_exact_rank(geom: Geometry, k: int, seed: int):
    """Dense N x N matrix with planted uniform-BLR structure of exact rank k.

    Pairs of boxes at lattice Chebyshev distance <= 1 (the box itself and its
    touching neighbours) get dense N(0,1) blocks; every other block is
    ``Ustar_i @ S_ij @ Vstar_j.T`` with ``Ustar_i``, ``Vstar_j`` the Q factors of
    Gaussian m x k matrices (signs fixed so R has a positive diagonal) and
    ``S_ij`` N(0,1).  Returns (A column-major, Ustar list, Vstar list).
    """
    g = rng(seed, STREAM_SYNTH_A)
    b = geom.nboxes
    bp = geom.box_ptr
    ustar, vstar = [], []
    for i in range(b):
        for lst in (ustar, vstar):
            mi = int(bp[i + 1] - bp[i])
            q, rr = np.linalg.qr(g.standard_normal((mi, k)))
            q = q * np.sign(np.diag(rr))[None, :]
            lst.append(q)
    A = np.zeros((geom.n, geom.n), order="F")
    lat = geom.lattice.astype(np.int64)
    for i in range(b):
        for j in range(b):
            ri = slice(bp[i], bp[i + 1])
            cj = slice(bp[j], bp[j + 1])
            if np.max(np.abs(lat[i] - lat[j])) <= 1:
                A[ri, cj] = g.standard_normal((bp[i + 1] - bp[i], bp[j + 1] - bp[j]))
            else:
                A[ri, cj] = ustar[i] @ g.standard_normal((k, k)) @ vstar[j].T
    return A, ustar, vstar


def planted_ragged_rank(geom: Geometry, ranks_u, ranks_v, seed: int):
    """Dense N x N matrix with planted uniform-BLR structure of per-box ranks.

    As ``planted_exact_rank`` but far block (i, j) is ``Ustar_i @ S_ij @ Vstar_j.T`` with
    ``Ustar_i`` m_i x ranks_u[i] and ``Vstar_j`` m_j x ranks_v[j] orthonormal and S_ij
    N(0,1), so box row i has far-field rank ranks_u[i] and box column j rank ranks_v[j].
    Returns (A column-major, Ustar list, Vstar list).
    """
    g = rng(seed, STREAM_SYNTH_A)
    b = geom.nboxes
    bp = geom.box_ptr
    ustar, vstar = [], []
    for i in range(b):
        mi = int(bp[i + 1] - bp[i])
        for lst, kk in ((ustar, int(ranks_u[i])), (vstar, int(ranks_v[i]))):
            q, rr = np.linalg.qr(g.standard_normal((mi, kk)))
            lst.append(q * np.sign(np.diag(rr))[None, :])
    A = np.zeros((geom.n, geom.n), order="F")
    lat = geom.lattice.astype(np.int64)
    for i in range(b):
        for j in range(b):
            ri = slice(bp[i], bp[i + 1])
            cj = slice(bp[j], bp[j + 1])
            if np.max(np.abs(lat[i] - lat[j])) <= 1:
                A[ri, cj] = g.standard_normal((bp[i + 1] - bp[i], bp[j + 1] - bp[j]))
            else:
                A[ri, cj] = ustar[i] @ g.standard_normal((ustar[i].shape[1], vstar[j].shape[1])) @ vstar[j].T
    return A, ustar, vstar


def slab_front(B: int, q: int):
    """The frontal face of a thin slab (Section 7.2) as a compression geometry: the n x n face
    points (n = B q, cell-centred in the unit square) in B x B boxes of q x q points, box-major
    as ``grid_geometry``, and the plane index x + n y of every row (the permutation a slab
    operator needs to map plan rows to grid points)."""
    g = grid_geometry(2, B, q)
    n = B * q
    ix = np.floor(g.pts[:, 0] * n).astype(np.int64)
    iy = np.floor(g.pts[:, 1] * n).astype(np.int64)
    return g, ix + n * iy


def blocks_for_rank(n: int, k: int, dim: int) -> int:
    """Block count that balances storage and matvecs for flat uBLR (Section 7 sizing rule)."""
    return int(math.floor(math.sqrt((3 ** dim) * n / k)))


# ---------------------------------------------------------------------------
# Standard workloads (seeds 20250100 + c).
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    dim: int
    boxes_per_axis: tuple
    pts_per_box_axis: tuple
    k: int
    kind: str                 # "planted" (dense A) or a kernel name
    seed: int
    p: int = 10
    extra_tag_cols: int = 3
    jitter: float = 0.0
    notes: str = ""
    extra: dict = field(default_factory=dict)

    def geometry(self) -> Geometry:
        return grid_geometry(self.dim, self.boxes_per_axis, self.pts_per_box_axis,
                             self.jitter, self.seed)

    @property
    def r(self) -> int:
        return self.k + self.p


WORKLOADS = {
    # 64x64 grid, 8x8 boxes of 64 points, planted exact rank 8, dense A.
    "planted_2d_n4096": Workload("planted_2d_n4096", 2, (8, 8), (8, 8), 8, "planted", 20250101),
    # 2D Laplace log|x-y| on a 256x256 grid, 16x16 boxes of 256 points, k=32.
    "laplace2d_n65536": Workload("laplace2d_n65536", 2, (16, 16), (16, 16), 32, "log", 20250102),
    # 3D 1/|x-y| on a 48^3 grid, 8^3 boxes of 216 points, k=48.
    "invr3d_n110592": Workload("invr3d_n110592", 3, (8, 8, 8), (6, 6, 6), 48, "inv_r", 20250103),
    # 2D Laplace on 512x512, 32x32 boxes of 256, k=48 (largest serving job).
    "laplace2d_n262144": Workload("laplace2d_n262144", 2, (32, 32), (16, 16), 48, "log", 20250105),
    # Reduced sizes used for element-wise parity.
    "laplace2d_n16384": Workload("laplace2d_n16384", 2, (8, 8), (16, 16), 32, "log", 20250102),
    "laplace2d_ragged": Workload("laplace2d_ragged", 2, (6, 5), (15, 13), 20, "log", 20250112,
                                 jitter=0.25),
}


def uneven_batch_jobs(njobs: int, seed: int, n_lo: int = 4096, n_hi: int = 131072):
    """Job shapes for batched compression: N target uniform, box shape from a fixed
    menu (m = 64..512), rank uniform in 8..min(64, m-10), kernel from three kinds,
    jittered grids."""
    g = rng(seed, STREAM_JOBS)
    shapes = [(8, 8), (8, 16), (16, 8), (16, 16), (16, 32), (32, 16)]
    kinds = ["log", "exp", "cos"]
    jobs = []
    for t in range(njobs):
        ntarget = int(g.integers(n_lo, n_hi + 1))
        qx, qy = shapes[int(g.integers(0, len(shapes)))]
        m = qx * qy
        B = max(4, int(round(math.sqrt(ntarget / m))))
        k = int(g.integers(8, min(64, m - 10) + 1))
        kind = kinds[int(g.integers(0, 3))]
        jobs.append(Workload(f"job{t}", 2, (B, B), (qx, qy), k, kind, seed * 1000 + t,
                             jitter=0.25))
    return jobs


def irregular_grid_geometry(widths_per_axis, jitter: float = 0.0, seed: int = 0) -> Geometry:
    """Cell-centred grid whose boxes have uneven sizes.

    ``widths_per_axis[t]`` lists the number of grid points of each box along
    axis t (so box sizes differ); the grid has sum(widths) points on that axis.
    Boxes are numbered x fastest and points inside a box are ordered x fastest.
    """
    dim = len(widths_per_axis)
    W = [list(map(int, w)) for w in widths_per_axis]
    B = [len(w) for w in W]
    n_axis = [sum(w) for w in W]
    starts = [np.concatenate([[0], np.cumsum(w)[:-1]]) for w in W]
    nb = int(np.prod(B))
    lattice = np.zeros((nb, dim), dtype=np.int32)
    pts_list, sizes = [], []
    for i in range(nb):
        rem = i
        for t in range(dim):
            lattice[i, t] = rem % B[t]
            rem //= B[t]
        axes = [np.arange(starts[t][lattice[i, t]], starts[t][lattice[i, t]] + W[t][lattice[i, t]])
                for t in range(dim)]
        mesh = np.meshgrid(*axes, indexing="ij")          # axis 0 = x
        g = np.stack([m.reshape(-1, order="F") for m in mesh], axis=1)
        pts_list.append((g + 0.5) / np.array(n_axis, dtype=float))
        sizes.append(g.shape[0])
    pts = np.concatenate(pts_list, axis=0)
    if jitter:
        h = 1.0 / np.array(n_axis, dtype=float)
        pts = pts + jitter * rng(seed, STREAM_JITTER).uniform(-1.0, 1.0, size=pts.shape) * h[None, :]
    box_ptr = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return Geometry(dim, np.ascontiguousarray(pts), box_ptr, lattice, tuple(B), tuple(0 for _ in B))


STREAM_POINTS = 10


def kd_geometry(n: int, dim: int, levels: int, seed: int, nboxes: int = 0):
    """Uniformly random points in [0,1]^dim tessellated by median splits.

    The unit cube is halved ``levels`` times, cycling through the axes; each cut
    lies midway between the two middle points of the cell along that axis, so
    the 2^levels boxes hold n / 2^levels points each, up to one (the geometry of
    Section 7: the domain is subdivided until every box reaches the desired
    cardinality).  Boxes are numbered in tree order and rows are box-major.
    With ``nboxes`` > 0 the count need not be a power of two: a cell that is to
    hold c boxes is cut, along the axis of its depth, into cells for c // 2 and
    c - c // 2 boxes, at the point rank n_cell (c // 2) / c, so every box holds
    n / nboxes points up to one (``levels`` is then ignored).

    Returns (Geometry with ``lattice`` None, near lists, cells) where ``cells``
    is (b, dim, 2) with the closed [lo, hi] range of every box per axis and
    ``near[i]`` lists, ascending, every box whose cell shares a boundary point
    with box i's (box i included, Section 2.5).
    """
    pts0 = rng(seed, STREAM_POINTS).uniform(0.0, 1.0, size=(n, dim))
    target = nboxes if nboxes > 0 else 2 ** levels
    boxes = [(np.arange(n), np.array([[0.0, 1.0]] * dim), target)]
    depth = 0
    while any(c > 1 for _, _, c in boxes):
        ax = depth % dim
        nxt = []
        for idx, cell, c in boxes:
            if c == 1:
                nxt.append((idx, cell, c))
                continue
            order = idx[np.argsort(pts0[idx, ax], kind="stable")]
            c_lo = c // 2
            h = (len(order) * c_lo) // c
            cut = 0.5 * (pts0[order[h - 1], ax] + pts0[order[h], ax])
            lo_cell, hi_cell = cell.copy(), cell.copy()
            lo_cell[ax, 1] = cut
            hi_cell[ax, 0] = cut
            nxt += [(order[:h], lo_cell, c_lo), (order[h:], hi_cell, c - c_lo)]
        boxes = nxt
        depth += 1
    boxes = [(idx, cell) for idx, cell, _ in boxes]
    pts = np.concatenate([pts0[idx] for idx, _ in boxes], axis=0)
    box_ptr = np.concatenate([[0], np.cumsum([len(idx) for idx, _ in boxes])]).astype(np.int64)
    cells = np.stack([cell for _, cell in boxes])
    b = len(boxes)
    near = []
    for i in range(b):
        touch = np.all((cells[:, :, 0] <= cells[i, :, 1]) & (cells[i, :, 0] <= cells[:, :, 1]), axis=1)
        near.append([int(j) for j in np.flatnonzero(touch)])
    geom = Geometry(dim, np.ascontiguousarray(pts), box_ptr, None, (b,), (0,))
    return geom, near, cells
