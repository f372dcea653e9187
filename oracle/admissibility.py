"""Strong admissibility on a box lattice (oracle; test infrastructure only).

Section 2.5: the neighbours of a box are the boxes sharing a boundary with it,
itself included, at most 3^d of them; the far field is the complement.  On a
regular lattice of boxes "sharing a boundary" (faces, edges or corners) is
lattice Chebyshev distance <= 1.
"""
from __future__ import annotations

import numpy as np


def near_lists(lattice: np.ndarray) -> list[list[int]]:
    """N_i = {j : max_t |lat_i,t - lat_j,t| <= 1}, ascending, i included (Section 2.5)."""
    lat = np.asarray(lattice, dtype=np.int64)
    b = lat.shape[0]
    out = []
    for i in range(b):
        out.append([j for j in range(b) if int(np.max(np.abs(lat[i] - lat[j]))) <= 1])
    return out


def far_lists(near: list[list[int]], nboxes: int) -> list[list[int]]:
    """F_i = [b] minus N_i, ascending (Section 2.5, definition of the far field)."""
    return [[j for j in range(nboxes) if j not in set(ni)] for ni in near]


def colours(lattice: np.ndarray) -> np.ndarray:
    """Probe colour of each box for step (III) (Section 6.1, the sparse identity probes).

    Reading: colour(i) = sum_t (lat_i,t mod 3) 3^t, which gives 3^d colour
    classes such that no two boxes of one class are both neighbours of the
    same box; in 1D this puts the identity blocks on boxes 1, 4, 7 as in the
    probe figure.
    """
    lat = np.asarray(lattice, dtype=np.int64)
    d = lat.shape[1]
    return np.array([sum(int(lat[i, t] % 3) * 3 ** t for t in range(d)) for i in range(lat.shape[0])],
                    dtype=np.int64)


def greedy_colours(near: list[list[int]]) -> np.ndarray:
    """Probe colours for caller-given neighbour lists (reading of Section 6.1 for a general
    neighbour relation): the probes need every box's neighbours to carry distinct colours,
    i.e. two boxes that share a neighbour differ.  Boxes are taken in index order and each
    gets the smallest colour not used by an earlier box within two neighbour steps."""
    b = len(near)
    colour = [-1] * b
    for i in range(b):
        taken = set()
        for j in near[i]:
            for l in near[j]:
                if colour[l] >= 0:
                    taken.add(colour[l])
        c = 0
        while c in taken:
            c += 1
        colour[i] = c
    return np.array(colour, dtype=np.int64)


def lists_and_colours(lattice, near=None):
    """(near, colours): the lattice rule and its mod-3 colours, or the given lists with
    greedy colours."""
    if near is None:
        return near_lists(lattice), colours(lattice)
    near = [sorted(int(j) for j in n) for n in near]
    return near, greedy_colours(near)


def num_tag_columns(near: list[list[int]], extra: int = 3) -> int:
    """Columns of T: one more than the largest neighbour count (Section 4.1), plus
    ``extra`` columns that make every null space at least (extra+1)-dimensional
    (Section 5.3; the experiments use 3 additional columns, Section 7)."""
    return max(len(n) for n in near) + 1 + int(extra)
