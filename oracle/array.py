"""Baselines and redundant-baseline bookkeeping (oracle).

Sec. 2.1 (eq. rime_integral): a baseline is b_pq = r_p - r_q.
Sec. 3.1: the hexagonal array has many physically distinct baselines that
share one vector; the model is evaluated once per unique vector and then
broadcast to every physical baseline (30 unique -> 1785 physical for the
HERA-91 layout with 0 < |b| < 60 m).  A visibility of -b is the complex
conjugate of that of b for a real sky and beam, so "unique" is taken modulo
sign.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


def baseline_pairs(n_ant: int) -> np.ndarray:
    """All pairs (i, j) with i < j, lexicographic order, shape [n_bl][2]."""
    return np.array([(i, j) for i in range(n_ant) for j in range(i + 1, n_ant)],
                    dtype=np.int64).reshape(-1, 2)


def baseline_vectors(ant_enu: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """b_ij = r_i - r_j in metres, shape [n_bl][3] (eq. rime_integral)."""
    return ant_enu[pairs[:, 0]] - ant_enu[pairs[:, 1]]


def _canonical(d: Tuple[int, int]) -> bool:
    return d[0] > 0 or (d[0] == 0 and d[1] > 0)


def unique_lattice(ant_ij: np.ndarray, pairs: np.ndarray):
    """Unique baselines from integer lattice differences, modulo sign.

    Returns (ubl [n_ubl][2] int, u_of_bl [n_bl] int, sign_of_bl [n_bl] +-1).
    The canonical representative has its first non-zero lattice coordinate
    positive; the list is sorted lexicographically.  Physical baseline k has
    lattice vector sign_of_bl[k] * ubl[u_of_bl[k]].
    """
    d = ant_ij[pairs[:, 0]] - ant_ij[pairs[:, 1]]
    canon = []
    signs = np.empty(len(d), dtype=np.int64)
    for k, (a, b) in enumerate(d):
        if a == 0 and b == 0:
            raise ValueError("zero-length baseline (two antennas at one site)")
        if _canonical((a, b)):
            canon.append((int(a), int(b)))
            signs[k] = 1
        else:
            canon.append((int(-a), int(-b)))
            signs[k] = -1
    ubl = sorted(set(canon))
    index = {v: i for i, v in enumerate(ubl)}
    u_of_bl = np.array([index[v] for v in canon], dtype=np.int64)
    return np.asarray(ubl, dtype=np.int64).reshape(-1, 2), u_of_bl, signs


def unique_by_vector(bvec: np.ndarray, decimals: int = 6):
    """Unique baselines by comparing rounded metre vectors, modulo sign.

    An independent route to the same grouping as ``unique_lattice`` (it never
    looks at lattice coordinates); used to cross-check it.
    Returns (n_ubl, groups) where groups maps a canonical rounded vector to
    the sorted list of physical baseline indices with sign.
    """
    groups = {}
    for k, b in enumerate(np.round(bvec[:, :2], decimals) + 0.0):
        key = (float(b[0]), float(b[1]))
        neg = (float(-b[0]) + 0.0, float(-b[1]) + 0.0)
        if key in groups:
            groups[key].append((k, 1))
        elif neg in groups:
            groups[neg].append((k, -1))
        else:
            groups[key] = [(k, 1)]
    return len(groups), groups
