"""Structured P1 triangulation of the unit square (oracle).

N x N nodes at (i h, j h), h = 1/(N-1).  Every cell (i, j) is cut along its
"/" diagonal into T1 = {(i,j), (i+1,j), (i+1,j+1)} and
T2 = {(i,j), (i+1,j+1), (i,j+1)}; element e = 2 (j (N-1) + i) + {0, 1}.
Boundary nodes carry the homogeneous Dirichlet condition A = 0 and are not
unknowns; interior node (i, j) has DoF index (j-1)(N-2) + (i-1).

The paper's FE model (Eq. (2)) uses H(curl) functions w_i; in 2-D with
A = A_z e_z these are w_i = N_i e_z with P1 nodal N_i, so the element
matrices of Eq. (4) reduce to the scalar P1 ones built in ``fem``.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Mesh:
    n: int                 # nodes per side
    h: float
    xy: np.ndarray         # [n*n, 2] node coordinates
    tri: np.ndarray        # [n_elem, 3] node indices (counter-clockwise)
    centroid: np.ndarray   # [n_elem, 2]
    area: np.ndarray       # [n_elem]
    dof: np.ndarray        # [n*n] interior DoF index or -1
    n_dof: int


def build(n: int) -> Mesh:
    if n < 3:
        raise ValueError("need at least 3 nodes per side")
    h = 1.0 / (n - 1)
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xy = np.stack([ii.ravel() * h, jj.ravel() * h], axis=1)
    tris = []
    for j in range(n - 1):
        for i in range(n - 1):
            p00 = j * n + i
            p10 = j * n + i + 1
            p11 = (j + 1) * n + i + 1
            p01 = (j + 1) * n + i
            tris.append((p00, p10, p11))
            tris.append((p00, p11, p01))
    tri = np.asarray(tris, dtype=np.int64)
    v = xy[tri]
    centroid = v.mean(axis=1)
    e1 = v[:, 1] - v[:, 0]
    e2 = v[:, 2] - v[:, 0]
    area = 0.5 * (e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0])
    dof = -np.ones(n * n, dtype=np.int64)
    k = 0
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            dof[j * n + i] = k
            k += 1
    return Mesh(n, h, xy, tri, centroid, area, dof, k)


def in_box(c: np.ndarray, box) -> np.ndarray:
    x0, x1, y0, y1 = box
    return (c[:, 0] >= x0) & (c[:, 0] <= x1) & (c[:, 1] >= y0) & (c[:, 1] <= y1)


def conductor_mask(m: Mesh, problem) -> np.ndarray:
    """Elements whose centroid lies in the conductor box."""
    return in_box(m.centroid, problem.conductor)


def strip_mask(m: Mesh, problem) -> np.ndarray:
    """Elements whose centroid lies in the source strip (full height)."""
    x0, x1 = problem.strip
    return (m.centroid[:, 0] >= x0) & (m.centroid[:, 0] <= x1)
