"""Icosahedral horizontal grid hierarchy and its spherical geometry (oracle).

Paper: the horizontal grid is an icosahedral grid whose points are projected
onto the sphere and whose coarse triangles each consist of four finer ones
(Section 4.1, Section 4.2). The geometric quantities of the finite-volume
scheme (cell areas |T|, centres r_T, edge lengths |S_TT'| and outward edge
normals n_TT') are those of Appendix A.

Readings (the paper leaves these open):
  * base icosahedron: poles (0,0,+-1) plus two rings of five vertices at
    latitude +-atan(1/2), longitudes 72 i (north ring) and 36 + 72 i (south
    ring); faces listed north cap, upper band, lower band, south cap, each
    counter-clockwise seen from outside;
  * refinement of face (a,b,c): children (a,m_ab,m_ca), (m_ab,b,m_bc),
    (m_ca,m_bc,c), (m_ab,m_bc,m_ca) with m = normalise((p+q)/2); child i of
    cell P is cell 4P+i; neighbour j of (a,b,c) lies across edge (a,b),
    (b,c), (c,a) for j = 0, 1, 2;
  * cell centre r_T: spherical circumcentre; |T|: spherical excess; |S_TT'|:
    great-circle arc; n_TT': unit tangent normal to the edge pointing out of
    T; the centre-to-centre factor uses 3-D chord vectors as printed.

Pins (tests/test_oracle_mesh.py): Euler counts, symmetric 3-regular
adjacency, nesting of children, total area 4 pi, children areas summing to
the parent's, equidistant circumcentres, symmetric positive edge factors.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _normalise(v: np.ndarray) -> np.ndarray:
    return v / np.sqrt(np.sum(v * v, axis=-1, keepdims=True))


def _dot(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    return np.sum(a * b, axis=-1)


def icosahedron():
    """The 12 vertices and 20 counter-clockwise faces of the base grid."""
    lat = math.atan(0.5)
    verts = np.zeros((12, 3))
    verts[0] = (0.0, 0.0, 1.0)
    verts[11] = (0.0, 0.0, -1.0)
    for i in range(5):
        lon_n = 2.0 * math.pi * i / 5.0
        lon_s = lon_n + math.pi / 5.0
        verts[1 + i] = (math.cos(lat) * math.cos(lon_n), math.cos(lat) * math.sin(lon_n), math.sin(lat))
        verts[6 + i] = (math.cos(lat) * math.cos(lon_s), math.cos(lat) * math.sin(lon_s), -math.sin(lat))
    faces = []
    north = [1 + i for i in range(5)]
    south = [6 + i for i in range(5)]
    for i in range(5):
        faces.append((0, north[i], north[(i + 1) % 5]))
    for i in range(5):
        faces.append((north[i], south[i], north[(i + 1) % 5]))
    for i in range(5):
        faces.append((north[(i + 1) % 5], south[i], south[(i + 1) % 5]))
    for i in range(5):
        faces.append((11, south[(i + 1) % 5], south[i]))
    return verts, np.array(faces, dtype=np.int64)


def _edge_keys(faces: np.ndarray, nv: int) -> np.ndarray:
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    p = np.stack([a, b, c], axis=1)
    q = np.stack([b, c, a], axis=1)
    return np.minimum(p, q) * nv + np.maximum(p, q)


def refine(verts: np.ndarray, faces: np.ndarray):
    """One step of 1:4 refinement with midpoints projected onto the sphere."""
    nv = len(verts)
    keys = _edge_keys(faces, nv)
    uniq, inv = np.unique(keys.ravel(), return_inverse=True)
    lo, hi = uniq // nv, uniq % nv
    mids = _normalise(0.5 * (verts[lo] + verts[hi]))
    mid_id = nv + inv.reshape(-1, 3)          # ids of m_ab, m_bc, m_ca
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    mab, mbc, mca = mid_id[:, 0], mid_id[:, 1], mid_id[:, 2]
    kids = np.stack(
        [
            np.stack([a, mab, mca], axis=1),
            np.stack([mab, b, mbc], axis=1),
            np.stack([mca, mbc, c], axis=1),
            np.stack([mab, mbc, mca], axis=1),
        ],
        axis=1,
    )
    return np.concatenate([verts, mids]), kids.reshape(-1, 3)


def neighbours(faces: np.ndarray, nv: int) -> np.ndarray:
    """nbr[T, j] = the cell sharing edge j of T (every edge has two cells)."""
    flat = _edge_keys(faces, nv).ravel()
    order = np.argsort(flat, kind="stable")
    srt = flat[order]
    if not np.all(srt[0::2] == srt[1::2]):
        raise ValueError("mesh is not closed: an edge is not shared by exactly two cells")
    first, second = order[0::2], order[1::2]
    nbr = np.empty(len(flat), dtype=np.int64)
    nbr[first] = second // 3
    nbr[second] = first // 3
    return nbr.reshape(-1, 3)


@dataclass
class Mesh:
    refinement: int
    verts: np.ndarray     # [nv, 3]
    faces: np.ndarray     # [n, 3] vertex ids, counter-clockwise
    nbr: np.ndarray       # [n, 3]
    centre: np.ndarray    # [n, 3] spherical circumcentres
    area: np.ndarray      # [n] spherical areas
    arc: np.ndarray       # [n, 3] great-circle length of edge j
    normal: np.ndarray    # [n, 3, 3] outward unit tangent normal of edge j
    g: np.ndarray         # [n, 3] |S| n.(r_T' - r_T) / |r_T' - r_T|^2

    @property
    def n(self) -> int:
        return len(self.faces)


def geometry(refinement: int, verts: np.ndarray, faces: np.ndarray) -> Mesh:
    nbr = neighbours(faces, len(verts))
    A, B, C = verts[faces[:, 0]], verts[faces[:, 1]], verts[faces[:, 2]]
    centre = _normalise(np.cross(B - A, C - A))
    # spherical excess E: tan(E/2) = |a.(b x c)| / (1 + a.b + b.c + c.a)
    num = np.abs(_dot(A, np.cross(B, C)))
    den = 1.0 + _dot(A, B) + _dot(B, C) + _dot(C, A)
    area = 2.0 * np.arctan2(num, den)
    arc = np.zeros((len(faces), 3))
    normal = np.zeros((len(faces), 3, 3))
    g = np.zeros((len(faces), 3))
    for j, (P, Q) in enumerate(((A, B), (B, C), (C, A))):
        cr = np.cross(P, Q)
        arc[:, j] = np.arctan2(np.sqrt(_dot(cr, cr)), _dot(P, Q))
        # edge P->Q of a counter-clockwise face has the interior on its left,
        # where P x Q points; the outward normal is the opposite direction
        nrm = _normalise(np.cross(Q, P))
        normal[:, j] = nrm
        d = centre[nbr[:, j]] - centre
        g[:, j] = arc[:, j] * _dot(nrm, d) / _dot(d, d)
    return Mesh(refinement, verts, faces, nbr, centre, area, arc, normal, g)


def hierarchy(refinement: int) -> list[Mesh]:
    """Meshes for refinements 0..refinement (index = refinement)."""
    verts, faces = icosahedron()
    out = [geometry(0, verts, faces)]
    for r in range(1, refinement + 1):
        verts, faces = refine(verts, faces)
        out.append(geometry(r, verts, faces))
    return out
