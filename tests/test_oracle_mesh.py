"""Pins of the oracle's icosahedral mesh and geometry (paper Section 4.2,
Appendix A): Euler counts, adjacency, nesting, closed-form base geometry,
area conservation, circumcentres and symmetric positive edge factors."""
import math
import os

import numpy as np
import pytest

from oracle import mesh

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "icosahedron_base.txt")


@pytest.fixture(scope="module")
def meshes():
    return mesh.hierarchy(4)


def _golden():
    out = {}
    for line in open(GOLDEN):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            out[k] = float(v)
    return out


def test_euler_counts(meshes):
    for m in meshes:
        n = m.refinement
        assert m.n == 20 * 4 ** n
        assert len(np.unique(m.faces)) == 10 * 4 ** n + 2      # V - E + F = 2
        # every edge shared by exactly two cells: 3F = 2E, E = 30 4^n
        f = np.asarray(m.faces)
        e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
        e.sort(axis=1)
        _, counts = np.unique(e, axis=0, return_counts=True)
        assert len(counts) == 30 * 4 ** n and np.all(counts == 2)


def test_adjacency(meshes):
    for m in meshes:
        T = np.arange(m.n)
        nb = m.nbr
        assert np.all(nb != T[:, None])
        assert np.all(nb[:, 0] != nb[:, 1]) and np.all(nb[:, 1] != nb[:, 2]) and np.all(nb[:, 0] != nb[:, 2])
        back = (nb[nb] == T[:, None, None]).sum(axis=2)          # T appears once among nbr[nbr[T, j]]
        assert np.all(back == 1)
        # cells across edge j share exactly the two vertices of that edge
        for j, (p, q) in enumerate(((0, 1), (1, 2), (2, 0))):
            e = np.sort(m.faces[:, [p, q]], axis=1)
            other = m.faces[nb[:, j]]
            assert np.all((other == e[:, :1]).any(axis=1) & (other == e[:, 1:]).any(axis=1))


def test_nesting(meshes):
    for coarse, fine in zip(meshes[:-1], meshes[1:]):
        kids = fine.faces.reshape(-1, 4, 3)
        a, b, c = coarse.faces[:, 0], coarse.faces[:, 1], coarse.faces[:, 2]
        assert np.all(kids[:, 0, 0] == a) and np.all(kids[:, 1, 1] == b) and np.all(kids[:, 2, 2] == c)
        # the middle child is made of the three edge midpoints
        mids = fine.verts[kids[:, 3]]
        va, vb, vc = (fine.verts[x] for x in (a, b, c))
        for (p, q), col in (((va, vb), 0), ((vb, vc), 1), ((vc, va), 2)):
            s = p + q
            assert np.allclose(mids[:, col], s / np.linalg.norm(s, axis=1, keepdims=True), atol=1e-15)
        # children areas tile the parent exactly
        assert np.allclose(fine.area.reshape(-1, 4).sum(axis=1), coarse.area, rtol=1e-13, atol=0)


def test_closed_form_base_geometry(meshes):
    gold = _golden()
    m = meshes[0]
    assert np.allclose(m.arc, gold["edge_arc"], rtol=1e-15, atol=0)
    assert np.allclose(m.area, gold["face_area"], rtol=2e-15, atol=0)
    d = np.linalg.norm(m.centre[m.nbr] - m.centre[:, None, :], axis=2)
    assert np.allclose(d, gold["centre_chord"], rtol=1e-14, atol=0)
    assert np.allclose(m.g, gold["flux_factor"], rtol=1e-14, atol=0)


def test_total_area_and_centres(meshes):
    for m in meshes:
        assert abs(m.area.sum() - 4 * math.pi) < 1e-12
        assert np.all(m.area > 0)
        dist = np.linalg.norm(m.verts[m.faces] - m.centre[:, None, :], axis=2)
        assert np.allclose(dist, dist[:, :1], rtol=0, atol=2e-14)
        assert np.allclose(np.linalg.norm(m.centre, axis=1), 1.0, atol=1e-15)
        # the centre lies on the outward side of its face
        assert np.all(np.sum(m.centre * m.verts[m.faces[:, 0]], axis=1) > 0)


def test_edge_factor_symmetric_positive(meshes):
    for m in meshes:
        assert np.all(m.g > 0)
        T = np.arange(m.n)
        for j in range(3):
            nb = m.nbr[:, j]
            jb = np.argmax(m.nbr[nb] == T[:, None], axis=1)
            assert np.allclose(m.g[nb, jb], m.g[:, j], rtol=1e-13, atol=0)
            assert np.allclose(m.arc[nb, jb], m.arc[:, j], rtol=1e-14, atol=0)
            # the outward normal is tangent at the edge and orthogonal to it
            p, q = m.verts[m.faces[:, j]], m.verts[m.faces[:, (j + 1) % 3]]
            nrm = m.normal[:, j]
            assert np.allclose(np.sum(nrm * (p + q), axis=1), 0, atol=1e-14)
            assert np.allclose(np.sum(nrm * (q - p), axis=1), 0, atol=1e-14)
            # pointing away from the cell: the opposite vertex is behind it
            opp = m.verts[m.faces[:, (j + 2) % 3]]
            assert np.all(np.sum(nrm * (opp - p), axis=1) < 0)
