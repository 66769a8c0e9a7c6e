"""Synthetic closed surface meshes for the BEM workloads (geometry only).

Each generator returns a dict with the tesserae of a closed triangulated
surface, in Angstrom:
  cen     (N, 3) barycentres
  nrm     (N, 3) outward unit normals (the triangle's plane normal)
  area    (N,)   areas (Angstrom^2)
  r_enc   radius of the sphere about the origin that encloses every vertex
  verts, tris    the vertices and the vertex triples

The sphere is an icosahedron whose faces are split into four, k times, with
the new vertices pushed out to the sphere (20 * 4^k tesserae); the rod is a
prolate spheroid, the same mesh stretched along z; the dimer is two spheres
side by side along x with a surface-to-surface gap.
"""
from __future__ import annotations

import numpy as np


def _icosahedron():
    t = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
                  [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11], [1, 5, 9], [5, 11, 4], [11, 10, 2],
                  [10, 7, 6], [7, 1, 8], [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9], [4, 9, 5], [2, 4, 11],
                  [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    return v / np.linalg.norm(v, axis=1)[:, None], f


def unit_icosphere(k: int):
    """Vertices on the unit sphere and faces after k four-way splits."""
    v, f = _icosahedron()
    verts = [p for p in v]
    for _ in range(k):
        mid = {}

        def midpoint(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in mid:
                p = verts[a] + verts[b]
                verts.append(p / np.linalg.norm(p))
                mid[key] = len(verts) - 1
            return mid[key]

        nf = []
        for a, b, c in f:
            ab, bc, ca = midpoint(a, b), midpoint(b, c), midpoint(c, a)
            nf += [[a, ab, ca], [b, bc, ab], [c, ca, bc], [ab, bc, ca]]
        f = np.array(nf, dtype=np.int64)
    return np.array(verts), f


def _tesserae(verts, tris, centre_of=None):
    p = verts[tris]
    cen = p.mean(axis=1)
    cr = np.cross(p[:, 1] - p[:, 0], p[:, 2] - p[:, 0])
    area = 0.5 * np.linalg.norm(cr, axis=1)
    nrm = cr / (2.0 * area)[:, None]
    # outward: away from the centre of the body the tessera belongs to
    ref = cen if centre_of is None else cen - centre_of
    nrm *= np.sign(np.einsum("ij,ij->i", nrm, ref))[:, None]
    return dict(cen=np.ascontiguousarray(cen), nrm=np.ascontiguousarray(nrm), area=np.ascontiguousarray(area),
                r_enc=float(np.linalg.norm(verts, axis=1).max()), verts=verts, tris=tris)


def sphere(radius: float, k: int):
    """Icosphere of the given radius (Angstrom), 20 * 4^k tesserae."""
    v, f = unit_icosphere(k)
    return _tesserae(v * radius, f)


def sphere_n(n: int, radius: float):
    """The icosphere with the fewest tesserae >= n."""
    k = 0
    while 20 * 4 ** k < n:
        k += 1
    return sphere(radius, k)


def spheroid(a: float, c: float, k: int):
    """Prolate spheroid (semi-axes a, a, c along x, y, z; the rod-like body)."""
    v, f = unit_icosphere(k)
    v = v * np.array([a, a, c])
    return _tesserae(v, f)


def sphere_dimer(radius: float, gap: float, k: int):
    """Two icospheres on the x axis, surfaces gap apart (the gap dimer)."""
    v, f = unit_icosphere(k)
    shift = radius + 0.5 * gap
    parts = []
    for sx in (-shift, shift):
        c = np.array([sx, 0.0, 0.0])
        parts.append(_tesserae(v * radius + c, f, centre_of=c))
    out = {key: np.concatenate([parts[0][key], parts[1][key]]) for key in ("cen", "nrm", "area")}
    verts = np.concatenate([parts[0]["verts"], parts[1]["verts"]])
    out.update(r_enc=float(np.linalg.norm(verts, axis=1).max()), verts=verts,
               tris=np.concatenate([f, f + len(v)]))
    return out
