"""Seeded synthetic nanostructure generators (input data only).

These build the atomic geometries that stand in for the paper's workloads
(fcc noble-metal clusters and rods, gap dimers, honeycomb graphene flakes;
Section 5 lists the shapes its GEOM interface produces).  Every coordinate is
in Angstrom, as the paper's input geometry is.  Nothing in this module
evaluates any equation of the response model: it only places atoms.

Exact-size selection: when a workload asks for exactly N atoms, the N sites
with the smallest shape metric are kept and ties inside a degenerate shell are
broken by lexicographic (x, y, z) order of the unjittered site, so the result
is a pure function of (shape, N, seed).
"""
from __future__ import annotations

import numpy as np

FCC_A = 4.08          # Ag/Au lattice constant, Angstrom
CC_BOND = 1.42        # graphene C-C distance, Angstrom

_FCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.0, 0.5, 0.5],
                       [0.5, 0.0, 0.5], [0.5, 0.5, 0.0]])


def _fcc_block(half_extent: float, a: float = FCC_A) -> np.ndarray:
    """All atom-centred fcc sites inside a cube of half-width half_extent."""
    n = int(np.ceil(half_extent / a)) + 1
    g = np.arange(-n, n + 1)
    cx, cy, cz = np.meshgrid(g, g, g, indexing="ij")
    cells = np.stack([cx.ravel(), cy.ravel(), cz.ravel()], axis=1).astype(np.float64)
    pts = (cells[:, None, :] + _FCC_BASIS[None]).reshape(-1, 3) * a
    m = np.all(np.abs(pts) <= half_extent + 1e-9, axis=1)
    return pts[m]


def _take_smallest(pts: np.ndarray, metric: np.ndarray, n: int) -> np.ndarray:
    """Keep the n sites of smallest metric; ties broken by (x, y, z)."""
    if n > len(pts):
        raise ValueError(f"only {len(pts)} candidate sites for n={n}")
    key = np.round(metric, 9)
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0], key))
    return pts[order[:n]]


def _jitter(pts: np.ndarray, amp: float, seed: int) -> np.ndarray:
    if amp <= 0:
        return pts.copy()
    rng = np.random.default_rng(seed)
    return pts + rng.uniform(-amp, amp, size=pts.shape)


def fcc_sphere_radius(radius: float, jitter: float = 0.01, seed: int = 1,
                      a: float = FCC_A) -> np.ndarray:
    """Atom-centred fcc sphere: every site with |r| <= radius (Angstrom)."""
    pts = _fcc_block(radius + a, a)
    pts = pts[np.linalg.norm(pts, axis=1) <= radius + 1e-9]
    pts = pts[np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0]))]
    return _jitter(pts, jitter, seed)


def fcc_sphere_n(n: int, jitter: float = 0.01, seed: int = 2,
                 a: float = FCC_A) -> np.ndarray:
    """Atom-centred fcc sphere of exactly n atoms (n nearest sites)."""
    r_est = (3.0 * n * a ** 3 / 4.0 / (4.0 * np.pi)) ** (1.0 / 3.0)
    pts = _fcc_block(r_est * 1.15 + 2 * a, a)
    sel = _take_smallest(pts, np.linalg.norm(pts, axis=1), n)
    return _jitter(sel, jitter, seed)


def fcc_rod_n(n: int, aspect: float = 3.0, jitter: float = 0.01, seed: int = 3,
              a: float = FCC_A) -> np.ndarray:
    """fcc rod along z with length/diameter = aspect, exactly n atoms.

    The shape metric is max(rho/R, |z|/(aspect*R)) so that the level sets are
    flat-ended cylinders of the requested aspect ratio."""
    vol = n * a ** 3 / 4.0
    r_est = (vol / (np.pi * 2.0 * aspect)) ** (1.0 / 3.0)
    half = max(r_est, aspect * r_est) * 1.2 + 2 * a
    pts = _fcc_block(half, a)
    rho = np.hypot(pts[:, 0], pts[:, 1])
    metric = np.maximum(rho / r_est, np.abs(pts[:, 2]) / (aspect * r_est))
    sel = _take_smallest(pts, metric, n)
    return _jitter(sel, jitter, seed)


def gap_dimer(n_total: int, gap: float, jitter: float = 0.01, seed: int = 5,
              a: float = FCC_A) -> np.ndarray:
    """Two identical fcc spheres along x separated by a surface gap (Angstrom)."""
    n1 = n_total // 2
    s = fcc_sphere_n(n1, jitter=0.0, a=a)
    s2 = fcc_sphere_n(n_total - n1, jitter=0.0, a=a)
    x_max = s[:, 0].max()
    x_min2 = s2[:, 0].min()
    shift = x_max - x_min2 + gap
    left = s - np.array([shift / 2.0, 0.0, 0.0])
    right = s2 + np.array([shift / 2.0, 0.0, 0.0])
    return _jitter(np.concatenate([left, right]), jitter, seed)


def _honeycomb_block(half_x: float, half_y: float, b: float = CC_BOND) -> np.ndarray:
    """Planar honeycomb (z = 0) with armchair direction along x."""
    a1 = np.array([1.5 * b, np.sqrt(3) / 2 * b])
    a2 = np.array([1.5 * b, -np.sqrt(3) / 2 * b])
    basis = np.array([[0.0, 0.0], [b, 0.0]])
    n = int(np.ceil(max(half_x, half_y) / b)) + 2
    g = np.arange(-n, n + 1)
    i, j = np.meshgrid(g, g, indexing="ij")
    cells = i.ravel()[:, None] * a1 + j.ravel()[:, None] * a2
    pts = (cells[:, None, :] + basis[None]).reshape(-1, 2)
    m = (np.abs(pts[:, 0]) <= half_x) & (np.abs(pts[:, 1]) <= half_y)
    pts = pts[m]
    return np.concatenate([pts, np.zeros((len(pts), 1))], axis=1)


def graphene_disk_n(n: int, jitter: float = 0.0, seed: int = 4) -> np.ndarray:
    """Honeycomb disk of exactly n atoms (2.619 Angstrom^2 per atom)."""
    area = n * 3 * np.sqrt(3) / 4 * CC_BOND ** 2
    r_est = np.sqrt(area / np.pi)
    pts = _honeycomb_block(r_est * 1.2 + 3, r_est * 1.2 + 3)
    sel = _take_smallest(pts, np.hypot(pts[:, 0], pts[:, 1]), n)
    return _jitter(sel, jitter, seed)


def graphene_ribbon_n(n: int, width: float, zigzag: bool = False, jitter: float = 0.0,
                      seed: int = 4) -> np.ndarray:
    """Honeycomb ribbon of exactly n atoms and the given width (Angstrom).

    The long axis is x for armchair edges and y for zigzag edges (the lattice is
    generated with its armchair direction along x)."""
    area = n * 3 * np.sqrt(3) / 4 * CC_BOND ** 2
    length = area / width
    if zigzag:
        pts = _honeycomb_block(width / 2 + 3, length / 2 * 1.3 + 3)
        metric = np.maximum(np.abs(pts[:, 0]) / (width / 2), np.abs(pts[:, 1]) / (length / 2))
    else:
        pts = _honeycomb_block(length / 2 * 1.3 + 3, width / 2 + 3)
        metric = np.maximum(np.abs(pts[:, 1]) / (width / 2), np.abs(pts[:, 0]) / (length / 2))
    sel = _take_smallest(pts, metric, n)
    return _jitter(sel, jitter, seed)


def two_atoms(distance: float, axis: int = 0) -> np.ndarray:
    p = np.zeros((2, 3))
    p[1, axis] = distance
    return p


def alloy_types(n: int, frac_b: float, seed: int = 6) -> np.ndarray:
    """Random substitutional alloy: exactly round(frac_b * n) atoms of type B (1),
    chosen by a seeded permutation, the rest type A (0)."""
    nb = int(round(frac_b * n))
    t = np.zeros(n, dtype=np.int32)
    t[np.random.default_rng(seed).permutation(n)[:nb]] = 1
    return t


def core_shell_types(xyz: np.ndarray, core_radius: float) -> np.ndarray:
    """Core (type A, 0) within core_radius of the centroid, shell (type B, 1) outside."""
    c = xyz.mean(axis=0)
    return (np.linalg.norm(xyz - c, axis=1) > core_radius).astype(np.int32)
