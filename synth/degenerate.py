"""Inputs with exact and near ties: ideal rings, cube corners, lattices.

Geometry only (no part of the method's arithmetic): seeded-free, closed-form
constructions that put many weighted points on one sphere and many radical
planes through one line, the inputs on which the weighted Delaunay
tetrahedrization is not unique.
"""
import numpy as np


def ring(n=6, d=1.39, r=1.7, h=None):
    """Ideal planar ring (C6 by default: C-C 1.39 A, r 1.7 A); with h, a
    hydrogen (r 1.2 A) radially h A outside each ring atom (C6H6 with h = 1.09)."""
    ang = np.arange(n) * 2 * np.pi / n
    xyz = np.stack([d * np.cos(ang), d * np.sin(ang), np.zeros(n)], 1)
    rad = np.full(n, r)
    if h is not None:
        xyz = np.concatenate([xyz, np.stack([(d + h) * np.cos(ang), (d + h) * np.sin(ang), np.zeros(n)], 1)])
        rad = np.concatenate([rad, np.full(n, 1.2)])
    return xyz, rad


def square_ring(s=1.5, r=1.7):
    """Four atoms on a square with exactly representable coordinates."""
    return np.array([[s, 0, 0], [0, s, 0], [-s, 0, 0], [0, -s, 0]], float), np.full(4, r)


def cube(s, r=1.7):
    """Eight equal atoms on the corners of a cube of side s (exact coordinates)."""
    return np.array([[x, y, z] for x in (0, s) for y in (0, s) for z in (0, s)], float), np.full(8, r)


def lattice(m, s, r=1.7):
    """m x m x m simple cubic lattice of spacing s."""
    g = np.array([[x, y, z] for x in range(m) for y in range(m) for z in range(m)], float) * s
    return g, np.full(len(g), r)


def octahedron(s, centre=False):
    """Six atoms on the axes at distance s, optionally with one at the centre."""
    v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float) * s
    if centre:
        v = np.concatenate([[[0.0, 0.0, 0.0]], v])
    return v, np.full(len(v), 1.7)


def fcc(s):
    """Face-centred cubic patch: the even points of a 3 x 3 x 3 grid of spacing s."""
    p = [[x, y, z] for x in range(3) for y in range(3) for z in range(3) if (x + y + z) % 2 == 0]
    return np.array(p, float) * s, np.full(len(p), 1.6)


def regular_tetrahedron(d, r=1.7):
    """Four equal atoms on a regular tetrahedron scaled by d."""
    u = np.array([[1, 0, -1 / np.sqrt(2)], [-1, 0, -1 / np.sqrt(2)], [0, 1, 1 / np.sqrt(2)], [0, -1, 1 / np.sqrt(2)]])
    return u * d, np.full(4, r)


def tangent_pair():
    """Two balls touching exactly with probe 1.5: r = 1.5, R = 3, centres 6 apart."""
    return np.array([[0.0, 0, 0], [6.0, 0, 0]]), np.array([1.5, 1.5])


def tangent_triple():
    """Three balls (r = 1.5, probe 1.5) pairwise touching exactly (side 6)."""
    return np.array([[0.0, 0, 0], [6.0, 0, 0], [3.0, np.sqrt(27.0), 0]]), np.full(3, 1.5)


def coincident_smaller():
    """A 1.2 A atom on the centre of a 1.7 A atom, and a third atom nearby."""
    return np.array([[0.0, 0, 0], [0.0, 0, 0], [2.0, 0, 0]]), np.array([1.7, 1.2, 1.5])


def coincident_equal():
    """Two equal atoms with one centre (invalid input)."""
    return np.array([[0.0, 0, 0], [0.0, 0, 0], [2.0, 0, 0]]), np.array([1.7, 1.7, 1.5])


# (name, input, slice-integral nodes, Euler characteristic of the union of balls)
CASES = [
    ("C6 ring", ring(), 96, 1),
    ("C6H6 ring", ring(h=1.09), 96, 1),
    ("square ring, exact coordinates", square_ring(), 96, 1),
    ("cube corners s=2", cube(2.0), 96, 1),
    ("cube corners s=3", cube(3.0), 96, 1),
    # s = 4: the cube's centre is 3.46 A from the corners, outside the 3.1 A
    # balls, while the faces' centres (2.83 A) are covered: one cavity
    ("cube corners s=4", cube(4.0), 96, 2),
    ("octahedron", octahedron(2.0), 96, 1),
    ("octahedron + centre", octahedron(2.0, True), 96, 1),
    ("3x3x3 lattice s=2", lattice(3, 2.0), 96, 1),
    ("3x3x3 lattice s=3", lattice(3, 3.0), 96, 1),
    # s = 4: the centre of each of the 8 lattice cubes is 3.46 A from its
    # corners, outside the 3.1 A balls: 8 cavities
    ("3x3x3 lattice s=4", lattice(3, 4.0), 400, 9),
    ("4x4x4 lattice s=2.5", lattice(4, 2.5), 96, 1),
    ("fcc", fcc(2.0), 96, 1),
]
