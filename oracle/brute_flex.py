"""Independent numpy brute force for the flexible-molecule oracle.

TEST INFRASTRUCTURE ONLY (only ``tests/`` import it).  Written again from the
definitions, sharing nothing with ``flex_oracle.c`` or the HIP library: the
bodies from their vertex coordinates, the bonds from the body's edges, the
flips as the vertex permutations that 180 degree rotations about the body's
symmetry axes induce (found numerically here, not tabulated), the energy of
Eq. 1 over all atom pairs plus Eq. 2 over the bonds, vectorised.
"""
from __future__ import annotations

import math

import numpy as np

from .brute import philox4x32_10, quat_to_matrix, uniform53, uniform53_left, uniform_open

TRIANGLE, SQUARE, TETRAHEDRON = 0, 1, 2


def body(geometry, side):
    """Vertices of the ideal body of edge `side` around its centroid."""
    if geometry == TRIANGLE:
        ang = np.array([0.0, 2 * np.pi / 3, -2 * np.pi / 3])
        r = side / np.sqrt(3.0)
        return np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(3)], axis=1)
    if geometry == SQUARE:  # a ring 0-1-2-3, counter-clockwise from (+, +)
        ang = np.pi / 4 + np.arange(4) * np.pi / 2
        r = side / np.sqrt(2.0)
        return np.stack([r * np.cos(ang), r * np.sin(ang), np.zeros(4)], axis=1)
    v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], dtype=float)
    return v * side / (2 * np.sqrt(2.0))


def bonds(geometry):
    """Bonded atom pairs: the edges of the ideal body (shortest vertex pairs)."""
    v = body(geometry, 1.0)
    n = len(v)
    d = np.linalg.norm(v[:, None] - v[None], axis=-1)
    return [(i, j) for i in range(n) for j in range(i + 1, n) if abs(d[i, j] - 1.0) < 1e-9]


def flips(geometry):
    """Type permutations of the flips, new_type[s] = old_type[perm[s]]: the
    180 degree rotations about the body's two-fold axes, in the order the
    oracle numbers them (triangle: the median through vertex q; square: the
    diagonal through vertex 0, the one through vertex 1, the bisector of edge
    01, the bisector of edge 12; tetrahedron: the axis through the midpoint of
    edge 01, of 02, of 03).  Each permutation is found by rotating the ideal
    body and matching vertices."""
    v = body(geometry, 1.0)
    mid = lambda i, j: 0.5 * (v[i] + v[j])  # noqa: E731
    if geometry == TRIANGLE:
        axes = [v[0], v[1], v[2]]
    elif geometry == SQUARE:
        axes = [v[0], v[1], mid(0, 1), mid(1, 2)]
    else:
        axes = [mid(0, 1), mid(0, 2), mid(0, 3)]
    out = []
    for a in axes:
        a = a / np.linalg.norm(a)
        R = 2.0 * np.outer(a, a) - np.eye(3)  # rotation by pi about a
        w = v @ R.T  # where each vertex goes
        to = [int(np.argmin(np.linalg.norm(v - w[t], axis=1))) for t in range(len(v))]
        assert np.allclose(v[to], w), "not a symmetry of the body"
        # the atom that lands on vertex s came from vertex t with to[t] = s
        out.append(tuple(to.index(s) for s in range(len(v))))
    return out


def _wca(r2, sig):
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        sr6 = (sig * sig / r2) ** 3
        u = 4.0 * (sr6 * sr6 - sr6 + 0.25)
    return np.where(r2 < (2.0 ** (1.0 / 3.0)) * sig * sig, u, 0.0)


def energy(pos, types, box, geometry, sigma):
    """Eq. 1 over every pair of distinct atoms plus Eq. 2 over the bonds
    (infinite when a bond reaches 1.5 sigma_ij)."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(body(geometry, 1.0))
    N = len(pos)
    sg = np.asarray(sigma, dtype=np.float64)[np.asarray(types)]
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(-1)
    sig = 0.5 * (sg[:, None] + sg[None, :])
    iu = np.triu_indices(N, 1)
    e = float(_wca(r2[iu], sig[iu]).sum())
    for m in range(N // n):
        for i, j in bonds(geometry):
            a, b = n * m + i, n * m + j
            lim = 1.5 * sig[a, b]
            if not r2[a, b] < lim * lim:
                return math.inf
            x2 = r2[a, b] / (lim * lim)
            e += -33.75 * math.log(1.0 - x2)
    return e


def terms_touching(pos, types, box, geometry, sigma, changed):
    """Pair terms in range (WCA inside its cut-off; every bond) among the
    pairs that involve an atom of `changed`."""
    pos = np.asarray(pos, dtype=np.float64).reshape(-1, 3)
    n = len(body(geometry, 1.0))
    sg = np.asarray(sigma, dtype=np.float64)[np.asarray(types)]
    bset = {(min(i, j), max(i, j)) for i, j in bonds(geometry)}
    count = 0
    seen = set()
    for a in changed:
        d = pos - pos[a]
        d -= box * np.round(d / box)
        r2 = (d * d).sum(-1)
        for j in range(len(pos)):
            if j == a or (min(a, j), max(a, j)) in seen:
                continue
            seen.add((min(a, j), max(a, j)))
            s = 0.5 * (sg[a] + sg[j])
            if r2[j] < (2.0 ** (1.0 / 3.0)) * s * s:
                count += 1
            if j // n == a // n and (min(a % n, j % n), max(a % n, j % n)) in bset:
                count += 1
    return count


class Replayer:
    """Replays the flexible oracle's decision log from the definitions."""

    def __init__(self, params, box):
        self.p = params
        self.box = box
        self.n = len(body(params.geometry, 1.0))
        self.sigma = params.sigma or ((0.9, 1.0, 1.1) if params.geometry == TRIANGLE else
                                      (0.9, 0.9 + 0.2 / 3, 0.9 + 0.4 / 3, 1.1))
        self.flips = flips(params.geometry)
        self.key = (params.seed & 0xFFFFFFFF, params.seed >> 32)

    def draw(self, slot, sweep, tag):
        return philox4x32_10([slot, sweep & 0xFFFFFFFF, sweep >> 32, tag], self.key)

    def shift(self, sweep):
        g = self.draw(0xFFFFFFFF, sweep, 3)
        return (self.box / self.p.cells_per_side) * uniform_open(g[:3])

    def cell(self, x, h):
        nc = self.p.cells_per_side
        w = self.box / nc
        idx = np.minimum(np.floor(np.mod(np.asarray(x) - h, self.box) / w).astype(int), nc - 1)
        return int(idx[0] + nc * (idx[1] + nc * idx[2]))

    def propose(self, pos, types, a, slot, sweep, restricted):
        """(move, (pos', types') or None for a cell exit, u_acc, changed atoms, flip kind)"""
        b0 = self.draw(slot, sweep, 0)
        b1 = self.draw(slot, sweep, 1)
        u_acc = uniform53(b0[0], b0[1])
        u_type = uniform_open(b0[2])
        pr = uniform_open(b1[:3])
        pos2, types2 = pos.copy(), types.copy()
        if u_type < self.p.p_flip:
            K = len(self.flips)
            q = min(int(K * pr[0]), K - 1)
            base = self.n * (a // self.n)
            old = types[base:base + self.n].copy()
            for s in range(self.n):
                types2[base + s] = old[self.flips[q][s]]
            changed = [base + s for s in range(self.n) if types2[base + s] != types[base + s]]
            return 2, (pos2, types2), u_acc, changed, q
        pos2[a] = np.mod(pos[a] + self.p.max_displacement * (2 * pr - 1), self.box)
        if restricted:
            h = self.shift(sweep)
            if self.cell(pos2[a], h) != self.cell(pos[a], h):
                return 0, None, u_acc, [], 255
        return 0, (pos2, types2), u_acc, [a], 255

    def energy(self, pos, types):
        return energy(pos, types, self.box, self.p.geometry, self.sigma)

    def terms(self, pos, types, changed):
        return terms_touching(pos, types, self.box, self.p.geometry, self.sigma, changed)


def lattice(params, box, side):
    """The lattice start: ideal bodies at simple-cubic sites, Shoemake
    orientations from the tag-2 Philox block of each molecule."""
    M = params.n_molecules
    nl = round(M ** (1 / 3))
    a = box / nl
    v = body(params.geometry, side)
    m = np.arange(M)
    c = np.stack([(m % nl + 0.5) * a, ((m // nl) % nl + 0.5) * a, (m // (nl * nl) + 0.5) * a], 1)
    key = (params.seed & 0xFFFFFFFF, params.seed >> 32)
    g = np.array([philox4x32_10([k, 0xFFFFFFFF, 0xFFFFFFFF, 2], key) for k in range(M)])
    u1, u2, u3 = (uniform_open(g[:, i]) for i in range(3))
    q = np.stack([np.sqrt(u1) * np.cos(2 * np.pi * u3), np.sqrt(1 - u1) * np.sin(2 * np.pi * u2),
                  np.sqrt(1 - u1) * np.cos(2 * np.pi * u2), np.sqrt(u1) * np.sin(2 * np.pi * u3)], 1)
    R = quat_to_matrix(q)
    pos = c[:, None, :] + np.einsum("mij,sj->msi", R, v)
    return np.mod(pos.reshape(-1, 3), box)
