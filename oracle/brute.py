"""Independent numpy brute force used to pin the C oracle.

TEST INFRASTRUCTURE ONLY (only ``tests/`` import it).  Nothing here is shared
with the C oracle or with the HIP library: Philox, the rigid body, the
energy and the proposals are written again from their definitions (Sec. II.A
Eq. 1 for the energy, Sec. II.B for the moves), vectorised over all site
pairs instead of looping, so that a slip in either implementation shows up as
a disagreement.
"""
from __future__ import annotations

import math

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32-10 (Salmon et al., SC'11) on numpy uint64 lanes.

    ``ctr``: (..., 4) and ``key``: (..., 2) integer arrays.  Returns (..., 4)."""
    c = np.asarray(ctr, dtype=np.uint64) & MASK32
    k = np.asarray(key, dtype=np.uint64) & MASK32
    x = [c[..., i].copy() for i in range(4)]
    k0, k1 = k[..., 0].copy(), k[..., 1].copy()
    for rnd in range(10):
        if rnd:
            k0 = (k0 + np.uint64(0x9E3779B9)) & MASK32
            k1 = (k1 + np.uint64(0xBB67AE85)) & MASK32
        p0 = np.uint64(0xD2511F53) * x[0]
        p1 = np.uint64(0xCD9E8D57) * x[2]
        x = [
            ((p1 >> np.uint64(32)) ^ x[1] ^ k0) & MASK32,
            p1 & MASK32,
            ((p0 >> np.uint64(32)) ^ x[3] ^ k1) & MASK32,
            p0 & MASK32,
        ]
    return np.stack(x, axis=-1).astype(np.uint32)


def uniform_open(w):
    """32-bit word -> (0, 1): (w + 1/2) / 2^32."""
    return (np.asarray(w, dtype=np.float64) + 0.5) / 4294967296.0


def uniform53(lo, hi):
    """Two words -> (0, 1] with 53 random bits."""
    v = (int(hi) << 32) | int(lo)
    return ((v >> 11) + 1) / 9007199254740992.0


def uniform53_left(lo, hi):
    v = (int(hi) << 32) | int(lo)
    return (v >> 11) / 9007199254740992.0


def quat_to_matrix(q):
    """Rotation matrices of unit quaternions (w, x, y, z), shape (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    m = np.empty(q.shape[:-1] + (3, 3))
    m[..., 0, 0] = w * w + x * x - y * y - z * z
    m[..., 0, 1] = 2 * (x * y - w * z)
    m[..., 0, 2] = 2 * (x * z + w * y)
    m[..., 1, 0] = 2 * (x * y + w * z)
    m[..., 1, 1] = w * w - x * x + y * y - z * z
    m[..., 1, 2] = 2 * (y * z - w * x)
    m[..., 2, 0] = 2 * (x * z - w * y)
    m[..., 2, 1] = 2 * (y * z + w * x)
    m[..., 2, 2] = w * w - x * x - y * y + z * z
    return m


def triangle(bond):
    """Vertices of an equilateral triangle of side ``bond`` around its centroid:
    site 0 on +x, sites 1 and 2 symmetric about the x axis."""
    ang = np.array([0.0, 2 * np.pi / 3, -2 * np.pi / 3])
    rad = bond / np.sqrt(3.0)
    return np.stack([rad * np.cos(ang), rad * np.sin(ang), np.zeros(3)], axis=1)


def sites(com, quat, bond):
    """(M, 3, 3) site positions c + R(q) b_s."""
    b = triangle(bond)
    R = quat_to_matrix(quat)
    return np.asarray(com)[:, None, :] + np.einsum("mij,sj->msi", R, b)


def wca_matrix(r2, sig):
    """Eq. (1) elementwise: 4[(s/r)^12 - (s/r)^6 + 1/4] below 2^(1/6) s."""
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        sr6 = (sig * sig / r2) ** 3
        u = 4.0 * (sr6 * sr6 - sr6 + 0.25)
    return np.where(r2 < (2.0 ** (1.0 / 3.0)) * sig * sig, u, 0.0)


def energy(com, quat, types, box, bond, sigma=(0.9, 1.0, 1.1)):
    """Total inter-molecular energy: every pair of sites of distinct molecules."""
    pos = sites(com, quat, bond).reshape(-1, 3)
    ty = np.asarray(types).reshape(-1)
    mol = np.repeat(np.arange(len(com)), 3)
    d = pos[:, None, :] - pos[None, :, :]
    d -= box * np.round(d / box)
    r2 = (d * d).sum(-1)
    sg = np.asarray(sigma)
    sig = 0.5 * (sg[ty][:, None] + sg[ty][None, :])
    other = mol[:, None] != mol[None, :]
    np.fill_diagonal(r2, 1.0)
    u = wca_matrix(r2, sig)
    return 0.5 * float(u[other].sum())


def interacting_pairs(com, quat, types, box, bond, m, moved, sigma=(0.9, 1.0, 1.1)):
    """Number of (moved site of molecule m, site of another molecule) pairs
    closer than their cut-off 2^(1/6) sigma_ij (Eq. 1), nearest image per
    site pair."""
    pos = sites(com, quat, bond)
    sg = np.asarray(sigma)
    ty = np.asarray(types)
    others = np.array([j for j in range(len(com)) if j != m], dtype=int)
    n = 0
    for a in moved:
        d = pos[others].reshape(-1, 3) - pos[m, a]
        d -= box * np.round(d / box)
        r2 = (d * d).sum(-1)
        sij = 0.5 * (sg[ty[m, a]] + sg[ty[others].reshape(-1)])
        n += int(np.count_nonzero(r2 < (2.0 ** (1.0 / 3.0)) * sij * sij))
    return n


def lattice_quaternions(n_molecules, seed):
    """Orientations of the lattice start: Shoemake's uniform unit quaternion
    (Graphics Gems III, 1992) from the three uniforms (u1, u2, u3) of the
    Philox block (m, 2^32 - 1, 2^32 - 1, 2) of molecule m:
    (sqrt(u1) cos 2 pi u3, sqrt(1 - u1) sin 2 pi u2, sqrt(1 - u1) cos 2 pi u2,
    sqrt(u1) sin 2 pi u3)."""
    m = np.arange(n_molecules, dtype=np.uint64)
    ctr = np.stack([m, np.full_like(m, 0xFFFFFFFF), np.full_like(m, 0xFFFFFFFF),
                    np.full_like(m, 2)], axis=1)
    key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64), (n_molecules, 1))
    g = philox4x32_10(ctr, key)
    u1, u2, u3 = (uniform_open(g[:, i]) for i in range(3))
    return np.stack([np.sqrt(u1) * np.cos(2 * np.pi * u3), np.sqrt(1 - u1) * np.sin(2 * np.pi * u2),
                     np.sqrt(1 - u1) * np.cos(2 * np.pi * u2), np.sqrt(u1) * np.sin(2 * np.pi * u3)],
                    axis=1)


class Replayer:
    """Replays the oracle's decision log step by step from the definitions."""

    def __init__(self, params, box, bond):
        self.p = params
        self.box = box
        self.bond = bond
        self.key = (params.seed & 0xFFFFFFFF, params.seed >> 32)

    def draw(self, slot, sweep, tag):
        return philox4x32_10([slot, sweep & 0xFFFFFFFF, sweep >> 32, tag], self.key)

    def cell(self, c, h):
        nc = self.p.cells_per_side
        w = self.box / nc
        g = np.mod(np.asarray(c) - h, self.box)
        idx = np.minimum(np.floor(g / w).astype(int), nc - 1)
        return int(idx[0] + nc * (idx[1] + nc * idx[2]))

    def shift(self, sweep):
        g = self.draw(0xFFFFFFFF, sweep, 3)
        return (self.box / self.p.cells_per_side) * uniform_open(g[:3])

    def propose(self, com, quat, types, m, slot, sweep, restricted):
        """(move kind, new state or None for a cell exit, u_acc, moved sites)"""
        b0 = self.draw(slot, sweep, 0)
        b1 = self.draw(slot, sweep, 1)
        u_acc = uniform53(b0[0], b0[1])
        u_type = uniform_open(b0[2])
        pr = uniform_open(b1[:3])
        com2, quat2, types2 = com.copy(), quat.copy(), types.copy()
        p = self.p
        if u_type < p.p_flip:
            move = 2
            a = min(int(3 * pr[0]), 2)
            s1, s2 = (a + 1) % 3, (a + 2) % 3
            types2[m, s1], types2[m, s2] = types[m, s2], types[m, s1]
            moved = (s1, s2)
        elif u_type < p.p_flip + p.p_translate:
            move = 0
            com2[m] = np.mod(com[m] + p.max_displacement * (2 * pr - 1), self.box)
            if restricted:
                h = self.shift(sweep)
                if self.cell(com2[m], h) != self.cell(com[m], h):
                    return move, None, u_acc, ()
            moved = (0, 1, 2)
        else:
            move = 1
            z = 2 * pr[0] - 1
            phi = 2 * math.pi * pr[1]
            axis = np.array([math.sqrt(1 - z * z) * math.cos(phi),
                             math.sqrt(1 - z * z) * math.sin(phi), z])
            th = p.max_rotation * (2 * pr[2] - 1)
            d = np.concatenate([[math.cos(th / 2)], axis * math.sin(th / 2)])
            q = quat[m]
            prod = np.array([
                d[0] * q[0] - d[1:] @ q[1:],
                *(d[0] * q[1:] + q[0] * d[1:] + np.cross(d[1:], q[1:])),
            ])
            quat2[m] = prod / np.linalg.norm(prod)
            moved = (0, 1, 2)
        return move, (com2, quat2, types2), u_acc, moved

    def energy(self, com, quat, types):
        return energy(com, quat, types, self.box, self.bond, self.p.sigma)

    def pairs(self, com, quat, types, m, moved):
        return interacting_pairs(com, quat, types, self.box, self.bond, m, moved, self.p.sigma)
