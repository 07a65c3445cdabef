"""Geometry of the zonal Shack-Hartmann problem (oracle side).

Everything here is integer bookkeeping except the taper weights.  The rules:

G1  A subaperture (i, j) (row i, column j, 0 <= i, j < N) is valid when more
    than half of its area is illuminated (Sec. 5: only subapertures with more
    than 50 % illuminated surface are kept).  The area is sampled on an
    ss x ss grid of cell centres; a sample is illuminated when its distance r
    (in pitches) from the pupil centre (N/2, N/2) satisfies
    eps*N/2 <= r <= N/2.  With coordinates scaled by 2*ss every test is an
    exact integer comparison against (ss*N)^2, and the obscuration bound is the
    double (eps*N*ss)^2.
G2  Actuator node (i, j), 0 <= i, j <= N, is valid when it is a corner of at
    least one valid subaperture (Fried geometry: each subaperture lies between
    four actuators, Sec. 4.1 and App. B).  Valid nodes are numbered row-major.
G3  The slope vector is [x-slopes of the valid subapertures in row-major order;
    y-slopes in the same order] (p = 2 p_sap, App. B).
G4  Fried slopes (App. B: two slopes from the four corner actuators), with i
    the row (y) and j the column (x), in radians per subaperture:
      sx = ((phi[i,j+1] - phi[i,j]) + (phi[i+1,j+1] - phi[i+1,j])) / 2
      sy = ((phi[i+1,j] - phi[i,j]) + (phi[i+1,j+1] - phi[i,j+1])) / 2
G5  Domains (Sec. 4.1): the subaperture grid is cut into b x b blocks,
    nb = ceil(N / b) per side.  Node (i, j) is owned by block
    (min(i // b, nb-1), min(j // b, nb-1)).  A block with at least one valid
    node is a domain; domains are numbered row-major by block.  The local state
    is the owned valid nodes in ascending index order.  The observation region
    is every valid subaperture with I*b - h <= i < min((I+1)*b, N) + h (same for
    j), giving the local slope list [its x-slopes; its y-slopes] in ascending
    global slope order.
G6  Taper (Sec. 4.1: the inverse square root of the noise covariance is
    multiplied by a function decreasing from one to zero with the distance from
    the centre of the observation region): f = GC(dist / c) with GC the
    Gaspari-Cohn fifth-order piecewise rational function (Gaspari & Cohn 1999,
    Q. J. R. Meteorol. Soc. 125, eq. 4.10), support 2c, and dist the distance in
    pitches from the subaperture centre (i + 1/2, j + 1/2) to the centre of the
    unclipped block, ((I + 1/2) b, (J + 1/2) b).  c = 0 means no taper (f = 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


def pupil_mask(n_sub: int, obscuration: float, ss: int = 64) -> np.ndarray:
    """G1: boolean (N, N) mask of valid subapertures of an annular pupil."""
    N = int(n_sub)
    outer = (ss * N) ** 2
    inner = (float(obscuration) * N * ss) ** 2
    s = np.arange(ss, dtype=np.int64)
    mask = np.zeros((N, N), dtype=bool)
    for i in range(N):
        ys = 2 * ss * i + 2 * s + 1 - ss * N
        for j in range(N):
            xs = 2 * ss * j + 2 * s + 1 - ss * N
            r2 = ys[:, None] ** 2 + xs[None, :] ** 2
            lit = np.count_nonzero((r2 <= outer) & (r2.astype(np.float64) >= inner))
            mask[i, j] = 2 * lit > ss * ss
    return mask


def square_mask(n_sub: int) -> np.ndarray:
    """All N x N subapertures valid (the square pupil of the smallest case)."""
    return np.ones((n_sub, n_sub), dtype=bool)


@dataclass
class Geometry:
    """Valid subapertures, valid nodes and their numbering (G1-G3)."""
    mask: np.ndarray                     # (N, N) bool
    node_valid: np.ndarray = field(init=False)   # (N+1, N+1) bool
    node_index: np.ndarray = field(init=False)   # (N+1, N+1) int, -1 if invalid
    subaps: np.ndarray = field(init=False)       # (p_sap, 2) int (i, j) row-major

    def __post_init__(self):
        m = np.asarray(self.mask, dtype=bool)
        N = m.shape[0]
        nv = np.zeros((N + 1, N + 1), dtype=bool)
        for i in range(N):
            for j in range(N):
                if m[i, j]:
                    nv[i, j] = nv[i + 1, j] = nv[i, j + 1] = nv[i + 1, j + 1] = True
        idx = -np.ones((N + 1, N + 1), dtype=np.int64)
        k = 0
        for i in range(N + 1):
            for j in range(N + 1):
                if nv[i, j]:
                    idx[i, j] = k
                    k += 1
        self.mask = m
        self.node_valid = nv
        self.node_index = idx
        self.subaps = np.array([(i, j) for i in range(N) for j in range(N) if m[i, j]],
                               dtype=np.int64).reshape(-1, 2)

    @property
    def n_sub(self) -> int:
        return self.mask.shape[0]

    @property
    def n_nodes(self) -> int:
        return int(self.node_valid.sum())

    @property
    def n_subaps(self) -> int:
        return int(self.subaps.shape[0])

    @property
    def n_slopes(self) -> int:
        return 2 * self.n_subaps

    def node_coords(self) -> np.ndarray:
        """(n, 2) grid coordinates (i, j) of the valid nodes in index order."""
        return np.argwhere(self.node_valid)


def slope_matrix(geom: Geometry) -> np.ndarray:
    """G4 as a dense (p, n) matrix D; only for small grids."""
    n, ps = geom.n_nodes, geom.n_subaps
    D = np.zeros((2 * ps, n))
    idx = geom.node_index
    for k, (i, j) in enumerate(geom.subaps):
        a, b_, c, d = idx[i, j], idx[i, j + 1], idx[i + 1, j], idx[i + 1, j + 1]
        D[k, b_] += 0.5
        D[k, a] -= 0.5
        D[k, d] += 0.5
        D[k, c] -= 0.5
        D[ps + k, c] += 0.5
        D[ps + k, a] -= 0.5
        D[ps + k, d] += 0.5
        D[ps + k, b_] -= 0.5
    return D


def apply_slopes(geom: Geometry, phase: np.ndarray) -> np.ndarray:
    """G4 applied to node values; `phase` is (n,) or (n, m) in node index order."""
    phase = np.asarray(phase, dtype=np.float64)
    idx = geom.node_index
    i, j = geom.subaps[:, 0], geom.subaps[:, 1]
    p00, p01 = phase[idx[i, j]], phase[idx[i, j + 1]]
    p10, p11 = phase[idx[i + 1, j]], phase[idx[i + 1, j + 1]]
    sx = 0.5 * ((p01 - p00) + (p11 - p10))
    sy = 0.5 * ((p10 - p00) + (p11 - p01))
    return np.concatenate([sx, sy], axis=0)


def apply_slopes_adjoint(geom: Geometry, s: np.ndarray) -> np.ndarray:
    """D^T s: the transpose of G4 applied to slope vectors (p,) or (p, m),
    each subaperture scattering its two slopes back onto its four corners."""
    s = np.asarray(s, dtype=np.float64)
    ps = geom.n_subaps
    sx, sy = s[:ps], s[ps:]
    idx = geom.node_index
    i, j = geom.subaps[:, 0], geom.subaps[:, 1]
    out = np.zeros((geom.n_nodes,) + s.shape[1:])
    np.add.at(out, idx[i, j], -0.5 * sx - 0.5 * sy)
    np.add.at(out, idx[i, j + 1], 0.5 * sx - 0.5 * sy)
    np.add.at(out, idx[i + 1, j], -0.5 * sx + 0.5 * sy)
    np.add.at(out, idx[i + 1, j + 1], 0.5 * sx + 0.5 * sy)
    return out


@dataclass
class Domain:
    block: tuple            # (I, J)
    owned: np.ndarray       # ascending global node indices (n_l,)
    obs: np.ndarray         # global slope indices (p_l,): x block then y block
    obs_subaps: np.ndarray  # (p_l / 2, 2) subaperture coordinates of the region


def domains(geom: Geometry, b: int, h: int) -> list[Domain]:
    """G5: the domain list with owned nodes and observation regions."""
    N = geom.n_sub
    nb = -(-N // b)
    owner = {}
    for i in range(N + 1):
        for j in range(N + 1):
            if geom.node_valid[i, j]:
                blk = (min(i // b, nb - 1), min(j // b, nb - 1))
                owner.setdefault(blk, []).append(int(geom.node_index[i, j]))
    sub_id = {(int(i), int(j)): k for k, (i, j) in enumerate(geom.subaps)}
    ps = geom.n_subaps
    out = []
    for I in range(nb):
        for J in range(nb):
            if (I, J) not in owner:
                continue
            owned = np.array(sorted(owner[(I, J)]), dtype=np.int64)
            rows = range(max(I * b - h, 0), min(min((I + 1) * b, N) + h, N))
            cols = range(max(J * b - h, 0), min(min((J + 1) * b, N) + h, N))
            ks = sorted(sub_id[(i, j)] for i in rows for j in cols if (i, j) in sub_id)
            ks = np.array(ks, dtype=np.int64)
            obs = np.concatenate([ks, ks + ps]).astype(np.int64)
            out.append(Domain((I, J), owned, obs, geom.subaps[ks].reshape(-1, 2)))
    return out


def owner_map(geom: Geometry, doms: list[Domain]) -> np.ndarray:
    """(n,) domain number owning each valid node."""
    own = -np.ones(geom.n_nodes, dtype=np.int64)
    for k, d in enumerate(doms):
        own[d.owned] = k
    return own


def gaspari_cohn(z) -> np.ndarray:
    """Gaspari & Cohn (1999) compactly supported fifth-order correlation
    function of z = r / c, equal to 1 at z = 0 and 0 for z >= 2."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    out = np.zeros_like(z)
    a = z <= 1.0
    za = z[a]
    out[a] = (((-0.25 * za + 0.5) * za + 0.625) * za - 5.0 / 3.0) * za * za + 1.0
    bm = (z > 1.0) & (z < 2.0)
    zb = z[bm]
    out[bm] = ((((zb / 12.0 - 0.5) * zb + 0.625) * zb + 5.0 / 3.0) * zb - 5.0) * zb \
        + 4.0 - 2.0 / (3.0 * zb)
    return out


def taper(dom: Domain, b: int, c: float) -> np.ndarray:
    """G6: taper weight f for each local slope (x block then y block)."""
    n2 = dom.obs.shape[0]
    if c <= 0.0:
        return np.ones(n2)
    I, J = dom.block
    cy, cx = (I + 0.5) * b, (J + 0.5) * b
    sy = dom.obs_subaps[:, 0] + 0.5
    sx = dom.obs_subaps[:, 1] + 0.5
    dist = np.sqrt((sy - cy) ** 2 + (sx - cx) ** 2)
    f = gaspari_cohn(dist / c)
    return np.concatenate([f, f])


def taper_dist(dom: Domain, b: int) -> np.ndarray:
    """Distances (in pitches) used by the taper, per local slope."""
    I, J = dom.block
    cy, cx = (I + 0.5) * b, (J + 0.5) * b
    d = np.sqrt((dom.obs_subaps[:, 0] + 0.5 - cy) ** 2 + (dom.obs_subaps[:, 1] + 0.5 - cx) ** 2)
    return np.concatenate([d, d])


def gaspari_cohn_deriv(z) -> np.ndarray:
    """d GC / d z (used by the taper-width gradient)."""
    z = np.abs(np.asarray(z, dtype=np.float64))
    out = np.zeros_like(z)
    a = z <= 1.0
    za = z[a]
    out[a] = (((-1.25 * za + 2.0) * za + 1.875) * za - 10.0 / 3.0) * za
    bm = (z > 1.0) & (z < 2.0)
    zb = z[bm]
    out[bm] = (((5.0 / 12.0 * zb - 2.0) * zb + 1.875) * zb + 10.0 / 3.0) * zb - 5.0 \
        + 2.0 / (3.0 * zb * zb)
    return out


def geometry_for(n_sub: int, obscuration: float | None) -> Geometry:
    """Square pupil when obscuration is None, else the annulus rule."""
    if obscuration is None:
        return Geometry(square_mask(n_sub))
    return Geometry(pupil_mask(n_sub, obscuration))


__all__ = ["pupil_mask", "square_mask", "Geometry", "slope_matrix", "apply_slopes", "apply_slopes_adjoint",
           "Domain", "domains", "owner_map", "gaspari_cohn", "gaspari_cohn_deriv",
           "taper", "taper_dist", "geometry_for"]
