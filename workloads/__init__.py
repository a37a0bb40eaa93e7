"""Seeded synthetic inputs for the D3M factor/solve path.

This module is shared by the CPU oracle, the tests and the benchmark.  It only
*generates inputs* (a tetrahedral mesh of the unit cube, a box partition of
its tetrahedra, per-tetrahedron relative permittivities, plane-wave incidence
parameters, receiver points) and holds none of the method's arithmetic: no
element matrices, no assembly, no factorisation.  The oracle and the HIP
library each build everything else from these arrays independently.

The paper's own workloads (PEC plates and dielectric spheres, Section III)
ship no meshes, so every workload here is a structured cube mesh whose sizes,
permittivity statistics and right-hand-side counts follow the five standard
configurations described in the module-level ``CONFIGS`` table.
"""
from __future__ import annotations

import itertools
import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem",
    "kuhn_cube_mesh",
    "box_partition",
    "make_problem",
    "make_config",
    "make_batch_config",
    "make_pec_config",
    "plate_faces",
    "box_shell_faces",
    "CONFIGS",
]

# The six axis permutations, in lexicographic order; each gives one Kuhn
# tetrahedron v0, v0+e_a, v0+e_a+e_b, v0+(1,1,1) of a hexahedron.
_PERMS = list(itertools.permutations(range(3)))


def kuhn_cube_mesh(n: int):
    """Unit cube split into n^3 hexahedra, each cut into 6 Kuhn tetrahedra.

    Returns ``xyz`` (float64 [n_v, 3]) and ``tets`` (int64 [n_t, 4]).
    Vertex (i, j, k) -> id (i*(n+1)+j)*(n+1)+k at (i/n, j/n, k/n).  Tetrahedra
    are listed hex by hex (hex (i,j,k) -> (i*n+j)*n+k) and permutation by
    permutation; the four vertex ids of each tetrahedron are increasing.
    """
    if n < 1:
        raise ValueError("n must be >= 1")
    m = n + 1
    g = np.arange(m, dtype=np.float64) / n
    xi, yi, zi = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([xi.ravel(), yi.ravel(), zi.ravel()], axis=1)

    ii, jj, kk = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    base = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)  # [n^3, 3]
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for p, perm in enumerate(_PERMS):
        c = base.copy()
        verts = [c.copy()]
        for ax in perm:
            c[:, ax] += 1
            verts.append(c.copy())
        for v, cc in enumerate(verts):
            tets[:, p, v] = (cc[:, 0] * m + cc[:, 1]) * m + cc[:, 2]
    return xyz, tets.reshape(-1, 4)


def _uniform_cuts(n: int, p: int):
    return [math.ceil(b * n / p) for b in range(p + 1)]


def box_partition(n: int, parts=(1, 1, 1), cuts=None):
    """Box partition of the Kuhn mesh: every tetrahedron of hex (i,j,k) goes to
    box (bx, by, bz) with id (bx*py + by)*pz + bz.

    ``cuts`` (optional) gives, per axis, the increasing hex indices
    [0, c1, ..., n] that bound the boxes; by default the boxes are
    floor(i*p/n).
    """
    px, py, pz = parts
    if cuts is None:
        cuts = [_uniform_cuts(n, px), _uniform_cuts(n, py), _uniform_cuts(n, pz)]
    owner = []
    for ax, p in enumerate((px, py, pz)):
        c = np.asarray(cuts[ax])
        if len(c) != p + 1 or c[0] != 0 or c[-1] != n or np.any(np.diff(c) <= 0):
            raise ValueError(f"bad cuts on axis {ax}: {c}")
        owner.append(np.searchsorted(c, np.arange(n), side="right") - 1)
    ii, jj, kk = np.meshgrid(owner[0], owner[1], owner[2], indexing="ij")
    hex_part = ((ii * py + jj) * pz + kk).ravel().astype(np.int32)
    return np.repeat(hex_part, 6)


def plate_faces(n: int, tets, axis: int, level: int, lo, hi):
    """Triangles of the Kuhn mesh lying in the plane x_axis = level / n inside
    the rectangle lo <= (other two coordinates) * n <= hi (hex units, lo and
    hi pairs for the two remaining axes in increasing axis order).  Returned
    as vertex-id triples [nf, 3], each triangle once."""
    m = n + 1
    ijk = lambda v: np.stack([v // (m * m), (v // m) % m, v % m], axis=-1)
    faces = np.concatenate([tets[:, [0, 1, 2]], tets[:, [0, 1, 3]], tets[:, [0, 2, 3]], tets[:, [1, 2, 3]]])
    c = ijk(faces)  # [nf, 3 vertices, 3 axes]
    others = [a for a in range(3) if a != axis]
    on = np.all(c[:, :, axis] == level, axis=1)
    for o, a in enumerate(others):
        on &= np.all((c[:, :, a] >= lo[o]) & (c[:, :, a] <= hi[o]), axis=1)
    return np.unique(np.sort(faces[on], axis=1), axis=0)


def box_shell_faces(n: int, tets, lo, hi):
    """Triangles on the six sides of the box lo <= x, y, z <= hi (hex units)."""
    out = []
    for axis in range(3):
        o = [a for a in range(3) if a != axis]
        for level in (lo[axis], hi[axis]):
            out.append(plate_faces(n, tets, axis, level, [lo[o[0]], lo[o[1]]], [hi[o[0]], hi[o[1]]]))
    return np.unique(np.concatenate(out), axis=0)


def _draw_dipoles(rng, count, keep_out=None):
    """Dipole positions uniform in [0.1, 0.9]^3 (redrawn while keep_out(pos) is
    true) and unit current moments with a uniform random phase."""
    pos = np.empty((count, 3))
    for i in range(count):
        while True:
            r = rng.uniform(0.1, 0.9, 3)
            if keep_out is None or not keep_out(r):
                break
        pos[i] = r
    u = rng.standard_normal((count, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    phase = np.exp(1j * rng.uniform(0.0, 2.0 * math.pi, count))
    return pos, u * phase[:, None]


def _tet_centroids(xyz, tets):
    return xyz[tets].mean(axis=1)


def _draw_plane_waves(rng, nrhs):
    d = rng.standard_normal((nrhs, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    h = rng.standard_normal((nrhs, 3))
    p = h - np.sum(h * d, axis=1, keepdims=True) * d
    p /= np.linalg.norm(p, axis=1, keepdims=True)
    return d, p


@dataclass
class Problem:
    """One synthetic D3M workload (inputs only)."""

    name: str
    n: int
    parts: tuple
    xyz: np.ndarray
    tets: np.ndarray
    part: np.ndarray
    eps_r: np.ndarray
    k: float
    alpha: complex
    dirs: np.ndarray
    pols: np.ndarray
    receivers: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    learnable: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    fd_tets: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int64))
    fd_h: float = 1e-6
    precision: str = "fp64"
    # PEC triangles (vertex-id triples) and point-dipole sources (one
    # right-hand side each, after the plane waves): position, current moment
    pec_faces: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), dtype=np.int64))
    dip_pos: np.ndarray = field(default_factory=lambda: np.zeros((0, 3)))
    dip_moment: np.ndarray = field(default_factory=lambda: np.zeros((0, 3), dtype=np.complex128))

    @property
    def nrhs(self) -> int:
        return int(self.dirs.shape[0])

    @property
    def n_sub(self) -> int:
        return int(self.part.max()) + 1 if self.part.size else 0


def make_problem(n, parts=(1, 1, 1), *, eps="one", k=2 * math.pi, nrhs=1,
                 seed=0, alpha=None, cuts=None, dirs=None, pols=None,
                 name="custom"):
    """Small custom workload for tests.

    ``eps``: "one" (free space), ("uniform", lo, hi) per tetrahedron, or an
    explicit array.  ``alpha`` defaults to -j*k.
    """
    xyz, tets = kuhn_cube_mesh(n)
    part = box_partition(n, parts, cuts)
    rng = np.random.default_rng(seed)
    nt = tets.shape[0]
    if isinstance(eps, str) and eps == "one":
        eps_r = np.ones(nt)
    elif isinstance(eps, tuple) and eps[0] == "uniform":
        eps_r = rng.uniform(eps[1], eps[2], nt)
    else:
        eps_r = np.asarray(eps, dtype=np.float64).copy()
    if dirs is None:
        dirs, pols = _draw_plane_waves(rng, nrhs)
    if alpha is None:
        alpha = -1j * k
    return Problem(name=name, n=n, parts=tuple(parts), xyz=xyz, tets=tets,
                   part=part, eps_r=eps_r, k=float(k), alpha=complex(alpha),
                   dirs=np.asarray(dirs, float), pols=np.asarray(pols, float))


CONFIGS = {
    1: "6^3 hexes, 2x2x1 boxes, eps_r = 1, k = 2*pi, 1 RHS (+z, x-polarised)",
    2: "24^3 hexes, 4x4x4 boxes, eps_r ~ U[1,4], k = 6*pi, 8 RHS",
    3: "32 independent problems, 12^3..32^3 hexes of side 1/8, jittered boxes, eps_r ~ U[1,4], k = 2*pi, 16 RHS each",
    4: "48^3 hexes, 8x8x8 boxes, eps_r = clip(lognormal(0.5, 0.3), 1, 10), k = 12*pi, 32 RHS",
    5: "32^3 hexes, 4x4x4 boxes, dielectric sphere r = 0.3 (eps_r ~ U[1,6] inside), k = 4*pi, 4 RHS, 64 receivers",
}


def make_config(i: int, seed: int | None = None) -> Problem:
    """Configurations 1, 2, 4, 5 (configuration 3 is a batch: make_batch_config).

    Draw order from ``numpy.random.default_rng(seed)`` (seed defaults to the
    configuration number): eps_r per tetrahedron in array order, then RHS
    directions, then polarisations, then receivers, then finite-difference
    tetrahedra.
    """
    seed = i if seed is None else seed
    rng = np.random.default_rng(seed)
    if i == 1:
        n, parts, k, nrhs = 6, (2, 2, 1), 2 * math.pi, 1
        xyz, tets = kuhn_cube_mesh(n)
        eps_r = np.ones(tets.shape[0])
        dirs = np.array([[0.0, 0.0, 1.0]])
        pols = np.array([[1.0, 0.0, 0.0]])
        return Problem("cfg1", n, parts, xyz, tets, box_partition(n, parts), eps_r,
                       k, -1j * k, dirs, pols)
    if i == 2:
        n, parts, k, nrhs = 24, (4, 4, 4), 6 * math.pi, 8
        xyz, tets = kuhn_cube_mesh(n)
        eps_r = rng.uniform(1.0, 4.0, tets.shape[0])
        dirs, pols = _draw_plane_waves(rng, nrhs)
        return Problem("cfg2", n, parts, xyz, tets, box_partition(n, parts), eps_r,
                       k, -1j * k, dirs, pols)
    if i == 4:
        n, parts, k, nrhs = 48, (8, 8, 8), 12 * math.pi, 32
        xyz, tets = kuhn_cube_mesh(n)
        eps_r = np.clip(rng.lognormal(0.5, 0.3, tets.shape[0]), 1.0, 10.0)
        dirs, pols = _draw_plane_waves(rng, nrhs)
        return Problem("cfg4", n, parts, xyz, tets, box_partition(n, parts), eps_r,
                       k, -1j * k, dirs, pols, precision="fp32_ir")
    if i == 5:
        n, parts, k, nrhs = 32, (4, 4, 4), 4 * math.pi, 4
        xyz, tets = kuhn_cube_mesh(n)
        cen = _tet_centroids(xyz, tets)
        inside = np.linalg.norm(cen - 0.5, axis=1) < 0.3
        draw = rng.uniform(1.0, 6.0, tets.shape[0])
        eps_r = np.where(inside, draw, 1.0)
        dirs, pols = _draw_plane_waves(rng, nrhs)
        # receivers: uniform in the shell 0.35 <= |r - c| <= 0.45
        u = rng.standard_normal((64, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = np.cbrt(rng.uniform(0.35 ** 3, 0.45 ** 3, 64))
        receivers = 0.5 + u * r[:, None]
        learnable = np.nonzero(inside)[0]
        fd_tets = np.sort(rng.choice(learnable, 20, replace=False))
        return Problem("cfg5", n, parts, xyz, tets, box_partition(n, parts), eps_r,
                       k, -1j * k, dirs, pols, receivers=receivers,
                       learnable=learnable, fd_tets=fd_tets, fd_h=1e-6)
    if i == 3:
        raise ValueError("configuration 3 is a batch; use make_batch_config()")
    raise ValueError(f"unknown configuration {i}")


def make_large_subdomain_config(seed: int = 8, n: int = 32, nrhs: int = 16) -> Problem:
    """The batch workload's largest subdomains on their own: an ``n``^3-hex
    cube (32: the top of the 12^3..32^3 range) in 2x2x2 box subdomains (the
    bottom of the 8..64 range, so 16^3 hexes and 31,024 edges each),
    eps_r ~ U[1, 4], hexes of an eighth of a wavelength (k = 2 pi n / 8),
    ``nrhs`` plane waves."""
    return make_problem(n, (2, 2, 2), eps=("uniform", 1, 4), k=2 * math.pi * n / 8, nrhs=nrhs, seed=seed)


def make_pec_config(seed: int = 6, n: int = 24, parts=(4, 4, 4), n_pw: int = 4, n_dip: int = 4) -> Problem:
    """PEC plates and impressed currents (the second workload of the paper's
    BVP: perfectly conducting scatterers, J_imp sources).  The paper's
    plate meshes are not given; this cube stands in: n^3 hexes in box
    subdomains, free space (eps_r = 1), k = 6*pi (wavelength 1/3, eight hexes
    per wavelength at n = 24), two square PEC plates -- one in the plane
    z = 1/2 (a subdomain interface for 4x4x4 boxes) over 1/4 <= x, y <= 3/4
    (1.5 wavelengths), one in the plane x = 3/8 (inside a subdomain) over
    1/8 <= y, z <= 3/8 -- and n_pw plane waves followed by n_dip point dipoles
    (kept more than 1/12 away from the plates' planes).  Draw order: plane
    waves, then dipoles."""
    rng = np.random.default_rng(seed)
    xyz, tets = kuhn_cube_mesh(n)
    k = 6 * math.pi
    q = n // 8
    pec = np.unique(np.concatenate([
        plate_faces(n, tets, 2, 4 * q, [2 * q, 2 * q], [6 * q, 6 * q]),
        plate_faces(n, tets, 0, 3 * q, [q, q], [3 * q, 3 * q])]), axis=0)
    dirs, pols = _draw_plane_waves(rng, n_pw)
    far = 1.0 / 12
    keep_out = lambda r: abs(r[2] - 0.5) < far or abs(r[0] - 0.375) < far
    dpos, dmom = _draw_dipoles(rng, n_dip, keep_out)
    return Problem("pec_plates", n, tuple(parts), xyz, tets, box_partition(n, parts), np.ones(tets.shape[0]),
                   k, -1j * k, dirs, pols, pec_faces=pec, dip_pos=dpos, dip_moment=dmom)


def make_batch_config(seed: int = 3, count: int = 32, n_range=(12, 32), nrhs=16, hex_size=0.125):
    """Configuration 3: ``count`` independent cube problems at one frequency.

    n ~ U{n_range}; boxes per axis p = clip(ceil(n/8), 2, 4); box cuts at
    round(b*n/p) plus a seeded jitter in {-1, 0, +1} (keeping >= 2 hexes per
    box); eps_r ~ U[1, 4]; ``nrhs`` plane waves each.  Every cube has hexes
    of side ``hex_size`` (1/8: eight hexes per free-space wavelength at
    k = 2*pi), so problem b is a cube of side n*hex_size wavelengths.  This is
    the unit cube at k = 2*pi*n/8 rescaled by n/8: stiffness, mass, absorbing
    and Robin terms of the edge-element system all scale by the same factor,
    so the two systems differ by one scalar and have the same solution up to
    that factor.  A shared k lets the problems be factored as one batch.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=count)
    k = 2 * math.pi
    probs = []
    for b, n in enumerate(ns):
        n = int(n)
        p = int(min(max(math.ceil(n / 8), 2), 4))
        cuts = []
        for _ax in range(3):
            c = [0]
            for m in range(1, p):
                c.append(int(round(m * n / p)) + int(rng.integers(-1, 2)))
            c.append(n)
            # keep at least two hexes per box
            for m in range(1, p):
                c[m] = max(c[m], c[m - 1] + 2)
            for m in range(p - 1, 0, -1):
                c[m] = min(c[m], c[m + 1] - 2)
            cuts.append(c)
        xyz, tets = kuhn_cube_mesh(n)
        xyz = xyz * (n * hex_size)
        part = box_partition(n, (p, p, p), cuts)
        eps_r = rng.uniform(1.0, 4.0, tets.shape[0])
        dirs, pols = _draw_plane_waves(rng, nrhs)
        probs.append(Problem(f"cfg3[{b}]", n, (p, p, p), xyz, tets, part, eps_r,
                             k, -1j * k, dirs, pols))
    return probs
