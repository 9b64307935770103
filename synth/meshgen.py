"""Seeded synthetic boundary meshes and boundary-condition recipes.

This module is an *input generator*: it writes vertex coordinates, triangle
connectivity (oriented so that the right-hand-rule normal points out of the
elastic domain), a per-element boundary-condition kind and the spatial shape
of the prescribed boundary value.  It contains none of the boundary-element
arithmetic (no kernels, no quadrature, no assembly), so both the CPU oracle
and the GPU path may consume its output.

Workloads mirror the paper's examples: a pressurised spherical cavity in full
space (an exterior Neumann problem), a prismatic rod with a step traction at
one end and the other end fixed (Section 4.1, the paper's first example), and
an elastic block with many spherical cavities loaded by a step traction on one
face and fixed on the opposite face (Section 4.3, the porous-solid example).

Boundary-condition kinds: 0 = traction prescribed (displacement unknown),
1 = displacement prescribed (traction unknown).  ``bc_shape`` is the
prescribed vector per element; the Laplace-domain value at parameter s is
``bc_shape * load_factor(s)`` with ``load_factor = 1/s`` for a Heaviside step.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

TRACTION = 0
DISPLACEMENT = 1


@dataclass
class Mesh:
    xyz: np.ndarray            # (nv, 3) float64
    tri: np.ndarray            # (nt, 3) int32, normal = (v1-v0)x(v2-v0) points out of the solid
    bc_kind: np.ndarray        # (nt,) int8
    bc_shape: np.ndarray       # (nt, 3) float64
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_unknowns(self) -> int:
        return 3 * self.n_tri


def _face_normals(xyz, tri):
    p0, p1, p2 = xyz[tri[:, 0]], xyz[tri[:, 1]], xyz[tri[:, 2]]
    c = np.cross(p1 - p0, p2 - p0)
    return c / np.linalg.norm(c, axis=1, keepdims=True)


def _orient(xyz, tri, want_dir):
    """Flip triangles whose right-hand normal disagrees with ``want_dir`` (nt,3)."""
    nrm = _face_normals(xyz, tri)
    flip = np.einsum("ij,ij->i", nrm, want_dir) < 0
    tri = tri.copy()
    tri[flip] = tri[flip][:, [0, 2, 1]]
    return tri


def icosphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0), inward: bool = True):
    """Icosahedron refined ``level`` times by edge midpoints projected onto the sphere.

    20*4**level triangles, 10*4**level+2 vertices.  ``inward`` orients the
    normals toward the centre (a cavity: the solid is outside)."""
    phi = (1.0 + 5.0 ** 0.5) / 2.0
    v = [(-1, phi, 0), (1, phi, 0), (-1, -phi, 0), (1, -phi, 0),
         (0, -1, phi), (0, 1, phi), (0, -1, -phi), (0, 1, -phi),
         (phi, 0, -1), (phi, 0, 1), (-phi, 0, -1), (-phi, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = [np.array(p, dtype=np.float64) / np.linalg.norm(p) for p in v]
    faces = [tuple(t) for t in f]
    for _ in range(level):
        cache = {}

        def mid(a, b):
            key = (a, b) if a < b else (b, a)
            if key not in cache:
                m = verts[a] + verts[b]
                verts.append(m / np.linalg.norm(m))
                cache[key] = len(verts) - 1
            return cache[key]

        nf = []
        for a, b, c in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = nf
    xyz = np.array(verts) * radius + np.asarray(center, dtype=np.float64)
    tri = np.array(faces, dtype=np.int32)
    cen = xyz[tri].mean(axis=1)
    outward = cen - np.asarray(center, dtype=np.float64)
    tri = _orient(xyz, tri, -outward if inward else outward)
    return xyz, tri


def box(lo, hi, nx: int, ny: int, nz: int):
    """Closed surface of the box [lo, hi] with an (nx, ny, nz) grid of squares
    per face pair, two triangles per square, outward normals, shared vertices.

    Returns xyz, tri and a per-triangle face id: 0/1 = x-/x+, 2/3 = y-/y+,
    4/5 = z-/z+."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    n = (nx, ny, nz)
    index = {}
    verts = []

    def vid(ijk):
        if ijk not in index:
            index[ijk] = len(verts)
            verts.append(lo + (hi - lo) * np.array(ijk, dtype=np.float64) / np.array(n, dtype=np.float64))
        return index[ijk]

    tris, fid, outdir = [], [], []
    for axis in range(3):
        a1, a2 = [d for d in range(3) if d != axis]
        for side in (0, 1):
            for i in range(n[a1]):
                for j in range(n[a2]):
                    def g(di, dj):
                        ijk = [0, 0, 0]
                        ijk[axis] = side * n[axis]
                        ijk[a1] = i + di
                        ijk[a2] = j + dj
                        return vid(tuple(ijk))
                    q = (g(0, 0), g(1, 0), g(1, 1), g(0, 1))
                    # alternate the diagonal so the pattern has no preferred direction
                    if (i + j) % 2 == 0:
                        tt = [(q[0], q[1], q[2]), (q[0], q[2], q[3])]
                    else:
                        tt = [(q[0], q[1], q[3]), (q[1], q[2], q[3])]
                    d = np.zeros(3)
                    d[axis] = 1.0 if side else -1.0
                    for t in tt:
                        tris.append(t)
                        fid.append(2 * axis + side)
                        outdir.append(d)
    xyz = np.array(verts)
    tri = _orient(xyz, np.array(tris, dtype=np.int32), np.array(outdir))
    return xyz, tri, np.array(fid, dtype=np.int8)


def _merge(parts):
    xyz_all, tri_all, off = [], [], 0
    for xyz, tri in parts:
        xyz_all.append(xyz)
        tri_all.append(tri + off)
        off += xyz.shape[0]
    return np.concatenate(xyz_all), np.concatenate(tri_all).astype(np.int32)


def cavity(level: int, radius: float = 1.0) -> Mesh:
    """Spherical cavity of radius ``radius`` in full space under unit internal
    pressure: traction prescribed everywhere, t = -p n with n pointing into the
    cavity (out of the solid), so ``bc_shape = -n``."""
    xyz, tri = icosphere(level, radius, inward=True)
    nrm = _face_normals(xyz, tri)
    nt = tri.shape[0]
    return Mesh(xyz, tri, np.zeros(nt, np.int8), -nrm, name=f"cavity_L{level}",
                meta={"level": level, "radius": radius})


@dataclass
class QuadMesh:
    """Six-node (curved quadratic) triangles: corners v0 v1 v2, then the
    mid-edge nodes of edges 01, 12, 20; the corner order follows the same
    orientation rule as ``Mesh.tri``.  Loads are given as a pressure per element
    (traction -p n on the surface, n out of the solid), since the normal varies
    over a curved element."""
    xyz: np.ndarray            # (nv, 3) float64
    tri6: np.ndarray           # (nt, 6) int32
    bc_kind: np.ndarray        # (nt,) int8
    pressure: np.ndarray       # (nt,) float64
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_tri(self) -> int:
        return int(self.tri6.shape[0])

    @property
    def n_nodes(self) -> int:
        """Unknown-carrying points: six per element."""
        return 6 * self.n_tri

    @property
    def n_unknowns(self) -> int:
        return 18 * self.n_tri


def quadratic_sphere(level: int, radius: float = 1.0, center=(0.0, 0.0, 0.0), inward: bool = True):
    """The icosphere of ``level`` with a node at each edge midpoint projected
    onto the sphere: (xyz, tri6)."""
    xyz, tri = icosphere(level, radius, center, inward)
    c = np.asarray(center, dtype=np.float64)
    pts = [p for p in xyz]
    cache = {}

    def mid(a, b):
        key = (a, b) if a < b else (b, a)
        if key not in cache:
            m = 0.5 * (xyz[a] + xyz[b]) - c
            pts.append(c + radius * m / np.linalg.norm(m))
            cache[key] = len(pts) - 1
        return cache[key]

    tri6 = np.array([(a, b, cc, mid(a, b), mid(b, cc), mid(cc, a)) for a, b, cc in tri], dtype=np.int32)
    return np.array(pts), tri6


def cavity_quadratic(level: int, radius: float = 1.0) -> QuadMesh:
    """The spherical cavity under unit internal pressure on six-node elements
    (20 * 4**level elements, 120 * 4**level unknown-carrying points)."""
    xyz, tri6 = quadratic_sphere(level, radius, inward=True)
    nt = tri6.shape[0]
    return QuadMesh(xyz, tri6, np.zeros(nt, np.int8), np.ones(nt), name=f"cavity_q{level}",
                    meta={"level": level, "radius": radius})


def rod(length: float, width: float, n_w: int, n_l: int) -> Mesh:
    """Prismatic rod [0,w]^2 x [0,L]: fixed at z=0 (u=0), unit axial traction
    +e_z on z=L, lateral faces traction free (the paper's first example, in
    unit material)."""
    xyz, tri, fid = box((0, 0, 0), (width, width, length), n_w, n_w, n_l)
    nt = tri.shape[0]
    kind = np.zeros(nt, np.int8)
    shape = np.zeros((nt, 3))
    kind[fid == 4] = DISPLACEMENT
    shape[fid == 5] = (0.0, 0.0, 1.0)
    return Mesh(xyz, tri, kind, shape, name=f"rod_{n_w}x{n_l}",
                meta={"length": length, "width": width})


def porous_block(side: float, n_face: int, voids, void_level) -> Mesh:
    """Cube [0,side]^3 (n_face x n_face squares per face) with spherical voids.

    ``voids`` is a list of (cx, cy, cz, r); ``void_level`` an int or a list.
    Loads follow the paper's porous-solid example: step traction +e_z on the
    z=0 face, z=side face fixed, every other surface traction free."""
    xyz, tri, fid = box((0, 0, 0), (side, side, side), n_face, n_face, n_face)
    nt_box = tri.shape[0]
    parts = [(xyz, tri)]
    levels = void_level if isinstance(void_level, (list, tuple, np.ndarray)) else [void_level] * len(voids)
    for (cx, cy, cz, r), lv in zip(voids, levels):
        parts.append(icosphere(int(lv), r, center=(cx, cy, cz), inward=True))
    xyz, tri = _merge(parts)
    nt = tri.shape[0]
    kind = np.zeros(nt, np.int8)
    shape = np.zeros((nt, 3))
    kind[:nt_box][fid == 5] = DISPLACEMENT
    shape[:nt_box][fid == 4] = (0.0, 0.0, 1.0)
    return Mesh(xyz, tri, kind, shape, name="porous_block",
                meta={"side": side, "n_face": n_face, "voids": [list(map(float, v)) for v in voids],
                      "void_levels": [int(l) for l in levels]})


def lattice_voids(side: float, per_axis: int, rmin: float, rmax: float, gap: float, seed: int):
    """One void per cell of a per_axis^3 lattice; radius ~U[rmin, rmax]; the
    centre is uniform in the cell shrunk by r+gap, so voids never overlap each
    other or the outer faces."""
    rng = np.random.default_rng(seed)
    cell = side / per_axis
    out = []
    for i in range(per_axis):
        for j in range(per_axis):
            for k in range(per_axis):
                r = rng.uniform(rmin, rmax)
                lo = np.array([i, j, k]) * cell + r + gap
                hi = np.array([i + 1, j + 1, k + 1]) * cell - r - gap
                c = rng.uniform(lo, hi)
                out.append((c[0], c[1], c[2], r))
    return out


def random_block(seed: int, side: float = 4.0) -> Mesh:
    """Seeded block for the batched workload: 1-8 voids placed in distinct cells
    of the 2x2x2 lattice, r~U[0.2,0.5], void level in {1,2,3}; the face
    resolution and void level are chosen so the unknown count lands near a
    target drawn from U[2000, 20000]."""
    rng = np.random.default_rng(seed)
    n_voids = int(rng.integers(1, 9))
    cells = rng.permutation(8)[:n_voids]
    target = int(rng.integers(2000, 20001))
    cell = side / 2
    voids = []
    for c in cells:
        i, j, k = (c >> 2) & 1, (c >> 1) & 1, c & 1
        r = rng.uniform(0.2, 0.5)
        lo = np.array([i, j, k]) * cell + r + 0.1
        hi = np.array([i + 1, j + 1, k + 1]) * cell - r - 0.1
        ctr = rng.uniform(lo, hi)
        voids.append((ctr[0], ctr[1], ctr[2], r))
    best = None
    for lv in (1, 2, 3):
        nv_el = n_voids * 20 * 4 ** lv
        for n in range(4, 40):
            nu = 3 * (12 * n * n + nv_el)
            err = abs(nu - target) / target
            if best is None or err < best[0]:
                best = (err, n, lv)
    _, n, lv = best
    m = porous_block(side, n, voids, lv)
    m.name = f"random_block_{seed}"
    m.meta.update({"seed": seed, "target_unknowns": target})
    return m


def lattice_block(per_axis: int, n_face: int, void_level: int, seed: int, side: float = 4.0,
                  rmin: float = 0.2, rmax: float = 0.5) -> Mesh:
    """Porous block with per_axis^3 voids in a lattice (the learned and
    full-size workloads: 27 voids, n_face=20, level 2 gives 13,440 elements)."""
    cell = side / per_axis
    rmax = min(rmax, cell / 2 - 0.05 - 1e-9)
    voids = lattice_voids(side, per_axis, rmin, rmax, 0.05 if per_axis > 3 else 0.1, seed)
    m = porous_block(side, n_face, voids, void_level)
    m.name = f"lattice_block_{per_axis}^3_n{n_face}_L{void_level}"
    m.meta.update({"seed": seed})
    return m


def fsm_parameters(T: float, kappa: float, Ns: int):
    """Frequency grid of the Fourier-series method (Section 2.2): period T,
    abscissa eta = kappa ln10 / T, frequencies s_k = eta + i k 2pi/T."""
    eta = kappa * np.log(10.0) / T
    dw = 2 * np.pi / T
    return eta, dw


def cavity_frequencies(n: int, T: float = 20.0):
    """Laplace parameters of the cavity workloads: s_k = 5/T + i k pi/T."""
    return (5.0 / T) + 1j * np.arange(n) * np.pi / T


def block_frequencies(n: int = 24, T: float = 300.0, kappa: float = 3.0, Ns: int = 512, seed: int = 0):
    """Laplace parameters of the porous-block workloads: n points on the line
    Re s = eta of the band omega in [0, Omega_s], Omega_s = (Ns/2) 2pi/T:
    omega = 0 plus n-1 seeded uniform draws, sorted (the mix of low and high
    frequencies that an adaptive sampling round asks for)."""
    eta, dw = fsm_parameters(T, kappa, Ns)
    om_max = (Ns // 2) * dw
    rng = np.random.default_rng(seed)
    om = np.sort(np.concatenate([[0.0], rng.uniform(0.0, om_max, n - 1)]))
    return eta + 1j * om
