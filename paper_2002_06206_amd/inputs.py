"""Seeded synthetic inputs shared by the HIP path, the oracle and the tests.

This module holds no arithmetic of the immersed boundary method itself: it
only builds triangle soups (the immersed surface Gamma_IB of Sec. 2, given as
an arbitrary, possibly "dirty" set of triangles), grid descriptions and seeded
random arrays.  Every geometry is returned as a C-contiguous float64 array of
shape (ntri, 3, 3): triangle, vertex, xyz.

The workloads stand in for the paper's geometries (sphere set, flat plate,
full vehicle, Sec. 3), which are not available: sizes, triangle counts and
defect kinds follow the dirty-geometry taxonomy of Sec. 2.3 (gaps, overlaps,
flipped faces, intersections, zero thickness, sub-cell channels).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

# Face order used everywhere: -x, +x, -y, +y, -z, +z.
PERIODIC, INFLOW, OUTFLOW, SLIP = 0, 1, 2, 3


@dataclasses.dataclass
class Case:
    """A complete synthetic problem: grid, boundary kinds, geometry and flow constants."""
    name: str
    n: tuple            # cells (nx, ny, nz)
    dx: float
    origin: tuple
    bc: tuple           # six face kinds, order -x,+x,-y,+y,-z,+z
    u_in: tuple
    tri: np.ndarray     # (ntri, 3, 3) float64
    nu: float
    dt: float
    steps: int
    csm: bool = True
    deadend: bool = False
    ref_length: float = 1.0   # length used for Re and for the drag reference area
    ref_area: float = 1.0


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotation matrix (QR of a Gaussian matrix, sign-fixed)."""
    a = rng.standard_normal((3, 3))
    q, r = np.linalg.qr(a)
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def rot_z(deg: float) -> np.ndarray:
    t = math.radians(deg)
    c, s = math.cos(t), math.sin(t)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _icosahedron():
    p = (1.0 + math.sqrt(5.0)) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], dtype=np.float64)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], dtype=np.int64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    return v, f


def icosphere(level: int, radius: float, centre, rot: np.ndarray | None = None) -> np.ndarray:
    """Icosahedron subdivided `level` times (20*4^level triangles), projected to the sphere."""
    v, f = _icosahedron()
    verts = [tuple(x) for x in v]
    for _ in range(level):
        cache = {}
        nv = list(verts)
        nf = []

        def mid(a, b):
            key = (min(a, b), max(a, b))
            if key not in cache:
                m = (np.asarray(nv[a]) + np.asarray(nv[b])) * 0.5
                m = m / np.linalg.norm(m)
                cache[key] = len(nv)
                nv.append(tuple(m))
            return cache[key]

        for a, b, c in f:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            nf += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        verts, f = nv, np.array(nf, dtype=np.int64)
    vv = np.asarray(verts, dtype=np.float64)
    if rot is not None:
        vv = vv @ rot.T
    vv = vv * radius + np.asarray(centre, dtype=np.float64)
    return np.ascontiguousarray(vv[f])


def uv_ellipsoid(semi, centre, rot, nu_: int = 32, nv_: int = 32) -> np.ndarray:
    """UV-sphere mesh scaled to an ellipsoid: nu_ longitudes, nv_ latitude bands."""
    tris = []
    th = np.linspace(0.0, math.pi, nv_ + 1)
    ph = np.linspace(0.0, 2 * math.pi, nu_ + 1)

    def pt(i, j):
        return np.array([math.sin(th[i]) * math.cos(ph[j]),
                         math.sin(th[i]) * math.sin(ph[j]),
                         math.cos(th[i])])
    for i in range(nv_):
        for j in range(nu_):
            a, b, c, d = pt(i, j), pt(i, j + 1), pt(i + 1, j), pt(i + 1, j + 1)
            if i == 0:
                tris.append((a, d, c))
            elif i == nv_ - 1:
                tris.append((a, b, c))
            else:
                tris.append((a, b, c))
                tris.append((b, d, c))
    t = np.array(tris, dtype=np.float64) * np.asarray(semi, dtype=np.float64)
    t = t @ np.asarray(rot).T + np.asarray(centre, dtype=np.float64)
    return np.ascontiguousarray(t)


def rectangle(centre, e1, e2, n1: int = 1, n2: int = 1) -> np.ndarray:
    """Planar rectangle centre +- e1/2 +- e2/2, split into n1*n2 quads, 2 triangles each."""
    c = np.asarray(centre, dtype=np.float64)
    e1 = np.asarray(e1, dtype=np.float64)
    e2 = np.asarray(e2, dtype=np.float64)
    out = []
    for a in range(n1):
        for b in range(n2):
            p00 = c + e1 * (a / n1 - 0.5) + e2 * (b / n2 - 0.5)
            p10 = c + e1 * ((a + 1) / n1 - 0.5) + e2 * (b / n2 - 0.5)
            p01 = c + e1 * (a / n1 - 0.5) + e2 * ((b + 1) / n2 - 0.5)
            p11 = c + e1 * ((a + 1) / n1 - 0.5) + e2 * ((b + 1) / n2 - 0.5)
            out.append((p00, p10, p11))
            out.append((p00, p11, p01))
    return np.ascontiguousarray(np.array(out, dtype=np.float64))


def disc(centre, normal_rot, radius: float, nseg: int = 64) -> np.ndarray:
    """Zero-thickness disc as a fan of nseg triangles in the local xy plane."""
    c = np.asarray(centre, dtype=np.float64)
    out = []
    for s in range(nseg):
        a0 = 2 * math.pi * s / nseg
        a1 = 2 * math.pi * (s + 1) / nseg
        p0 = np.array([radius * math.cos(a0), radius * math.sin(a0), 0.0])
        p1 = np.array([radius * math.cos(a1), radius * math.sin(a1), 0.0])
        out.append((np.zeros(3), p0, p1))
    t = np.array(out) @ np.asarray(normal_rot).T + c
    return np.ascontiguousarray(t)


def extruded_polygon(xy: np.ndarray, z0: float, z1: float) -> np.ndarray:
    """Closed polygon (m,2) extruded along z from z0 to z1 as 2m side triangles (no caps)."""
    m = len(xy)
    out = []
    for s in range(m):
        a = xy[s]
        b = xy[(s + 1) % m]
        p0 = (a[0], a[1], z0)
        p1 = (b[0], b[1], z0)
        p2 = (b[0], b[1], z1)
        p3 = (a[0], a[1], z1)
        out.append((p0, p1, p2))
        out.append((p0, p2, p3))
    return np.ascontiguousarray(np.array(out, dtype=np.float64))


def delete_fraction(tri: np.ndarray, frac: float, rng) -> np.ndarray:
    keep = rng.random(len(tri)) >= frac
    return np.ascontiguousarray(tri[keep])


def flip_fraction(tri: np.ndarray, frac: float, rng) -> np.ndarray:
    t = tri.copy()
    sel = rng.random(len(t)) < frac
    t[sel] = t[sel][:, [0, 2, 1], :]
    return np.ascontiguousarray(t)


# ---------------------------------------------------------------- workloads

def case_sphere32(seed: int = 0) -> Case:
    """32^3 cells, icosphere (320 triangles) of diameter 8 cells at the centre,
    inflow U=1, Re=100 on the diameter, CSM on, CFL 0.3."""
    rng = np.random.default_rng(seed)
    tri = icosphere(2, 4.0, (16.0, 16.0, 16.0), random_rotation(rng))
    return Case("sphere32", (32, 32, 32), 1.0, (0.0, 0.0, 0.0),
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=8.0 / 100.0, dt=0.3, steps=100, ref_length=8.0,
                ref_area=math.pi * 64.0 / 4.0)


def dirty_sphere(n: int, radius: float, seed: int, level: int = 5):
    """Icosphere with the dirty defects: 2% gaps, a duplicate shell 0.1 cell out with
    its own 2% gaps, 10% flipped triangles and an internal zero-thickness disc."""
    rng = np.random.default_rng(seed)
    c = (n / 2.0, n / 2.0, n / 2.0)
    rot = random_rotation(rng)
    outer = icosphere(level, radius, c, rot)
    outer = delete_fraction(outer, 0.02, rng)
    shell = icosphere(level, radius + 0.1, c, rot)
    shell = delete_fraction(shell, 0.02, rng)
    d = disc(c, random_rotation(rng), radius * 0.5, 64)
    tri = np.concatenate([outer, shell, d])
    tri = flip_fraction(tri, 0.10, rng)
    perm = rng.permutation(len(tri))
    return np.ascontiguousarray(tri[perm])


def case_dirty_sphere128(seed: int = 0) -> Case:
    """128^3 cells, dirty icosphere of diameter 24 cells (20,480 triangles per shell), Re=1e4."""
    tri = dirty_sphere(128, 12.0, seed)
    return Case("dirty_sphere128", (128, 128, 128), 1.0, (0.0, 0.0, 0.0),
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=24.0 / 1e4, dt=0.3, steps=500, ref_length=24.0,
                ref_area=math.pi * 24.0 ** 2 / 4.0)


def case_plate256(seed: int = 0, n: int = 256) -> Case:
    """Zero-thickness flat plate of 64x64 cells (8,192 triangles) at 30 deg incidence, Re=1e5."""
    c = np.array([n / 2.0, n / 2.0, n / 2.0])
    chord = 64.0 * n / 256.0
    r = rot_z(30.0)
    e1 = r @ np.array([chord, 0.0, 0.0])
    e2 = np.array([0.0, 0.0, chord])
    m = int(round(chord))
    tri = rectangle(c + np.array([0.013, 0.027, 0.0]), e1, e2, m, m)
    return Case("plate%d" % n, (n, n, n), 1.0, (0.0, 0.0, 0.0),
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=chord / 1e5, dt=0.3, steps=1000, ref_length=chord,
                ref_area=chord * chord)


def ellipsoid_field(n: int, seed: int, n_ell: int = 40, n_plate: int = 5,
                    gap: float = 0.03, uv: int = 32):
    """40 overlapping ellipsoids (semi-axes U[4,20], UV mesh ~2k triangles, 3% gaps)
    plus 5 thin plates (sides U[16,64]) with random pose; sizes scale with n/256."""
    rng = np.random.default_rng(seed)
    s = n / 256.0
    parts = []
    for _ in range(n_ell):
        semi = rng.uniform(4.0, 20.0, 3) * s
        centre = rng.uniform(32.0, 224.0, 3) * s
        e = uv_ellipsoid(semi, centre, random_rotation(rng), uv, uv)
        parts.append(delete_fraction(e, gap, rng))
    for _ in range(n_plate):
        a, b = rng.uniform(16.0, 64.0, 2) * s
        centre = rng.uniform(32.0, 224.0, 3) * s
        r = random_rotation(rng)
        parts.append(rectangle(centre, r[:, 0] * a, r[:, 1] * b))
    tri = np.concatenate(parts)
    return np.ascontiguousarray(tri[rng.permutation(len(tri))])


def case_ellipsoids256(seed: int = 0, n: int = 256) -> Case:
    """256^3 cells, 40 ellipsoids + 5 plates, Re=1e4 on the mean ellipsoid diameter (24 cells)."""
    tri = ellipsoid_field(n, seed)
    return Case("ellipsoids%d" % n, (n, n, n), 1.0, (0.0, 0.0, 0.0),
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=24.0 * n / 256.0 / 1e4, dt=0.3, steps=1000, ref_length=24.0)


def vehicle_like(n: int, seed: int, target_tri: int = 1_000_000):
    """Synthetic full-vehicle-like assembly: overlapping boxes and ellipsoids,
    intersecting zero-thickness plates, nested internal parts, 1% gaps and
    sub-cell channels (plate pairs 0.3-0.8 cell apart)."""
    rng = np.random.default_rng(seed)
    s = n / 1024.0
    parts = []
    body_c = np.array([0.45, 0.5, 0.42]) * n
    # main body: a large subdivided box (zero-thickness panels) and a nested inner box
    for scale, sub in ((1.0, 96), (0.6, 48)):
        ext = np.array([420.0, 170.0, 130.0]) * s * scale
        for ax in range(3):
            for sgn in (-1.0, 1.0):
                u = (ax + 1) % 3
                v = (ax + 2) % 3
                c = body_c.copy()
                c[ax] += sgn * ext[ax] / 2
                e1 = np.zeros(3)
                e1[u] = ext[u]
                e2 = np.zeros(3)
                e2[v] = ext[v]
                parts.append(rectangle(c, e1, e2, sub, sub))
    # wheels, mirrors, engine parts: ellipsoids
    n_ell = 160
    for _ in range(n_ell):
        semi = rng.uniform(6.0, 60.0, 3) * s
        centre = body_c + rng.uniform(-0.5, 0.5, 3) * np.array([480.0, 200.0, 160.0]) * s
        parts.append(uv_ellipsoid(semi, centre, random_rotation(rng), 48, 48))
    # intersecting plates
    for _ in range(200):
        a, b = rng.uniform(20.0, 200.0, 2) * s
        centre = body_c + rng.uniform(-0.5, 0.5, 3) * np.array([480.0, 200.0, 160.0]) * s
        r = random_rotation(rng)
        parts.append(rectangle(centre, r[:, 0] * a, r[:, 1] * b, 8, 8))
    # sub-cell channels: parallel plate pairs 0.3-0.8 cell apart
    for _ in range(60):
        a, b = rng.uniform(20.0, 80.0, 2) * s
        centre = body_c + rng.uniform(-0.5, 0.5, 3) * np.array([480.0, 200.0, 160.0]) * s
        r = random_rotation(rng)
        gapw = rng.uniform(0.3, 0.8)
        parts.append(rectangle(centre, r[:, 0] * a, r[:, 1] * b, 4, 4))
        parts.append(rectangle(centre + r[:, 2] * gapw, r[:, 0] * a, r[:, 1] * b, 4, 4))
    tri = np.concatenate(parts)
    if len(tri) > target_tri:
        tri = tri[rng.choice(len(tri), target_tri, replace=False)]
    tri = delete_fraction(tri, 0.01, rng)
    return np.ascontiguousarray(tri[rng.permutation(len(tri))])


def case_vehicle(n: int = 1024, seed: int = 0) -> Case:
    tri = vehicle_like(n, seed)
    return Case("vehicle%d" % n, (n, n, n), 1.0, (0.0, 0.0, 0.0),
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=512.0 * n / 1024.0 / 1e6, dt=0.3, steps=200, deadend=True,
                ref_length=512.0 * n / 1024.0)


# ------------------------------------------------------- verification geometry

def tgv_circle(n: int, nz: int = 4, radius: float = 1.0, m: int = 1024) -> np.ndarray:
    """Circle of radius 1 about the origin (m-gon), extruded through the z-extent."""
    dx = 4.0 / n
    a = 2 * math.pi * (np.arange(m) + 0.5) / m
    xy = np.stack([radius * np.cos(a), radius * np.sin(a)], axis=1)
    return extruded_polygon(xy, -dx, (nz + 1) * dx)


def tgv_square(n: int, nz: int = 4, rotated: bool = True) -> np.ndarray:
    """Square of side sqrt(2) about the origin; rotated=True puts its vertices on the unit circle."""
    dx = 4.0 / n
    if rotated:
        xy = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
    else:
        h = math.sqrt(2.0) / 2
        xy = np.array([[h, -h], [h, h], [-h, h], [-h, -h]])
    return extruded_polygon(xy, -dx, (nz + 1) * dx)


def channel_planes(y_lo: float, y_hi: float, lo: float, hi: float) -> np.ndarray:
    """Two planes y=y_lo and y=y_hi spanning [lo,hi] in x and z (2 triangles each)."""
    c = (lo + hi) / 2.0
    L = hi - lo
    p1 = rectangle((c, y_lo, c), (L, 0, 0), (0, 0, L))
    p2 = rectangle((c, y_hi, c), (L, 0, 0), (0, 0, L))
    return np.ascontiguousarray(np.concatenate([p1, p2]))


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.standard_normal(shape) * scale)


# ------------------------------------------------------------------ learned preconditioner

CNN_LAYERS = (("W1", 1, 16), ("W2", 16, 16), ("Wg", 1, 16))


def cnn_init_weights(seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded normal initial weights of the learned preconditioner, flat float32 in the
    layout W1[t, 0, co], W2[t, ci, co], Wg[t, 0, co] (t = 27 taps).  Standard
    deviations 0.05 (W1), 0.3 / sqrt(27 * 16) (W2) and 0.1 (Wg) keep the untrained
    operator a small addition to Jacobi; `scale` multiplies W1 and W2."""
    rng = np.random.default_rng(seed)
    std = {"W1": 0.05 * scale, "W2": 0.3 / math.sqrt(27 * 16) * scale, "Wg": 0.1}
    parts = [rng.standard_normal(27 * ci * co) * std[name] for name, ci, co in CNN_LAYERS]
    return np.ascontiguousarray(np.concatenate(parts).astype(np.float32))


def case_ellipsoid_window(seed: int, n: int = 64, field_n: int = 256) -> Case:
    """An n^3 window of the field_n^3 ellipsoid field of the given seed (same object
    sizes as the full workload), centred on a seeded triangle of the field so that it
    always holds geometry; inflow U=1 on -x, outflow on +x, slip elsewhere.  Used for
    training pairs and held-out evaluation of the learned preconditioner."""
    tri = ellipsoid_field(field_n, seed)
    rng = np.random.default_rng(seed + 7919)
    c = tri[rng.integers(len(tri)), 0]
    o = tuple(float(v) for v in np.clip(c - n / 2.0 + rng.uniform(-0.5, 0.5, 3), 0.0, field_n - n))
    return Case("ellipsoid_window%d" % n, (n, n, n), 1.0, o,
                (INFLOW, OUTFLOW, SLIP, SLIP, SLIP, SLIP), (1.0, 0.0, 0.0), tri,
                nu=24.0 / 1e4, dt=0.3, steps=100, ref_length=24.0)
