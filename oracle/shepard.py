"""Near-field surface force oracle (test infrastructure only; the product path never
imports it): Shepard interpolation of the cell-centre pressure at the surface vertices,
split into the front and back side of each triangle (eq. (force)).

What is computed (plain FP64 numpy, one vertex at a time in the paper's notation):

* For a surface point X (a triangle vertex) the surrounding grid points x^(k) are the
  cell centres of the eight cells whose centres span the dual cell containing X
  (cells (i0 + a, j0 + b, k0 + c), a, b, c in {0, 1}, i0 = floor((X - origin)/dx - 1/2));
  points outside the domain are dropped.  Every cell holds a pressure in this method
  (there is no solid/fluid classification; a closed body's interior is its own
  pressure component).
* The weight of x^(k) is S = delta(n . (X - x^(k))) / |X - x^(k)|^2 with n the unit
  normal of the triangle (right-handed vertex order).  The delta selects a side: the
  front value f+(X) averages the points with n . (x^(k) - X) > 0, the back value f-(X)
  those with n . (x^(k) - X) < 0; points in the triangle's plane belong to neither.
  f(X) = sum S f_k / sum S (a point at distance 0 lies in the plane and is dropped).
  A side without points has no value.
* A triangle's side value is the mean of its vertices' values on that side (over the
  vertices that have one); its pressure force is A n (p- - p+), a side without value
  contributing nothing.  The force on the surface is the sum over triangles.

Readings (the paper leaves these open): the eight dual-cell points as the
"surrounding fluid points", the sign convention of the front/back split, vertex values
combined per triangle by their mean, and the triangle area as the integration weight.

Thin-plate filter Z of eq. (force_filter) (optional, `thin_filter`): a surrounding point
x^(k) gets weight zero at the vertex X when the segment from X to x^(k) crosses a
triangle of the surface at a parameter t in (T_MIN, 1] (t = 0 at X; contacts at X
itself, where the neighbouring triangles of the vertex meet, do not count).  Such a
point lies behind another surface, as the back side of a plate thinner than a cell does
from its front face; the paper cancels exactly those values.  The crossing test is
Moller and Trumbore's (J. Graphics Tools 2, 1997; the paper names the method for its
ray tests), edges inclusive, with its FP64 operations in one fixed order.
"""
from __future__ import annotations

import numpy as np

from . import flow


def triangle_frames(tri: np.ndarray):
    """Unit normals (right-handed vertex order) and areas of triangles (ntri, 3, 3);
    degenerate triangles get normal 0 and area 0 (non-finite ones NaN).  Sums are
    written out left to right (one fixed FP64 operation order)."""
    tri = np.asarray(tri, dtype=np.float64)
    e1 = tri[:, 1] - tri[:, 0]
    e2 = tri[:, 2] - tri[:, 0]
    c = np.stack([e1[:, 1] * e2[:, 2] - e1[:, 2] * e2[:, 1],
                  e1[:, 2] * e2[:, 0] - e1[:, 0] * e2[:, 2],
                  e1[:, 0] * e2[:, 1] - e1[:, 1] * e2[:, 0]], axis=1)
    two_a = np.sqrt(c[:, 0] * c[:, 0] + c[:, 1] * c[:, 1] + c[:, 2] * c[:, 2])
    n = np.zeros_like(c)
    ok = two_a > 0.0
    n[ok] = c[ok] / two_a[ok, None]
    return n, 0.5 * two_a


T_MIN = 1e-6


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0])


def _dot(a, b):
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]


def segment_hits(P, Q, tri: np.ndarray) -> np.ndarray:
    """For each triangle (ntri, 3, 3): whether the segment P + t (Q - P) meets it at
    some t in (T_MIN, 1] (Moller-Trumbore, edges inclusive, parallel never)."""
    D = tuple(float(Q[a]) - float(P[a]) for a in range(3))
    V0, V1, V2 = tri[:, 0], tri[:, 1], tri[:, 2]
    E1 = (V1[:, 0] - V0[:, 0], V1[:, 1] - V0[:, 1], V1[:, 2] - V0[:, 2])
    E2 = (V2[:, 0] - V0[:, 0], V2[:, 1] - V0[:, 1], V2[:, 2] - V0[:, 2])
    Pv = _cross(D, E2)
    det = _dot(E1, Pv)
    ok = det != 0.0
    inv = np.divide(1.0, det, out=np.zeros_like(det), where=ok)
    T = (float(P[0]) - V0[:, 0], float(P[1]) - V0[:, 1], float(P[2]) - V0[:, 2])
    u = _dot(T, Pv) * inv
    Qv = _cross(T, E1)
    v = _dot(D, Qv) * inv
    t = _dot(E2, Qv) * inv
    return ok & (u >= 0.0) & (u <= 1.0) & (v >= 0.0) & (u + v <= 1.0) & (t > T_MIN) & (t <= 1.0)


def vertex_values(g: flow.Grid, p: np.ndarray, X: np.ndarray, n: np.ndarray, occluders=None):
    """Front and back Shepard values of p at point X for normal n (eq. (force)); None
    for a side without points.  occluders (ntri, 3, 3): apply the thin-plate filter Z
    against these triangles."""
    nz, ny, nx = g.shape
    o = np.asarray(g.origin, dtype=np.float64)
    fb = np.floor((X - o) / g.dx - 0.5)
    lim = np.array([nx, ny, nz], dtype=np.float64) + 1.0
    if not np.all((fb >= -2.0) & (fb <= lim)):
        return None, None   # dual cell wholly outside the grid (or a non-finite X)
    base = fb.astype(np.int64)
    num = {1: 0.0, -1: 0.0}
    den = {1: 0.0, -1: 0.0}
    for c in range(2):
        for b in range(2):
            for a in range(2):
                i, j, k = base[0] + a, base[1] + b, base[2] + c
                if not (0 <= i < nx and 0 <= j < ny and 0 <= k < nz):
                    continue
                x = o + (np.array([i, j, k], dtype=np.float64) + 0.5) * g.dx
                r = x - X
                s = float(n[0] * r[0] + n[1] * r[1] + n[2] * r[2])
                if s == 0.0:
                    continue
                if occluders is not None and len(occluders) and np.any(segment_hits(X, x, occluders)):
                    continue
                side = 1 if s > 0.0 else -1
                d2 = float(r[0] * r[0] + r[1] * r[1] + r[2] * r[2])
                num[side] += float(p[k, j, i]) / d2
                den[side] += 1.0 / d2
    out = []
    for side in (1, -1):
        out.append(num[side] / den[side] if den[side] > 0.0 else None)
    return out[0], out[1]


def _near(tri: np.ndarray, lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    """Triangles whose bounding box meets the box [lo, hi] (a prefilter only)."""
    tmin = tri.min(axis=1)
    tmax = tri.max(axis=1)
    return tri[np.all((tmax >= lo) & (tmin <= hi), axis=1)]


def surface_pressure(g: flow.Grid, p: np.ndarray, tri: np.ndarray, thin_filter: bool = False, surface=None):
    """Per triangle: (front, back) pressure (NaN for a side without value), and the
    total pressure force sum A n (p- - p+) over the triangles.  thin_filter: the filter
    Z of eq. (force_filter) against the triangles of `surface` (default: tri itself)."""
    tri = np.asarray(tri, dtype=np.float64)
    surf = tri if surface is None else np.asarray(surface, dtype=np.float64)
    n, area = triangle_frames(tri)
    side = np.full((len(tri), 2), np.nan)
    force = np.zeros(3)
    for t in range(len(tri)):
        if not (area[t] > 0.0 and np.isfinite(area[t])):   # degenerate, overflowing or non-finite
            continue
        occ = None
        if thin_filter:
            lo = tri[t].min(axis=0) - 2.0 * g.dx
            hi = tri[t].max(axis=0) + 2.0 * g.dx
            occ = _near(surf, lo, hi)
        vals = [vertex_values(g, p, tri[t, v], n[t], occ) for v in range(3)]
        for s in range(2):
            have = [vv[s] for vv in vals if vv[s] is not None]
            if have:
                side[t, s] = sum(have) / len(have)
        pf = 0.0 if np.isnan(side[t, 0]) else side[t, 0]
        pb = 0.0 if np.isnan(side[t, 1]) else side[t, 1]
        force += area[t] * n[t] * (pb - pf)
    return side, force
