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
The thin-plate filter Z of eq. (force_filter) is not included.
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


def vertex_values(g: flow.Grid, p: np.ndarray, X: np.ndarray, n: np.ndarray):
    """Front and back Shepard values of p at point X for normal n (eq. (force)); None
    for a side without points."""
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
                side = 1 if s > 0.0 else -1
                d2 = float(r[0] * r[0] + r[1] * r[1] + r[2] * r[2])
                num[side] += float(p[k, j, i]) / d2
                den[side] += 1.0 / d2
    out = []
    for side in (1, -1):
        out.append(num[side] / den[side] if den[side] > 0.0 else None)
    return out[0], out[1]


def surface_pressure(g: flow.Grid, p: np.ndarray, tri: np.ndarray):
    """Per triangle: (front, back) pressure (NaN for a side without value), and the
    total pressure force sum A n (p- - p+) over the triangles."""
    tri = np.asarray(tri, dtype=np.float64)
    n, area = triangle_frames(tri)
    side = np.full((len(tri), 2), np.nan)
    force = np.zeros(3)
    for t in range(len(tri)):
        if not (area[t] > 0.0 and np.isfinite(area[t])):   # degenerate, overflowing or non-finite
            continue
        vals = [vertex_values(g, p, tri[t, v], n[t]) for v in range(3)]
        for s in range(2):
            have = [vv[s] for vv in vals if vv[s] is not None]
            if have:
                side[t, s] = sum(have) / len(have)
        pf = 0.0 if np.isnan(side[t, 0]) else side[t, 0]
        pb = 0.0 if np.isnan(side[t, 1]) else side[t, 1]
        force += area[t] * n[t] * (pb - pf)
    return side, force
