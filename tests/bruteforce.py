"""Exact brute-force references used to pin the oracle (pure Python, Fractions).

Every segment between two face-adjacent cell centres is tested against every
triangle with exact rational arithmetic, solving the segment/triangle system
P0 + t (P1 - P0) = A + beta (B - A) + gamma (C - A) by Cramer's rule
(the Moller-Trumbore system, Sec. 2.3.1, solved exactly).  A triangle whose
plane is parallel to the segment never blocks it.
"""
from fractions import Fraction as Fr


def _det3(a, b, c):
    return (a[0] * (b[1] * c[2] - b[2] * c[1])
            - a[1] * (b[0] * c[2] - b[2] * c[0])
            + a[2] * (b[0] * c[1] - b[1] * c[0]))


def seg_tri(P0, P1, A, B, C, eps=0):
    """Exact closed-segment / closed-triangle test; returns the parameter t in [0,1] or None.
    eps > 0 widens the triangle: barycentric coordinates down to -eps count as inside
    (the ray test's tolerance)."""
    D = [P1[i] - P0[i] for i in range(3)]
    E1 = [B[i] - A[i] for i in range(3)]
    E2 = [C[i] - A[i] for i in range(3)]
    R = [P0[i] - A[i] for i in range(3)]
    # t*D - beta*E1 - gamma*E2 = -R  ->  columns (D, -E1, -E2)
    M = [[D[i], -E1[i], -E2[i]] for i in range(3)]
    cols = list(zip(*M))
    det = _det3(*cols)
    if det == 0:
        return None
    rhs = [-R[i] for i in range(3)]

    def rep(j):
        cc = list(cols)
        cc[j] = tuple(rhs)
        return _det3(*cc)
    t = Fr(rep(0)) / det
    beta = Fr(rep(1)) / det
    gamma = Fr(rep(2)) / det
    e = Fr(eps)
    if t < 0 or t > 1 or beta < -e or gamma < -e or beta + gamma > 1 + e:
        return None
    return t


def brute_tag(tri, n, dx, origin, eps=0):
    """Returns dict (flat cell, dir) -> exact theta (Fraction) over all blocked pairs."""
    nx, ny, nz = n
    dxf = Fr(dx)
    org = [Fr(o) for o in origin]
    T = [[[Fr(float(v)) for v in vert] for vert in t] for t in tri]

    def centre(i, j, k):
        return [org[0] + (Fr(i) + Fr(1, 2)) * dxf, org[1] + (Fr(j) + Fr(1, 2)) * dxf,
                org[2] + (Fr(k) + Fr(1, 2)) * dxf]
    out = {}
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                ca = i + nx * (j + ny * k)
                for ax, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    i2, j2, k2 = i + di, j + dj, k + dk
                    if i2 >= nx or j2 >= ny or k2 >= nz:
                        continue
                    cb = i2 + nx * (j2 + ny * k2)
                    P0, P1 = centre(i, j, k), centre(i2, j2, k2)
                    best = None
                    for (A, B, C) in T:
                        t = seg_tri(P0, P1, A, B, C, eps)
                        if t is not None:
                            best = t if best is None else min(best, t)
                    if best is None:
                        continue
                    worst = None
                    for (A, B, C) in T:
                        t = seg_tri(P0, P1, A, B, C, eps)
                        if t is not None:
                            worst = t if worst is None else max(worst, t)
                    out[(ca, 2 * ax + 1)] = best
                    out[(cb, 2 * ax)] = 1 - worst
    return out


def inside_parity(pt, tri):
    """Ray parity along +x with a slightly skewed direction (generic position)."""
    P0 = [Fr(v) for v in pt]
    P1 = [P0[0] + Fr(10 ** 6), P0[1] + Fr(1, 7919), P0[2] + Fr(1, 104729)]
    cnt = 0
    for t in tri:
        # the ray moves < 1e-3 in y and z: triangles whose y/z extent misses it cannot count
        if (min(t[:, 1]) > pt[1] + 1e-3 or max(t[:, 1]) < pt[1] - 1e-3
                or min(t[:, 2]) > pt[2] + 1e-3 or max(t[:, 2]) < pt[2] - 1e-3):
            continue
        A, B, C = ([Fr(float(v)) for v in vert] for vert in t)
        if seg_tri(P0, P1, A, B, C) is not None:
            cnt += 1
    return cnt % 2
