"""Pins for the tagging oracle (Sec. 2.3.1: ghost cells behind grid-line crossings).

The oracle (C, exact bignum signs) is checked against things it does not share
code with: exact rational brute force over every segment x every triangle,
hand-built geometries with known answers, inside/outside ray parity of closed
meshes, and the topology-free invariances the method claims.
"""
import itertools
import math
from fractions import Fraction as Fr

import numpy as np
import pytest

from bruteforce import brute_tag, inside_parity
from oracle import tagging
from paper_2002_06206_amd import inputs


def _o2d_exact(pu, pv, au, av, bu, bv):
    F = Fr
    d = (F(au) - F(pu)) * (F(bv) - F(pv)) - (F(av) - F(pv)) * (F(bu) - F(pu))
    return (d > 0) - (d < 0)


def test_orient2d_sign_matches_rationals():
    rng = np.random.default_rng(1)
    for _ in range(3000):
        v = rng.uniform(-50, 50, 6)
        if rng.random() < 0.5:
            # put p exactly on the line a-b with a dyadic parameter (exactly representable)
            t = rng.integers(-8, 9) / 8.0
            v[0] = v[2] + t * (v[4] - v[2])
            v[1] = v[3] + t * (v[5] - v[3])
            if rng.random() < 0.5:
                v[0] = np.nextafter(v[0], np.inf)
        got = tagging.orient2d_sign(*v)
        assert got == _o2d_exact(*v)


def test_orient2d_sign_extreme_exponents():
    cases = [(0.5, 0.5, 1e-300, 1e-300, 1.0, 1.0),
             (1e-200, 3e-200, 2e-200, 6e-200, 4e-200, 12e-200),
             (0.5, 0.5, 0.5 + 2 ** -52, 0.5, 0.5, 0.5 + 2 ** -52),
             (1e10, 1e-10, -1e10, 1e-10, 0.0, 1e-10 + 1e-26)]
    for c in cases:
        assert tagging.orient2d_sign(*c) == _o2d_exact(*c)


def test_crossing_sign_matches_rationals():
    rng = np.random.default_rng(2)
    for _ in range(800):
        A, B, C = rng.uniform(-10, 10, (3, 3))
        k = int(rng.integers(0, 3))
        u, v = (k + 1) % 3, (k + 2) % 3
        pu, pv = rng.uniform(-5, 5, 2)
        t = rng.uniform(-10, 10)
        if rng.random() < 0.3:
            # exact plane hit: t equal to a vertex coordinate on a vertex line
            pu, pv, t = A[u], A[v], A[k]
        F = Fr
        w_a = (F(B[u]) - F(pu)) * (F(C[v]) - F(pv)) - (F(B[v]) - F(pv)) * (F(C[u]) - F(pu))
        w_b = (F(C[u]) - F(pu)) * (F(A[v]) - F(pv)) - (F(C[v]) - F(pv)) * (F(A[u]) - F(pu))
        w_c = (F(A[u]) - F(pu)) * (F(B[v]) - F(pv)) - (F(A[v]) - F(pv)) * (F(B[u]) - F(pu))
        s = w_a * (F(A[k]) - F(t)) + w_b * (F(B[k]) - F(t)) + w_c * (F(C[k]) - F(t))
        assert tagging.crossing_sign(pu, pv, t, A, B, C, k) == (s > 0) - (s < 0)


def _compare_brute(tri, n, dx=1.0, origin=(0.0, 0.0, 0.0), eps=0.0):
    blocked, theta = tagging.tag(tri, n, dx, origin, eps)
    ref = brute_tag(tri, n, dx, origin, eps)
    bf = blocked.ravel()
    tf = theta.reshape(-1, 6)
    got = {(c, d) for c in range(len(bf)) for d in range(6) if (bf[c] >> d) & 1}
    assert got == set(ref.keys())
    for (c, d), t in ref.items():
        assert abs(tf[c, d] - float(t)) <= 1e-12
    open_ = [(c, d) for c in range(len(bf)) for d in range(6) if not (bf[c] >> d) & 1]
    assert all(tf[c, d] == 2.0 for c, d in open_)
    return blocked, theta


def test_brute_force_random_soup():
    rng = np.random.default_rng(3)
    n = (6, 5, 4)
    tri = rng.uniform(0.0, 6.0, (14, 3, 3)) * np.array([1.0, 5 / 6, 4 / 6])
    _compare_brute(tri, n)


def test_brute_force_snapped_soup_with_ties():
    # vertices on a half-cell lattice: edges and vertices land on grid lines and centres
    rng = np.random.default_rng(4)
    n = (5, 5, 5)
    tri = rng.integers(0, 11, (16, 3, 3)) * 0.5
    _compare_brute(tri, n)


def test_brute_force_nonunit_grid():
    rng = np.random.default_rng(5)
    n = (5, 4, 4)
    dx = 0.3
    origin = (-0.7, 0.2, 1.1)
    tri = rng.uniform(0, 1, (10, 3, 3)) * np.array([5, 4, 4]) * dx + np.array(origin)
    _compare_brute(tri, n, dx, origin)


def _box(lo, hi):
    """Closed axis-aligned box surface, 12 triangles."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    c = (lo + hi) / 2
    e = hi - lo
    out = []
    for ax in range(3):
        u, v = (ax + 1) % 3, (ax + 2) % 3
        for s in (-1, 1):
            cc = c.copy()
            cc[ax] += s * e[ax] / 2
            e1 = np.zeros(3)
            e1[u] = e[u]
            e2 = np.zeros(3)
            e2[v] = e[v]
            out.append(inputs.rectangle(cc, e1, e2))
    return np.concatenate(out)


def test_box_fractional_offsets_known_answer():
    # box [2.3, 5.8] x [1.6, 4.1] x [3.2, 5.45] on a unit grid (centres at i+0.5)
    lo, hi = (2.3, 1.6, 3.2), (5.8, 4.1, 5.45)
    n = (8, 7, 8)
    blocked, theta = tagging.tag(_box(lo, hi), n, 1.0, (0, 0, 0))
    cen = [np.arange(n[a]) + 0.5 for a in range(3)]
    exp_b = np.zeros((n[2], n[1], n[0]), np.uint8)
    exp_t = np.full((n[2], n[1], n[0], 6), 2.0)
    for k, j, i in itertools.product(range(n[2]), range(n[1]), range(n[0])):
        p = (cen[0][i], cen[1][j], cen[2][k])
        for ax in range(3):
            u, v = (ax + 1) % 3, (ax + 2) % 3
            if not (lo[u] <= p[u] <= hi[u] and lo[v] <= p[v] <= hi[v]):
                continue
            for s in (-1, 1):
                q = p[ax] + s
                for wall in (lo[ax], hi[ax]):
                    if min(p[ax], q) <= wall <= max(p[ax], q) and 0 <= q < n[ax]:
                        d = 2 * ax + (1 if s > 0 else 0)
                        exp_b[k, j, i] |= 1 << d
                        exp_t[k, j, i, d] = min(exp_t[k, j, i, d], abs(wall - p[ax]))
    assert np.array_equal(blocked, exp_b)
    np.testing.assert_allclose(theta, exp_t, rtol=0, atol=1e-14)


def test_box_through_centres_ties():
    # faces exactly on cell centres: hits at both adjacent segments with theta 0 and 1
    lo, hi = (2.5, 2.5, 2.5), (4.5, 5.5, 3.5)
    n = (7, 8, 6)
    blocked, theta = tagging.tag(_box(lo, hi), n, 1.0, (0, 0, 0))
    # the cell whose centre lies on the -x face (x=2.5 -> i=2) at j=3,k=2 (y=3.5,z=2.5 inside)
    c = (2, 3, 2)
    assert blocked[c[2], c[1], c[0]] & 0b11 == 0b11
    assert theta[c[2], c[1], c[0], 0] == 0.0 and theta[c[2], c[1], c[0], 1] == 0.0
    assert theta[c[2], c[1], c[0] - 1, 1] == 1.0
    assert theta[c[2], c[1], c[0] + 1, 0] == 1.0
    _compare_brute(_box(lo, hi), n)


def test_shared_edge_on_grid_line_does_not_leak():
    # a square split along its diagonal; the diagonal passes exactly through grid lines
    sq = inputs.rectangle((3.0, 3.0, 2.3), (4.0, 0, 0), (0, 4.0, 0))  # z-plane, diag through (x.5, x.5)
    blocked, theta = tagging.tag(sq, (6, 6, 5), 1.0, (0, 0, 0))
    for j in range(1, 5):
        for i in range(1, 5):
            assert blocked[1, j, i] & (1 << 5)
            assert blocked[2, j, i] & (1 << 4)
            assert abs(theta[1, j, i, 5] - 0.8) < 1e-14
            assert abs(theta[2, j, i, 4] - 0.2) < 1e-14
    # exactly the 16 z-segments under the square are blocked, once, from both sides
    assert np.count_nonzero(blocked) == 32
    assert set(np.unique(blocked[blocked != 0]).tolist()) <= {16, 32}


def test_watertight_parity_no_leak():
    tri = inputs.icosphere(2, 3.3, (5.1, 4.9, 5.05), inputs.random_rotation(np.random.default_rng(7)))
    n = (10, 10, 10)
    blocked, _ = tagging.tag(tri, n, 1.0, (0, 0, 0))
    par = np.zeros((10, 10, 10), np.int8)
    for k, j, i in itertools.product(range(10), repeat=3):
        par[k, j, i] = inside_parity((i + 0.5, j + 0.5, k + 0.5), tri)
    assert par.sum() > 50
    for ax, npax in ((0, 2), (1, 1), (2, 0)):
        a = np.moveaxis(par, npax, -1)
        b = np.moveaxis(blocked, npax, -1)
        differ = a[..., :-1] != a[..., 1:]
        blk = (b[..., :-1] >> (2 * ax + 1)) & 1
        assert np.all(blk[differ] == 1), "a parity change without a blocked segment is a leak"


def test_topology_free_invariances():
    rng = np.random.default_rng(8)
    tri = inputs.dirty_sphere(24, 6.0, seed=3, level=3)
    n = (24, 24, 24)
    b0, t0 = tagging.tag(tri, n, 1.0, (0, 0, 0))
    variants = {
        "flip": tri[:, [0, 2, 1], :],
        "rotate": tri[:, [1, 2, 0], :],
        "permute": tri[rng.permutation(len(tri))],
        "duplicate": np.concatenate([tri, tri[: len(tri) // 3]]),
    }
    for name, t in variants.items():
        b, th = tagging.tag(np.ascontiguousarray(t), n, 1.0, (0, 0, 0))
        assert np.array_equal(b, b0), name
        np.testing.assert_allclose(th, t0, rtol=0, atol=1e-13, err_msg=name)
    # permutation and duplication keep each triangle's vertex order: theta bit-identical
    for name in ("permute", "duplicate"):
        _, th = tagging.tag(np.ascontiguousarray(variants[name]), n, 1.0, (0, 0, 0))
        assert np.array_equal(th, t0), name


def test_gap_opens_only_its_own_segments():
    tri = inputs.icosphere(3, 5.0, (8.2, 7.9, 8.1), inputs.random_rotation(np.random.default_rng(9)))
    n = (16, 16, 16)
    b0, _ = tagging.tag(tri, n, 1.0, (0, 0, 0))
    for drop in (0, 57, 300):
        keep = np.ones(len(tri), bool)
        keep[drop] = False
        b1, _ = tagging.tag(np.ascontiguousarray(tri[keep]), n, 1.0, (0, 0, 0))
        alone, _ = tagging.tag(np.ascontiguousarray(tri[drop:drop + 1]), n, 1.0, (0, 0, 0))
        # opened bits are a subset of what the dropped triangle blocks on its own
        opened = b0 & ~b1
        assert np.all((opened & ~alone) == 0)
        assert np.all((b1 & ~b0) == 0)


def test_geometry_outside_domain_ignored():
    tri = _box((-3.0, -3.0, -3.0), (-1.0, -1.0, -1.0))
    b, th = tagging.tag(tri, (4, 4, 4), 1.0, (0, 0, 0))
    assert b.sum() == 0 and np.all(th == 2.0)


# ------------------------------------------------- tolerance of the ray test

@pytest.mark.parametrize("eps", [0.02, 0.1, 0.5])
def test_bary_eps_brute_force_random_soup(eps):
    """With the tolerance the oracle blocks exactly the segments that meet some triangle
    widened to barycentric coordinates >= -eps, solved in rational arithmetic, and its
    theta is the nearest such crossing (rounding aside)."""
    rng = np.random.default_rng(13)
    n = (6, 5, 4)
    tri = rng.uniform(0.0, 6.0, (14, 3, 3)) * np.array([1.0, 5 / 6, 4 / 6])
    _compare_brute(tri, n, eps=eps)


def test_bary_eps_closes_a_gap_between_triangles():
    """Two triangles of a plate z = 2.3 that leave a slit between them: the grid line
    through the slit passes at barycentric distance 0.0204 from the nearer triangle, so
    it leaks at eps = 0 and 0.015 and is blocked from 0.025 on, with theta the plane's
    distance from the cell centre."""
    h = 3.0
    # the line x = y = 1.5 would lie on the hypotenuse x + y = 3 of a right triangle with
    # 3-cell legs; the legs end at 2.94 instead (barycentric distance 0.0204 from the
    # line); the second triangle's hypotenuse x + y = 3.56 is 0.23 away
    A1 = [(0.0, 0.0, 2.3), (h - 0.06, 0.0, 2.3), (0.0, h - 0.06, 2.3)]
    A2 = [(h, h, 2.3), (0.56, h, 2.3), (h, 0.56, 2.3)]
    tri = np.array([A1, A2])
    n = (4, 4, 4)
    seg = (1 + 4 * (1 + 4 * 1), 5)     # cell (1, 1, 1), +z: crosses z = 2.3 only through the slit
    for eps, blocked in ((0.0, False), (0.015, False), (0.025, True), (0.2, True)):
        b, th = tagging.tag(tri, n, 1.0, (0, 0, 0), eps)
        bit = (b.ravel()[seg[0]] >> seg[1]) & 1
        assert bool(bit) == blocked, eps
        if blocked:
            assert abs(th.reshape(-1, 6)[seg] - 0.8) < 1e-12
            assert (b.ravel()[seg[0] + 16] >> 4) & 1          # the cell above sees it too


def test_bary_eps_is_monotone():
    """A larger tolerance blocks a superset of segments, and where both block, the
    nearest crossing can only come closer."""
    tri = inputs.dirty_sphere(16, 5.0, seed=3, level=3) + np.array([0.3, -0.2, 0.1])
    n = (16, 16, 16)
    prev_b, prev_t = tagging.tag(tri, n, 1.0, (0, 0, 0), 0.0)
    for eps in (0.01, 0.05, 0.2):
        b, t = tagging.tag(tri, n, 1.0, (0, 0, 0), eps)
        assert np.all((prev_b & ~b) == 0)
        both = (prev_b[..., None] >> np.arange(6)) & (b[..., None] >> np.arange(6)) & 1
        assert np.all(t[both == 1] <= prev_t[both == 1])
        assert (b & ~prev_b).any() or eps == 0.01
        prev_b, prev_t = b, t
    with pytest.raises(ValueError):
        tagging.tag(tri, n, 1.0, (0, 0, 0), 0.6)
