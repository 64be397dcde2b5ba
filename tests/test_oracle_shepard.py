"""Pins of the near-field surface force oracle (oracle/shepard.py, eq. (force)): closed
forms where the Shepard weights are equal or the pressure is piecewise constant, the
dropping of in-plane points, orientation invariance of the force, and the zero net
force of a closed surface."""
import numpy as np

from oracle import flow, shepard

S = flow.SLIP


def _grid(n, dx=1.0, origin=(0.0, 0.0, 0.0)):
    return flow.Grid(n, dx, origin, (S,) * 6)


def _square(z, lo, hi, up=True):
    """Two triangles covering [lo, hi]^2 in the plane z, normal +z (or -z)."""
    a, b, c, d = (lo, lo, z), (hi, lo, z), (hi, hi, z), (lo, hi, z)
    t = [[a, b, c], [a, c, d]] if up else [[a, c, b], [a, d, c]]
    return np.array(t, dtype=np.float64)


def test_equidistant_points_give_the_mean_of_each_side():
    # a vertex at the centre of a dual cell: the eight cell centres are equidistant,
    # so each side's Shepard value is the plain mean of its four cells
    g = _grid((4, 4, 4))
    p = np.random.default_rng(0).standard_normal(g.shape)
    X = np.array([2.0, 2.0, 2.0])
    for axis in range(3):
        n = np.zeros(3)
        n[axis] = 1.0
        f, b = shepard.vertex_values(g, p, X, n)
        sl_f = [slice(1, 3)] * 3
        sl_b = [slice(1, 3)] * 3
        sl_f[2 - axis] = slice(2, 3)   # array order (z, y, x)
        sl_b[2 - axis] = slice(1, 2)
        assert abs(f - p[tuple(sl_f)].mean()) < 1e-15
        assert abs(b - p[tuple(sl_b)].mean()) < 1e-15


def test_points_in_the_plane_are_dropped():
    # the plane through a row of cell centres: those four points belong to neither
    # side; the front value is the mean of the row above (equal distances), and the
    # back side has no point
    g = _grid((4, 4, 4))
    p = np.random.default_rng(1).standard_normal(g.shape)
    f, b = shepard.vertex_values(g, p, np.array([2.0, 2.0, 1.5]), np.array([0.0, 0.0, 1.0]))
    assert abs(f - p[2, 1:3, 1:3].mean()) < 1e-15
    assert b is None


def test_two_sided_plate_closed_form_and_orientation():
    # a plate in z = 3 (between cell centres) with p = +1 above and -1 below: every
    # front value is +1 and every back value -1 for the upward normal, so the force is
    # A n (p- - p+) = -2 A e_z; flipping the orientation swaps the sides and the
    # normal, and the force stays the same
    g = _grid((6, 6, 6))
    zc = (np.arange(6) + 0.5)[:, None, None] * np.ones((6, 6, 6))
    p = np.where(zc > 3.0, 1.0, -1.0)
    for up in (True, False):
        tri = _square(3.0, 1.25, 4.5, up)
        side, force = shepard.surface_pressure(g, p, tri)
        sgn = 1.0 if up else -1.0
        np.testing.assert_array_equal(side[:, 0], sgn)
        np.testing.assert_array_equal(side[:, 1], -sgn)
        area = (4.5 - 1.25) ** 2
        np.testing.assert_allclose(force, [0.0, 0.0, -2.0 * area], rtol=0, atol=1e-12)


def _box(lo, hi):
    """Closed surface of the cube [lo, hi]^3: 12 triangles, outward normals."""
    v = lambda i, j, k: tuple(hi if b else lo for b in (i, j, k))  # noqa: E731
    faces = [  # four corners in counter-clockwise order seen from outside
        [v(0, 0, 0), v(0, 1, 0), v(1, 1, 0), v(1, 0, 0)],   # -z
        [v(0, 0, 1), v(1, 0, 1), v(1, 1, 1), v(0, 1, 1)],   # +z
        [v(0, 0, 0), v(1, 0, 0), v(1, 0, 1), v(0, 0, 1)],   # -y
        [v(0, 1, 0), v(0, 1, 1), v(1, 1, 1), v(1, 1, 0)],   # +y
        [v(0, 0, 0), v(0, 0, 1), v(0, 1, 1), v(0, 1, 0)],   # -x
        [v(1, 0, 0), v(1, 1, 0), v(1, 1, 1), v(1, 0, 1)],   # +x
    ]
    tri = []
    for a, b, c, d in faces:
        tri += [[a, b, c], [a, c, d]]
    return np.array(tri, dtype=np.float64)


def test_closed_box_piecewise_pressure():
    # box [1, 3]^3 (faces between cell centres, corners at dual-cell centres) with
    # p = c_in in its 8 interior cells and c_out outside.  Every vertex is a corner:
    # its 4 front points are outside (c_out); of its 4 back points one is interior, so
    # the back value is (c_in + 3 c_out) / 4.  The net force sum A n (p- - p+) vanishes
    # because sum A n = 0 over a closed surface.
    g = _grid((5, 5, 5))
    c_in, c_out = 2.5, -0.75
    p = np.full(g.shape, c_out)
    p[1:3, 1:3, 1:3] = c_in
    tri = _box(1.0, 3.0)
    n, area = shepard.triangle_frames(tri)
    assert np.allclose(np.sum(area[:, None] * n, axis=0), 0.0, atol=1e-14)
    cent = tri.mean(axis=1)
    assert np.all(np.sum(n * (cent - 2.0), axis=1) > 0.0)   # outward
    side, force = shepard.surface_pressure(g, p, tri)
    np.testing.assert_allclose(side[:, 0], c_out, rtol=0, atol=1e-15)
    np.testing.assert_allclose(side[:, 1], (c_in + 3 * c_out) / 4, rtol=0, atol=1e-15)
    np.testing.assert_allclose(force, 0.0, atol=1e-12)


def test_degenerate_triangle_and_domain_edge():
    # a zero-area triangle contributes nothing; a vertex at the domain corner keeps
    # only the in-domain points (here one per side at most)
    g = _grid((3, 3, 3))
    p = np.random.default_rng(2).standard_normal(g.shape)
    tri = np.array([[[1.0, 1.0, 1.0], [2.0, 2.0, 2.0], [3.0, 3.0, 3.0]]])
    side, force = shepard.surface_pressure(g, p, tri)
    assert np.all(np.isnan(side)) and np.all(force == 0.0)
    f, b = shepard.vertex_values(g, p, np.array([0.0, 0.0, 0.0]), np.array([1.0, 1.0, 1.0]) / np.sqrt(3.0))
    assert abs(f - p[0, 0, 0]) < 1e-15 and b is None


def test_inverse_square_weights_worked_example():
    # vertex X = (2.25, 2, 2), normal (1, 1, 0)/sqrt(2): front points are the two cell
    # centres (2.5, 2.5, z); back points are (2.5, 1.5, z) at d^2 = 9/16 and the four
    # (1.5, y, z) at d^2 = 17/16.  With p = 1 on the (2.5, 1.5, z) pair and 0 on the
    # rest, the back value is (2 * 16/9) / (2 * 16/9 + 4 * 16/17) = 17/35 by hand
    # (weights 1/d would give 0.407).
    g = _grid((4, 4, 4))
    p = np.zeros(g.shape)
    p[1:3, 1, 2] = 1.0        # cells x = 2.5 (i = 2), y = 1.5 (j = 1), z = 1.5, 2.5
    p[1:3, 2, 2] = 7.0        # the front pair (2.5, 2.5, z)
    f, b = shepard.vertex_values(g, p, np.array([2.25, 2.0, 2.0]), np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0))
    assert abs(f - 7.0) < 1e-15
    assert abs(b - 17.0 / 35.0) < 1e-15


# ------------------------------------------------------------ thin-plate filter Z

def test_segment_crossing_cases():
    tri = np.array([[[0.0, 0.0, 1.0], [2.0, 0.0, 1.0], [0.0, 2.0, 1.0]]])
    hit = lambda P, Q: bool(shepard.segment_hits(np.array(P), np.array(Q), tri)[0])  # noqa: E731
    assert hit((0.5, 0.5, 0.0), (0.5, 0.5, 2.0))          # through the interior
    assert not hit((1.5, 1.5, 0.0), (1.5, 1.5, 2.0))      # beside the hypotenuse
    assert hit((1.0, 1.0, 0.0), (1.0, 1.0, 2.0))          # through the hypotenuse (edges count)
    assert hit((0.5, 0.5, 0.0), (0.5, 0.5, 1.0))          # ending on it (t = 1)
    assert not hit((0.5, 0.5, 1.0), (0.5, 0.5, 2.0))      # starting on it (t = 0)
    assert not hit((0.5, 0.5, 0.0), (0.5, 0.5, 0.9))      # stopping short
    assert not hit((0.5, 0.5, 1.0), (1.5, 0.2, 1.0))      # in its plane


def _plate(z, lo, hi, up):
    a, b, c, d = (lo, lo, z), (hi, lo, z), (hi, hi, z), (lo, hi, z)
    return np.array([[a, b, c], [a, c, d]] if up else [[a, c, b], [a, d, c]], dtype=np.float64)


def _sheet(z, up, n=3, L=6.0):
    """Triangulated square [0, L]^2 in the plane z on an (n+1)^2 vertex grid."""
    xs = np.linspace(0.0, L, n + 1)
    tri = []
    for i in range(n):
        for j in range(n):
            a, b = (xs[i], xs[j], z), (xs[i + 1], xs[j], z)
            c, d = (xs[i + 1], xs[j + 1], z), (xs[i], xs[j + 1], z)
            tri += [[a, b, c], [a, c, d]] if up else [[a, c, b], [a, d, c]]
    return np.array(tri, dtype=np.float64)


def test_thin_plate_filter_counts_the_plate_once():
    # a plate 0.3 cells thick across the whole domain between the cell centres z = 2.5
    # and 3.5 (faces at 3.15 with normal +z and 2.85 with -z), p = +1 above, -1 below.
    # Unfiltered, each face also averages the points beyond the other face and the force
    # is counted twice (-4 A e_z, A = 36); the filter cancels those values: -2 A e_z,
    # every triangle with its front value only
    g = flow.Grid((6, 6, 6), 1.0, (0.0, 0.0, 0.0), (flow.SLIP,) * 6)
    zc = (np.arange(6) + 0.5)[:, None, None] * np.ones((6, 6, 6))
    p = np.where(zc > 3.0, 1.0, -1.0)
    up, lo = _sheet(3.15, True), _sheet(2.85, False)
    tri = np.concatenate([up, lo])
    side, f_raw = shepard.surface_pressure(g, p, tri)
    np.testing.assert_allclose(f_raw, [0.0, 0.0, -4.0 * 36.0], atol=1e-11)
    side, f = shepard.surface_pressure(g, p, tri, thin_filter=True)
    np.testing.assert_allclose(f, [0.0, 0.0, -2.0 * 36.0], atol=1e-11)
    nu = len(up)
    assert np.all(side[:nu, 0] == 1.0) and np.all(np.isnan(side[:nu, 1]))     # upper face: front only
    assert np.all(side[nu:, 0] == -1.0) and np.all(np.isnan(side[nu:, 1]))    # lower face: front only


def test_filter_leaves_single_surfaces_unchanged():
    g = flow.Grid((6, 6, 6), 1.0, (0.0, 0.0, 0.0), (flow.SLIP,) * 6)
    p = np.random.default_rng(8).standard_normal((6, 6, 6))
    for tri in (_plate(3.0, 1.25, 4.5, True), _box(1.0, 3.0)):
        s0, f0 = shepard.surface_pressure(g, p, tri)
        s1, f1 = shepard.surface_pressure(g, p, tri, thin_filter=True)
        assert np.array_equal(np.isnan(s0), np.isnan(s1)) and np.array_equal(s0[~np.isnan(s0)], s1[~np.isnan(s1)])
        assert np.array_equal(f0, f1)
