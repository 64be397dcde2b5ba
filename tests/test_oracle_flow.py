"""Pins for the FP64 flow oracle against closed forms, textbook identities and the
paper's own verification results (Sec. 2.4, Taylor-Green vortex).
"""
import math

import numpy as np
import pytest

from oracle import flow, tagging
from paper_2002_06206_amd import inputs

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


def empty(g):
    return np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0)


# ------------------------------------------------------------ ghost values

@pytest.mark.parametrize("theta", [0.0, 0.1, 0.25, 0.4999, 0.5, 0.7, 0.93, 1.0])
@pytest.mark.parametrize("opp_blocked", [False, True])
def test_ghost_reproduces_linear_field_through_wall(theta, opp_blocked):
    """Both branches of eq. (q_axis) give the exact ghost for a field that is linear
    along the axis and equals q_IB at the wall (first-order Taylor reading, Sec. 2.3.2).
    With the opposite face also blocked and theta < 0.5 (Reading G1) the ghost is
    the mirror value 2 q_IB - q_c, which is checked directly."""
    g = flow.Grid((6, 3, 3), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
    blocked, th = empty(g)
    c = (1, 1, 2)   # (k, j, i)
    blocked[c] |= 1 << 1          # +x face blocked at distance theta
    th[c + (1,)] = theta
    blocked[1, 1, 3] |= 1 << 0
    th[1, 1, 3, 0] = 1.0 - theta
    if opp_blocked:
        blocked[c] |= 1 << 0
        th[c + (0,)] = 0.9
        blocked[1, 1, 1] |= 1 << 1
        th[1, 1, 1, 1] = 0.1
    st = flow.build_stencils(g, blocked, th)
    alpha, beta = 0.37, -1.3
    x = np.arange(6) + 0.5
    q = np.broadcast_to(alpha + beta * x, g.shape).copy()
    X = flow.cut_points(st)
    wall = np.zeros((st.ncut, 3))
    wall[:, 0] = alpha + beta * X[:, 0]
    ghost = flow.neighbour(st, q, 0, 1, wall)[c]
    if opp_blocked and theta < 0.5:
        # G1: 2 q_IB - q_c is exact for any field that is odd about the wall
        q_ib = alpha + beta * (x[2] + theta)
        assert abs(ghost - (2 * q_ib - q[c])) < 1e-13
    else:
        assert abs(ghost - (alpha + beta * x[3])) < 1e-12


def test_ghost_branches_continuous_at_half():
    g = flow.Grid((6, 3, 3), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
    vals = []
    for t in (0.5, 0.5 - 1e-12):
        blocked, th = empty(g)
        blocked[1, 1, 2] |= 2
        th[1, 1, 2, 1] = t
        blocked[1, 1, 3] |= 1
        th[1, 1, 3, 0] = 1 - t
        st = flow.build_stencils(g, blocked, th)
        rng = np.random.default_rng(0)
        q = rng.standard_normal(g.shape)
        wall = np.full((st.ncut, 3), 0.8)
        vals.append(flow.neighbour(st, q, 0, 1, wall)[1, 1, 2])
    assert abs(vals[0] - vals[1]) < 1e-10
    # both equal 2 q_IB - q_c at theta = 0.5
    assert abs(vals[0] - (2 * 0.8 - q[1, 1, 2])) < 1e-12


# ---------------------------------------------------------------- CSM

def _linear_velocity(g, G):
    x = [g.origin[a] + (np.arange(g.n[a]) + 0.5) * g.dx for a in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    pos = [X, Y, Z]
    return [sum(G[i][j] * pos[j] for j in range(3)) for i in range(3)]


def _csm_interior(G, dx=0.5):
    g = flow.Grid((6, 6, 6), dx, (0.0, 0.0, 0.0), (S,) * 6)
    st = flow.build_stencils(g, *empty(g))
    nut = flow.csm_nut(st, _linear_velocity(g, G))
    return nut[1:-1, 1:-1, 1:-1], g


def test_csm_pure_shear_is_zero():
    nut, _ = _csm_interior(np.array([[0, 2.0, 0], [0, 0, 0], [0, 0, 0]]))
    assert np.all(nut == 0.0)


def test_csm_rigid_rotation_is_zero():
    nut, _ = _csm_interior(np.array([[0, -1.5, 0], [1.5, 0, 0], [0, 0, 0]]))
    assert np.all(np.abs(nut) < 1e-15)


def test_csm_pure_strain():
    G = np.diag([1.0, -0.4, -0.6])
    nut, g = _csm_interior(G)
    # W = 0 -> Q = -E -> F_CS = -1 -> nu_t = dx^2 |S| / 20
    np.testing.assert_allclose(nut, g.dx ** 2 * np.sqrt(np.sum(G * G)) / 20.0, rtol=1e-14)


def test_csm_random_gradient_alternative_formula():
    rng = np.random.default_rng(11)
    for _ in range(10):
        G = rng.standard_normal((3, 3))
        nut, g = _csm_interior(G)
        # Q = -G_ij G_ji / 2 and E = G_ij G_ij / 2 (no split into S and W)
        F = -np.sum(G * G.T) / np.sum(G * G)
        assert abs(F) <= 1.0
        Sn = np.sqrt(np.sum((0.5 * (G + G.T)) ** 2))
        np.testing.assert_allclose(nut, g.dx ** 2 * Sn * abs(F) ** 1.5 / 20.0, rtol=1e-12)


# ------------------------------------------------------------ Laplacian

def test_laplacian_periodic_cosine_exact_eigenvalue():
    n, dx = (16, 12, 8), 0.25
    g = flow.Grid(n, dx, (0.0, 0.0, 0.0), (P,) * 6)
    st = flow.build_stencils(g, *empty(g))
    L = [n[a] * dx for a in range(3)]
    x = [(np.arange(n[a]) + 0.5) * dx for a in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    kx, ky, kz = 2 * math.pi / L[0], 4 * math.pi / L[1], 2 * math.pi / L[2]
    p = np.cos(kx * X) * np.cos(ky * Y) * np.sin(kz * Z)
    lam = sum((2 * math.cos(k * dx) - 2) / dx ** 2 for k in (kx, ky, kz))
    np.testing.assert_allclose(flow.laplacian(st, p), lam * p, atol=1e-11)


def _random_geometry_stencil(seed=0, bc=(I, O, S, S, P, P)):
    rng = np.random.default_rng(seed)
    g = flow.Grid((9, 8, 7), 1.0, (0.0, 0.0, 0.0), bc)
    tri = np.concatenate([inputs.icosphere(1, 2.2, (4.3, 4.1, 3.6), inputs.random_rotation(rng)),
                          inputs.rectangle((6.2, 3.1, 3.3), (0, 5.0, 0), (0, 0, 4.0))])
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    return g, flow.build_stencils(g, b, th)


def test_laplacian_energy_form_and_symmetry():
    """x.(-L x) equals the sum over open faces of (x_c - x_nb)^2 plus 2 x_c^2 per
    outlet face (graph-Laplacian energy), and -L is symmetric."""
    g, st = _random_geometry_stencil()
    rng = np.random.default_rng(1)
    x = rng.standard_normal(g.shape)
    y = rng.standard_normal(g.shape)
    energy = 0.0
    xf = x.ravel()
    n = g.n
    bl = st.blocked.ravel()
    for c in range(g.ncell):
        i, j, k = c % n[0], (c // n[0]) % n[1], c // (n[0] * n[1])
        for ax, (di, dj, dk) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
            co = [i, j, k]
            co[ax] += 1
            if co[ax] == n[ax]:
                if g.bc[2 * ax + 1] == P:
                    co[ax] = 0
                else:
                    if g.bc[2 * ax + 1] == O:
                        energy += 2 * xf[c] ** 2
                    continue
            if (bl[c] >> (2 * ax + 1)) & 1:
                continue
            nb = co[0] + n[0] * (co[1] + n[1] * co[2])
            energy += (xf[c] - xf[nb]) ** 2
        if i == 0 and g.bc[0] == O:
            energy += 2 * xf[c] ** 2
    assert abs(np.sum(x * -flow.laplacian(st, x)) - energy) < 1e-10 * energy
    assert abs(np.sum(y * flow.laplacian(st, x)) - np.sum(x * flow.laplacian(st, y))) < 1e-10


def test_pcg_recovers_manufactured_solution():
    g, st = _random_geometry_stencil(2, bc=(P,) * 6)
    rng = np.random.default_rng(3)
    p_true = flow.remove_component_means(st, rng.standard_normal(g.shape))
    b = flow.laplacian(st, p_true)
    x, it = flow.pcg(st, b, np.zeros(g.shape), 1e-13, 5000)
    x = flow.remove_component_means(st, x)
    assert it > 5
    assert np.max(np.abs(x - p_true)) < 1e-9


def test_pcg_manufactured_with_outlet():
    g, st = _random_geometry_stencil(4)
    rng = np.random.default_rng(5)
    p_true = flow.remove_component_means(st, rng.standard_normal(g.shape))
    b = flow.laplacian(st, p_true)
    x, it = flow.pcg(st, b, rng.standard_normal(g.shape), 1e-13, 5000)
    x = flow.remove_component_means(st, x)
    assert np.max(np.abs(x - p_true)) < 1e-9


def test_continuous_poisson_second_order():
    errs = []
    for N in (8, 16, 32):
        L = 1.0
        dx = L / N
        g = flow.Grid((N, N, N), dx, (0.0, 0.0, 0.0), (P,) * 6)
        st = flow.build_stencils(g, *empty(g))
        x = (np.arange(N) + 0.5) * dx
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
        w = 2 * math.pi
        p = np.cos(w * X) * np.cos(w * Y) * np.cos(w * Z)
        b = -3 * w * w * p
        sol, _ = flow.pcg(st, b, np.zeros(g.shape), 1e-12, 5000)
        sol = flow.remove_component_means(st, sol)
        errs.append(np.sqrt(np.mean((sol - p) ** 2)))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) > 1.9


# ------------------------------------------------------- full steps

def _sphere_state(seed=0, n=12):
    rng = np.random.default_rng(seed)
    g = flow.Grid((n, n, n), 1.0, (0.0, 0.0, 0.0), (I, O, S, S, S, S), (1.0, 0.0, 0.0))
    tri = inputs.icosphere(2, 2.6, (n / 2 + 0.13, n / 2 - 0.07, n / 2 + 0.21), inputs.random_rotation(rng))
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, b, th)
    u, U, p, h = flow.init_state(st, (1.0, 0.0, 0.0))
    return g, st, u, U, p, h


def test_divergence_identity_after_projection():
    """P3: after the correction, div U^{n+1} = dt (b - L p) cell by cell, and the
    right-hand side sums to zero on every enclosed component."""
    g, st, u, U, p, h = _sphere_state()
    prm = flow.StepParams(dt=0.3, nu=0.05, tol=1e-6)
    for n in range(3):
        u, U, p, h, stats = flow.step(st, u, U, p, h, prm, n)
    b = stats["b"]
    div = flow.divergence(g, U)
    res = b - flow.laplacian(st, p)
    np.testing.assert_allclose(div, prm.dt * res, atol=1e-12 * np.max(np.abs(b)) * prm.dt + 1e-15)
    for cells in st.comps:
        assert abs(b.ravel()[cells].sum()) < 1e-10 * np.max(np.abs(b))
    assert len(st.comps) >= 1   # the watertight sphere interior is an enclosed fluid component


def test_mass_conservation_tight_tolerance():
    g, st, u, U, p, h = _sphere_state(1)
    prm = flow.StepParams(dt=0.3, nu=0.05, tol=1e-13)
    for n in range(3):
        u, U, p, h, stats = flow.step(st, u, U, p, h, prm, n)
    assert stats["div_linf"] < 1e-10
    assert stats["rel_residual"] < 1e-12


def _tgv(N, steps, dt, ib=None, nz=4):
    dx = 4.0 / N
    g = flow.Grid((N, N, nz), dx, (-2.0, -2.0, 0.0), (P,) * 6)
    if ib is None:
        blocked, theta = empty(g)
    else:
        tri = inputs.tgv_circle(N, nz) if ib == "circle" else inputs.tgv_square(N, nz)
        blocked, theta = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, blocked, theta)
    X = flow.cut_points(st)
    nu = 0.01

    def exact(x, y, t):
        e = math.exp(-2 * math.pi ** 2 * nu * t)
        return -np.cos(np.pi * x) * np.sin(np.pi * y) * e, np.sin(np.pi * x) * np.cos(np.pi * y) * e
    xc = -2 + (np.arange(N) + 0.5) * dx
    Z, Y, Xg = np.meshgrid(np.arange(nz), xc, xc, indexing="ij")
    u1, u2 = exact(Xg, Y, 0.0)
    u = [u1, u2, np.zeros(g.shape)]
    U1, _ = exact(Xg + dx / 2, Y, 0.0)
    _, U2 = exact(Xg, Y + dx / 2, 0.0)
    U = [U1, U2, np.zeros(g.shape)]
    p = np.zeros(g.shape)
    h = [np.zeros(g.shape)] * 3
    prm = flow.StepParams(dt=dt, nu=nu, csm=False, tol=1e-12)
    for n in range(steps):
        wall = None
        if st.ncut:
            wx, wy = exact(X[:, 0], X[:, 1], (n + 1) * dt)
            wall = np.stack([wx, wy, np.zeros_like(wx)], axis=1)
        u, U, p, h, stats = flow.step(st, u, U, p, h, prm, n, wall)
    e1, _ = exact(Xg, Y, steps * dt)
    return np.sqrt(np.mean((u[0] - e1) ** 2))


def test_tgv_second_order_without_ib():
    """Sec. 2.4: the solver without IB is second order in space (Taylor-Green, Re = 100)."""
    errs = [_tgv(N, 60, 0.005) for N in (16, 32, 64)]
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.9, orders


@pytest.mark.slow
def test_tgv_circle_ib_order():
    """Sec. 2.4: with the circular IB the L2 slope is about 1.34 overall (first-order
    wall interpolation), close to 2 on the coarse grids."""
    errs = [_tgv(N, 60, 0.005, "circle") for N in (16, 32, 64)]
    overall = math.log2(errs[0] / errs[2]) / 2
    assert overall >= 1.3, errs


@pytest.mark.slow
def test_tgv_square_ib_order():
    """Sec. 2.4: with the square IB (side sqrt(2), vertices on the unit circle) the
    paper reports an L2 slope of 1.37.  On the paper's two coarsest grids (N = 40, 80,
    t = 0.3) the oracle's slope is 1.44; the bar, 1.3, leaves room below the paper's 1.37
    for the difference in grids and time."""
    errs = [_tgv(N, 60, 0.005, "square") for N in (40, 80)]
    order = math.log2(errs[0] / errs[1])
    assert order >= 1.3, errs


def test_poiseuille_fixed_point_and_force_balance():
    """Poiseuille flow between two immersed planes at sub-cell offsets.  The steady
    1-D profile solving nu u'' + g = 0 with the eq. (q_axis) ghost rows must be an
    exact fixed point of the 3-D step (advection cancels, Q = 0 so the CSM gives
    nu_t = 0, the pressure stays 0), and the viscous wall force must balance the
    body force on every cell exactly."""
    ny = 16
    nu, gx = 0.1, 1e-3
    for delta in (0.0, 0.1, 0.25, 0.5, 0.75, 0.9):
        g = flow.Grid((4, ny, 4), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
        y_lo, y_hi = 3.5 + delta, 3.5 + delta + 7.3
        tri = inputs.channel_planes(y_lo, y_hi, -2.0, 10.0)
        b, th = tagging.tag(tri, g.n, g.dx, g.origin)
        st = flow.build_stencils(g, b, th)
        # 1-D system on the column: rows j, neighbours j+-1 or the ghost of eq. (q_axis)
        col = [st.blocked[0, j, 0] for j in range(ny)]
        A = np.zeros((ny, ny))
        rhs = np.full(ny, -gx)
        for j in range(ny):
            for d, s in ((2, -1), (3, 1)):
                if (col[j] >> d) & 1:
                    t = th[0, j, 0, d]
                    od = d ^ 1
                    A[j, j] -= nu
                    if t >= 0.5:
                        A[j, j] += nu * (t - 1) / t
                    elif (col[j] >> od) & 1:
                        A[j, j] += -nu
                    else:
                        A[j, j] += -2 * t * nu
                        A[j, (j - s) % ny] += (2 * t - 1) * nu
                else:
                    A[j, j] -= nu
                    A[j, (j + s) % ny] += nu
        prof = np.linalg.solve(A, rhs)
        u = [np.broadcast_to(prof[None, :, None], g.shape).copy(), np.zeros(g.shape), np.zeros(g.shape)]
        U = [u[0].copy(), np.zeros(g.shape), np.zeros(g.shape)]
        p = np.zeros(g.shape)
        h = [np.zeros(g.shape)] * 3
        prm = flow.StepParams(dt=1.0, nu=nu, body=(gx, 0.0, 0.0), tol=1e-12)
        un, Un, pn, H, stats = flow.step(st, u, U, p, h, prm, 0)
        assert np.max(np.abs(un[0] - u[0])) < 1e-13, delta
        assert np.max(np.abs(un[1])) < 1e-14 and np.max(np.abs(pn)) < 1e-12
        assert np.max(np.abs(stats["nut"])) == 0.0
        Fp, Fv = flow.forces(st, un, pn, stats["nut"], nu)
        assert abs(Fv[0] - gx * g.ncell) < 1e-12, (delta, Fv)


def test_poiseuille_converges_to_parabola():
    """The oracle's steady channel profile approaches u = g/(2 nu)(y - y_lo)(y_hi - y).
    The steady state is found directly: the momentum right-hand side is affine in a
    y-only profile (advection cancels, nu_t = 0), so its matrix is assembled column
    by column from the oracle itself and solved."""
    nu, gx = 0.1, 1e-3
    errs = []
    for N in (8, 16, 32, 64):
        dx = 1.0 / N
        ny = N + 4
        g = flow.Grid((2, ny, 2), dx, (0.0, -2 * dx, 0.0), (P,) * 6)
        y_lo, y_hi = 0.3 * dx, 1.0 - 0.2 * dx
        tri = inputs.channel_planes(y_lo, y_hi, -1.0, 2.0)
        b, th = tagging.tag(tri, g.n, g.dx, g.origin)
        st = flow.build_stencils(g, b, th)
        zero = [np.zeros(g.shape)] * 3
        base = flow.momentum_rhs(st, zero, zero, np.zeros(g.shape), nu, (gx, 0, 0), None)[0][0, :, 0]
        M = np.zeros((ny, ny))
        for j in range(ny):
            e = np.zeros(g.shape)
            e[:, j, :] = 1.0
            M[:, j] = flow.momentum_rhs(st, [e, zero[1], zero[2]], zero, np.zeros(g.shape), nu,
                                        (gx, 0, 0), None)[0][0, :, 0] - base
        prof = np.linalg.solve(M, -base)
        y = g.origin[1] + (np.arange(ny) + 0.5) * dx
        exact = gx / (2 * nu) * (y - y_lo) * (y_hi - y)
        inside = (y > y_lo) & (y < y_hi)
        errs.append(np.max(np.abs(prof[inside] - exact[inside])) / np.max(exact))
    order = math.log2(errs[0] / errs[3]) / 3
    assert order > 0.9, errs


# ------------------------------------------------------------ forces

def test_forces_uniform_pressure_zero_velocity():
    g, st, u, U, p, h = _sphere_state(2)
    z = [np.zeros(g.shape)] * 3
    Fp, Fv = flow.forces(st, z, np.full(g.shape, 3.7), None, 0.1)
    np.testing.assert_allclose(Fp, 0.0, atol=1e-12)
    np.testing.assert_allclose(Fv, 0.0, atol=0)


def test_forces_sealed_box_linear_pressure():
    """Closed box of cells with p = g x inside and 0 outside: the blocked-face pressure
    sum telescopes per x-row to g dx^3 (n_row - 1)."""
    g = flow.Grid((10, 9, 8), 0.5, (0.0, 0.0, 0.0), (S,) * 6)
    lo, hi = np.array([1.1, 0.8, 1.3]), np.array([3.6, 3.4, 2.9])
    from test_oracle_tagging import _box
    b, th = tagging.tag(_box(lo, hi), g.n, g.dx, g.origin)
    st = flow.build_stencils(g, b, th)
    x = [(np.arange(g.n[a]) + 0.5) * g.dx for a in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    inside = (X > lo[0]) & (X < hi[0]) & (Y > lo[1]) & (Y < hi[1]) & (Z > lo[2]) & (Z < hi[2])
    gp = 2.5
    p = np.where(inside, gp * X, 0.0)
    Fp, _ = flow.forces(st, [np.zeros(g.shape)] * 3, p, None, 0.0)
    rows = inside.sum(axis=2)
    expect = gp * g.dx ** 3 * np.sum(np.where(rows > 0, rows - 1, 0))
    assert abs(Fp[0] - expect) < 1e-12 * abs(expect)
    assert abs(Fp[1]) < 1e-12 and abs(Fp[2]) < 1e-12


# ----------------------------------------------------------- dead-end

def test_deadend_filter_closes_pocket():
    g = flow.Grid((5, 5, 5), 1.0, (0.0, 0.0, 0.0), (S,) * 6)
    b, th = empty(g)
    c = (2, 2, 2)
    for d in range(5):           # five blocked faces, +z open
        b[c] |= 1 << d
        th[c + (d,)] = 0.4
    for d, nb in ((0, (2, 2, 1)), (1, (2, 2, 3)), (2, (2, 1, 2)), (3, (2, 3, 2)), (4, (1, 2, 2))):
        b[nb] |= 1 << (d ^ 1)
        th[nb + (d ^ 1,)] = 0.6
    st = flow.build_stencils(g, b, th, deadend=True)
    assert st.deadend[c] and st.blocked[c] == 0x3F
    assert th[c + (5,)] == 2.0 and st.theta[c + (5,)] == 0.0
    assert st.blocked[3, 2, 2] & 1 << 4 and st.theta[3, 2, 2, 4] == 1.0
    assert st.deadend.sum() == 1
    # the pocket is an isolated enclosed cell
    assert st.flags[c] & (1 << 15)


def test_variable_step_ab2_integrates_linear_forcing_exactly():
    """Second-order Adams-Bashforth with r = dt/dt_prev integrates a right-hand side
    that is linear in time exactly: with a uniform periodic flow and body force
    g(t) = a + b t, every increment after the Euler start equals the integral of g."""
    g = flow.Grid((4, 4, 4), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
    st = flow.build_stencils(g, *empty(g))
    u, U, p, h = flow.init_state(st, (0.3, 0.0, 0.0))
    a, b = 0.7, -0.45
    t = 0.0
    dts = [0.1, 0.13, 0.07, 0.2, 0.05, 0.11]
    dt_prev = 0.0
    for n, dt in enumerate(dts):
        u0 = u[0][0, 0, 0]
        prm = flow.StepParams(dt=dt, nu=0.01, csm=False, body=(a + b * t, 0.0, 0.0), tol=1e-12, dt_prev=dt_prev)
        u, U, p, h, _ = flow.step(st, u, U, p, h, prm, n)
        if n > 0:
            exact = a * dt + b * ((t + dt) ** 2 - t ** 2) / 2
            assert abs((u[0][0, 0, 0] - u0) - exact) < 1e-14
        t += dt
        dt_prev = dt
