"""Pins of the Crank-Nicolson predictor oracle (eq. (crank-nicolson), BiCGStab of
Sec. 2.1): BiCGStab against a dense direct solve and its exact special cases, the
momentum operator against the already pinned affine right-hand side, the amplification
factor of a Fourier mode in closed form, energy conservation of the Cayley transform
for pure central advection, and dead-end cells held at their wall velocity."""
import numpy as np

from oracle import flow, tagging
from paper_2002_06206_amd import inputs

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


def test_bicgstab_matches_dense_solve():
    rng = np.random.default_rng(3)
    n = 40
    A = 3.0 * np.eye(n) + rng.standard_normal((n, n)) / np.sqrt(n)
    assert np.max(np.abs(A - A.T)) > 0.1          # genuinely nonsymmetric
    b = rng.standard_normal(n)
    x, it, status = flow.bicgstab(lambda q: A @ q, b, np.zeros(n), 1e-13, 200)
    xs = np.linalg.solve(A, b)
    assert status == "converged" and 0 < it < n
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-11
    assert np.linalg.norm(b - A @ x) <= 1e-13 * np.linalg.norm(b) * 1.0001


def test_bicgstab_special_cases():
    # A = c I: the first half step already solves it (s = 0), x = x0 + r/c exactly
    b = np.array([1.0, -2.0, 0.5, 4.0])
    x, it, status = flow.bicgstab(lambda q: 2.5 * q, b, np.zeros(4), 1e-14, 50)
    assert status == "converged" and it == 1
    assert np.array_equal(x, b / 2.5)
    # zero right-hand side: zero solution without iterating
    x, it, status = flow.bicgstab(lambda q: 2.5 * q, np.zeros(4), np.ones(4), 1e-14, 50)
    assert status == "converged" and it == 0 and not np.any(x)
    # exact initial guess: converged at the first check
    x, it, status = flow.bicgstab(lambda q: 2.5 * q, b, b / 2.5, 1e-14, 50)
    assert it == 0 and status == "converged"
    # a rotation by 90 degrees: <r0, A r0> = 0, the textbook breakdown
    R = np.array([[0.0, 1.0], [-1.0, 0.0]])
    _, it, status = flow.bicgstab(lambda q: R @ q, np.array([1.0, 0.0]), np.zeros(2), 1e-12, 10)
    assert status == "breakdown" and it == 0
    # the cap
    rng = np.random.default_rng(4)
    A = 3.0 * np.eye(30) + rng.standard_normal((30, 30))
    _, it, status = flow.bicgstab(lambda q: A @ q, rng.standard_normal(30), np.zeros(30), 1e-15, 2)
    assert status == "max_iter" and it == 2


def _geometry_case():
    rng = np.random.default_rng(7)
    g = flow.Grid((9, 8, 7), 1.0, (0.0, 0.0, 0.0), (I, O, S, S, P, P), (0.9, 0.2, -0.1))
    tri = np.concatenate([inputs.icosphere(1, 2.2, (4.3, 4.1, 3.6), inputs.random_rotation(rng)),
                          inputs.rectangle((6.2, 3.1, 3.3), (0, 5.0, 0), (0, 0, 4.0))])
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, b, th)
    wall = rng.standard_normal((st.ncut, 3)) * 0.3
    u = [rng.standard_normal(g.shape) for _ in range(3)]
    U = [rng.standard_normal(g.shape) for _ in range(3)]
    nut = np.abs(rng.standard_normal(g.shape)) * 0.05
    return g, st, wall, u, U, nut


def test_operator_is_the_linear_part_of_the_right_hand_side():
    # H(u) = L u + H(0): inflow, outflow, slip and periodic faces, blocked faces with
    # moving walls, eddy viscosity and a body force
    g, st, wall, u, U, nut = _geometry_case()
    assert st.ncut > 50
    nu, body = 0.03, (0.4, -0.2, 0.1)
    H = flow.momentum_rhs(st, u, U, nut, nu, body, wall)
    H0 = flow.momentum_rhs(st, [np.zeros(g.shape)] * 3, U, nut, nu, body, wall)
    for m in range(3):
        L = flow.momentum_operator(st, u[m], m, U, nut, nu)
        scale = np.max(np.abs(H[m])) + np.max(np.abs(H0[m]))
        assert np.max(np.abs((H[m] - H0[m]) - L)) < 1e-13 * scale
        assert np.max(np.abs(L)) > 0.1


def _fourier_case(nu, dt, modes=(2, 1, 1)):
    g = flow.Grid((16, 8, 8), 0.5, (0.0, 0.0, 0.0), (P,) * 6)
    st = flow.build_stencils(g, np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0))
    u0 = (0.8, -0.5, 0.3)
    _, U, _, _ = flow.init_state(st, u0)
    k = [2.0 * np.pi * modes[a] / (g.n[a] * g.dx) for a in range(3)]
    zc, yc, xc = np.meshgrid(*[(np.arange(g.n[a]) + 0.5) * g.dx for a in (2, 1, 0)], indexing="ij")
    theta = k[0] * xc + k[1] * yc + k[2] * zc
    lam = sum(-1j * u0[a] * np.sin(k[a] * g.dx) / g.dx - 2.0 * nu * (1.0 - np.cos(k[a] * g.dx)) / g.dx ** 2
              for a in range(3))
    return g, st, u0, U, theta, lam


def test_fourier_mode_amplification_closed_form():
    # uniform advecting velocity and a Fourier mode on a periodic box: L e^{i theta} =
    # lambda e^{i theta} with lambda = sum_a [-i U_a sin(k_a dx)/dx - 2 nu (1 - cos(k_a dx))/dx^2],
    # and one Crank-Nicolson step multiplies the mode by (1 + dt lambda/2) / (1 - dt lambda/2)
    nu, dt = 0.05, 0.4
    g, st, u0, U, theta, lam = _fourier_case(nu, dt)
    amp, phase = (0.3, -0.2, 0.15), (0.0, 1.1, -0.7)
    u = [u0[m] + amp[m] * np.cos(theta + phase[m]) for m in range(3)]
    us, H, iters = flow.cn_predictor(st, u, U, np.zeros(g.shape), nu, dt, (0.0, 0.0, 0.0), None, 1e-14, 100)
    G = (1.0 + 0.5 * dt * lam) / (1.0 - 0.5 * dt * lam)
    for m in range(3):
        exact = u0[m] + np.real(G * amp[m] * np.exp(1j * (theta + phase[m])))
        assert np.max(np.abs(us[m] - exact)) < 1e-13
        euler = u0[m] + np.real((1.0 + dt * lam) * amp[m] * np.exp(1j * (theta + phase[m])))
        assert np.max(np.abs(us[m] - euler)) > 1e-3      # the test tells the schemes apart
        # H^n is the explicit right-hand side: lambda times the mode
        assert np.max(np.abs(H[m] - np.real(lam * amp[m] * np.exp(1j * (theta + phase[m]))))) < 1e-13
    assert all(0 < it <= 50 for it in iters)


def test_pure_central_advection_conserves_energy():
    # uniform U, nu = 0: central advection is skew-symmetric, its Crank-Nicolson step an
    # orthogonal (Cayley) map, so sum u^2 is kept at any dt; viscosity makes it decrease
    g, st, u0, U, _, _ = _fourier_case(0.0, 1.0)
    rng = np.random.default_rng(11)
    u = [rng.standard_normal(g.shape) for _ in range(3)]
    dt = 1.5                                          # advective CFL 2.4
    us, _, _ = flow.cn_predictor(st, u, U, np.zeros(g.shape), 0.0, dt, (0.0, 0.0, 0.0), None, 1e-15, 400)
    for m in range(3):
        e0, e1 = np.sum(u[m] ** 2), np.sum(us[m] ** 2)
        assert abs(e1 - e0) < 1e-12 * e0
    us, _, _ = flow.cn_predictor(st, u, U, np.zeros(g.shape), 0.2, dt, (0.0, 0.0, 0.0), None, 1e-15, 400)
    for m in range(3):
        assert np.sum(us[m] ** 2) < 0.9 * np.sum(u[m] ** 2)


def test_deadend_cells_hold_their_wall_velocity():
    g = flow.Grid((5, 5, 5), 1.0, (0.0, 0.0, 0.0), (S,) * 6)
    b = np.zeros(g.shape, np.uint8)
    th = np.full(g.shape + (6,), 2.0)
    c = (2, 2, 2)
    for d in range(5):
        b[c] |= 1 << d
        th[c + (d,)] = 0.4
    for d, nb in ((0, (2, 2, 1)), (1, (2, 2, 3)), (2, (2, 1, 2)), (3, (2, 3, 2)), (4, (1, 2, 2))):
        b[nb] |= 1 << (d ^ 1)
        th[nb + (d ^ 1,)] = 0.6
    st = flow.build_stencils(g, b, th, deadend=True)
    assert st.deadend.sum() == 1
    rng = np.random.default_rng(5)
    wall = rng.standard_normal((st.ncut, 3))
    u = [rng.standard_normal(g.shape) for _ in range(3)]
    _, U, _, _ = flow.init_state(st, (0.2, 0.1, 0.0), wall)
    us, H, _ = flow.cn_predictor(st, u, U, np.zeros(g.shape), 0.05, 0.3, (0.0, 0.0, 0.0), wall, 1e-14, 100)
    dv = flow.dead_velocity(st, wall)
    sel = st.blocked.ravel()[st.cut_cell] == 0x3F
    for m in range(3):
        assert us[m][c] == dv[m][c]
        assert abs(dv[m][c] - np.mean(wall[sel, m])) < 1e-15
        assert H[m][c] == 0.0


def test_cn_step_projects_to_a_divergence_free_field():
    rng = np.random.default_rng(0)
    n = 12
    g = flow.Grid((n, n, n), 1.0, (0.0, 0.0, 0.0), (I, O, S, S, S, S), (1.0, 0.0, 0.0))
    tri = inputs.icosphere(2, 2.6, (n / 2 + 0.13, n / 2 - 0.07, n / 2 + 0.21), inputs.random_rotation(rng))
    st = flow.build_stencils(g, *tagging.tag(tri, g.n, g.dx, g.origin))
    u, U, p, h = flow.init_state(st, (1.0, 0.0, 0.0))
    for k in range(2):
        prm = flow.StepParams(dt=0.6, nu=0.01, tol=1e-12, scheme="cn", mom_tol=1e-12)
        u, U, p, h, stats = flow.step(st, u, U, p, h, prm, k)
        assert stats["div_linf"] < 1e-9 and stats["mom_iters"][0] > 0   # v, w start from a zero right-hand side
