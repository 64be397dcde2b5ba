"""Pins of the hybrid central/QUICK face value of the momentum oracle (Sec. 3: central
differences blended with 10 % QUICK; two-deep ghosts of the dummy cells, Sec. 2.3.1):
flux-form QUICK advection exact for cubic profiles (central is not), the Fourier symbol
of the blend for both flow directions and the Crank-Nicolson amplification with the
blend explicit, pairwise cancellation of face fluxes (conservation) with a non-uniform
face velocity, and linear exactness through a wall (first and second ghost)."""
import numpy as np
import pytest

from oracle import flow

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


def _open(g):
    return flow.build_stencils(g, np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0))


def _uniform_U(g, st, u0):
    _, U, _, _ = flow.init_state(st, u0)
    return U


@pytest.mark.parametrize("U0", [0.7, -0.7])
def test_quick_advection_exact_for_cubics(U0):
    # q = x^3 along x on a periodic box in y, z: QUICK face values carry a constant
    # error for a cubic, which cancels in the flux difference, so the advection term is
    # -U (q(x + dx/2) - q(x - dx/2)) / dx exactly; the central face value does not
    g = flow.Grid((14, 3, 3), 0.5, (0.0, 0.0, 0.0), (S, S, P, P, P, P))
    st = _open(g)
    xc = (np.arange(g.n[0]) + 0.5) * g.dx
    q = np.broadcast_to(xc ** 3 - 2.0 * xc ** 2 + 0.3 * xc, g.shape).copy()
    U = [np.full(g.shape, U0), np.zeros(g.shape), np.zeros(g.shape)]
    zero = [np.zeros(g.shape)] * 2
    f = lambda x: x ** 3 - 2.0 * x ** 2 + 0.3 * x  # noqa: E731
    exact = -U0 * (f(xc + 0.5 * g.dx) - f(xc - 0.5 * g.dx)) / g.dx
    inner = slice(2, g.n[0] - 2)
    Hq = flow.momentum_rhs(st, [q] + zero, U, np.zeros(g.shape), 0.0, (0, 0, 0), None, quick=1.0)[0]
    Hc = flow.momentum_rhs(st, [q] + zero, U, np.zeros(g.shape), 0.0, (0, 0, 0), None, quick=0.0)[0]
    assert np.max(np.abs(Hq[1, 1, inner] - exact[inner])) < 1e-12 * np.max(np.abs(exact))
    assert np.max(np.abs(Hc[1, 1, inner] - exact[inner])) > 1e-3
    # the blend is the linear combination of the two
    Hb = flow.momentum_rhs(st, [q] + zero, U, np.zeros(g.shape), 0.0, (0, 0, 0), None, quick=0.1)[0]
    assert np.max(np.abs(Hb - (0.9 * Hc + 0.1 * Hq))) < 1e-12 * np.max(np.abs(Hc))


def test_quick_fourier_symbol_and_crank_nicolson_closed_form():
    # uniform U with components of both signs on a periodic box, nu > 0: the right-hand
    # side of a Fourier mode is lambda times the mode with
    #   lambda = sum_a [-(U_a/dx)(1 - e^{-i kappa_a}) Phi_a - 2 nu (1 - cos kappa_a)/dx^2],
    #   Phi_a = (1-w)(1 + e^{i kappa})/2 + w (6 + 3 e^{i kappa} - e^{-i kappa})/8   (U_a > 0)
    #   Phi_a = (1-w)(1 + e^{i kappa})/2 + w (6 e^{i kappa} + 3 - e^{2 i kappa})/8  (U_a < 0)
    # and a Crank-Nicolson step with the blend explicit multiplies it by
    # 1 + dt lambda / (1 - dt lambda_c / 2), lambda_c the central symbol
    g = flow.Grid((16, 8, 8), 0.5, (0.0, 0.0, 0.0), (P,) * 6)
    st = _open(g)
    u0 = (0.8, -0.5, 0.3)
    U = _uniform_U(g, st, u0)
    nu, dt, w = 0.02, 0.4, 0.1
    modes = (2, 1, 1)
    kap = [2.0 * np.pi * modes[a] / g.n[a] for a in range(3)]
    zc, yc, xc = np.meshgrid(*[np.arange(g.n[a]) for a in (2, 1, 0)], indexing="ij")
    theta = kap[0] * xc + kap[1] * yc + kap[2] * zc

    def symbol(weight):
        lam = 0.0
        for a in range(3):
            e = np.exp(1j * kap[a])
            cen = (1.0 + e) / 2.0
            qk = (6.0 + 3.0 * e - 1.0 / e) / 8.0 if u0[a] > 0 else (6.0 * e + 3.0 - e * e) / 8.0
            phi = (1.0 - weight) * cen + weight * qk
            lam += -(u0[a] / g.dx) * (1.0 - 1.0 / e) * phi - 2.0 * nu * (1.0 - np.cos(kap[a])) / g.dx ** 2
        return lam

    lam, lam_c = symbol(w), symbol(0.0)
    assert lam.real < lam_c.real < 0.0                 # QUICK adds dissipation
    amp, phase = (0.3, -0.2, 0.15), (0.0, 1.1, -0.7)
    u = [u0[m] + amp[m] * np.cos(theta + phase[m]) for m in range(3)]
    H = flow.momentum_rhs(st, u, U, np.zeros(g.shape), nu, (0, 0, 0), None, quick=w)
    us, _, _ = flow.cn_predictor(st, u, U, np.zeros(g.shape), nu, dt, (0, 0, 0), None, 1e-14, 100, quick=w)
    G = 1.0 + dt * lam / (1.0 - 0.5 * dt * lam_c)
    for m in range(3):
        mode = amp[m] * np.exp(1j * (theta + phase[m]))
        assert np.max(np.abs(H[m] - np.real(lam * mode))) < 1e-13
        assert np.max(np.abs(us[m] - (u0[m] + np.real(G * mode)))) < 1e-13


def test_quick_face_fluxes_cancel_pairwise():
    # periodic box, random q and a random (not divergence-free) face velocity, nu = 0:
    # every face flux enters the two cells with opposite signs, so the advection terms
    # sum to zero, which needs both cells to build the same QUICK face value
    g = flow.Grid((10, 9, 8), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
    st = _open(g)
    rng = np.random.default_rng(4)
    q = rng.standard_normal(g.shape)
    U = [rng.standard_normal(g.shape) for _ in range(3)]
    zero = [np.zeros(g.shape)] * 2
    for w in (0.1, 1.0):
        H = flow.momentum_rhs(st, [q] + zero, U, np.zeros(g.shape), 0.0, (0, 0, 0), None, quick=w)[0]
        assert abs(np.sum(H)) < 1e-12 * np.sum(np.abs(H))
        assert np.max(np.abs(H)) > 0.1


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.8])
@pytest.mark.parametrize("U0", [0.6, -0.6])
def test_quick_linear_exactness_through_a_wall(theta, U0):
    # a linear field along x with the wall value taken from it: the first ghost of
    # eq. (q_axis) and the second ghost 2 G1 - q_c both equal the field's values, so the
    # QUICK and the central face values agree everywhere (both exact for linear data),
    # also on the faces whose QUICK stencil reaches through the wall
    g = flow.Grid((10, 3, 3), 1.0, (0.0, 0.0, 0.0), (S, S, P, P, P, P))
    blocked = np.zeros(g.shape, np.uint8)
    th = np.full(g.shape + (6,), 2.0)
    for j in range(3):
        for k in range(3):
            blocked[k, j, 4] |= 1 << 1           # wall between x-cells 4 and 5
            th[k, j, 4, 1] = theta
            blocked[k, j, 5] |= 1 << 0
            th[k, j, 5, 0] = 1.0 - theta
    st = flow.build_stencils(g, blocked, th)
    alpha, beta = 0.4, -1.1
    xc = (np.arange(g.n[0]) + 0.5) * g.dx
    q = np.broadcast_to(alpha + beta * xc, g.shape).copy()
    X = flow.cut_points(st)
    wall = np.zeros((st.ncut, 3))
    wall[:, 1] = alpha + beta * X[:, 0]          # component 1 (tangential to the wall)
    U = [np.full(g.shape, U0), np.zeros(g.shape), np.zeros(g.shape)]
    u = [np.zeros(g.shape), q, np.zeros(g.shape)]
    Hq = flow.momentum_rhs(st, u, U, np.zeros(g.shape), 0.0, (0, 0, 0), wall, quick=1.0)[1]
    Hc = flow.momentum_rhs(st, u, U, np.zeros(g.shape), 0.0, (0, 0, 0), wall, quick=0.0)[1]
    inner = slice(2, g.n[0] - 2)                 # away from the slip faces in x
    assert np.max(np.abs(Hq[:, :, inner] - Hc[:, :, inner])) < 1e-12
    assert np.max(np.abs(Hc[:, :, 4:6])) > 0.1   # the wall cells carry flux
