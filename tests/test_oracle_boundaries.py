"""Pins for the oracle's outer boundaries (Reading R10: the paper leaves the domain
faces open, Sec. 2.1) and for the eddy viscosity on blocked faces (Reading G4), against
closed forms that do not restate the ghost formulas:

* discrete eigenmodes of the 3-point diffusion operator.  On a cell-centred grid the
  modes sin(pi (i + 1/2)/n) (zero value on both faces), cos(pi (i + 1/2)/n) (zero
  gradient on both faces) and sin(pi (i + 1/2)/(2n)) (zero value on the first face,
  zero gradient on the last) are exact eigenvectors with eigenvalues
  -4 sin^2(pi/(2n))/dx^2, -4 sin^2(pi/(2n))/dx^2 and -4 sin^2(pi/(4n))/dx^2.  Inflow
  (Dirichlet u_in), outflow (zero gradient) and slip (zero normal velocity,
  zero-gradient tangential velocity) select which mode each velocity component must
  follow along each axis;
* the inflow face carries the prescribed velocity: its advective flux is u_in times
  the transported inflow value;
* uniform flow u = U_in through an empty inflow/outflow/slip channel is a steady
  solution of the whole step with p = 0;
* Couette flow between immersed walls at sub-cell offsets (a lower wall moving at
  U_b, an upper one at rest) with a uniform eddy viscosity between them is steady:
  the eq. (q_axis) ghosts are exact for the linear profile, so H = 0 in every channel
  cell, whatever the velocity and eddy viscosity beyond the walls.
"""
import math

import numpy as np
import pytest

from oracle import flow, tagging
from paper_2002_06206_amd import inputs

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


def _empty_stencil(g):
    blocked = np.zeros(g.shape, np.uint8)
    theta = np.full(g.shape + (6,), 2.0)
    return flow.build_stencils(g, blocked, theta)


def _centres(n):
    return np.arange(n) + 0.5


def _lam(n, dx, quarter=False):
    a = math.pi / (4 * n) if quarter else math.pi / (2 * n)
    return -4.0 * math.sin(a) ** 2 / dx ** 2


@pytest.mark.parametrize("dx", [1.0, 0.25])
def test_outer_boundary_diffusion_follows_discrete_eigenmodes(dx):
    """Channel with inflow at -x, outflow at +x and slip walls on y and z; face velocity
    zero, no eddy viscosity, no body force.  Each velocity component is a sum of the
    eigenmodes its boundary kinds select, so the momentum right-hand side is
    nu * (eigenvalue) * mode, term by term, to round-off."""
    n = (12, 10, 8)
    u_in = (1.3, 0.0, 0.0)
    g = flow.Grid(n, dx, (0.0, 0.0, 0.0), (I, O, S, S, S, S), u_in)
    st = _empty_stencil(g)
    nu = 0.07
    xi, yj, zk = (_centres(n[a]) for a in range(3))
    Z, Y, X = np.meshgrid(zk, yj, xi, indexing="ij")
    sx_dn = np.sin(math.pi * X / (2 * n[0]))       # value 0 at the inflow face, zero gradient at the outflow
    cy = np.cos(math.pi * Y / n[1])                  # zero gradient at both y faces
    cz = np.cos(math.pi * Z / n[2])
    sy = np.sin(math.pi * Y / n[1])                  # zero value at both y faces
    sz = np.sin(math.pi * Z / n[2])
    lx, ly, lz = _lam(n[0], dx, quarter=True), _lam(n[1], dx), _lam(n[2], dx)
    A, B, C, D, E = 0.8, -0.35, 0.6, 0.45, -0.7
    # u: tangential to the slip walls (zero gradient), Dirichlet u_in at the inflow
    u = u_in[0] + sx_dn * (A + B * cy + C * cz)
    # v, w: normal to their slip walls (zero value there), zero at the inflow
    v = D * sx_dn * sy
    w = E * sx_dn * sz
    zero = [np.zeros(g.shape)] * 3
    H = flow.momentum_rhs(st, [u, v, w], zero, np.zeros(g.shape), nu, (0.0, 0.0, 0.0), None)
    # the only advective flux is the inflow face's: u_in times the prescribed inflow value
    inflow = np.zeros(g.shape)
    inflow[:, :, 0] = u_in[0] * u_in[0] / dx
    exp_u = nu * sx_dn * (lx * A + (lx + ly) * B * cy + (lx + lz) * C * cz) + inflow
    exp_v = nu * (lx + ly) * v
    exp_w = nu * (lx + lz) * w
    scale = nu * abs(lx + ly + lz) + abs(inflow).max()
    for got, exp in ((H[0], exp_u), (H[1], exp_v), (H[2], exp_w)):
        assert np.max(np.abs(got - exp)) < 1e-12 * scale


@pytest.mark.parametrize("dx", [1.0, 0.5])
def test_uniform_inflow_is_a_steady_state_of_the_step(dx):
    """u = U_in e_x with consistent face velocities in an empty inflow / outflow / slip
    channel: one whole step (CSM on, AB2) leaves u and U unchanged and p = 0."""
    n = (10, 8, 6)
    u_in = (0.9, 0.0, 0.0)
    g = flow.Grid(n, dx, (0.0, 0.0, 0.0), (I, O, S, S, S, S), u_in)
    st = _empty_stencil(g)
    u, U, p, h = flow.init_state(st, u_in)
    prm = flow.StepParams(dt=0.2 * dx, nu=0.03, tol=1e-13)
    for k in range(2):
        u2, U2, p2, h, stats = flow.step(st, u, U, p, h, prm, k)
        for m in range(3):
            assert np.max(np.abs(u2[m] - u[m])) < 1e-14
            assert np.max(np.abs(U2[m] - U[m])) < 1e-14
        assert np.max(np.abs(p2)) < 1e-13
        assert np.max(np.abs(stats["nut"])) == 0.0
        u, U, p = u2, U2, p2


def _couette(delta_lo, delta_hi, seed):
    """Periodic in x and z, slip on y; immersed planes at y_lo (moving at U_b along x)
    and y_hi (at rest).  Returns the stencil, the wall velocities per cut and the
    channel mask."""
    ny = 20
    g = flow.Grid((4, ny, 4), 1.0, (0.0, 0.0, 0.0), (P, P, S, S, P, P))
    y_lo, y_hi = 4.0 + delta_lo, 13.0 + delta_hi
    tri = inputs.channel_planes(y_lo, y_hi, -2.0, 10.0)
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, b, th)
    X = flow.cut_points(st)
    Ub = 0.8
    wall = np.zeros((st.ncut, 3))
    wall[np.abs(X[:, 1] - y_lo) < 1e-9, 0] = Ub
    assert np.all((np.abs(X[:, 1] - y_lo) < 1e-9) | (np.abs(X[:, 1] - y_hi) < 1e-9))
    y = _centres(ny)
    chan = (y > y_lo) & (y < y_hi)
    prof = Ub * (y_hi - y) / (y_hi - y_lo)      # linear, U_b at y_lo and 0 at y_hi
    rng = np.random.default_rng(seed)
    outside = rng.standard_normal(ny)
    u_col = np.where(chan, prof, outside)
    return g, st, wall, chan, u_col, rng


@pytest.mark.parametrize("deltas", [(0.0, 0.0), (0.1, 0.75), (0.25, 0.5), (0.5, 0.9), (0.75, 0.1), (0.9, 0.3)])
def test_couette_between_immersed_walls_is_steady_with_own_side_eddy_viscosity(deltas):
    """With a uniform eddy viscosity nu_1 in the channel and a different, random one
    beyond the walls, Couette flow is steady in the channel: H = 0 there.  A wall flux
    that took any part of the other side's eddy viscosity would leave a residual shear
    of (nu_t,f - nu_1) * du/dy at the wall rows."""
    g, st, wall, chan, u_col, rng = _couette(*deltas, seed=3)
    shape = g.shape
    u = np.broadcast_to(u_col[None, :, None], shape).copy()
    nu1 = 0.021
    nut_col = np.where(chan, nu1, 0.05 + rng.uniform(0.0, 0.3, g.n[1]))
    nut = np.broadcast_to(nut_col[None, :, None], shape).copy()
    zero = np.zeros(shape)
    U = [u.copy(), zero.copy(), zero.copy()]
    H = flow.momentum_rhs(st, [u, zero, zero], U, nut, 0.01, (0.0, 0.0, 0.0), wall)
    mask = np.broadcast_to(chan[None, :, None], shape)
    for m in range(3):
        assert np.max(np.abs(H[m][mask])) < 1e-14, (deltas, m)
    # the eddy viscosity beyond the walls matters there (the check above is not vacuous)
    H2 = flow.momentum_rhs(st, [u, zero, zero], U, np.full(shape, nu1), 0.01, (0.0, 0.0, 0.0), wall)
    assert np.max(np.abs(H2[0][~mask] - H[0][~mask])) > 1e-6
