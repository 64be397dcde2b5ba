"""Pins of the red-black SOR oracle (oracle/flow.py rbsor; Sec. 2.1, the paper's
alternative Poisson solver): the Gauss-Seidel property of each half sweep at omega = 1
(every cell of the colour just updated satisfies its own equation), the solution of a
walled problem with an outlet against the pinned conjugate-gradient solve, the gauge
freedom of an enclosed component, the classical optimal-omega speed-up over
Gauss-Seidel, and the rejection of odd periodic counts."""
import math

import numpy as np
import pytest

from oracle import flow, tagging
from paper_2002_06206_amd import inputs

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


def _walled(bc=(I, O, S, S, P, P), n=(10, 8, 6)):
    rng = np.random.default_rng(0)
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), bc)
    tri = np.concatenate([inputs.icosphere(1, 2.2, (4.3, 4.1, 3.1), inputs.random_rotation(rng)),
                          inputs.rectangle((7.2, 3.1, 3.0), (0, 5.0, 0), (0, 0, 4.0))])
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    return g, flow.build_stencils(g, b, th), rng


def test_half_sweeps_are_gauss_seidel_at_omega_one():
    g, st, rng = _walled()
    b = rng.standard_normal(g.shape)
    x = rng.standard_normal(g.shape)
    ii, jj, kk = np.meshgrid(np.arange(g.n[2]), np.arange(g.n[1]), np.arange(g.n[0]), indexing="ij")
    colour = (ii + jj + kk) % 2
    has = flow.jacobi_diag(st) > 0
    # one sweep of the oracle, then the residual of each colour right after its half
    x1, it, _ = flow.rbsor(st, b, x, 1.0, 0.0, 1)
    assert it == 1
    # black residuals vanish after the full sweep (their update was last)
    r = b - flow.laplacian(st, x1)
    assert np.max(np.abs(r[(colour == 1) & has])) < 1e-12 * np.max(np.abs(b))
    # red residuals vanish after the red half (rebuilt by hand from the definition)
    diag = -flow.jacobi_diag(st)
    xr = np.where((colour == 0) & has, x + (b - flow.laplacian(st, x)) / np.where(has, diag, 1.0), x)
    rr = b - flow.laplacian(st, xr)
    assert np.max(np.abs(rr[(colour == 0) & has])) < 1e-12 * np.max(np.abs(b))
    assert np.max(np.abs(r[(colour == 0) & has])) > 1e-3       # ... and not after the black half


def test_solution_matches_conjugate_gradients_with_outlet():
    g, st, rng = _walled()
    b = rng.standard_normal(g.shape)
    b = flow.remove_component_means(st, b)
    x, it, ok = flow.rbsor(st, b, np.zeros(g.shape), 1.7, 1e-11, 20000, check_every=4)
    assert ok and it % 4 == 0 and it > 0
    xc, _ = flow.pcg(st, b, np.zeros(g.shape), 1e-13, 20000)
    x = flow.remove_component_means(st, x)
    xc = flow.remove_component_means(st, xc)
    assert np.linalg.norm(x - xc) / np.linalg.norm(xc) < 1e-8
    assert np.linalg.norm(b - flow.laplacian(st, x)) <= 1e-11 * np.linalg.norm(b)


def test_enclosed_component_converges_up_to_its_constant():
    # a closed box (a pure Neumann component): b compatible, the solution is unique up
    # to the component's constant, which the gauge removes
    g = flow.Grid((10, 10, 10), 1.0, (0.0, 0.0, 0.0), (I, O, S, S, S, S))
    from test_oracle_tagging import _box
    tri = _box((2.0, 2.0, 2.0), (8.0, 8.0, 8.0))     # faces between cell centres
    st = flow.build_stencils(g, *tagging.tag(tri, g.n, g.dx, g.origin))
    assert len(st.comps) == 1
    rng = np.random.default_rng(3)
    b = flow.remove_component_means(st, rng.standard_normal(g.shape))
    x, _, ok = flow.rbsor(st, b, rng.standard_normal(g.shape), 1.6, 1e-10, 20000, check_every=2)
    xc, _ = flow.pcg(st, b, np.zeros(g.shape), 1e-13, 20000)
    assert ok
    d = flow.remove_component_means(st, x) - flow.remove_component_means(st, xc)
    assert np.linalg.norm(d) / np.linalg.norm(xc) < 1e-7


def test_optimal_omega_beats_gauss_seidel():
    # a long channel with an outlet (p = 0 on the +x face), Neumann elsewhere: with
    # omega near 2/(1 + sin(pi/2n)) SOR needs several times fewer sweeps than omega = 1
    g = flow.Grid((24, 4, 4), 1.0, (0.0, 0.0, 0.0), (I, O, S, S, S, S))
    st = flow.build_stencils(g, np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0))
    rng = np.random.default_rng(5)
    b = rng.standard_normal(g.shape)
    _, it_gs, ok1 = flow.rbsor(st, b, np.zeros(g.shape), 1.0, 1e-8, 100000)
    w = 2.0 / (1.0 + math.sin(math.pi / (2 * g.n[0])))
    _, it_sor, ok2 = flow.rbsor(st, b, np.zeros(g.shape), w, 1e-8, 100000)
    assert ok1 and ok2
    assert it_gs > 4 * it_sor


def test_odd_periodic_count_rejected_and_zero_rhs():
    g = flow.Grid((9, 4, 4), 1.0, (0.0, 0.0, 0.0), (P, P, S, S, S, S))
    st = flow.build_stencils(g, np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0))
    with pytest.raises(ValueError):
        flow.rbsor(st, np.ones(g.shape), np.zeros(g.shape), 1.5, 1e-8, 10)
    g, st, rng = _walled()
    x, it, ok = flow.rbsor(st, np.zeros(g.shape), rng.standard_normal(g.shape), 1.5, 1e-8, 10)
    assert ok and it == 0 and not np.any(x)
