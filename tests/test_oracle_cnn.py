"""Pins for the CNN-preconditioner oracle (oracle/cnn.py) against library routines
(scipy's n-d correlation, torch's bfloat16 conversion, scipy's scalar minimiser, a
dense solve), brute-force loops, adjoint identities, finite differences and the
closed forms of Adam and conjugate gradients, and the network's four-cell receptive
field (window evaluation equals the full one).
"""
import numpy as np
import pytest
import scipy.ndimage
import scipy.optimize
import torch

from oracle import cnn, flow, tagging
from paper_2002_06206_amd import inputs

P, I, O, S = flow.PERIODIC, flow.INFLOW, flow.OUTFLOW, flow.SLIP


# ------------------------------------------------------------------ bf16

def test_bf16_round_matches_torch_including_ties():
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(20000) * np.exp(rng.uniform(-30, 30, 20000))).astype(np.float32)
    # exact ties: low 16 bits = 0x8000, both parities of the kept part
    u = rng.integers(0x00800000, 0x7F000000, 4000, dtype=np.uint32)
    ties = ((u & 0xFFFF0000) | 0x8000).view(np.float32)
    a = np.concatenate([a, ties, -ties, np.float32([0.0, -0.0, 1.0, 3.0e38])])
    ref = torch.from_numpy(a).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(cnn.bf16_round(a), ref)


def test_bf16_round_closed_forms():
    # bfloat16 keeps 7 fraction bits: the spacing at 1 is 2^-7
    assert cnn.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0                    # tie -> even
    assert cnn.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6    # tie -> even (up)
    assert cnn.bf16_round(np.array([1.0 + 2.0 ** -8 + 2.0 ** -12]))[0] == 1.0 + 2.0 ** -7
    assert np.isnan(cnn.bf16_round(np.array([np.nan]))[0])


# ------------------------------------------------------------------ convolution

def test_conv_forward_matches_scipy_correlate():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((5, 6, 7, 3))
    w = rng.standard_normal((27, 3, 2))
    y = cnn.conv_forward(x, w)
    for co in range(2):
        ref = np.zeros(x.shape[:3])
        for ci in range(3):
            k = w[:, ci, co].reshape(3, 3, 3)     # [dz+1, dy+1, dx+1]
            ref += scipy.ndimage.correlate(x[..., ci], k, mode="constant", cval=0.0)
        np.testing.assert_allclose(y[..., co], ref, rtol=0, atol=1e-12)


def test_conv_forward_brute_force_loops():
    rng = np.random.default_rng(2)
    nz, ny, nx = 3, 4, 5
    x = rng.standard_normal((nz, ny, nx, 2))
    w = rng.standard_normal((27, 2, 3))
    y = cnn.conv_forward(x, w)
    for z in range(nz):
        for yy in range(ny):
            for xx in range(nx):
                for co in range(3):
                    acc = 0.0
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, y2, x2 = z + dz, yy + dy, xx + dx
                                if 0 <= zz < nz and 0 <= y2 < ny and 0 <= x2 < nx:
                                    t = (dz + 1) * 9 + (dy + 1) * 3 + (dx + 1)
                                    for ci in range(2):
                                        acc += x[zz, y2, x2, ci] * w[t, ci, co]
                    assert abs(y[z, yy, xx, co] - acc) < 1e-12


def test_conv_backward_adjoint_identities():
    """conv_forward is bilinear in (x, w); its two backward maps are the adjoints:
    <conv(x, w), g> = <x, bwd_data(g, w)> = <w, bwd_weight(x, g)>."""
    rng = np.random.default_rng(3)
    x = rng.standard_normal((4, 5, 6, 16))
    w = rng.standard_normal((27, 16, 4))
    g = rng.standard_normal((4, 5, 6, 4))
    lhs = np.sum(cnn.conv_forward(x, w) * g)
    assert abs(lhs - np.sum(x * cnn.conv_backward_data(g, w))) < 1e-9 * abs(lhs)
    assert abs(lhs - np.sum(w * cnn.conv_backward_weight(x, g))) < 1e-9 * abs(lhs)


def test_network_backward_matches_finite_differences():
    rng = np.random.default_rng(4)
    x = rng.standard_normal((4, 5, 6))
    g = rng.uniform(0, 1, (4, 5, 6))
    ws = cnn.split_weights(inputs.cnn_init_weights(7, scale=5.0).astype(np.float64))
    ws[2] = ws[2] * 15.0   # gate weights large enough that part of the gate is clamped
    R = rng.standard_normal((4, 5, 6))

    def J(ws_, x_, g_):
        y, _ = cnn.forward(x_, g_, ws_)
        return float(np.sum(y * R))

    # the gate's pre-activations cover both the linear part of hsig (|v| < 2) and its
    # clamps, so the checks below see both branches of its slope
    inside = np.mean(np.abs(cnn.conv_forward(g[..., None], ws[2])) < 2.0)
    assert 0.2 < inside < 0.9, inside
    y, saved = cnn.forward(x, g, ws)
    dws, dx, dg = cnn.backward(saved, ws, R)
    assert np.max(np.abs(dws[2])) > 0.0
    h = 1e-6
    for l in range(3):
        for _ in range(8):
            idx = tuple(rng.integers(0, s) for s in ws[l].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h
            wm[l][idx] -= h
            fd = (J(wp, x, g) - J(wm, x, g)) / (2 * h)
            assert abs(fd - dws[l][idx]) < 1e-6 * max(1e-3, abs(fd)), (l, idx, fd, dws[l][idx])
    for arr, grad in ((x, dx), (g, dg)):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in arr.shape)
            ap, am = arr.copy(), arr.copy()
            ap[idx] += h
            am[idx] -= h
            args_p = (ap, g) if arr is x else (x, ap)
            args_m = (am, g) if arr is x else (x, am)
            fd = (J(ws, *args_p) - J(ws, *args_m)) / (2 * h)
            assert abs(fd - grad[idx]) < 1e-6 * max(1e-3, abs(fd))


def test_network_is_linear_symmetric_and_positive():
    """K^T K with a fixed geometry gate: linear in x, self-adjoint, x.net(x) = |Kx|^2 >= 0."""
    rng = np.random.default_rng(5)
    g = rng.uniform(0, 1, (5, 6, 7))
    u, v = rng.standard_normal((2, 5, 6, 7))
    ws = cnn.split_weights(inputs.cnn_init_weights(1, scale=4.0).astype(np.float64))
    nu, _ = cnn.forward(u, g, ws)
    nv, _ = cnn.forward(v, g, ws)
    nuv, _ = cnn.forward(2.5 * u - 0.7 * v, g, ws)
    np.testing.assert_allclose(nuv, 2.5 * nu - 0.7 * nv, rtol=1e-10, atol=1e-12 * np.max(np.abs(nu)))
    assert abs(np.sum(u * nv) - np.sum(v * nu)) < 1e-10 * np.sqrt(np.sum(nu * nu) * np.sum(v * v))
    assert np.sum(u * nu) > 0.0 and np.sum(v * nv) > 0.0


# ------------------------------------------------------------------ preconditioner and loss

def _plate_stencil(n=(10, 8, 6), seed=0):
    """Open geometry (a plate) with an outlet: A is nonsingular."""
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), (I, O, S, S, S, S))
    tri = inputs.rectangle((4.4, 3.7, 2.9), (0, 4.0, 0.7), (0.5, 0, 3.0))
    b, th = tagging.tag(tri, g.n, g.dx, g.origin)
    return g, flow.build_stencils(g, b, th)


def _dense_A(st):
    g = st.grid
    N = g.ncell
    A = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        A[:, j] = cnn.apply_A(st, e.reshape(g.shape)).ravel()
        e[j] = 0.0
    return A


def test_geometry_channel_closed_form():
    g = flow.Grid((4, 5, 6), 1.0, (0.0, 0.0, 0.0), (P,) * 6)
    st = flow.build_stencils(g, *(np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0)))
    assert np.all(cnn.geometry_channel(st) == 1.0)
    g = flow.Grid((4, 5, 6), 1.0, (0.0, 0.0, 0.0), (S,) * 6)
    st = flow.build_stencils(g, *(np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0)))
    gc = cnn.geometry_channel(st)
    assert gc[0, 0, 0] == 3.0 / 6.0 and gc[2, 2, 1] == 1.0 and gc[0, 2, 2] == 5.0 / 6.0


def test_zero_weights_give_jacobi():
    g, st = _plate_stencil()
    r = np.random.default_rng(6).standard_normal(g.shape)
    ws = [np.zeros((27, ci, co)) for _, ci, co in cnn.LAYERS]
    z = cnn.precondition(st, r, ws)
    np.testing.assert_allclose(z, r / flow.jacobi_diag(st), rtol=1e-15)


@pytest.mark.parametrize("omega", [0.0, 0.8])
def test_loss_is_the_minimum_energy_distance(omega):
    """loss = min_a |p - a p_hat|_A^2 / |p|_A^2, checked with a dense solve for p and a
    scalar minimiser for a (p_hat from the additive and the smoothed form)."""
    g, st = _plate_stencil()
    A = _dense_A(st)
    assert np.allclose(A, A.T)
    rng = np.random.default_rng(8)
    b = rng.standard_normal(g.shape)
    p = np.linalg.solve(A, -b.ravel()).reshape(g.shape)        # L p = b  <=>  A p = -b
    ws = cnn.split_weights(inputs.cnn_init_weights(3, scale=3.0).astype(np.float64))
    ph = cnn.precondition(st, -b, ws, omega=omega)
    pA = p.ravel() @ A @ p.ravel()

    def E(a):
        e = p.ravel() - a * ph.ravel()
        return e @ A @ e / pA

    res = scipy.optimize.minimize_scalar(E, bracket=(0.0, 1.0), tol=1e-12)
    loss = cnn.loss_only(st, b, p, ws, omega=omega)
    assert 0.0 < loss < 1.0
    assert abs(loss - res.fun) < 1e-10
    # the training loss evaluates the same p_hat
    assert abs(cnn.loss_and_grad(st, b, p, ws, omega=omega)[0] - loss) < 1e-13


def test_loss_scale_invariance():
    g, st = _plate_stencil()
    A = _dense_A(st)
    rng = np.random.default_rng(9)
    b = rng.standard_normal(g.shape)
    p = np.linalg.solve(A, -b.ravel()).reshape(g.shape)
    ws = cnn.split_weights(inputs.cnn_init_weights(4, scale=3.0).astype(np.float64))
    l1 = cnn.loss_only(st, b, p, ws)
    l2 = cnn.loss_only(st, 1e-3 * b, 1e-3 * p, ws)
    assert abs(l1 - l2) < 1e-12


@pytest.mark.parametrize("omega", [0.0, 0.8])
def test_loss_gradient_matches_finite_differences(omega):
    """The analytic gradient (through the smoothing steps too) against central
    differences of the loss, which is evaluated from the preconditioner itself."""
    g, st = _plate_stencil()
    A = _dense_A(st)
    rng = np.random.default_rng(10)
    b = rng.standard_normal(g.shape)
    p = np.linalg.solve(A, -b.ravel()).reshape(g.shape)
    ws = cnn.split_weights(inputs.cnn_init_weights(5, scale=3.0).astype(np.float64))
    loss, dws = cnn.loss_and_grad(st, b, p, ws, omega=omega)
    assert abs(loss - cnn.loss_only(st, b, p, ws, omega=omega)) < 1e-13
    h = 1e-6
    for l in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, s) for s in ws[l].shape)
            wp = [w.copy() for w in ws]
            wm = [w.copy() for w in ws]
            wp[l][idx] += h
            wm[l][idx] -= h
            fd = (cnn.loss_only(st, b, p, wp, omega=omega) - cnn.loss_only(st, b, p, wm, omega=omega)) / (2 * h)
            assert abs(fd - dws[l][idx]) < 1e-6 * max(1e-3, abs(fd)), (l, idx, fd, dws[l][idx])


def test_two_level_form_matches_its_matrix():
    """The smoothed preconditioner (three sequential steps) equals the matrix
    2S - S A S + (I - S A) C (I - A S), S = omega D^-1, assembled from dense A and the
    dense additive preconditioner C: a dropped term, a wrong sign or the unsmoothed
    residual fed to the network changes it."""
    g, st = _plate_stencil()
    A = _dense_A(st)
    N = g.ncell
    ws = cnn.split_weights(inputs.cnn_init_weights(7, scale=3.0).astype(np.float64))
    C = np.zeros((N, N))
    e = np.zeros(N)
    for j in range(N):
        e[j] = 1.0
        C[:, j] = cnn.precondition(st, e.reshape(g.shape), ws).ravel()
        e[j] = 0.0
    omega = 0.8
    S = np.diag(omega / flow.jacobi_diag(st).ravel())
    I_ = np.eye(N)
    M = 2.0 * S - S @ A @ S + (I_ - S @ A) @ C @ (I_ - A @ S)
    assert np.allclose(M, M.T, rtol=0, atol=1e-12 * np.abs(M).max())
    assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0.0
    rng = np.random.default_rng(13)
    for _ in range(3):
        r = rng.standard_normal(g.shape)
        z = cnn.precondition(st, r, ws, omega=omega)
        np.testing.assert_allclose(z.ravel(), M @ r.ravel(), rtol=0, atol=1e-12 * np.abs(M @ r.ravel()).max())


def test_two_level_form_on_a_fourier_mode():
    """Zero weights on a periodic box: A has the Fourier modes as eigenvectors with
    lambda = sum over axes of 2 (1 - cos(2 pi m / n)) / dx^2 and D = 6 / dx^2, so the
    smoothed preconditioner scales a mode by 2 s - s^2 lambda + (1 - s lambda)^2 / D,
    s = omega / D."""
    n = (8, 6, 10)
    dx = 0.5
    g = flow.Grid(n, dx, (0.0, 0.0, 0.0), (P,) * 6)
    st = flow.build_stencils(g, np.zeros(g.shape, np.uint8), np.full(g.shape + (6,), 2.0))
    ws = [np.zeros((27, ci, co)) for _, ci, co in cnn.LAYERS]
    kz, ky, kx = np.meshgrid(np.arange(n[2]), np.arange(n[1]), np.arange(n[0]), indexing="ij")
    for m, omega in (((1, 2, 3), 6.0 / 7.0), ((4, 3, 5), 0.5), ((0, 1, 0), 1.0)):
        r = np.cos(2 * np.pi * (m[0] * kx / n[0] + m[1] * ky / n[1] + m[2] * kz / n[2]))
        lam = sum(2.0 * (1.0 - np.cos(2 * np.pi * m[a] / n[a])) for a in range(3)) / dx ** 2
        D = 6.0 / dx ** 2
        sm = omega / D
        factor = 2.0 * sm - sm * sm * lam + (1.0 - sm * lam) ** 2 / D
        z = cnn.precondition(st, r, ws, omega=omega)
        np.testing.assert_allclose(z, factor * r, rtol=0, atol=1e-13 * D ** -1)


def test_two_level_jacobi_needs_fewer_iterations():
    """With zero weights the smoothed form is a degree-two polynomial in D^-1 A around
    Jacobi; FCG(1) on it converges to the dense solution in fewer iterations than
    Jacobi-PCG."""
    g, st = _plate_stencil()
    A = _dense_A(st)
    rng = np.random.default_rng(14)
    b = rng.standard_normal(g.shape)
    p = np.linalg.solve(A, -b.ravel()).reshape(g.shape)
    ws = [np.zeros((27, ci, co)) for _, ci, co in cnn.LAYERS]
    x, it = cnn.fcg(st, b, np.zeros(g.shape), lambda r: cnn.precondition(st, r, ws, omega=6.0 / 7.0), 1e-10, 500)
    _, it_j = flow.pcg(st, b, np.zeros(g.shape), 1e-10, 500)
    assert np.max(np.abs(x - p)) < 1e-7 * np.max(np.abs(p))
    assert it < it_j, (it, it_j)


def test_adam_first_steps_closed_form():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    w0 = np.array([1.0, 2.0, 3.0, 4.0])
    m = np.zeros(4)
    v = np.zeros(4)
    w1, m, v = cnn.adam(w0, g, m, v, 1, 0.01)
    # first step: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    np.testing.assert_allclose(w1, w0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14)
    # second step with the same gradient: bias corrections make m_hat = g, v_hat = g^2 again
    w2, m, v = cnn.adam(w1, g, m, v, 2, 0.01)
    np.testing.assert_allclose(w2, w1 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


# ------------------------------------------------------------------ flexible CG

def test_fcg_with_jacobi_equals_pcg():
    """With a fixed symmetric positive definite preconditioner the Polak-Ribiere beta
    equals the Fletcher-Reeves one (r_k is orthogonal to z_{k-1} = M^-1 r_{k-1}), so
    FCG(1) reproduces Jacobi-PCG."""
    g, st = _plate_stencil()
    rng = np.random.default_rng(11)
    b = rng.standard_normal(g.shape)
    minv = cnn.jacobi_inverse(st)
    x1, it1 = cnn.fcg(st, b, np.zeros(g.shape), lambda r: minv * r, 1e-10, 500)
    x2, it2 = flow.pcg(st, b, np.zeros(g.shape), 1e-10, 500)
    assert abs(it1 - it2) <= 1
    assert np.max(np.abs(x1 - x2)) < 1e-7 * np.max(np.abs(x2))


@pytest.mark.parametrize("omega", [0.0, 6.0 / 7.0])
def test_fcg_with_learned_preconditioner_solves(omega):
    """The learned operator is symmetric positive definite (Jacobi plus K^T K, alone or
    between the two damped Jacobi steps): FCG(1) converges to the dense solution."""
    g, st = _plate_stencil()
    A = _dense_A(st)
    rng = np.random.default_rng(12)
    b = rng.standard_normal(g.shape)
    p = np.linalg.solve(A, -b.ravel()).reshape(g.shape)
    ws = cnn.split_weights(inputs.cnn_init_weights(6, scale=4.0).astype(np.float64))
    x, it = cnn.fcg(st, b, np.zeros(g.shape), lambda r: cnn.precondition(st, r, ws, omega=omega), 1e-10, 500)
    assert it > 3
    assert np.max(np.abs(x - p)) < 1e-7 * np.max(np.abs(p))


def test_network_receptive_field_is_four_cells():
    # four 3^3 layers: the output at a cell depends on the input and the geometry
    # channel within 4 cells, so the network evaluated on the 9^3 window around a cell
    # (clipped at the grid faces, where both forms pad with zeros) gives the full
    # evaluation's value exactly; a 7^3 window does not (the full-size sampled parity
    # test of the device preconditioner relies on the first fact)
    rng = np.random.default_rng(41)
    shape = (14, 13, 15)
    x = rng.standard_normal(shape)
    g = rng.random(shape)
    ws = cnn.split_weights(inputs.cnn_init_weights(5, scale=4.0).astype(np.float64))
    full, _ = cnn.forward(x, g, ws, bf16=True)
    short = 0
    for (k, j, i) in [(7, 6, 7), (0, 0, 0), (13, 12, 14), (2, 9, 4), (11, 3, 10)]:
        for R, exact in ((4, True), (3, False)):
            lo = (max(0, k - R), max(0, j - R), max(0, i - R))
            win = tuple(slice(lo[a], min(shape[a], c + R + 1)) for a, c in enumerate((k, j, i)))
            y, _ = cnn.forward(x[win], g[win], ws, bf16=True)
            v = y[k - lo[0], j - lo[1], i - lo[2]]
            if exact:
                assert v == full[k, j, i]
            elif v != full[k, j, i]:
                short += 1
    assert short >= 1   # the interior cell's 7^3 window misses part of its dependence
