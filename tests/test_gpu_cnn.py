"""GPU parity of the learned preconditioner (BF16 MFMA kernels, FP32 accumulation)
against the FP64 oracle of oracle/cnn.py through the C ABI.

Tolerances.  The oracle takes every BF16 rounding the GPU takes (input, hidden
activations, backward signals, weights) and sums exactly in FP64; the GPU sums the
same BF16 products in FP32 (relative error ~ K * 2^-24, K <= 432 products).  The two
therefore differ only where that FP32 error moves a value across a BF16 rounding
boundary, which flips one stored activation by one BF16 unit (2^-8 relative) with
probability ~ 1e-4 per value.  The resulting relative L2 differences measured at
the seeds below are 6e-6 to 6e-5 (the kernels are deterministic, so a seed gives the
same value on every run); each bar is about three times its measured value (stated
next to it), so one wrong tap or channel confined to a tile edge fails.  The loss,
which lies in [0, 1], is checked to 1e-4 absolute.
"""
import numpy as np
import pytest

from oracle import cnn, flow, tagging
from paper_2002_06206_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2002_06206_amd import ibm
else:  # collected on CPU machines, skipped by the marker filter
    ibm = None

RAGGED = (37, 13, 9)   # nx, ny, nz: two or more 32x8x4 tiles per axis with ragged tails


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.sqrt(np.sum(b * b))
    return np.sqrt(np.sum((a - b) ** 2)) / den if den > 0 else np.sqrt(np.sum(a * a))


def _layers(flat):
    return cnn.split_weights(np.asarray(flat, dtype=np.float64))


def _ws_bf16(flat):
    return cnn.split_weights(cnn.bf16_round(np.asarray(flat, dtype=np.float32)))


def _input(rng, shape):
    """cells x 2: channel 0 the network input x, channel 1 the geometry g in [0, 1]."""
    x = np.stack([rng.standard_normal(shape), rng.uniform(0.0, 1.0, shape)], axis=-1)
    return torch.from_numpy(x).to(torch.bfloat16)


def _forward_case(seed=0, n=RAGGED):
    rng = np.random.default_rng(seed)
    shape = (n[2], n[1], n[0])
    xb = _input(rng, shape)
    w = inputs.cnn_init_weights(seed + 3, scale=4.0)
    net = ibm.Network(int(np.prod(n)), w)
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    ibm.ibm_cnn_forward(net.net, xb.cuda().contiguous(), y, n)
    return net, w, xb.double().numpy(), y.cpu().numpy()


def test_forward_matches_oracle_ragged_grid():
    print("case cnn forward", RAGGED, flush=True)
    net, w, x, y = _forward_case()
    yo, _ = cnn.forward(x[..., 0], x[..., 1], _layers(w), bf16=True)
    e = rel_l2(y, yo)
    print("forward rel L2 %.2e" % e, flush=True)
    assert np.all(np.isfinite(y))
    assert e < 6e-5          # measured 2.0e-5
    # without the BF16 rounding points the FP64 network is still close (stated, loose)
    yf, _ = cnn.forward(x[..., 0], x[..., 1], _layers(w), bf16=False)
    assert rel_l2(y, yf) < 5e-2
    net.close()


def test_marching_forward_matches_oracle_ragged_grid():
    """The inference-only network runs the marching kernels of the solver path (z
    slabs of a 32 x 8 tile, gate computed on the fly): same oracle bar as the kept
    forward, on the ragged grid (several slabs, short last slab)."""
    rng = np.random.default_rng(21)
    shape = (RAGGED[2], RAGGED[1], RAGGED[0])
    xb = _input(rng, shape)
    w = inputs.cnn_init_weights(22, scale=4.0)
    net = ibm.Network(int(np.prod(RAGGED)), w, inference_only=True)
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    print("case cnn marching forward", RAGGED, flush=True)
    ibm.ibm_cnn_forward(net.net, xb.cuda().contiguous(), y, RAGGED)
    x = xb.double().numpy()
    yo, _ = cnn.forward(x[..., 0], x[..., 1], _layers(w), bf16=True)
    e = rel_l2(y.cpu().numpy(), yo)
    print("marching forward rel L2 %.2e" % e, flush=True)
    assert e < 4e-5          # measured 1.3e-5
    net.close()


def test_marching_forward_matches_kept_forward():
    """The two forward forms take the same BF16 roundings in the three 16-channel
    layers and accumulate their MFMA k-steps in the same order, so those activations
    agree bit for bit; the last (16 -> 1) layer of the marching form sums the same exact
    BF16 x BF16 products in another order (three FP32 partial sums per output instead of
    one chain), so the outputs differ only by FP32 summation error: at most ~432 * 2^-24
    of the sum of |products| per cell, bounded here by 1e-5 relative L2.  250 x 250 x 45
    gives 6-plane slabs with a short last slab and ragged x-y tiles."""
    n = (250, 250, 45)
    shape = (n[2], n[1], n[0])
    xb = _input(np.random.default_rng(23), shape).cuda().contiguous()
    w = inputs.cnn_init_weights(24, scale=4.0)
    ys = []
    for inference_only in (False, True):
        net = ibm.Network(int(np.prod(n)), w, inference_only=inference_only)
        y = torch.empty(shape, dtype=torch.float32, device="cuda")
        print("case cnn forward forms", n, "inference_only", inference_only, flush=True)
        ibm.ibm_cnn_forward(net.net, xb, y, n)
        torch.cuda.synchronize()
        ys.append(y.cpu().numpy())
        net.close()
    assert np.all(np.isfinite(ys[0])) and np.max(np.abs(ys[0])) > 0.0
    e = rel_l2(ys[1], ys[0])
    print("marching vs kept forward rel L2 %.2e" % e, flush=True)
    assert e < 1e-5


def test_forward_tile_edges_exact_zero_padding():
    """A unit impulse in x at the last cell of the first 32 x 8 x 4 tile: checked against
    the oracle at every cell, across tile boundaries and up to the domain faces (zero
    padding), and nothing outside the 9-cell reach of the four convolutions."""
    n = (64, 16, 8)
    shape = (n[2], n[1], n[0])
    rng = np.random.default_rng(12)
    x = np.zeros(shape + (2,))
    x[3, 7, 31, 0] = 1.0
    x[..., 1] = rng.uniform(0.0, 1.0, shape)
    xb = torch.from_numpy(x).to(torch.bfloat16)
    w = inputs.cnn_init_weights(11, scale=4.0)
    net = ibm.Network(int(np.prod(n)), w)
    y = torch.empty(shape, dtype=torch.float32, device="cuda")
    print("case cnn impulse", n, flush=True)
    ibm.ibm_cnn_forward(net.net, xb.cuda().contiguous(), y, n)
    xo = xb.double().numpy()
    yo, _ = cnn.forward(xo[..., 0], xo[..., 1], _layers(w), bf16=True)
    y = y.cpu().numpy()
    scale = np.max(np.abs(yo))
    assert scale > 0.0
    assert np.max(np.abs(y - yo)) <= 1e-2 * scale
    far = np.ones(shape, dtype=bool)
    far[0:8, 3:12, 27:36] = False
    assert np.all(y[far] == 0.0)
    net.close()


def test_backward_matches_oracle_ragged_grid():
    print("case cnn backward", RAGGED, flush=True)
    net, w, x, _ = _forward_case(1)
    rng = np.random.default_rng(5)
    shape = x.shape[:3]
    dy = rng.standard_normal(shape).astype(np.float32)
    dw = torch.empty(ibm.CNN_NWEIGHTS, dtype=torch.float32, device="cuda")
    dx = torch.empty(shape + (2,), dtype=torch.float32, device="cuda")
    ibm.ibm_cnn_backward(net.net, torch.from_numpy(dy).cuda(), dw, dx)
    _, saved = cnn.forward(x[..., 0], x[..., 1], _layers(w), bf16=True)
    dws, dxo, dgo = cnn.backward(saved, _layers(w), dy.astype(np.float64), bf16=True)
    gw = cnn.split_weights(dw.cpu().numpy())
    for l in range(3):
        e = rel_l2(gw[l], dws[l])
        print("%s weight-gradient rel L2 %.2e" % (cnn.LAYERS[l][0], e), flush=True)
        assert e < 1.6e-4    # measured 4.2e-5 (W1), 1.0e-5 (W2), 5.2e-5 (Wg)
    dxg = dx.cpu().numpy()
    e = rel_l2(dxg[..., 0], dxo)
    eg = rel_l2(dxg[..., 1], dgo)
    print("input-gradient rel L2 %.2e, geometry-gradient rel L2 %.2e" % (e, eg), flush=True)
    assert e < 2e-5 and eg < 1.8e-4    # measured 6.3e-6, 5.8e-5
    net.close()


def _geometry_case(seed=5, n=40):
    case = inputs.case_ellipsoids256(seed=seed, n=n)
    g = flow.Grid(case.n, case.dx, case.origin, case.bc, case.u_in)
    ob, ot = tagging.tag(case.tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, ob, ot)
    s = ibm.Solver(g.n, g.dx, g.origin, g.bc, g.u_in, ibm.MIXED)
    s.build(torch.from_numpy(ob).cuda(), torch.from_numpy(ot).cuda())
    rng = np.random.default_rng(seed + 100)
    p = flow.remove_component_means(st, rng.standard_normal(g.shape))
    b = flow.laplacian(st, p)
    return g, st, s, b, p


@pytest.mark.parametrize("omega", [0.0, 6.0 / 7.0])
def test_loss_and_gradient_match_oracle(omega):
    """The training loss and its weight gradient, for the network's map alone and
    through the smoothed form (the FP64 smoothing steps of the loss on both sides)."""
    g, st, s, b, p = _geometry_case()
    w = inputs.cnn_init_weights(2, scale=3.0)
    net = ibm.Network(g.ncell, w)
    dw = torch.empty(ibm.CNN_NWEIGHTS, dtype=torch.float32, device="cuda")
    print("case cnn loss", g.n, "omega", omega, flush=True)
    loss = net.loss(s, torch.from_numpy(b).cuda(), torch.from_numpy(p).cuda(), dw, omega=omega)
    lo, dws = cnn.loss_and_grad(st, b, p, _layers(w), bf16=True, omega=omega)
    print("loss gpu %.6f oracle %.6f" % (loss, lo), flush=True)
    assert 0.0 < loss < 1.0
    assert abs(loss - lo) < 1e-4
    gw = cnn.split_weights(dw.cpu().numpy())
    for l in range(3):
        e = rel_l2(gw[l], dws[l])
        print("%s loss-gradient rel L2 %.2e" % (cnn.LAYERS[l][0], e), flush=True)
        assert e < 8e-5      # measured 2.0e-5 (W1), 1.6e-5 (W2), 2.6e-5 (Wg) for omega = 0
    # the smoothed loss is a different function of the weights
    if omega > 0.0:
        assert abs(lo - cnn.loss_only(st, b, p, _layers(w), bf16=True)) > 1e-3
    net.close()
    s.close()


def test_train_step_is_adam_on_the_gradient():
    g, st, s, b, p = _geometry_case(6, 32)
    w0 = inputs.cnn_init_weights(4, scale=3.0)
    net = ibm.Network(g.ncell, w0)
    bt, pt = torch.from_numpy(b).cuda(), torch.from_numpy(p).cuda()
    dw = torch.empty(ibm.CNN_NWEIGHTS, dtype=torch.float32, device="cuda")
    print("case cnn adam", flush=True)
    l0 = net.loss(s, bt, pt, dw)
    lr = 1e-3
    l1 = net.train_step(s, bt, pt, lr)
    assert l1 == l0          # the step reports the loss before its update (same kernels)
    gr = dw.cpu().numpy().astype(np.float64)
    wexp, _, _ = cnn.adam(w0.astype(np.float64), gr, np.zeros_like(gr), np.zeros_like(gr), 1, lr)
    w1 = net.weights.astype(np.float64)
    assert np.max(np.abs(w1 - wexp)) <= 1e-6 * lr + 1e-7 * np.max(np.abs(w0))
    net.close()
    s.close()


def test_preconditioner_matches_oracle():
    g, st, s, b, p = _geometry_case(7, 40)
    w = inputs.cnn_init_weights(8, scale=3.0)
    net = ibm.Network(g.ncell, w)
    r = np.random.default_rng(9).standard_normal(g.shape).astype(np.float32)
    z = torch.empty(g.shape, dtype=torch.float32, device="cuda")
    print("case cnn precondition", flush=True)
    ibm.ibm_cnn_precondition(net.net, s.ctx, torch.from_numpy(r).cuda(), z)
    zo = cnn.precondition(st, r.astype(np.float64), _layers(w), bf16=True)
    e = rel_l2(z.cpu().numpy(), zo)
    print("preconditioner rel L2 %.2e" % e, flush=True)
    assert e < 8e-5          # measured 2.7e-5
    net.close()
    s.close()


def test_preconditioner_matches_oracle_ragged_rows():
    """The solver's marching launch on a grid whose ny is not a multiple of the 8-row
    tile (40 x 37 x 24): the partial row tile at the +y edge goes through the guarded
    loads and stores of the combine epilogue."""
    n = (40, 37, 24)
    rng = np.random.default_rng(31)
    tri = inputs.icosphere(2, 7.0, (19.6, 18.3, 11.7), inputs.random_rotation(rng))
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), (1, 2, 3, 3, 3, 3), (1.0, 0.0, 0.0))
    ob, ot = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, ob, ot)
    s = ibm.Solver(g.n, g.dx, g.origin, g.bc, g.u_in, ibm.MIXED)
    s.build(torch.from_numpy(ob).cuda(), torch.from_numpy(ot).cuda())
    w = inputs.cnn_init_weights(32, scale=3.0)
    net = ibm.Network(g.ncell, w)
    r = rng.standard_normal(g.shape).astype(np.float32)
    z = torch.empty(g.shape, dtype=torch.float32, device="cuda")
    print("case cnn precondition ragged rows", n, flush=True)
    ibm.ibm_cnn_precondition(net.net, s.ctx, torch.from_numpy(r).cuda(), z)
    zo = cnn.precondition(st, r.astype(np.float64), _layers(w), bf16=True)
    zg = z.cpu().numpy()
    e = rel_l2(zg, zo)
    e_edge = rel_l2(zg[:, 32:, :], zo[:, 32:, :])
    print("preconditioner rel L2 %.2e (rows 32-36: %.2e)" % (e, e_edge), flush=True)
    assert e < 1.4e-4 and e_edge < 1.4e-4    # measured 4.6e-5, 4.6e-5
    net.close()
    s.close()


OMEGA = 6.0 / 7.0   # the damped Jacobi weight of the smoothed form


@pytest.mark.parametrize("bc", ["walls", "periodic"])
def test_smoothed_preconditioner_matches_oracle(bc):
    """The two-level form z1 = S r, z2 = z1 + M(r - A z1), z = z2 + S(r - A z2),
    S = omega D^-1: the FP32 pre- and post-smoothing passes around the network's
    marching kernels against the oracle (the network in BF16 as above, the smoothing in
    FP64) on a 40 x 37 x 24 grid (ragged row tiles) with an immersed sphere, once with
    inflow, outflow and slip faces and once periodic in every direction (the passes'
    wrapped neighbours).  The smoothing passes add FP32 rounding of about 1e-7
    relative to the network's BF16 flips."""
    n = (40, 37, 24)
    rng = np.random.default_rng(33)
    tri = inputs.icosphere(2, 7.0, (19.6, 18.3, 11.7), inputs.random_rotation(rng))
    faces = (1, 2, 3, 3, 3, 3) if bc == "walls" else (0,) * 6
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), faces, (1.0, 0.0, 0.0))
    ob, ot = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, ob, ot)
    s = ibm.Solver(g.n, g.dx, g.origin, g.bc, g.u_in, ibm.MIXED)
    s.build(torch.from_numpy(ob).cuda(), torch.from_numpy(ot).cuda())
    w = inputs.cnn_init_weights(34, scale=3.0)
    net = ibm.Network(g.ncell, w)
    r = rng.standard_normal(g.shape).astype(np.float32)
    z = torch.empty(g.shape, dtype=torch.float32, device="cuda")
    print("case cnn smoothed precondition", bc, n, flush=True)
    ibm.ibm_cnn_precondition(net.net, s.ctx, torch.from_numpy(r).cuda(), z, OMEGA)
    zo = cnn.precondition(st, r.astype(np.float64), _layers(w), bf16=True, omega=OMEGA)
    zg = z.cpu().numpy()
    e = rel_l2(zg, zo)
    e_edge = rel_l2(zg[:, 32:, :], zo[:, 32:, :])
    print("smoothed preconditioner rel L2 %.2e (rows 32-36: %.2e)" % (e, e_edge), flush=True)
    assert np.all(np.isfinite(zg))
    assert e < 1.4e-4 and e_edge < 1.4e-4    # measured 5.2e-5 / 3.3e-5 (walls), 4.4e-5 / 3.1e-5 (periodic)
    # the smoothing changes the map: the unsmoothed one is far from it
    assert rel_l2(cnn.precondition(st, r.astype(np.float64), _layers(w), bf16=True), zo) > 1e-2
    net.close()
    s.close()


def test_smoothed_preconditioner_argument_errors():
    """The smoothed form needs nx % 4 == 0 and omega in (0, 1]."""
    g, st, s, b, p = _geometry_case(3, 32)
    net = ibm.Network(g.ncell, inputs.cnn_init_weights(1, scale=3.0))
    r = torch.ones(g.shape, dtype=torch.float32, device="cuda")
    z = torch.empty_like(r)
    print("case cnn smoothed argument errors", flush=True)
    for om in (-0.5, 1.5, float("nan")):
        with pytest.raises(ibm.IBMError):
            ibm.ibm_cnn_precondition(net.net, s.ctx, r, z, om)
    net.attach(s)
    x = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ibm.IBMError):
        s.poisson(torch.from_numpy(b).cuda(), x, tol=1e-6, kind=ibm.SOLVER_FCG_CNN, omega=1.5)
    net.close()
    s.close()
    n = RAGGED
    gr = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), (1, 2, 3, 3, 3, 3), (1.0, 0.0, 0.0))
    sr = ibm.Solver(gr.n, gr.dx, gr.origin, gr.bc, gr.u_in, ibm.MIXED)
    zeros = torch.zeros((n[2], n[1], n[0]), dtype=torch.uint8, device="cuda")
    sr.build(zeros, torch.full((n[2], n[1], n[0], 6), 2.0, dtype=torch.float64, device="cuda"))
    netr = ibm.Network(gr.ncell, inputs.cnn_init_weights(1, scale=3.0))
    rr = torch.ones((n[2], n[1], n[0]), dtype=torch.float32, device="cuda")
    with pytest.raises(ibm.IBMError):
        ibm.ibm_cnn_precondition(netr.net, sr.ctx, rr, torch.empty_like(rr), OMEGA)
    netr.close()
    sr.close()


@pytest.mark.parametrize("how", ["force_stall", "nan_weights"])
def test_fcg_cnn_falls_back_to_fp64(how):
    """A learned solve that stalls (the test hook) or whose network gives non-finite
    values (NaN weights) hands the solve to FP64 Jacobi PCG from the current x: the
    fallback is reported, x is finite and the FP64 residual meets the tolerance."""
    g, st, s, b, p = _geometry_case(3, 32)
    w = inputs.cnn_init_weights(1, scale=3.0)
    if how == "nan_weights":
        w = np.full_like(w, np.nan)
    net = ibm.Network(g.ncell, w)
    net.attach(s)
    x = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    print("case fcg cnn fallback", how, flush=True)
    rc, stats = s.poisson(torch.from_numpy(b).cuda(), x, tol=1e-10, max_iter=20000, kind=ibm.SOLVER_FCG_CNN,
                          inner_tol=0.1, inner_max_iter=500, force_stall=1 if how == "force_stall" else 0)
    print("  %s" % stats, flush=True)
    assert rc == 0 and stats["fallback_used"] == 1
    assert bool(torch.isfinite(x).all())
    assert stats["rel_residual"] <= 1e-10 * 1.0001
    net.close()
    s.close()


@pytest.mark.parametrize("omega", [0.0, OMEGA])
def test_fcg_cnn_solve_reaches_fp64_tolerance(omega):
    """The learned solve, without and with the smoothing steps, reaches the FP64
    tolerance and the dense solution."""
    g, st, s, b, p = _geometry_case(3, 48)
    net = ibm.Network(g.ncell, inputs.cnn_init_weights(1, scale=3.0))
    net.attach(s)
    bt = torch.from_numpy(b).cuda()
    print("case fcg cnn solve omega", omega, flush=True)
    for tol in (1e-6, 1e-10):
        x = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
        rc, stats = s.poisson(bt, x, tol=tol, max_iter=20000, kind=ibm.SOLVER_FCG_CNN, inner_tol=0.1,
                              inner_max_iter=500, omega=omega)
        print("tol %g: %s" % (tol, stats), flush=True)
        assert rc == 0 and stats["rel_residual"] <= tol * 1.0001
        assert stats["fallback_used"] == 0
    assert rel_l2(x.cpu().numpy(), p) < 1e-7
    net.close()
    s.close()


def test_steps_allocate_nothing():
    """ibm_step allocates nothing after set-up: the library's allocation count stays the
    same across learned (the network's map alone and between the smoothing steps),
    mixed-Jacobi and Crank-Nicolson steps, with and without the extrapolated pressure
    guess, once the network is attached and the Crank-Nicolson workspace prepared."""
    case = inputs.case_ellipsoid_window(103, 32)
    s = ibm.Solver(case.n, case.dx, case.origin, case.bc, case.u_in, ibm.MIXED)
    gb, _ = s.tag(case.tri, want_theta=False)
    s.build(gb)
    net = ibm.Network(int(np.prod(case.n)), inputs.cnn_init_weights(1, scale=3.0), inference_only=True)
    net.attach(s)
    s.prepare_crank_nicolson()
    st = s.new_state(case.u_in)
    p_prev = st["p"].clone()
    torch.cuda.synchronize()
    a0 = ibm.alloc_count()
    print("case steps allocate nothing", case.n, flush=True)
    kinds = [(ibm.SOLVER_FCG_CNN, "ab2"), (ibm.SOLVER_FCG_CNN, "ab2"), (ibm.SOLVER_FCG_JACOBI, "ab2"),
             (ibm.SOLVER_FCG_CNN, "cn")]
    for k, (kind, scheme) in enumerate(kinds):
        # the last two steps start their pressure solves from the extrapolated guess
        rc, stats = s.step(st, ibm.step_params(0.2, case.nu, step=k, dt_prev=0.2 if k else 0.0, tol=1e-6,
                                               kind=kind, inner_tol=1e-3, inner_max_iter=500, scheme=scheme,
                                               mom_tol=1e-6, p_prev=p_prev if k >= 2 else None,
                                               omega=OMEGA if k in (1, 3) else 0.0))
        assert rc == 0 and stats["fallback_used"] == 0
    torch.cuda.synchronize()
    assert ibm.alloc_count() == a0
    net.close()
    s.close()


def test_fcg_cnn_without_network_is_an_error():
    g, st, s, b, p = _geometry_case(3, 32)
    x = torch.zeros(g.shape, dtype=torch.float64, device="cuda")
    with pytest.raises(ibm.IBMError):
        s.poisson(torch.from_numpy(b).cuda(), x, tol=1e-6, kind=ibm.SOLVER_FCG_CNN)
    s.close()


def test_training_pairs_at_krylov_depth_solve_the_pressure_equation():
    """A training pair taken at Krylov depth k is (b - L x_k, p - x_k) with x_k the k-th
    Jacobi-PCG iterate from zero: it must satisfy L p' = b' to the accuracy of the
    step's solve (tol 1e-8 relative) like a depth-0 pair, and differ from the step's
    right-hand side."""
    from paper_2002_06206_amd import train
    print("case cnn depth pairs", flush=True)
    case = inputs.case_ellipsoid_window(101, 32)
    s0, p0 = train.generate_pairs(case, steps=6, every=1, first=2, depths=(0,))
    s1, p1 = train.generate_pairs(case, steps=6, every=1, first=2, depths=(0, 8))
    s2, p2 = train.generate_pairs(case, steps=6, every=1, first=2, depths=(0, -2))
    assert len(p0) == len(p1) == len(p2) == 4
    for s, pairs in ((s0, p0), (s1, p1), (s2, p2)):
        for b, p in pairs:
            e = float(torch.linalg.vector_norm(s.laplacian(p) - b) / torch.linalg.vector_norm(b))
            assert e < 1e-6, e
    # depth 0 pairs agree (same steps); depth 8 pairs carry the residual after 8 iterates
    assert torch.equal(p0[0][0], p1[0][0]) and torch.equal(p0[2][0], p1[2][0])
    r = float(torch.linalg.vector_norm(p1[1][0]) / torch.linalg.vector_norm(p0[1][0]))
    print("depth-8 residual / right-hand side %.3f" % r, flush=True)
    assert 0.0 < r < 1.0
    # after one damped Jacobi step: b' = b - L x with x = (6/7) b / diag(L)
    assert torch.equal(p0[0][0], p2[0][0])
    x = torch.where(train.laplacian_diagonal(s2) < 0.0, (6.0 / 7.0) * p0[1][0] / train.laplacian_diagonal(s2),
                    torch.zeros_like(p0[1][0]))
    e = float(torch.linalg.vector_norm(p2[1][0] - (p0[1][0] - s2.laplacian(x))) / torch.linalg.vector_norm(p0[1][0]))
    print("damped-Jacobi pair: residual mismatch %.1e" % e, flush=True)
    assert e < 1e-14
    s0.close()
    s1.close()
    s2.close()


@pytest.mark.parametrize("n", [(7, 9, 10), (25, 31, 6)])
def test_laplacian_diagonal_probe_matches_oracle(n):
    """The colouring probe of the operator's diagonal (training pairs after a damped
    Jacobi step) equals -diag(A) of the oracle exactly, with periodic x and y axes
    whose lengths defeat a fixed colouring (7 and 31 are 1 mod 2 and mod 3, 25 is 1 mod
    2, 3 and 4), an inflow and an outlet face in z and an immersed sphere."""
    from paper_2002_06206_amd import train
    rng = np.random.default_rng(51)
    tri = inputs.icosphere(2, 2.0, (n[0] / 2 + 0.1, n[1] / 2 + 0.2, n[2] / 2 + 0.3), inputs.random_rotation(rng))
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), (0, 0, 0, 0, 1, 2), (0.0, 0.0, 1.0))
    ob, ot = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, ob, ot)
    s = ibm.Solver(g.n, g.dx, g.origin, g.bc, g.u_in, ibm.FP64)
    s.build(torch.from_numpy(ob).cuda(), torch.from_numpy(ot).cuda())
    print("case laplacian diagonal probe", n, flush=True)
    d = train.laplacian_diagonal(s).cpu().numpy()
    np.testing.assert_array_equal(d, -flow.jacobi_diag(st))
    s.close()


def test_trained_preconditioner_gains_over_jacobi():
    """What the trained network gains: it is trained on the GPU (library kernels, Adam) on
    (b, p) pairs of the plain FP64 solver from seeded 48^3 windows of the ellipsoid field
    and evaluated on pairs of a held-out seed.  Held-out loss and the iterations of the
    mixed solve to 1e-6 from a zero guess are printed for FCG with the trained network
    and for the method without it (mixed Jacobi CG)."""
    from paper_2002_06206_amd import train
    n = 48
    print("case cnn gain: building pairs", flush=True)
    data = train.build_dataset(train.TRAIN_SEEDS[:3], n, steps=18, every=3)
    held = train.build_dataset(train.EVAL_SEEDS[:1], n, steps=18, every=3)
    net = ibm.Network(n ** 3, inputs.cnn_init_weights(0))
    l0 = train.mean_loss(net, held)
    train.train(net, data, 400, 2e-3)
    l1 = train.mean_loss(net, held)
    print("held-out loss %.4f -> %.4f" % (l0, l1), flush=True)
    s, pairs = held[0]
    it_j, it_c, it_s, t_j, t_c = [], [], [], 0.0, 0.0
    for b, p in pairs:
        st, t = train.solve_iterations(s, b, ibm.SOLVER_FCG_JACOBI, tol=1e-6, inner_tol=0.1, inner_max_iter=2000)
        assert st["status"] == 0 and st["fallback_used"] == 0
        it_j.append(st["iters_inner"])
        t_j += t
        net.attach(s)
        st, t = train.solve_iterations(s, b, ibm.SOLVER_FCG_CNN, tol=1e-6, inner_tol=0.1, inner_max_iter=2000)
        assert st["status"] == 0 and st["fallback_used"] == 0 and st["rel_residual"] <= 1e-6 * 1.0001
        it_c.append(st["iters_inner"])
        t_c += t
        st, _ = train.solve_iterations(s, b, ibm.SOLVER_FCG_CNN, tol=1e-6, inner_tol=0.1, inner_max_iter=2000,
                                       omega=OMEGA)
        assert st["status"] == 0 and st["fallback_used"] == 0 and st["rel_residual"] <= 1e-6 * 1.0001
        it_s.append(st["iters_inner"])
    print("held-out solves to 1e-6: Jacobi CG %s iterations (%.1f ms), trained FCG %s iterations (%.1f ms), "
          "with the smoothing steps %s" % (it_j, 1e3 * t_j, it_c, 1e3 * t_c, it_s), flush=True)
    assert l1 < 0.8 * l0
    assert np.mean(it_c) < 0.6 * np.mean(it_j)
    assert np.mean(it_s) < np.mean(it_c)
    net.close()
    for s_, _ in data + held:
        s_.close()
