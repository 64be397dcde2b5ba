"""Pins of the building-cube (BCM) grid oracle (oracle/bcm.py; Sec. 2.2): one level of
cubes reproduces the uniform-grid operator bit for bit; on two levels a constant field
stays constant across the halos with a zero operator, fine-to-coarse averages of a
linear field are exact and coarse-to-fine copies take the covering coarse cell; only
face halos are written; the listed-cube forms (used to sample large grids) equal the
full forms on the listed cubes."""
import numpy as np
import pytest

from oracle import bcm


def test_one_level_equals_the_uniform_grid():
    K, n, dx = (2, 3, 2), 4, 0.7
    C = bcm.Cubes(K, n, dx, (0.0, 0.0, 0.0), np.zeros(K[::-1], bool))
    rng = np.random.default_rng(0)
    N = (K[0] * n, K[1] * n, K[2] * n)
    u = rng.standard_normal(N[::-1])          # (z, y, x)
    data = np.zeros(C.size())
    s = C.side
    for q, (lvl, o) in enumerate(C.cubes):
        i0, j0, k0 = o // 2
        blk = data[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
        blk[bcm.H:bcm.H + n, bcm.H:bcm.H + n, bcm.H:bcm.H + n] = u[k0:k0 + n, j0:j0 + n, i0:i0 + n]
    ex = C.exchange(data)
    # every face halo (both layers) equals the uniform field padded symmetrically by two
    # cells: neighbour values inside the domain, mirrored cells 0 and 1 outside
    pad = np.pad(u, bcm.H, mode="symmetric")
    h = bcm.H
    for q, (lvl, o) in enumerate(C.cubes):
        i0, j0, k0 = o // 2
        blk = ex[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
        ref = pad[k0:k0 + n + 2 * h, j0:j0 + n + 2 * h, i0:i0 + n + 2 * h]
        for sl in ((slice(h, h + n), slice(h, h + n), slice(None)),
                   (slice(h, h + n), slice(None), slice(h, h + n)),
                   (slice(None), slice(h, h + n), slice(h, h + n))):
            assert np.array_equal(blk[sl], ref[sl])
    L = C.laplacian(ex)
    # the uniform grid with mirror (zero-gradient) boundaries, neighbours in the same order
    g = np.pad(u, 1, mode="edge")
    c = g[1:-1, 1:-1, 1:-1]
    ref = (g[1:-1, 1:-1, :-2] + g[1:-1, 1:-1, 2:] + g[1:-1, :-2, 1:-1] + g[1:-1, 2:, 1:-1] + g[:-2, 1:-1, 1:-1]
           + g[2:, 1:-1, 1:-1] - 6.0 * c) / (dx * dx)
    for q, (lvl, o) in enumerate(C.cubes):
        i0, j0, k0 = o // 2
        assert np.array_equal(C.interior(L, q), ref[k0:k0 + n, j0:j0 + n, i0:i0 + n])


def _two_level(seed=None):
    """The two-level test grid: two refined coarse cubes, or with a seed a random set of
    them (each coarse cube refined with probability 1/2)."""
    K, n, dx = (3, 2, 2), 4, 1.0
    refine = np.zeros(K[::-1], bool)
    if seed is None:
        refine[0, 0, 1] = True
        refine[1, 1, 2] = True
    else:
        refine = np.random.default_rng(seed).random(K[::-1]) < 0.5
    return bcm.Cubes(K, n, dx, (0.5, -1.0, 2.0), refine)


@pytest.mark.parametrize("seed", [None, 11, 12, 13])
def test_constant_field_on_two_levels(seed):
    C = _two_level(seed)
    assert len(C.cubes) == 3 * 2 * 2 + 7 * int(C.refine.sum())
    data = C.exchange(C.fill(lambda x, y, z: np.full_like(x, 3.25)))
    s, n, h = C.side, C.n, bcm.H
    for q in range(len(C.cubes)):
        blk = data[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
        assert np.all(blk[h:h + n, h:h + n, :] == 3.25)     # x-face halos
        assert np.all(blk[h:h + n, :, h:h + n] == 3.25)
        assert np.all(blk[:, h:h + n, h:h + n] == 3.25)
        assert blk[0, 0, 0] == 0.0                           # corners untouched
    assert np.max(np.abs(C.laplacian(data))) == 0.0


@pytest.mark.parametrize("seed", [None, 11, 12, 13])
def test_linear_field_averages_and_copies(seed):
    C = _two_level(seed)
    f = lambda x, y, z: 0.3 + 1.7 * x - 0.9 * y + 0.4 * z  # noqa: E731
    data = C.exchange(C.fill(f))
    n, h = C.n, bcm.H
    checked = {"avg": 0, "copy": 0}
    for q, (lvl, o) in enumerate(C.cubes):
        w = 1 if lvl == 1 else 2
        for axis in range(3):
            for sgn in (-1, 1):
                for layer in (1, 2):
                    c = [1, 2, 3]
                    c[axis] = n - 1 + layer if sgn > 0 else -layer
                    centre = o + (np.array(c) + 0.5) * w
                    hit = C.locate(centre)
                    if hit is None:
                        continue
                    q2, l2, cell = hit
                    v = data[C.index(q, *c)]
                    x = (centre * 0.5 * C.dx0) + C.origin
                    if lvl == 0 and l2 == 1:          # average of fine cells: exact for linear
                        assert abs(v - f(*x)) < 1e-12
                        checked["avg"] += 1
                    elif lvl == 1 and l2 == 0:        # copy of the covering coarse cell
                        cc = C.cell_centres(q2)[cell[2], cell[1], cell[0]]
                        assert v == data[C.index(q2, *cell)] and abs(v - f(*cc)) < 1e-12
                        checked["copy"] += 1
                    else:                             # same level: the neighbour's own cell
                        assert abs(v - f(*x)) < 1e-12
    mixed = 0 < C.refine.sum() < C.refine.size
    assert (checked["avg"] > 0 and checked["copy"] > 0) or not mixed
    # the operator of a linear field vanishes away from the level interfaces
    L = C.laplacian(data)
    for q, (lvl, o) in enumerate(C.cubes):
        inner = C.interior(L, q)[1:n - 1, 1:n - 1, 1:n - 1]   # clear of boundary and interface
        assert np.max(np.abs(inner)) < 1e-12


def test_rbsor_half_sweeps_and_convergence():
    # at omega = 1 a half sweep zeroes the residual of its colour (against the halos it
    # exchanged); on a consistent two-level system b = L u the iteration converges to u
    # up to the constant of the Neumann problem
    C = _two_level()
    u = C.exchange(C.fill(lambda x, y, z: np.sin(0.7 * x) + 0.3 * np.cos(0.5 * y + 0.2 * z)))
    b = C.laplacian(u)
    x0 = np.zeros(C.size())
    n = C.n
    kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    for colour in (0, 1):
        y = C.half_sweep(b, x0 + 0.1, 1.0, colour)
        r = b - C.laplacian(y)
        mine = (ii + jj + kk) % 2 == colour
        worst = max(np.max(np.abs(C.interior(r, q)[mine])) for q in range(len(C.cubes)))
        other = max(np.max(np.abs(C.interior(r, q)[~mine])) for q in range(len(C.cubes)))
        assert worst < 1e-12 * np.max(np.abs(b)) and other > 1e-3
    x = C.rbsor(b, x0, 1.6, 400)
    d = np.concatenate([(C.interior(x, q) - C.interior(u, q)).ravel() for q in range(len(C.cubes))])
    ref = np.concatenate([C.interior(u, q).ravel() for q in range(len(C.cubes))])
    assert np.std(d) < 1e-6 * np.std(ref)


def test_listed_cubes_equal_the_full_grid():
    # the listed-cube forms of the exchange, the operator and a sweep (used to sample
    # the large grid) give the full forms' values on the listed cubes: halos of a cube
    # and of the cubes its halos read from are filled before its second half sweep
    K, n = (3, 2, 2), 4
    refine = np.zeros(K[::-1], bool)
    refine[0, 1, 1] = refine[1, 0, 2] = True
    C = bcm.Cubes(K, n, 0.9, (0.0, 0.0, 0.0), refine)
    rng = np.random.default_rng(12)
    x0 = rng.standard_normal(C.size())
    b = rng.standard_normal(C.size())
    full_ex = C.exchange(x0)
    full_L = C.laplacian(full_ex)
    full_sw = C.rbsor(b, x0, 1.4, 1)
    s3 = C.side ** 3
    for q in (0, 3, len(C.cubes) - 1):
        ex = C.exchange(x0, [q])
        assert np.array_equal(ex[q * s3:(q + 1) * s3], full_ex[q * s3:(q + 1) * s3])
        assert np.array_equal(C.interior(C.laplacian(ex, [q]), q), C.interior(full_L, q))
        d1, s1, d8, s8 = C.halo_sources([q])
        src = sorted(set((np.concatenate([s1, s8.ravel()]) // s3).tolist()) | {q})
        x1 = C.half_sweep(b, x0, 1.4, 0, src)
        x2 = C.half_sweep(b, x1, 1.4, 1, [q])
        assert np.array_equal(C.interior(x2, q), C.interior(full_sw, q))
        # a cube of the list updates nothing outside its own storage
        other = np.ones(C.size(), bool)
        for r in src:
            other[r * s3:(r + 1) * s3] = False
        assert np.array_equal(x1[other], x0[other])


# ----------------------------------------------- immersed geometry on the cubes

def _scatter(C, u):
    """Cube storage holding the level-0 uniform field u (z, y, x) in every (coarse) cube."""
    data = np.zeros(C.size())
    s, n = C.side, C.n
    for q, (lvl, o) in enumerate(C.cubes):
        i0, j0, k0 = o // 2
        blk = data[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
        blk[bcm.H:bcm.H + n, bcm.H:bcm.H + n, bcm.H:bcm.H + n] = u[k0:k0 + n, j0:j0 + n, i0:i0 + n]
    return data


def _sphere(centre, radius, seed=0):
    from paper_2002_06206_amd import inputs
    return inputs.icosphere(3, radius, centre, inputs.random_rotation(np.random.default_rng(seed)))


def test_one_level_with_geometry_equals_the_uniform_pressure_operator():
    """One level of cubes carrying the blocked bits of a tagged sphere is the uniform
    grid's pressure operator with those bits and zero-gradient (slip) domain faces: the
    flow oracle's L p over open faces (Neumann ghost behind blocked faces, Sec. 2.3.2
    reading G3), to rounding (the two sum the same terms in a different order)."""
    from oracle import flow, tagging
    K, n, dx = (3, 2, 2), 8, 0.5
    N = (K[0] * n, K[1] * n, K[2] * n)
    C = bcm.Cubes(K, n, dx, (0.0, 0.0, 0.0), np.zeros(K[::-1], bool))
    tri = _sphere((6.1, 3.9, 4.2), 2.7)
    blocked, theta = tagging.tag(tri, N, dx, (0.0, 0.0, 0.0))
    assert np.count_nonzero(blocked) > 50
    C.set_blocked(0, blocked)
    S = flow.SLIP
    g = flow.Grid(N, dx, (0.0, 0.0, 0.0), (S,) * 6)
    st = flow.build_stencils(g, blocked, theta)
    u = np.random.default_rng(4).standard_normal(N[::-1])
    L = C.laplacian(C.exchange(_scatter(C, u)))
    ref = flow.laplacian(st, u)
    got = np.zeros(N[::-1])
    for q, (lvl, o) in enumerate(C.cubes):
        i0, j0, k0 = o // 2
        got[k0:k0 + n, j0:j0 + n, i0:i0 + n] = C.interior(L, q)
    assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_two_level_geometry_masks_and_sor():
    """Two levels with a sphere inside the refined cubes: every cube cell takes the bits
    of its own level's tagging (blocked faces seen from both cells within a level), and
    red-black SOR with the open-face diagonal drives the residual of a consistent system
    b = L u down on both levels; a planted mistake (the blocked neighbour's own value
    instead of the ghost) changes the operator next to the wall."""
    from oracle import tagging
    K, n, dx0 = (2, 2, 2), 8, 1.0
    refine = np.zeros(K[::-1], bool)
    refine[0, 0, 0] = refine[0, 0, 1] = True
    C = bcm.Cubes(K, n, dx0, (0.0, 0.0, 0.0), refine)
    tri = _sphere((8.0, 4.1, 3.9), 2.6, seed=2)
    for lvl in (0, 1):
        shape = C.level_shape(lvl)
        dx = C.dx(lvl)
        b, _ = tagging.tag(tri, shape[::-1], dx, (0.0, 0.0, 0.0))
        C.set_blocked(lvl, b)
        if lvl == 1:
            # within the level grid a blocked face is blocked from both sides
            assert np.count_nonzero(b) > 50
            assert np.array_equal((b >> 1) & 1, np.roll((b >> 0) & 1, -1, axis=2) * (np.arange(shape[2]) <
                                                                                    shape[2] - 1))
    fine = [q for q, (l, _) in enumerate(C.cubes) if l == 1]
    assert sum(np.count_nonzero(C.mask[q]) for q in fine) > 50
    u = C.fill(lambda x, y, z: np.sin(0.7 * x) * np.cos(0.4 * y) + 0.3 * z)
    b = C.laplacian(C.exchange(u))
    x = np.zeros_like(u)
    r0 = np.linalg.norm(b)
    x = C.rbsor(b, x, 1.7, 300)
    r = np.linalg.norm(b - C.laplacian(C.exchange(x)))
    assert r < 1e-3 * r0, (r, r0)
    # planted mistake: ignore the masks
    L_masked = C.laplacian(C.exchange(u))
    mask = C.mask
    del C.mask
    L_plain = C.laplacian(C.exchange(u))
    C.mask = mask
    assert np.max(np.abs(L_masked - L_plain)) > 1e-3


# ------------------------------------------------ the pressure solve on the cubes

def _two_level_small():
    refine = np.zeros((1, 1, 2), bool)
    refine[0, 0, 1] = True
    return bcm.Cubes((2, 1, 1), 4, 1.0, (0.0, 0.0, 0.0), refine)


def _dense(C):
    m = len(C.cubes) * C.n ** 3
    A = np.zeros((m, m))
    for k in range(m):
        e = np.zeros(m)
        e[k] = 1.0
        A[:, k] = C.apply(e)
    return A


def _off_null(A, d):
    """The part of d orthogonal to the null space of A (from its SVD)."""
    _, sv, vt = np.linalg.svd(A)
    null = vt[sv < 1e-10 * sv[0]]
    return d - null.T @ (null @ d), len(null)


def test_pack_unpack_and_the_operator_on_packed_interiors():
    """pack / unpack are inverse on the interiors, and apply is exchange-then-L whatever
    the input's halos hold (the exchange rewrites every face halo L reads)."""
    C = _two_level_small()
    data = np.random.default_rng(3).standard_normal(C.size())
    v = C.pack(data)
    assert v.shape == (len(C.cubes) * C.n ** 3,)
    assert np.array_equal(C.pack(C.unpack(v)), v)
    assert np.array_equal(C.apply(v), C.pack(C.laplacian(C.exchange(data))))
    assert np.array_equal(C.pack(C.unpack(v)), C.pack(data))


@pytest.mark.parametrize("geometry", [False, True])
def test_bicgstab_on_cubes_equals_the_dense_solve(geometry):
    """On a two-level grid (one coarse cube, one refined into 8), with and without a
    blocked slab, BiCGStab on the cubes reaches the solution of the dense system built
    from the operator, up to the null space (the constants of the all-Neumann problem,
    one per component); the all-Neumann operator annihilates constants."""
    C = _two_level_small()
    if geometry:
        for lvl in (0, 1):
            nz, ny, nx = C.level_shape(lvl)
            blk = np.zeros((nz, ny, nx), np.uint8)
            f = 1 if lvl == 0 else 2
            j = 2 * f                     # a wall between rows j - 1 and j, over part of x
            blk[:, j - 1, : 3 * nx // 4] |= 8
            blk[:, j, : 3 * nx // 4] |= 4
            C.set_blocked(lvl, blk)
    A = _dense(C)
    m = A.shape[0]
    assert np.max(np.abs(A @ np.ones(m))) < 1e-12
    u = np.random.default_rng(7).standard_normal(m)
    b = C.unpack(A @ u)
    x, it, status = C.bicgstab(b, np.zeros_like(b), 1e-12, 4000)
    assert status == "converged" and it > 5
    xs = np.linalg.lstsq(A, A @ u, rcond=None)[0]
    d, nnull = _off_null(A, C.pack(x) - xs)
    assert nnull == 1
    assert np.linalg.norm(d) <= 1e-8 * np.linalg.norm(xs)
    assert C.residual(b, x) <= 1e-12


def test_sor_solve_stops_at_the_first_check_below_tol():
    """SOR to a tolerance is plain red-black SOR stopped at the first multiple of
    check_every whose true residual is at or below tol: the same sweeps give the same
    x bit for bit, one group fewer is still above tol, and the cap is honoured."""
    C = _two_level_small()
    u = C.fill(lambda x, y, z: np.sin(0.7 * x) * np.cos(0.4 * y) + 0.3 * z)
    b = C.laplacian(C.exchange(u))
    x0 = np.zeros_like(b)
    x, sweeps, status = C.sor_solve(b, x0, 1.6, 1e-6, 10, 5000)
    assert status == "converged" and sweeps % 10 == 0 and sweeps >= 20
    assert C.residual(b, x) <= 1e-6
    assert np.array_equal(x, C.rbsor(b, x0, 1.6, sweeps))
    assert C.residual(b, C.rbsor(b, x0, 1.6, sweeps - 10)) > 1e-6
    x2, s2, st2 = C.sor_solve(b, x0, 1.6, 1e-6, 10, 25)
    assert st2 == "max_iter" and s2 == 25 and np.array_equal(x2, C.rbsor(b, x0, 1.6, 25))
    xz, sz, stz = C.sor_solve(np.zeros_like(b), x0, 1.6, 1e-6, 10, 100)
    assert stz == "converged" and sz == 0
