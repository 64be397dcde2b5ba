"""GPU parity of the building-cube grid (Sec. 2.2) against oracle/bcm.py through the C
ABI: cube order and levels equal to the oracle's, the halo exchange (copies, means of
8 fine cells, mirrors) and the 7-point operator on the cubes bit for bit, on a one-level
grid against the uniform operator, and on two levels with several refined cubes; red-black
SOR sweeps on the cubes bit for bit."""
import numpy as np
import pytest

from oracle import bcm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    from paper_2002_06206_amd import ibm
else:  # collected on CPU machines, skipped by the marker filter
    ibm = None


@pytest.mark.parametrize("K,n,cells", [((2, 3, 2), 4, ((0, 0, 1), (1, 2, 0))),
                                        ((3, 2, 2), 8, ((0, 0, 0), (1, 1, 2), (0, 1, 1))),
                                        ((2, 2, 2), 16, ())])
def test_exchange_and_operator_bit_exact(K, n, cells):
    refine = np.zeros(K[::-1], bool)
    for c in cells:
        refine[c] = True
    dx0, origin = 0.8, (0.5, -1.0, 2.0)
    print("case bcm", K, n, cells, flush=True)
    C = bcm.Cubes(K, n, dx0, origin, refine)
    G = ibm.BCM(K, n, dx0, origin, refine)
    assert G.ncubes == len(C.cubes) and G.size == C.size()
    assert np.array_equal(G.levels, [lv for lv, _ in C.cubes])
    assert np.array_equal(G.origins, np.array([o for _, o in C.cubes]))
    rng = np.random.default_rng(1)
    data = rng.standard_normal(C.size())
    ref = C.exchange(data)
    d = torch.from_numpy(data.copy()).cuda()
    G.exchange(d)
    got = d.cpu().numpy()
    assert np.array_equal(got, ref)
    y = torch.zeros_like(d)
    G.laplacian(d, y)
    L = C.laplacian(ref)
    for q in range(len(C.cubes)):
        assert np.array_equal(C.interior(y.cpu().numpy(), q), C.interior(L, q))
    G.close()


@pytest.mark.parametrize("K,n,cells", [((3, 2, 2), 4, ((0, 0, 1), (1, 1, 2))), ((2, 2, 1), 8, ((0, 1, 1),))])
def test_sor_sweeps_bit_exact(K, n, cells):
    refine = np.zeros(K[::-1], bool)
    for c in cells:
        refine[c] = True
    print("case bcm sor", K, n, cells, flush=True)
    C = bcm.Cubes(K, n, 1.0, (0.0, 0.0, 0.0), refine)
    G = ibm.BCM(K, n, 1.0, (0.0, 0.0, 0.0), refine)
    rng = np.random.default_rng(6)
    b = rng.standard_normal(C.size())
    x0 = rng.standard_normal(C.size())
    ref = C.rbsor(b, x0, 1.5, 3)
    x = torch.from_numpy(x0.copy()).cuda()
    G.sor(torch.from_numpy(b).cuda(), x, 1.5, 3)
    got = x.cpu().numpy()
    for q in range(len(C.cubes)):
        assert np.array_equal(C.interior(got, q), C.interior(ref, q))
    G.close()


def test_bad_arguments_rejected():
    with pytest.raises(ibm.IBMError):
        ibm.BCM((2, 2, 2), 5, 1.0, (0, 0, 0), np.zeros((2, 2, 2), bool))      # odd n
    with pytest.raises(ibm.IBMError):
        ibm.BCM((0, 2, 2), 4, 1.0, (0, 0, 0), np.zeros((2, 2, 0), bool))


def test_geometry_operator_and_sor_bit_exact():
    """Immersed geometry on two levels (a sphere across refined and coarse cubes): each
    level's blocked bits come from tagging that level's uniform grid (the oracle's
    tagger, the same bits the GPU tagging gives bit for bit); the masked operator and red-
    black SOR sweeps with the open-face diagonal bit-exact against the oracle."""
    from oracle import tagging
    from paper_2002_06206_amd import inputs
    K, n, dx0 = (3, 2, 2), 8, 1.0
    refine = np.zeros(K[::-1], bool)
    refine[0, 0, 1] = refine[0, 1, 1] = refine[1, 0, 1] = True
    C = bcm.Cubes(K, n, dx0, (0.0, 0.0, 0.0), refine)
    G = ibm.BCM(K, n, dx0, (0.0, 0.0, 0.0), refine)
    tri = inputs.icosphere(3, 3.3, (14.5, 7.7, 4.1), inputs.random_rotation(np.random.default_rng(3)))
    print("case bcm geometry", K, n, flush=True)
    for lvl in (0, 1):
        shape = C.level_shape(lvl)
        b, _ = tagging.tag(tri, shape[::-1], C.dx(lvl), (0.0, 0.0, 0.0))
        assert np.count_nonzero(b) > 20
        C.set_blocked(lvl, b)
        G.set_blocked(lvl, torch.from_numpy(np.ascontiguousarray(b)).cuda())
    assert sum(np.count_nonzero(C.mask[q]) for q in range(len(C.cubes)) if C.cubes[q][0] == 0) > 0
    assert sum(np.count_nonzero(C.mask[q]) for q in range(len(C.cubes)) if C.cubes[q][0] == 1) > 0
    rng = np.random.default_rng(8)
    data = rng.standard_normal(C.size())
    ref = C.exchange(data)
    d = torch.from_numpy(data.copy()).cuda()
    G.exchange(d)
    y = torch.zeros_like(d)
    G.laplacian(d, y)
    L = C.laplacian(ref)
    yg = y.cpu().numpy()
    for q in range(len(C.cubes)):
        assert np.array_equal(C.interior(yg, q), C.interior(L, q))
    b = rng.standard_normal(C.size())
    x0 = rng.standard_normal(C.size())
    refx = C.rbsor(b, x0, 1.6, 3)
    x = torch.from_numpy(x0.copy()).cuda()
    G.sor(torch.from_numpy(b).cuda(), x, 1.6, 3)
    got = x.cpu().numpy()
    for q in range(len(C.cubes)):
        assert np.array_equal(C.interior(got, q), C.interior(refx, q))
    G.close()
