"""CPU checks of the training driver's host logic (paper_2002_06206_amd/train.py) with
the oracle's operator standing in for the library's: the colouring probe of the
pressure operator's diagonal equals the oracle's Jacobi diagonal on grids whose
periodic lengths defeat a fixed colouring."""
import numpy as np
import pytest
import torch

from oracle import flow, tagging
from paper_2002_06206_amd import inputs, train


class _OracleSolver:
    """The two members laplacian_diagonal reads, with the oracle's operator on CPU tensors."""

    def __init__(self, st):
        self.st = st
        g = st.grid
        self.shape = g.shape
        self.dev = torch.device("cpu")
        self.calls = 0

    def laplacian(self, x):
        self.calls += 1
        return torch.from_numpy(flow.laplacian(self.st, x.numpy()))


@pytest.mark.parametrize("n, faces", [((7, 9, 10), (0, 0, 0, 0, 1, 2)), ((25, 31, 6), (0, 0, 0, 0, 1, 2)),
                                      ((12, 10, 8), (1, 2, 3, 3, 3, 3)), ((13, 16, 5), (0, 0, 3, 3, 0, 0))])
def test_laplacian_diagonal_probe(n, faces):
    rng = np.random.default_rng(52)
    tri = inputs.icosphere(2, 1.8, (n[0] / 2 + 0.1, n[1] / 2 + 0.2, n[2] / 2 + 0.3), inputs.random_rotation(rng))
    g = flow.Grid(n, 1.0, (0.0, 0.0, 0.0), faces, (0.0, 0.0, 1.0) if faces[4] == 1 else (1.0, 0.0, 0.0))
    ob, ot = tagging.tag(tri, g.n, g.dx, g.origin)
    st = flow.build_stencils(g, ob, ot)
    s = _OracleSolver(st)
    d = train.laplacian_diagonal(s).numpy()
    np.testing.assert_array_equal(d, -flow.jacobi_diag(st))
    # one probe per colour: the product of the per-axis moduli
    mods = []
    for m_n in n:
        m = 2
        while m_n % m == 1:
            m += 1
        mods.append(m)
    assert s.calls == mods[0] * mods[1] * mods[2]
