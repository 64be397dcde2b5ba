"""Oracle: plain FP64 CPU implementation of the immersed-boundary time step.

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
CPU-baseline leg of the benchmark; never by the product path.

Everything here is whole-array numpy in float64 with no blocking, fusion or
reordering beyond the definitions below.  Arrays are indexed [k, j, i]
(z, y, x), so the flat index is c = i + nx*(j + ny*k).  Directions are
numbered 0..5 = -x, +x, -y, +y, -z, +z (axis = dir // 2, sign = +1 for odd).

Paper passages followed (Onishi & Tsubokura, arXiv:2002.06206):
  * fractional step, face velocity, Poisson for the face divergence:
    Sec. 2.1, eq. (crank-nicolson) / (correction) / (poisson), Rhie-Chow;
    explicit Adams-Bashforth (the paper's own verification scheme, Sec. 2.4;
    AB "represents the same system", Sec. 2.1), and the Crank-Nicolson
    advection-diffusion predictor of eq. (crank-nicolson) solved by BiCGStab
    (Sec. 2.1) as the alternative scheme;
  * eddy viscosity and the coherent structure model: Sec. 2.3 (turbulence
    model), eqs. (Smagorinsky), (Q), (FCS), C1 = 1/20;
  * dummy cells, ghosts behind a grid-line crossing: Sec. 2.3.1;
  * axis-projected ghost value: Sec. 2.3.2, eq. (q_axis);
  * Dirichlet/Neumann ghost convention (zeta, eta): Sec. 2.3.2, eq. (Mittal);
  * dead-end filter: Sec. 3 (full vehicle), eq. (deadend_filter);
  * drag normalisation: eqs. (cd_sphere), (cd_flat_plate).
Readings taken where the paper is silent are named in comments (G1 ...).
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

PERIODIC, INFLOW, OUTFLOW, SLIP = 0, 1, 2, 3
FLUID, INC, ADJ = 0, 1, 2
# numpy axis of each grid axis k (x, y, z)
NPAX = (2, 1, 0)


@dataclasses.dataclass(frozen=True)
class Grid:
    n: tuple          # (nx, ny, nz)
    dx: float
    origin: tuple
    bc: tuple         # six kinds, order -x,+x,-y,+y,-z,+z
    u_in: tuple = (0.0, 0.0, 0.0)

    @property
    def shape(self):
        return (self.n[2], self.n[1], self.n[0])

    @property
    def ncell(self):
        return self.n[0] * self.n[1] * self.n[2]

    def periodic(self, k):
        return self.bc[2 * k] == PERIODIC


def _index_grid(g: Grid):
    kk, jj, ii = np.meshgrid(np.arange(g.n[2]), np.arange(g.n[1]), np.arange(g.n[0]), indexing="ij")
    return (ii, jj, kk)


@functools.lru_cache(maxsize=64)
def boundary_mask(g: Grid, d: int) -> np.ndarray:
    """(Cached; callers never modify the returned array.)  True where the face of each cell in direction d is a non-periodic domain face."""
    k, s = d // 2, (1 if d % 2 else -1)
    idx = _index_grid(g)[k]
    m = (idx == (g.n[k] - 1)) if s > 0 else (idx == 0)
    if g.periodic(k):
        return np.zeros(g.shape, dtype=bool)
    return m


def shifted(a: np.ndarray, k: int, s: int) -> np.ndarray:
    """Value of `a` at c + s*e_k, wrapping around (callers mask domain faces)."""
    return np.roll(a, -s, axis=NPAX[k])


# ------------------------------------------------------------------ stencils

@dataclasses.dataclass
class Stencil:
    grid: Grid
    blocked: np.ndarray       # uint8 (nz,ny,nx), effective blocked bits
    theta: np.ndarray         # (nz,ny,nx,6), 2.0 where open
    flags: np.ndarray         # uint16
    label: np.ndarray         # int32, minimum flat index of the component
    enclosed: np.ndarray      # bool per cell
    deadend: np.ndarray       # bool per cell
    cut_cell: np.ndarray      # flat cell index per cut (ordered by cell, then dir)
    cut_dir: np.ndarray
    cut_theta: np.ndarray
    a_ib: np.ndarray          # ghost = a_ib*q_IB + a_c*q_c + a_o*q_o  (eq. q_axis)
    a_c: np.ndarray
    a_o: np.ndarray
    cut_opp: np.ndarray       # flat index of the opposite neighbour, -1 when unused
    comps: list               # flat cell-index arrays of the enclosed components
    cache: dict = dataclasses.field(default_factory=dict)

    @property
    def ncut(self):
        return len(self.cut_cell)


def deadend_filter(g: Grid, blocked: np.ndarray, theta: np.ndarray):
    """Eq. (deadend_filter): a cell whose six axial neighbours are cut off in five
    or more directions has its IB forcing cancelled.  Reading R12: such a cell is
    closed on all six faces (theta 0 on its new cuts) and frozen at the wall
    velocity; each neighbour that saw it through an open face now sees a wall at
    its centre (theta 1).  One pass, decided on the unfiltered bits; when two
    contributions meet on one (cell, dir) the smaller theta is kept."""
    b = blocked.copy()
    th = theta.copy()
    cnt = np.zeros(g.shape, dtype=np.int32)
    for d in range(6):
        cnt += (blocked >> d) & 1
    dead = cnt >= 5
    for d in range(6):
        k, s = d // 2, (1 if d % 2 else -1)
        od = d ^ 1
        new = dead & (((blocked >> d) & 1) == 0) & ~boundary_mask(g, d)
        b[new] |= np.uint8(1 << d)
        th[..., d] = np.where(new, np.minimum(th[..., d], 0.0), th[..., d])
        # neighbour across d sees the dead-end centre as a wall at theta = 1
        nb_new = shifted(new, k, -s)   # cell c' = c + s e_k receives from c
        b[nb_new] |= np.uint8(1 << od)
        th[..., od] = np.where(nb_new, np.minimum(th[..., od], 1.0), th[..., od])
    return b, th, dead


def build_stencils(g: Grid, blocked: np.ndarray, theta: np.ndarray, deadend: bool = False) -> Stencil:
    """Stencil build: classes (Sec. 2.3.1, eq. dummy_cell_region), the axis-projected
    ghost coefficients of eq. (q_axis), dead-end filter, and the connectivity of
    the pressure problem (components over open faces)."""
    blocked = np.asarray(blocked, dtype=np.uint8).reshape(g.shape)
    theta = np.asarray(theta, dtype=np.float64).reshape(g.shape + (6,))
    if deadend:
        blocked, theta, dead = deadend_filter(g, blocked, theta)
    else:
        dead = np.zeros(g.shape, dtype=bool)

    bit = [((blocked >> d) & 1).astype(bool) for d in range(6)]
    # wall-including cells: the wall lies within the cell's own axial extent
    inc = np.zeros(g.shape, dtype=bool)
    for d in range(6):
        inc |= bit[d] & (theta[..., d] <= 0.5)
    adj = np.zeros(g.shape, dtype=bool)
    for d in range(6):
        k, s = d // 2, (1 if d % 2 else -1)
        adj |= shifted(inc, k, s) & ~boundary_mask(g, d)
    adj &= ~inc
    cls = np.where(inc, INC, np.where(adj, ADJ, FLUID)).astype(np.uint16)
    near = np.zeros(g.shape, dtype=np.uint16)
    for d in range(6):
        near |= ((bit[d] & (theta[..., d] < 0.5)).astype(np.uint16) << d)

    # connectivity over open faces (periodic wraps included)
    N = g.ncell
    flat = np.arange(N).reshape(g.shape)
    rows, cols = [], []
    outlet = np.zeros(g.shape, dtype=bool)
    for d in (1, 3, 5):
        k = d // 2
        open_ = ~bit[d] & ~boundary_mask(g, d)
        rows.append(flat[open_])
        cols.append(shifted(flat, k, +1)[open_])
    for d in range(6):
        if g.bc[d] == OUTFLOW:
            outlet |= boundary_mask(g, d)
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    adjm = sp.coo_matrix((np.ones(len(r)), (r, c)), shape=(N, N)).tocsr()
    ncomp, comp = connected_components(adjm, directed=False)
    minidx = np.full(ncomp, N, dtype=np.int64)
    np.minimum.at(minidx, comp, np.arange(N))
    label = minidx[comp].astype(np.int32).reshape(g.shape)
    has_out = np.zeros(ncomp, dtype=bool)
    has_out[comp[outlet.ravel()]] = True
    enclosed = ~has_out[comp].reshape(g.shape)
    enc_cells = np.flatnonzero(enclosed.ravel())
    ec = comp[enc_cells]
    order = np.argsort(ec, kind="stable")
    enc_cells, ec = enc_cells[order], ec[order]
    cuts_at = np.flatnonzero(np.diff(ec)) + 1
    comps = [a for a in np.split(enc_cells, cuts_at) if len(a)]

    flags = (blocked.astype(np.uint16) | (cls << 6) | (near << 8)
             | (dead.astype(np.uint16) << 14) | (enclosed.astype(np.uint16) << 15))

    # cut list, ordered by (cell, dir)
    bflat = blocked.ravel()
    cells, dirs = [], []
    for d in range(6):
        cc = np.flatnonzero((bflat >> d) & 1)
        cells.append(cc)
        dirs.append(np.full(len(cc), d, dtype=np.int64))
    cells = np.concatenate(cells)
    dirs = np.concatenate(dirs)
    order = np.lexsort((dirs, cells))
    cells, dirs = cells[order], dirs[order]
    th = theta.reshape(-1, 6)[cells, dirs]
    od = dirs ^ 1
    bm_all = np.stack([boundary_mask(g, d).ravel() for d in range(6)], axis=1)
    opp_blocked = ((bflat[cells] >> od) & 1) == 1
    opp_boundary = bm_all[cells, od]
    br1 = th >= 0.5
    g1 = ~br1 & (opp_blocked | opp_boundary)
    br2 = ~br1 & ~g1
    safe = np.where(br1, th, 1.0)
    # eq. (q_axis), first branch (theta >= 0.5): extrapolation through q_c and the
    # wall value; Reading G2: theta = 1 is included and gives q_GC = q_IB.
    # eq. (q_axis), second branch (theta < 0.5): sign-inverted linear interpolation
    # at the image point between the opposite neighbour and the cell.
    # Reading G1: when there is no fluid neighbour behind the cell (opposite face
    # blocked: sub-cell channel; or a domain face) the image point falls back onto
    # the cell centre, q_GC = 2 q_IB - q_c.
    a_ib = np.where(br1, 1.0 / safe, 2.0)
    a_c = np.where(br1, (safe - 1.0) / safe, np.where(g1, -1.0, -2.0 * th))
    a_o = np.where(br2, 2.0 * th - 1.0, 0.0)
    ci = cells % g.n[0]
    cj = (cells // g.n[0]) % g.n[1]
    ck = cells // (g.n[0] * g.n[1])
    coord = np.stack([ci, cj, ck], axis=1)
    ax = dirs // 2
    sgn = np.where(dirs % 2 == 1, 1, -1)
    oc = coord.copy()
    nn = np.array(g.n)
    oc[np.arange(len(ax)), ax] = (oc[np.arange(len(ax)), ax] - sgn) % nn[ax]
    opp_idx = oc[:, 0] + g.n[0] * (oc[:, 1] + g.n[1] * oc[:, 2])
    opp = np.where(br2, opp_idx, -1).astype(np.int64)
    return Stencil(g, blocked, theta, flags, label, enclosed, dead, cells, dirs, th,
                   a_ib, a_c, a_o, opp, comps)


def cut_points(st: Stencil) -> np.ndarray:
    """Crossing point X of every cut: the cell centre moved by theta*dx along the cut."""
    g = st.grid
    i = st.cut_cell % g.n[0]
    j = (st.cut_cell // g.n[0]) % g.n[1]
    k = st.cut_cell // (g.n[0] * g.n[1])
    X = np.stack([g.origin[0] + (i + 0.5) * g.dx,
                  g.origin[1] + (j + 0.5) * g.dx,
                  g.origin[2] + (k + 0.5) * g.dx], axis=1)
    ax = st.cut_dir // 2
    s = np.where(st.cut_dir % 2 == 1, 1.0, -1.0)
    X[np.arange(len(ax)), ax] += s * st.cut_theta * g.dx
    return X


# -------------------------------------------------------- neighbour values

def bc_ghost(g: Grid, q: np.ndarray, m: int, d: int) -> np.ndarray:
    """Ghost value of velocity component m behind domain face d (Reading R10):
    inflow: Dirichlet u_in on the face; outflow: zero gradient;
    slip: zero normal component, zero-gradient tangential components."""
    kind = g.bc[d]
    k = d // 2
    if kind == INFLOW:
        return 2.0 * g.u_in[m] - q
    if kind == SLIP and m == k:
        return -q
    return q.copy()


def neighbour(st: Stencil, q: np.ndarray, m: int, d: int, wall: np.ndarray | None) -> np.ndarray:
    """Value of velocity component m seen by every cell across its face d:
    the neighbour, the domain-face ghost, or the axis-projected ghost of
    eq. (q_axis) where the face is blocked."""
    g = st.grid
    k, s = d // 2, (1 if d % 2 else -1)
    out = shifted(q, k, s)
    bm = boundary_mask(g, d)
    out = np.where(bm, bc_ghost(g, q, m, d), out)
    sel = st.cut_dir == d
    if np.any(sel):
        cells = st.cut_cell[sel]
        qf = q.ravel()
        qib = wall[sel, m] if wall is not None else np.zeros(len(cells))
        qo = np.where(st.cut_opp[sel] >= 0, qf[np.maximum(st.cut_opp[sel], 0)], 0.0)
        ghost = st.a_ib[sel] * qib + st.a_c[sel] * qf[cells] + st.a_o[sel] * qo
        o = out.ravel().copy()
        o[cells] = ghost
        out = o.reshape(g.shape)
    return out


def face_nut(st: Stencil, nut: np.ndarray, d: int) -> np.ndarray:
    """Eddy viscosity on face d: average of the two cells on open interior faces,
    the cell's own value on blocked and domain faces (Reading G4)."""
    g = st.grid
    k, s = d // 2, (1 if d % 2 else -1)
    avg = 0.5 * (nut + shifted(nut, k, s))
    closed = boundary_mask(g, d) | (((st.blocked >> d) & 1) == 1)
    return np.where(closed, nut, avg)


def face_velocity(g: Grid, U: list, d: int) -> np.ndarray:
    """Normal face velocity on face d of every cell.  U[k] holds the +face of each cell;
    the -face of the first layer comes from the boundary kind."""
    k, s = d // 2, (1 if d % 2 else -1)
    if s > 0:
        return U[k]
    v = shifted(U[k], k, -1)
    if g.bc[d] != PERIODIC:
        bm = boundary_mask(g, d)
        val = g.u_in[k] if g.bc[d] == INFLOW else 0.0
        v = np.where(bm, val, v)
    return v


def wall_face_velocity(st: Stencil, wall: np.ndarray | None, k: int) -> np.ndarray:
    """Normal velocity on blocked +k faces: mean of the wall velocities of the two cuts
    that see the face (one from each side)."""
    g = st.grid
    out = np.zeros(g.ncell)
    if wall is None:
        return out.reshape(g.shape)
    d = 2 * k + 1
    sel_p = st.cut_dir == d
    sel_m = st.cut_dir == d - 1
    a = np.zeros(g.ncell)
    a[st.cut_cell[sel_p]] = wall[sel_p, k]
    b = np.zeros(g.ncell)
    b[st.cut_cell[sel_m]] = wall[sel_m, k]
    bsh = shifted(b.reshape(g.shape), k, +1)
    return 0.5 * (a.reshape(g.shape) + bsh)


# ---------------------------------------------------------------- initial state

def init_state(st: Stencil, u0, wall=None):
    """u = u0 everywhere, face velocities consistent with it (wall normal velocity on
    blocked faces, boundary values on domain faces), p = 0, H = 0."""
    g = st.grid
    u = [np.full(g.shape, float(u0[m])) for m in range(3)]
    U = []
    for k in range(3):
        d = 2 * k + 1
        Uk = np.full(g.shape, float(u0[k]))
        bm = boundary_mask(g, d)
        if g.bc[d] == INFLOW:
            Uk = np.where(bm, g.u_in[k], Uk)
        elif g.bc[d] == SLIP:
            Uk = np.where(bm, 0.0, Uk)
        blk = ((st.blocked >> d) & 1) == 1
        Uk = np.where(blk, wall_face_velocity(st, wall, k), Uk)
        U.append(Uk)
    p = np.zeros(g.shape)
    h = [np.zeros(g.shape) for _ in range(3)]
    return u, U, p, h


# ------------------------------------------------------------------- CSM

def csm_nut(st: Stencil, u: list, c1: float = 1.0 / 20.0, wall=None) -> np.ndarray:
    """Coherent structure model (Sec. 2.3, turbulence model):
    G_ij = du_i/dx_j by central differences (ghost values across blocked faces),
    S = (G+G^T)/2, W = (G-G^T)/2, Q = (W:W - S:S)/2, E = (W:W + S:S)/2,
    F_CS = Q/E, C = C1 |F_CS|^(3/2), nu_t = C dx^2 |S| with |S| = sqrt(S_ij S_ij)."""
    g = st.grid
    G = [[None] * 3 for _ in range(3)]
    for i in range(3):
        for j in range(3):
            qp = neighbour(st, u[i], i, 2 * j + 1, wall)
            qm = neighbour(st, u[i], i, 2 * j, wall)
            G[i][j] = (qp - qm) / (2.0 * g.dx)
    SS = np.zeros(g.shape)
    WW = np.zeros(g.shape)
    for i in range(3):
        for j in range(3):
            s_ = 0.5 * (G[i][j] + G[j][i])
            w_ = 0.5 * (G[i][j] - G[j][i])
            SS += s_ * s_
            WW += w_ * w_
    Q = 0.5 * (WW - SS)
    E = 0.5 * (WW + SS)
    F = np.divide(Q, E, out=np.zeros(g.shape), where=E > 0.0)
    C = c1 * np.abs(F) ** 1.5
    return C * g.dx * g.dx * np.sqrt(SS)


# ------------------------------------------------------------ predictor

def second_neighbour(st: Stencil, q: np.ndarray, m: int, d: int, wall, n1: np.ndarray) -> np.ndarray:
    """Value of component m two cells away across face d (the far cell of a QUICK
    stencil, the S2 ghost of the dummy cells, Sec. 2.3.1): across an open interior face,
    the neighbour's own value across its face d (its ghost or domain-face ghost where
    that face is closed); across a blocked or domain face, the ghost line of n1 continued
    one cell further, 2 n1 - q (Reading Q2).  n1 = neighbour(st, q, m, d, wall)."""
    g = st.grid
    k, s = d // 2, (1 if d % 2 else -1)
    closed = boundary_mask(g, d) | (((st.blocked >> d) & 1) == 1)
    far = shifted(n1, k, s)
    return np.where(closed, 2.0 * n1 - q, far)


def quick_face(q, n1, n2, b1, out):
    """QUICK face value (Leonard, 1979) between a cell (q) and its neighbour across the
    face (n1): with the flow leaving the cell through the face (out), upstream q,
    downstream n1 and far upstream b1 (the cell's value across its opposite face):
    (6 q + 3 n1 - b1)/8; otherwise upstream n1, downstream q, far upstream n2:
    (6 n1 + 3 q - n2)/8."""
    return np.where(out, (6.0 * q + 3.0 * n1 - b1) / 8.0, (6.0 * n1 + 3.0 * q - n2) / 8.0)


def momentum_rhs(st: Stencil, u: list, U: list, nut: np.ndarray, nu: float, body, wall, quick: float = 0.0) -> list:
    """H = -(1/dx) sum_f s U_f q_f + (1/dx^2) sum_f (nu + nu_t,f)(q_nb - q_c) + g,
    flux form with the stored face velocity U^n (Sec. 2.1; on blocked faces it
    holds the wall normal velocity of the last projection), the ghost of eq. (q_axis)
    behind blocked faces (direct forcing of eq. (forcing_term) realised through the
    ghost, Reading R9) and the face value q_f of the hybrid scheme (Sec. 3): central
    (q + q_nb)/2 blended with the QUICK value by the weight `quick` (0.1 in the paper's
    Ahmed-body and sphere runs; 0 = pure central)."""
    g = st.grid
    H = []
    for m in range(3):
        q = u[m]
        h = np.full(g.shape, float(body[m]))
        nbs = [neighbour(st, q, m, d, wall) for d in range(6)]
        for d in range(6):
            s = 1 if d % 2 else -1
            qn = nbs[d]
            Uf = face_velocity(g, U, d)
            qf = 0.5 * (q + qn)
            if quick != 0.0:
                qq = quick_face(q, qn, second_neighbour(st, q, m, d, wall, qn), nbs[d ^ 1], s * Uf > 0.0)
                qf = (1.0 - quick) * qf + quick * qq
            h = h - s * Uf * qf / g.dx + (nu + face_nut(st, nut, d)) * (qn - q) / (g.dx * g.dx)
        H.append(h)
    return H


def dead_velocity(st: Stencil, wall) -> list:
    """Velocity of dead-end cells: mean wall velocity over the cell's cuts."""
    g = st.grid
    out = []
    for m in range(3):
        acc = np.zeros(g.ncell)
        cnt = np.zeros(g.ncell)
        w = wall[:, m] if wall is not None else np.zeros(st.ncut)
        np.add.at(acc, st.cut_cell, w)
        np.add.at(cnt, st.cut_cell, 1.0)
        out.append(np.divide(acc, cnt, out=np.zeros(g.ncell), where=cnt > 0).reshape(g.shape))
    return out


def predictor(st, u, U, hprev, nut, nu, dt, body, step, wall, dt_prev=0.0, quick=0.0):
    """u* = u^n + dt ((1 + r/2) H^n - (r/2) H^{n-1}), r = dt/dt_prev: second-order
    Adams-Bashforth with a variable step (r = 1 gives 3/2, -1/2); forward Euler at step 0."""
    H = momentum_rhs(st, u, U, nut, nu, body, wall, quick)
    us = []
    dv = dead_velocity(st, wall) if st.deadend.any() else None
    r = dt / dt_prev if dt_prev > 0 else 1.0
    for m in range(3):
        if step == 0:
            v = u[m] + dt * H[m]
        else:
            v = u[m] + dt * ((1.0 + 0.5 * r) * H[m] - (0.5 * r) * hprev[m])
        if dv is not None:
            v = np.where(st.deadend, dv[m], v)
            H[m] = np.where(st.deadend, 0.0, H[m])
        us.append(v)
    return us, H


# ------------------------------------------------- Crank-Nicolson predictor

def hom_neighbour(st: Stencil, q: np.ndarray, m: int, d: int) -> np.ndarray:
    """Value of component m across face d as seen by the part of the momentum
    right-hand side that is linear in q: the neighbour, the domain-face ghost with a
    zero inflow velocity (inflow and the normal component at a slip face: -q;
    otherwise q), and the eq. (q_axis) ghost with a zero wall velocity
    (a_c q_c + a_o q_o).  The ghosts of `neighbour` are these plus terms that do not
    depend on q."""
    g = st.grid
    k, s = d // 2, (1 if d % 2 else -1)
    out = shifted(q, k, s)
    bm = boundary_mask(g, d)
    odd = g.bc[d] == INFLOW or (g.bc[d] == SLIP and m == k)
    out = np.where(bm, -q if odd else q, out)
    sel = st.cut_dir == d
    if np.any(sel):
        cells = st.cut_cell[sel]
        qf = q.ravel()
        qo = np.where(st.cut_opp[sel] >= 0, qf[np.maximum(st.cut_opp[sel], 0)], 0.0)
        o = out.ravel().copy()
        o[cells] = st.a_c[sel] * qf[cells] + st.a_o[sel] * qo
        out = o.reshape(g.shape)
    return out


def momentum_operator(st: Stencil, q: np.ndarray, m: int, U: list, nut: np.ndarray, nu: float) -> np.ndarray:
    """L_m q: the part of the momentum right-hand side of eq. (crank-nicolson) that is
    linear in velocity component m, with the advecting face velocity frozen at U^n and
    the eddy viscosity at its value from u^n:
    L q = -(1/dx) sum_f s U_f (q + q_nb)/2 + (1/dx^2) sum_f (nu + nu_t,f)(q_nb - q),
    q_nb from hom_neighbour.  The full right-hand side is H(u) = L u + (terms from the
    wall and inflow velocities and the body force)."""
    g = st.grid
    out = np.zeros(g.shape)
    for d in range(6):
        s = 1 if d % 2 else -1
        qn = hom_neighbour(st, q, m, d)
        Uf = face_velocity(g, U, d)
        out = out - s * Uf * (0.5 * (q + qn)) / g.dx + (nu + face_nut(st, nut, d)) * (qn - q) / (g.dx * g.dx)
    return out


def bicgstab(apply, b: np.ndarray, x0: np.ndarray, tol: float, max_iter: int):
    """BiCGStab (van der Vorst, SIAM J. Sci. Stat. Comput. 13, 1992), unpreconditioned,
    for A x = b with a nonsymmetric A (the solver the paper names for its implicit time
    integration, Sec. 2.1).  Stops when ||r|| <= tol ||b|| at the start of an iteration,
    or when ||s|| <= tol ||b|| halfway through one (x += alpha p only).  Returns
    (x, iterations, status), status 'converged', 'max_iter' or 'breakdown'
    (rho = 0, <r0, v> = 0 or omega = 0 with the residual not yet small)."""
    bb = float(np.sum(b * b))
    if bb == 0.0:
        return np.zeros_like(b), 0, "converged"
    tol2 = tol * tol * bb
    x = x0.copy()
    r = b - apply(x)
    r0 = r.copy()
    rho_old, alpha, omega = 1.0, 1.0, 1.0
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    for it in range(max_iter + 1):
        if float(np.sum(r * r)) <= tol2:
            return x, it, "converged"
        if it == max_iter:
            return x, it, "max_iter"
        rho = float(np.sum(r0 * r))
        if rho == 0.0:
            return x, it, "breakdown"
        beta = (rho / rho_old) * (alpha / omega)
        p = r + beta * (p - omega * v)
        v = apply(p)
        r0v = float(np.sum(r0 * v))
        if r0v == 0.0:
            return x, it, "breakdown"
        alpha = rho / r0v
        s = r - alpha * v
        if float(np.sum(s * s)) <= tol2:
            return x + alpha * p, it + 1, "converged"
        t = apply(s)
        omega = float(np.sum(t * s)) / float(np.sum(t * t))
        if omega == 0.0:
            return x, it, "breakdown"
        x = x + alpha * p + omega * s
        r = s - omega * t
        rho_old = rho
    raise AssertionError("unreachable")


def cn_matrix_apply(st: Stencil, q: np.ndarray, m: int, U: list, nut: np.ndarray, nu: float, dt: float):
    """(I - dt/2 L_m) q, with identity rows at dead-end cells (Reading R13)."""
    a = q - 0.5 * dt * momentum_operator(st, q, m, U, nut, nu)
    return np.where(st.deadend, q, a)


def cn_predictor(st, u, U, nut, nu, dt, body, wall, tol, max_iter, quick=0.0):
    """Crank-Nicolson predictor of eq. (crank-nicolson): advection (by the frozen U^n)
    and diffusion both taken half at u^n and half at u*, the wall, inflow and body
    terms whole.  With H the full right-hand side and L its linear part
    (momentum_operator), u* - u^n = dt [H(u^n) + L(u* - u^n)/2], so the increment
    delta = u* - u^n solves (I - dt/2 L) delta = dt H^n, one system per component,
    solved by BiCGStab from delta_0 = dt H^n (the explicit Euler increment).
    Dead-end cells are pinned at their mean wall velocity (identity rows).  With a QUICK
    blend the blended part of the face value stays explicit (in H^n only; L is the
    central operator, Reading Q3).
    Returns (u*, H^n with zeros at dead-end cells, iterations per component)."""
    H = momentum_rhs(st, u, U, nut, nu, body, wall, quick)
    dead = st.deadend
    dv = dead_velocity(st, wall) if dead.any() else None
    us, iters = [], []
    for m in range(3):
        b = dt * H[m]
        if dv is not None:
            b = np.where(dead, dv[m] - u[m], b)
        delta, it, status = bicgstab(lambda q, m=m: cn_matrix_apply(st, q, m, U, nut, nu, dt), b, b, tol, max_iter)
        if status != "converged":
            raise RuntimeError(f"momentum solve of component {m}: {status} after {it} iterations")
        v = u[m] + delta
        if dv is not None:
            v = np.where(dead, dv[m], v)
            H[m] = np.where(dead, 0.0, H[m])
        us.append(v)
        iters.append(it)
    return us, H, iters


# ---------------------------------------------------------- Poisson / projection

def face_predicted(st: Stencil, us: list, wall) -> list:
    """Predicted normal face velocity U* on the +face of each cell (Rhie-Chow style
    face velocity, Reading R6): central average on open faces, wall normal velocity
    on blocked faces, boundary value on domain faces."""
    g = st.grid
    out = []
    for k in range(3):
        d = 2 * k + 1
        v = 0.5 * (us[k] + shifted(us[k], k, +1))
        blk = ((st.blocked >> d) & 1) == 1
        v = np.where(blk, wall_face_velocity(st, wall, k), v)
        bm = boundary_mask(g, d)
        if g.bc[d] == INFLOW:
            v = np.where(bm, g.u_in[k], v)
        elif g.bc[d] == SLIP:
            v = np.where(bm, 0.0, v)
        elif g.bc[d] == OUTFLOW:
            v = np.where(bm, us[k], v)
        out.append(v)
    return out


def divergence(g: Grid, U: list) -> np.ndarray:
    div = np.zeros(g.shape)
    for k in range(3):
        div += (face_velocity(g, U, 2 * k + 1) - face_velocity(g, U, 2 * k)) / g.dx
    return div


def remove_component_means(st: Stencil, a: np.ndarray) -> np.ndarray:
    """Subtract the mean over every enclosed component (compatibility of the Neumann
    problem and gauge of the pressure, Reading G3)."""
    f = a.ravel().copy()
    for cells in st.comps:
        f[cells] -= f[cells].mean()
    return f.reshape(a.shape)


def poisson_rhs(st: Stencil, Us: list, dt: float) -> np.ndarray:
    """b = div(U*)/dt (eq. poisson), made compatible on enclosed components."""
    b = divergence(st.grid, Us) / dt
    return remove_component_means(st, b)


def open_face(st: Stencil, d: int) -> np.ndarray:
    key = ("open", d)
    if key not in st.cache:
        st.cache[key] = (((st.blocked >> d) & 1) == 0) & ~boundary_mask(st.grid, d)
    return st.cache[key]


def outlet_face(st: Stencil, d: int) -> np.ndarray:
    g = st.grid
    if g.bc[d] != OUTFLOW:
        return np.zeros(g.shape, dtype=bool)
    return boundary_mask(g, d)


def laplacian(st: Stencil, p: np.ndarray) -> np.ndarray:
    """L p = (1/dx^2) [ sum over open faces (p_nb - p_c) - 2 p_c per outlet face ].
    Blocked faces and inflow/slip faces carry the Neumann ghost p_GC = p_c
    (zeta = 1, eta = 0 in eq. (Mittal)), so they drop out."""
    g = st.grid
    out = np.zeros(g.shape)
    for d in range(6):
        k, s = d // 2, (1 if d % 2 else -1)
        out += np.where(open_face(st, d), shifted(p, k, s) - p, 0.0)
        out += np.where(outlet_face(st, d), -2.0 * p, 0.0)
    return out / (g.dx * g.dx)


def jacobi_diag(st: Stencil) -> np.ndarray:
    """Diagonal of A = -L."""
    g = st.grid
    dg = np.zeros(g.shape)
    for d in range(6):
        dg += open_face(st, d) + 2.0 * outlet_face(st, d)
    return dg / (g.dx * g.dx)


def pcg(st: Stencil, b: np.ndarray, x0: np.ndarray, tol: float, max_iter: int):
    """Jacobi-preconditioned conjugate gradients on A x = -b with A = -L (symmetric
    positive semi-definite), warm start x0.  Stops at the first iteration with
    ||r||_2 <= tol ||b||_2 (recursively updated residual).  Returns (x, iters)."""
    f = -b
    fn = np.sqrt(np.sum(f * f))
    if fn == 0.0:
        return np.zeros_like(x0), 0
    dg = jacobi_diag(st)
    minv = np.divide(1.0, dg, out=np.zeros_like(dg), where=dg > 0)
    x = x0.copy()
    r = f + laplacian(st, x)
    if np.sqrt(np.sum(r * r)) <= tol * fn:
        return x, 0
    z = minv * r
    d = z.copy()
    rz = np.sum(r * z)
    it = 0
    while it < max_iter:
        it += 1
        q = -laplacian(st, d)
        alpha = rz / np.sum(d * q)
        x = x + alpha * d
        r = r - alpha * q
        if np.sqrt(np.sum(r * r)) <= tol * fn:
            break
        z = minv * r
        rz_new = np.sum(r * z)
        beta = rz_new / rz
        rz = rz_new
        d = z + beta * d
    return x, it


def rbsor(st: Stencil, b: np.ndarray, x0: np.ndarray, omega: float, tol: float, max_iter: int,
          check_every: int = 1):
    """Red-black successive over-relaxation on L x = b (Sec. 2.1 names red-black SOR as
    the alternative to BiCGStab for the Poisson equation; Sec. 2.3.2 notes that it
    converges rapidly with these ghosts).  Cells are coloured by the parity of i + j + k;
    one sweep updates every cell of colour 0, then every cell of colour 1, each by
    x_c += omega (b_c - (L x)_c) / L_cc with the current values.  The neighbours of a
    cell all have the other colour (periodic axes need an even cell count), so a half
    sweep does not depend on the order of its cells.  Cells without open or outlet faces
    (L_cc = 0) keep their value.  The true residual is tested every `check_every` sweeps
    and after the last: ||b - L x|| <= tol ||b|| stops.  A zero b gives x = 0.
    Returns (x, sweeps, converged)."""
    g = st.grid
    for k in range(3):
        if g.periodic(k) and g.n[k] % 2:
            raise ValueError("red-black ordering needs an even cell count on periodic axes")
    bn = float(np.sqrt(np.sum(b * b)))
    if bn == 0.0:
        return np.zeros_like(x0), 0, True
    diag = -jacobi_diag(st)                      # L_cc
    ii, jj, kk = _index_grid(g)
    colour = (ii + jj + kk) % 2
    has = diag != 0.0
    safe = np.where(has, diag, 1.0)
    x = x0.copy()
    it = 0
    while True:
        if it % check_every == 0 or it == max_iter:
            r = b - laplacian(st, x)
            if float(np.sqrt(np.sum(r * r))) <= tol * bn:
                return x, it, True
            if it >= max_iter:
                return x, it, False
        for c in (0, 1):
            r = b - laplacian(st, x)
            x = np.where(has & (colour == c), x + omega * r / safe, x)
        it += 1


def project(st: Stencil, us: list, Us: list, p: np.ndarray, dt: float):
    """Correction, eq. (correction): U^{n+1} = U* - dt dp/dx on faces (compact
    difference), u^{n+1} = u* - dt (p_E - p_W)/(2dx) at centres; Neumann ghost
    p_c across blocked, inflow and slip faces, Dirichlet p = 0 on outlet faces."""
    g = st.grid
    U = []
    u = []
    for k in range(3):
        d = 2 * k + 1
        gradf = (shifted(p, k, +1) - p) / g.dx
        v = np.where(open_face(st, d), Us[k] - dt * gradf, Us[k])
        v = np.where(outlet_face(st, d), Us[k] + 2.0 * dt * p / g.dx, v)
        U.append(v)

        def pghost(dd):
            kk, s = dd // 2, (1 if dd % 2 else -1)
            val = np.where(open_face(st, dd), shifted(p, kk, s), p)
            return np.where(outlet_face(st, dd), -p, val)
        uk = us[k] - dt * (pghost(2 * k + 1) - pghost(2 * k)) / (2.0 * g.dx)
        if st.deadend.any():
            uk = np.where(st.deadend, us[k], uk)
        u.append(uk)
    return u, U


@dataclasses.dataclass
class StepParams:
    dt: float
    nu: float
    c1: float = 1.0 / 20.0
    csm: bool = True
    body: tuple = (0.0, 0.0, 0.0)
    tol: float = 1e-10
    max_iter: int = 10000
    dt_prev: float = 0.0
    scheme: str = "ab2"        # "ab2" (explicit) or "cn" (Crank-Nicolson + BiCGStab)
    mom_tol: float = 1e-10     # cn: relative residual of each component's system
    mom_max_iter: int = 200    # cn: BiCGStab iteration cap
    quick: float = 0.0         # weight of the QUICK face value in the hybrid scheme


def step(st: Stencil, u, U, p, hprev, prm: StepParams, step_index: int, wall=None):
    """One fractional step: CSM -> predictor (AB2, or Crank-Nicolson with BiCGStab) ->
    face velocity + Poisson RHS -> PCG -> gauge -> projection.
    Returns (u, U, p, H, stats)."""
    g = st.grid
    nut = csm_nut(st, u, prm.c1, wall) if prm.csm else np.zeros(g.shape)
    mom_iters = [0, 0, 0]
    if prm.scheme == "cn":
        us, H, mom_iters = cn_predictor(st, u, U, nut, prm.nu, prm.dt, prm.body, wall, prm.mom_tol,
                                        prm.mom_max_iter, prm.quick)
    elif prm.scheme == "ab2":
        us, H = predictor(st, u, U, hprev, nut, prm.nu, prm.dt, prm.body, step_index, wall, prm.dt_prev,
                          prm.quick)
    else:
        raise ValueError(prm.scheme)
    Us = face_predicted(st, us, wall)
    b = poisson_rhs(st, Us, prm.dt)
    pn, iters = pcg(st, b, p, prm.tol, prm.max_iter)
    pn = remove_component_means(st, pn)
    res = b - laplacian(st, pn)
    bn = np.sqrt(np.sum(b * b))
    un, Un = project(st, us, Us, pn, prm.dt)
    div = divergence(g, Un)
    stats = dict(iters=iters, rel_residual=float(np.sqrt(np.sum(res * res)) / bn) if bn > 0 else 0.0,
                 div_l2=float(np.sqrt(np.sum(div * div))), div_linf=float(np.max(np.abs(div))),
                 umax=float(max(np.max(np.abs(face_velocity(g, Un, d))) for d in range(6))),
                 nut=nut, b=b, mom_iters=mom_iters)
    return un, Un, pn, H, stats


# ------------------------------------------------------------------ forces

def forces(st: Stencil, u: list, p: np.ndarray, nut: np.ndarray | None, nu: float, wall=None):
    """Force on the immersed surface as the momentum flux through every blocked face
    (Reading R11): F += dx^2 [ s p_c e_k - (nu + nu_t,c) (q_GC - q_c)/dx ].
    Returns (F_pressure[3], F_viscous[3])."""
    g = st.grid
    Fp = np.zeros(3)
    Fv = np.zeros(3)
    pf = p.ravel()
    nt = nut.ravel() if nut is not None else np.zeros(g.ncell)
    s = np.where(st.cut_dir % 2 == 1, 1.0, -1.0)
    ax = st.cut_dir // 2
    A = g.dx * g.dx
    for k in range(3):
        Fp[k] = np.sum(np.where(ax == k, s * pf[st.cut_cell], 0.0)) * A
    for m in range(3):
        qf = u[m].ravel()
        qib = wall[:, m] if wall is not None else np.zeros(st.ncut)
        qo = np.where(st.cut_opp >= 0, qf[np.maximum(st.cut_opp, 0)], 0.0)
        ghost = st.a_ib * qib + st.a_c * qf[st.cut_cell] + st.a_o * qo
        Fv[m] = -np.sum((nu + nt[st.cut_cell]) * (ghost - qf[st.cut_cell]) / g.dx) * A
    return Fp, Fv
