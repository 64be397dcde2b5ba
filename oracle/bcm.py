"""Building-cube (BCM) two-level grid oracle (test infrastructure only; the product path
never imports it): cubes, halo exchange and the pressure operator on the cubes
(Sec. 2.2, discretization of the grid system).

What is computed (plain FP64 numpy, one halo cell at a time, from the definitions):

* The domain is tiled by K = (Kx, Ky, Kz) coarse cubes of n^3 cells of size dx0; a
  coarse cube marked for refinement is replaced by 8 fine cubes of n^3 cells of size
  dx0/2 (the two fixed levels of the paper, a factor of two apart).  Cube order: coarse
  cubes in z, y, x order; a refined one contributes its 8 fine cubes in z, y, x order.
* Every cube stores its n^3 cells with H = 2 halo layers on each face ((n + 2H)^3
  values, x fastest).  The exchange fills only the face halos (axis directions; edges and
  corners of the halo are not used by an axis stencil and are left alone).
* A halo cell of cube A takes its value from the cube that covers its centre: from a
  cube of the same level or a coarser one, the value of the cell that contains the centre
  (a copy, the paper's zero-order interpolation); from finer cubes, the mean of the 8
  fine cells inside the halo cell (the paper's averaging), summed in z, y, x order.
  Outside the domain the halo mirrors the cube's own cells (zero normal gradient): layer
  l takes interior cell l - 1 counted from the face.
* The operator on a cube: (L x)_c = (sum of the six axis neighbours - 6 x_c) / dx^2,
  the neighbours summed in the order -x, +x, -y, +y, -z, +z, read from the cube's own
  storage (halos included).

* Immersed geometry on the cubes (set_blocked): each level is tagged as a uniform grid
  of its own cell size over the whole domain (Sec. 2.3.1, the axis-projected segment
  test), and every cube takes the blocked bits of its cells from its level's grid.  A
  blocked face carries the pressure ghost p_GC = p_c (the Neumann case of eq. (Mittal),
  reading G3), so the operator adds x_c in place of the neighbour; a red-black SOR
  update divides by the number of open faces (-open / dx^2), and a cell without open
  faces keeps its value.

* The pressure solve on the cubes (Sec. 2.1 names BiCGStab and red-black SOR for the
  Poisson equation; Sec. 2.2 puts it on this grid): the unknowns are the cube
  interiors, the operator is "exchange, then L".  bicgstab runs the flow oracle's
  BiCGStab on that operator (stopping on the recursive residual); sor_solve runs
  red-black SOR in groups of check_every sweeps and stops at the first check where the
  true residual ||b - L x|| <= tol ||b|| (norms over the interiors).

Readings: n = 16 cells per cube axis (the paper's figure shows 8, its text gives the
structure only); mirror halos at the domain boundary (the paper omits the outer boundary
conditions); the cube order above (an interface, chosen to make the fine cubes of one
coarse cube contiguous); a cube cell's faces are blocked as the segments of its own
level's grid, also where the neighbour across the face belongs to the other level.
"""
from __future__ import annotations

import numpy as np

H = 2


class Cubes:
    def __init__(self, K, n, dx0, origin, refine):
        """refine: bool array (Kz, Ky, Kx)."""
        self.K = tuple(int(k) for k in K)
        self.n = int(n)
        self.dx0 = float(dx0)
        self.origin = np.asarray(origin, dtype=np.float64)
        self.refine = np.asarray(refine, dtype=bool)
        self.cubes = []          # (level, integer origin in fine-cell units (x, y, z))
        self.first = np.zeros(self.K[::-1], dtype=np.int64)   # first cube of each coarse cube
        for kz in range(self.K[2]):
            for ky in range(self.K[1]):
                for kx in range(self.K[0]):
                    self.first[kz, ky, kx] = len(self.cubes)
                    base = np.array([kx, ky, kz]) * 2 * self.n
                    if self.refine[kz, ky, kx]:
                        for cz in range(2):
                            for cy in range(2):
                                for cx in range(2):
                                    self.cubes.append((1, base + np.array([cx, cy, cz]) * self.n))
                    else:
                        self.cubes.append((0, base))
        self.side = self.n + 2 * H

    def dx(self, level):
        return self.dx0 if level == 0 else 0.5 * self.dx0

    def level_shape(self, level):
        """Cells (nz, ny, nx) of the uniform grid of one level over the whole domain."""
        f = 1 if level == 0 else 2
        return tuple(int(self.K[a] * self.n * f) for a in (2, 1, 0))

    def set_blocked(self, level, blocked):
        """Blocked bits of the cubes of one level from that level's uniform-grid tagging
        (uint8 array of level_shape(level)): cube cell (i, j, k) takes the bits of grid
        cell (origin + (i, j, k)) of its level."""
        blocked = np.asarray(blocked, dtype=np.uint8)
        assert blocked.shape == self.level_shape(level)
        if not hasattr(self, "mask"):
            self.mask = np.zeros((len(self.cubes), self.n, self.n, self.n), dtype=np.uint8)
        n = self.n
        for q, (lvl, o) in enumerate(self.cubes):
            if lvl != level:
                continue
            c0 = o // 2 if lvl == 0 else o
            self.mask[q] = blocked[c0[2]:c0[2] + n, c0[1]:c0[1] + n, c0[0]:c0[0] + n]

    def size(self):
        return len(self.cubes) * self.side ** 3

    def index(self, q, i, j, k):
        """Storage index of cell (i, j, k) of cube q (interior 0..n-1, halo -H..n+H-1)."""
        s = self.side
        return q * s ** 3 + (i + H) + s * ((j + H) + s * (k + H))

    def locate(self, p):
        """Cube and cell containing the point p (fine-cell units), or None outside."""
        K2 = np.array(self.K) * 2 * self.n
        if np.any(p < 0) or np.any(p >= K2):
            return None
        kc = (p // (2 * self.n)).astype(int)
        first = int(self.first[kc[2], kc[1], kc[0]])
        if self.refine[kc[2], kc[1], kc[0]]:
            sub = ((p - kc * 2 * self.n) // self.n).astype(int)
            q = first + sub[0] + 2 * sub[1] + 4 * sub[2]
            lvl, o = self.cubes[q]
            cell = (p - o).astype(int)
        else:
            q = first
            lvl, o = self.cubes[q]
            cell = ((p - o) // 2).astype(int)
        return q, lvl, cell

    def exchange(self, data, cubes=None):
        """Fills the face halos of every cube, or of the listed cubes only (returns a new
        array).  The sources of every halo cell are resolved once from the definition
        below (halo_sources) and kept; a mean adds its 8 values in their listed order."""
        key = None if cubes is None else tuple(sorted(int(q) for q in cubes))
        if not hasattr(self, "_plans"):
            self._plans = {}
        if key not in self._plans:
            self._plans[key] = self.halo_sources(key)
        dst1, src1, dst8, src8 = self._plans[key]
        out = data.copy()
        out[dst1] = data[src1]
        acc = np.zeros(len(dst8))
        for e in range(8):
            acc = acc + data[src8[:, e]]
        out[dst8] = acc / 8.0
        return out

    def halo_sources(self, cubes=None):
        """Per face-halo cell (of every cube, or of the listed cubes), its storage index and
        the indices it takes its value from: (dst of copies, their source, dst of means,
        their 8 sources in z, y, x order)."""
        dst1, src1, dst8, src8 = [], [], [], []
        n = self.n
        for q in (range(len(self.cubes)) if cubes is None else cubes):
            lvl, o = self.cubes[q]
            w = 1 if lvl == 1 else 2                     # this cube's cell size in fine units
            for axis in range(3):
                for sgn in (-1, 1):
                    for layer in range(1, H + 1):
                        ci = n - 1 + layer if sgn > 0 else -layer
                        for a in range(n):
                            for b in range(n):
                                c = [0, 0, 0]
                                c[axis] = ci
                                c[(axis + 1) % 3] = a
                                c[(axis + 2) % 3] = b
                                centre = o + (np.array(c) + 0.5) * w     # fine-cell units
                                hit = self.locate(centre)
                                dst = self.index(q, *c)
                                if hit is None:
                                    m = list(c)
                                    m[axis] = n - layer if sgn > 0 else layer - 1
                                    dst1.append(dst)
                                    src1.append(self.index(q, *m))
                                else:
                                    qq, l2, cell = hit
                                    if l2 <= lvl or lvl == 1:
                                        dst1.append(dst)
                                        src1.append(self.index(qq, *cell))
                                    else:
                                        # coarse halo cell over fine cells: the 8 inside it,
                                        # in z, y, x order
                                        lo = o + np.array(c) * 2
                                        srcs = []
                                        for dz in range(2):
                                            for dy in range(2):
                                                for dxx in range(2):
                                                    pp = lo + np.array([dxx, dy, dz]) + 0.5
                                                    q3, _, c3 = self.locate(pp)
                                                    srcs.append(self.index(q3, *c3))
                                        dst8.append(dst)
                                        src8.append(srcs)
        return (np.array(dst1, dtype=np.int64), np.array(src1, dtype=np.int64), np.array(dst8, dtype=np.int64),
                np.array(src8, dtype=np.int64).reshape(-1, 8))

    def laplacian(self, data, cubes=None):
        """(L x) on every cube interior, or on the listed cubes' (halos of the result and
        cubes not listed are zero)."""
        out = np.zeros_like(data)
        n, sd = self.n, self.side
        for q in (range(len(self.cubes)) if cubes is None else cubes):
            lvl, o = self.cubes[q]
            dx = self.dx(lvl)
            blk = data[q * sd ** 3:(q + 1) * sd ** 3].reshape(sd, sd, sd)
            ob = out[q * sd ** 3:(q + 1) * sd ** 3].reshape(sd, sd, sd)
            c = slice(H, H + n)
            m, p = slice(H - 1, H + n - 1), slice(H + 1, H + n + 1)
            xc = blk[c, c, c]
            nbs = (blk[c, c, m], blk[c, c, p], blk[c, m, c], blk[c, p, c], blk[m, c, c], blk[p, c, c])
            if hasattr(self, "mask"):
                # behind a blocked face the Neumann ghost p_GC = p_c
                nbs = tuple(np.where(((self.mask[q] >> d) & 1) == 1, xc, nbs[d]) for d in range(6))
            s = nbs[0]
            for d in range(1, 6):
                s = s + nbs[d]
            ob[c, c, c] = (s - 6.0 * xc) / (dx * dx)
        return out

    def open_faces(self, q):
        """Open faces (0..6) of cube q's cells."""
        if not hasattr(self, "mask"):
            return np.full((self.n,) * 3, 6)
        m = self.mask[q]
        return sum(((m >> d) & 1) == 0 for d in range(6)).astype(np.int64)

    def rbsor(self, b, x0, omega, sweeps):
        """Red-black SOR on the cubes (Sec. 2.1's alternative solver on the Sec. 2.2 grid):
        each half sweep exchanges the halos, then updates every interior cell of one
        colour (parity of its cube-local i + j + k; cube origins are multiples of n, so
        this is the parity within its level) in every cube by
        x_c += omega (b_c - (L x)_c) / (-open / dx^2) (open = 6 without geometry; a cell
        without open faces keeps its value), reading only cells of the other colour
        and the halo copies.  Returns x after `sweeps` sweeps (halos as last exchanged)."""
        x = x0.copy()
        for _ in range(sweeps):
            for c in (0, 1):
                x = self.half_sweep(b, x, omega, c)
        return x

    def half_sweep(self, b, x, omega, colour, cubes=None):
        """One half sweep: exchange, then the cells of one colour (see rbsor).  With a
        list of cubes, only their halos and interiors are updated; that equals the full
        half sweep on them when every cube their halos read from holds its full-sweep
        values."""
        n = self.n
        kk, jj, ii = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        mine = (ii + jj + kk) % 2 == colour
        s = self.side
        x = self.exchange(x, cubes)
        L = self.laplacian(x, cubes)
        for q in (range(len(self.cubes)) if cubes is None else cubes):
            lvl = self.cubes[q][0]
            dx = self.dx(lvl)
            nopen = self.open_faces(q)
            diag = -nopen / (dx * dx)
            blk = x[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
            inner = blk[H:H + n, H:H + n, H:H + n]
            r = self.interior(b, q) - self.interior(L, q)
            upd = mine & (nopen > 0)
            inner[...] = np.where(upd, inner + omega * r / np.where(upd, diag, 1.0), inner)
        return x

    # ------------------------------------------------------- the solve on the cubes
    def pack(self, data):
        """The interiors of every cube, concatenated in cube order ((k, j, i) inside)."""
        return np.concatenate([self.interior(data, q).ravel() for q in range(len(self.cubes))])

    def unpack(self, v):
        """Cube storage with v (as pack returns it) in the interiors and zero halos."""
        data = np.zeros(self.size())
        n, n3 = self.n, self.n ** 3
        for q in range(len(self.cubes)):
            self.interior(data, q)[...] = np.asarray(v[q * n3:(q + 1) * n3]).reshape(n, n, n)
        return data

    def apply(self, v):
        """The pressure operator on packed interiors: exchange the halos, then L."""
        return self.pack(self.laplacian(self.exchange(self.unpack(v))))

    def residual(self, b, x):
        """||b - L x|| / ||b|| over the interiors (x's halos exchanged first); 0 for b = 0."""
        r = self.pack(b) - self.pack(self.laplacian(self.exchange(x)))
        bb = float(np.sum(self.pack(b) ** 2))
        return 0.0 if bb == 0.0 else float(np.sqrt(np.sum(r * r) / bb))

    def bicgstab(self, b, x0, tol, max_iter):
        """BiCGStab for L x = b on the cubes (b, x0: cube storage, interiors used).
        Returns (x as cube storage with zero halos, iterations, status)."""
        from oracle import flow
        x, it, status = flow.bicgstab(self.apply, self.pack(b), self.pack(x0), tol, max_iter)
        return self.unpack(x), it, status

    def sor_solve(self, b, x0, omega, tol, check_every, max_sweeps):
        """Red-black SOR to a tolerance: the true residual is checked before the first
        sweep and after every check_every sweeps; returns (x, sweeps, status) at the
        first check with residual <= tol ('converged'), or after max_sweeps sweeps
        ('max_iter', with a last check there).  x keeps its halos as last exchanged."""
        x = x0.copy()
        sweeps = 0
        while True:
            if self.residual(b, x) <= tol:
                return x, sweeps, "converged"
            if sweeps >= max_sweeps:
                return x, sweeps, "max_iter"
            k = min(check_every, max_sweeps - sweeps)
            x = self.rbsor(b, x, omega, k)
            sweeps += k

    def cell_centres(self, q):
        """Physical centres (n, n, n, 3) of cube q's interior cells, array order (k, j, i)."""
        lvl, o = self.cubes[q]
        w = 1 if lvl == 1 else 2
        ax = [(o[a] + (np.arange(self.n) + 0.5) * w) * 0.5 * self.dx0 + self.origin[a] for a in range(3)]
        zz, yy, xx = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
        return np.stack([xx, yy, zz], axis=-1)

    def fill(self, f):
        """Cube storage with f(x, y, z) at every interior cell, zero halos."""
        data = np.zeros(self.size())
        s = self.side
        for q in range(len(self.cubes)):
            cc = self.cell_centres(q)
            block = data[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
            block[H:H + self.n, H:H + self.n, H:H + self.n] = f(cc[..., 0], cc[..., 1], cc[..., 2])
        return data

    def interior(self, data, q):
        s = self.side
        block = data[q * s ** 3:(q + 1) * s ** 3].reshape(s, s, s)
        return block[H:H + self.n, H:H + self.n, H:H + self.n]
