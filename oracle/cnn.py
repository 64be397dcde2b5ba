"""CNN preconditioner oracle: FP64 numpy reference of the learned part of the
pressure solve (test infrastructure only; the product path never imports it).

What is computed:

* A linear, symmetric positive semi-definite convolutional operator built from
  four 3x3x3 convolutions with 16 channels and a geometry gate:
      G      = hsig(Wg * g)                         (16 channels, per geometry)
      K x    = W2 * ((W1 * x) . G)                  (1 -> 16 channels)
      K^T y  = W1^T * ((W2^T * y) . G)              (16 -> 1, adjoint convolutions)
      net(x) = K^T K x
  with hsig(v) = min(max(v/4 + 1/2, 0), 1) (the "hard" logistic: the same value and
  slope as the logistic function at 0, clamped to [0, 1]), g the fraction of the six
  faces of a cell that are open pressure faces, "*"
  a zero-padded 3x3x3 cross-correlation, "^T *" its adjoint and "." the
  per-channel product.  The operator is linear in x, so a Krylov method sees a
  fixed preconditioner; x^T net(x) = |K x|^2 >= 0.
* The preconditioner  z = D^-1 r + s * net(r / s),  s = RMS(r), D the diagonal of
  the pressure operator A = -L: symmetric positive definite, Jacobi when the
  weights are zero.  (Dividing by s only keeps BF16 activations near unit size;
  in exact arithmetic s * net(r/s) = net(r).)
* Optionally (omega > 0) that preconditioner inside a symmetric two-level form with
  one damped Jacobi smoothing step S = omega D^-1 before and after it:
      z1 = S r,   z2 = z1 + M(r - A z1),   z = z2 + S(r - A z2),
  i.e. z = (2S - S A S) r + (I - S A) M (I - A S) r, symmetric because S, A and M
  are, and positive definite for 0 < omega < 1 (the eigenvalues of D^-1 A lie in
  [0, 2], so 2S - S A S is positive definite).  The smoothing takes the error components a convolution of four cells'
  reach leaves behind off the network.  The network can be trained as M alone or
  through this form (the loss below with the smoothed p_hat).
* Training loss for one (b, p) pair of the pressure equation L p = b, i.e.
  A p = f with f = -b:  the A-norm distance of p from the best multiple of the
  preconditioned right-hand side p_hat = M(f),
      loss = min_a |p - a p_hat|_A^2 / |p|_A^2 = 1 - (f.p_hat)^2 / ((f.p)(p_hat.A p_hat)),
  which is invariant to the scale of p_hat, as is the Krylov method it serves.
* Adam (Kingma and Ba, 2015) and flexible conjugate gradients FCG(1) (Notay,
  2000: the Polak-Ribiere form of beta), which tolerates the small asymmetry that
  BF16 rounding leaves in the preconditioner.

The paper itself runs plain Krylov pressure solves on CPU clusters; this part is
the learned extension layered on its pressure solve (eq. (poisson)).  Rounding
points that the GPU path takes in BF16 (network input, gate, every stored
activation and backward signal, weights) are reproduced by `bf16_round` when
`bf16=True`; with `bf16=False` everything is FP64.

Weight layout (also the flat FP32 layout the C ABI takes): W1[t, 0, co] (432),
W2[t, ci, co] (6912), Wg[t, 0, co] (432), in that order, tap
t = (dz+1)*9 + (dy+1)*3 + (dx+1) for offsets dx, dy, dz in {-1, 0, 1}.  Fields are
numpy arrays shaped (nz, ny, nx[, C]), x fastest in memory.
"""
from __future__ import annotations

import numpy as np

from . import flow

# (name, input channels, output channels) of the three weight tensors
LAYERS = (("W1", 1, 16), ("W2", 16, 16), ("Wg", 1, 16))
TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def n_weights() -> int:
    return sum(27 * ci * co for _, ci, co in LAYERS)


def split_weights(flat: np.ndarray) -> list:
    out, o = [], 0
    for _, ci, co in LAYERS:
        n = 27 * ci * co
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(27, ci, co))
        o += n
    return out


def join_weights(ws: list) -> np.ndarray:
    return np.concatenate([np.asarray(w, dtype=np.float64).reshape(-1) for w in ws])


# ------------------------------------------------------------------ bf16

def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (8-bit significand), ties to even, returned as
    float64.  bfloat16 is the upper half of an IEEE binary32: round the value to
    binary32 first, then drop the low 16 bits with round-half-even on them.
    NaN stays NaN; overflow goes to infinity."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    keep = u >> 16
    up = (low > 0x8000) | ((low == 0x8000) & ((keep & 1) == 1))
    keep = keep + up.astype(np.uint64)
    nan = np.isnan(f)
    r = (keep << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    return np.where(nan, np.nan, r)


# ------------------------------------------------------------------ convolution

def shift0(a: np.ndarray, dz: int, dy: int, dx: int) -> np.ndarray:
    """Value of `a` at (z+dz, y+dy, x+dx) for every cell (z, y, x), zero where that
    neighbour lies outside the grid.  `a` is shaped (nz, ny, nx, C)."""
    out = np.zeros_like(a)
    nz, ny, nx = a.shape[:3]

    def rng(n, d):
        lo, hi = max(0, -d), n - max(0, d)
        return slice(lo, hi), slice(lo + d, hi + d)

    (zo, zi), (yo, yi), (xo, xi) = rng(nz, dz), rng(ny, dy), rng(nx, dx)
    out[zo, yo, xo] = a[zi, yi, xi]
    return out


def conv_forward(x: np.ndarray, w: np.ndarray) -> np.ndarray:
    """y[c, co] = sum over taps t and input channels ci of x[c + off_t, ci] w[t, ci, co],
    zero padding (a cross-correlation, the convention of CNN layers)."""
    y = np.zeros(x.shape[:3] + (w.shape[2],))
    for t, (dz, dy, dx) in enumerate(TAPS):
        y += shift0(x, dz, dy, dx) @ w[t]
    return y


def conv_backward_data(dy: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of conv_forward in x: dx[c, ci] = sum_t sum_co w[t, ci, co] dy[c - off_t, co]."""
    dx = np.zeros(dy.shape[:3] + (w.shape[1],))
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        dx += shift0(dy, -dz, -dyy, -dxx) @ w[t].T
    return dx


def conv_backward_weight(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """Gradient in w: dw[t, ci, co] = sum_c x[c + off_t, ci] dy[c, co]."""
    ci, co = x.shape[3], dy.shape[3]
    dw = np.zeros((27, ci, co))
    dyf = dy.reshape(-1, co)
    for t, (dz, dyy, dxx) in enumerate(TAPS):
        dw[t] = shift0(x, dz, dyy, dxx).reshape(-1, ci).T @ dyf
    return dw


# ------------------------------------------------------------------ network

def hsig(v):
    """Gate nonlinearity: v/4 + 1/2 clamped to [0, 1]."""
    return np.clip(0.25 * v + 0.5, 0.0, 1.0)


def hsig_slope(G):
    """d hsig / dv expressed through the gate value: 1/4 strictly inside (0, 1), 0 where
    the clamp is active (at the kinks the one-sided slope of the clamp is taken)."""
    return np.where((G > 0.0) & (G < 1.0), 0.25, 0.0)


def forward(x: np.ndarray, g: np.ndarray, ws: list, bf16: bool = False):
    """net(x) = K^T K x (x, g: (nz, ny, nx)).  Returns (y, saved) with saved the
    activations the backward pass needs.  With bf16=True the input, the gate and
    every stored activation are rounded to bfloat16 and the weights taken as their
    bfloat16 values; sums are FP64 (exact products)."""
    rnd = bf16_round if bf16 else (lambda v: v)
    W1, W2, Wg = (rnd(w) for w in ws)
    x1 = rnd(x)[..., None]
    g1 = rnd(g)[..., None]
    G = rnd(hsig(conv_forward(g1, Wg)))
    u1 = conv_forward(x1, W1)
    a1 = rnd(u1 * G)
    y = rnd(conv_forward(a1, W2))
    v = conv_backward_data(y, W2)
    b = rnd(v * G)
    out = conv_backward_data(b, W1)[..., 0]
    saved = {"x": x1, "g": g1, "G": G, "u1": rnd(u1), "a1": a1, "y": y, "v": rnd(v), "b": b}
    return out, saved


def backward(saved: dict, ws: list, dy: np.ndarray, bf16: bool = False):
    """Gradients of a scalar J with dJ/d(net output) = dy (nz, ny, nx): returns
    (dws, dx, dg) with dws = [dW1, dW2, dWg] and dx, dg the gradients in the two
    inputs.  With bf16=True every backward signal is rounded to bfloat16 before it
    meets weights or activations, as on the GPU."""
    rnd = bf16_round if bf16 else (lambda v: v)
    W1, W2, Wg = (rnd(w) for w in ws)
    G = saved["G"]
    go = rnd(dy[..., None])
    # out = W1^T * b
    dW1 = conv_backward_weight(go, saved["b"])
    db = conv_forward(go, W1)
    # b = v . G
    dv = rnd(db * G)
    dG = db * saved["v"]
    # v = W2^T * y
    dW2 = conv_backward_weight(dv, saved["y"])
    dyy = rnd(conv_forward(dv, W2))
    # y = W2 * a1
    dW2 = dW2 + conv_backward_weight(saved["a1"], dyy)
    da1 = conv_backward_data(dyy, W2)
    # a1 = u1 . G
    du1 = rnd(da1 * G)
    dG = dG + da1 * saved["u1"]
    # u1 = W1 * x
    dW1 = dW1 + conv_backward_weight(saved["x"], du1)
    dx = conv_backward_data(du1, W1)[..., 0]
    # G = hsig(Wg * g)
    dpre = rnd(dG * hsig_slope(G))
    dWg = conv_backward_weight(saved["g"], dpre)
    dg = conv_backward_data(dpre, Wg)[..., 0]
    return [dW1, dW2, dWg], dx, dg


# ------------------------------------------------------------------ preconditioner

def geometry_channel(st: flow.Stencil) -> np.ndarray:
    """Fraction of the six faces of each cell that are open pressure faces."""
    n = np.zeros(st.grid.shape)
    for d in range(6):
        n += flow.open_face(st, d)
    return n / 6.0


def jacobi_inverse(st: flow.Stencil) -> np.ndarray:
    dg = flow.jacobi_diag(st)
    return np.divide(1.0, dg, out=np.zeros_like(dg), where=dg > 0)


def rms(r: np.ndarray) -> float:
    return float(np.sqrt(np.sum(r * r) / r.size))


def precondition(st: flow.Stencil, r: np.ndarray, ws: list, bf16: bool = False, omega: float = 0.0) -> np.ndarray:
    """z = D^-1 r + s net(r/s), s = RMS(r); z = 0 for r = 0.  omega > 0: that map M
    between two damped Jacobi steps S = omega D^-1, z1 = S r, z2 = z1 + M(r - A z1),
    z = z2 + S(r - A z2)."""
    if omega > 0.0:
        sm = omega * jacobi_inverse(st)
        z1 = sm * r
        z2 = z1 + precondition(st, r - apply_A(st, z1), ws, bf16)
        return z2 + sm * (r - apply_A(st, z2))
    s = rms(r)
    if s == 0.0:
        return np.zeros_like(r)
    y, _ = forward(r / s, geometry_channel(st), ws, bf16)
    return jacobi_inverse(st) * r + s * y


def apply_A(st: flow.Stencil, v: np.ndarray) -> np.ndarray:
    """The symmetric positive (semi-)definite pressure operator A = -L."""
    return -flow.laplacian(st, v)


def loss_and_grad(st: flow.Stencil, b: np.ndarray, p: np.ndarray, ws: list, bf16: bool = False,
                  omega: float = 0.0):
    """Scale-invariant A-norm loss of the preconditioned right-hand side for the pair
    (b, p), L p = b, and its gradient in the weights.  omega > 0: the preconditioner is
    the smoothed form of `precondition`, so the network sees r1 = f - A S f and its
    output reaches p_hat through (I - S A).  Returns (loss, dws)."""
    f = -b
    jinv = jacobi_inverse(st)
    if omega > 0.0:
        sm = omega * jinv
        t = sm * f
        r_in = f - apply_A(st, t)
    else:
        r_in = f
    s = rms(r_in)
    y, saved = forward(r_in / s, geometry_channel(st), ws, bf16)
    ph = jinv * r_in + s * y
    if omega > 0.0:
        z2 = t + ph
        ph = z2 + sm * (f - apply_A(st, z2))
    q = apply_A(st, ph)
    c = float(np.sum(f * ph))
    Q = float(np.sum(ph * q))
    B = float(np.sum(f * p))
    loss = 1.0 - c * c / (B * Q)
    # d loss / d p_hat = (2c/(BQ)) ((c/Q) A p_hat - f), chained through p_hat = ... + s y
    # (with the smoothing, p_hat = ... + (I - S A) s y, whose adjoint is I - A S)
    gph = (2.0 * c / (B * Q)) * ((c / Q) * q - f)
    if omega > 0.0:
        gph = gph - apply_A(st, sm * gph)
    dws, _, _ = backward(saved, ws, s * gph, bf16)
    return loss, dws


def loss_only(st, b, p, ws, bf16=False, omega: float = 0.0) -> float:
    f = -b
    ph = precondition(st, f, ws, bf16, omega)
    c = float(np.sum(f * ph))
    Q = float(np.sum(ph * apply_A(st, ph)))
    return 1.0 - c * c / (float(np.sum(f * p)) * Q)


def adam(w: np.ndarray, g: np.ndarray, m: np.ndarray, v: np.ndarray, t: int, lr: float,
         b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (step count t starting at 1) of the flat arrays; returns (w, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v


# ------------------------------------------------------------------ flexible CG

def fcg(st: flow.Stencil, b: np.ndarray, x0: np.ndarray, precond, tol: float, max_iter: int):
    """Flexible conjugate gradients FCG(1) on A x = -b (A = -L), warm start x0.

    Iteration: z = M(r); beta = <z, r - r_prev> / <z_prev, r_prev> (zero on the first
    iteration); d = z + beta d; alpha = <z, r> / <d, A d>; x += alpha d; r -= alpha A d.
    Stops at |r|_2 <= tol |b|_2 on the recursive residual.  Returns (x, iters)."""
    f = -b
    fn = np.sqrt(np.sum(f * f))
    if fn == 0.0:
        return np.zeros_like(x0), 0
    x = x0.copy()
    r = f - apply_A(st, x)
    it = 0
    d = None
    zr_prev = r_prev = None
    while np.sqrt(np.sum(r * r)) > tol * fn and it < max_iter:
        z = precond(r)
        zr = float(np.sum(z * r))
        if d is None:
            d = z.copy()
        else:
            beta = float(np.sum(z * (r - r_prev))) / zr_prev
            d = z + beta * d
        q = apply_A(st, d)
        alpha = zr / float(np.sum(d * q))
        x = x + alpha * d
        r_prev = r
        r = r - alpha * q
        zr_prev = zr
        it += 1
    return x, it

