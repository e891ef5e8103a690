"""CPU ORACLE -- test infrastructure only: the surrogate network in plain FP64 NumPy.

The surrogate maps the 4x4x4 psi patch of a pierced cell to the offset of the refined core sample
from the cell's first estimate x0 (the mean of its pierced-face centres, Sec. 3.3.1), plus a
confidence. Every step is written out from its definition:

  features   q = a + 4 b + 16 c over the patch nodes (offsets a-1, b-1, c-1 from the cell's min
             corner, x fastest); s = sqrt(mean_q |psi_q|^2) (s = 1 if the patch is all zero);
             f[2q] = Re psi_q / s, f[2q+1] = Im psi_q / s                      (128 inputs)
  network    Z1 = X W1 + b1, H1 = gelu(Z1), Z2 = H1 W2 + b2, H2 = gelu(Z2), Z3 = H2 W3 + b3,
             W1: 128xH, W2: HxH, W3: Hx4 (rows = inputs; the hidden width H, 128 in the library,
             is read from the parameters); gelu(x) = x Phi(x) with
             Phi(x) = (1 + erf(x / sqrt 2)) / 2 (erf from the platform's math library)
  outputs    delta = Z3[:, 0:3] (predicted x* - x0, cell units), conf = sigmoid(Z3[:, 3])
  loss       mean over the batch of  |delta - t|^2 + lam * bce(Z3[:, 3], y),
             bce(z, y) = log(1 + exp(z)) - y z,  y = [max_a |delta_a - t_a| < tol] taken from the
             current prediction and held constant (no gradient through y)
  Adam       m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, w -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

It shares no code with the GPU library and never imports it.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def features(re: np.ndarray, im: np.ndarray) -> np.ndarray:
    """128 inputs from one 4x4x4 patch given as arrays indexed [c][b][a] (z, y, x)."""
    re = np.asarray(re, np.float64).reshape(64)
    im = np.asarray(im, np.float64).reshape(64)
    s = np.sqrt(np.mean(re * re + im * im))
    if s == 0.0:
        s = 1.0
    f = np.empty(128, np.float64)
    f[0::2] = re / s
    f[1::2] = im / s
    return f


def first_estimate(desc: int) -> np.ndarray:
    """Mean of the centres of the cell's pierced faces (-x, +x, -y, +y, -z, +z), cell-local; the
    cell centre when no face is pierced."""
    acc = np.zeros(3)
    n = 0
    for face in range(6):
        if (desc >> (2 * face)) & 3:
            c = np.full(3, 0.5)
            c[face >> 1] = face & 1
            acc += c
            n += 1
    return acc / n if n else np.full(3, 0.5)


def gelu(x):
    return x * 0.5 * (1.0 + erf(x / np.sqrt(2.0)))


def gelu_grad(x):
    phi = np.exp(-0.5 * x * x) / np.sqrt(2.0 * np.pi)
    return 0.5 * (1.0 + erf(x / np.sqrt(2.0))) + x * phi


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def forward(P: dict, X: np.ndarray) -> dict:
    Z1 = X @ P["W1"] + P["b1"]
    H1 = gelu(Z1)
    Z2 = H1 @ P["W2"] + P["b2"]
    H2 = gelu(Z2)
    Z3 = H2 @ P["W3"] + P["b3"]
    return dict(X=X, Z1=Z1, H1=H1, Z2=Z2, H2=H2, Z3=Z3)


def conf_targets(Z3: np.ndarray, T: np.ndarray, tol: float) -> np.ndarray:
    return (np.abs(Z3[:, :3] - T).max(axis=1) < tol).astype(np.float64)


def loss_grad(P: dict, X: np.ndarray, T: np.ndarray, lam: float = 0.1, tol: float = 0.25, y=None):
    """Mean loss over the batch and its gradient with respect to every parameter. y (the confidence
    targets) is computed from the forward pass unless given. Returns (loss, grads, y)."""
    n = X.shape[0]
    F = forward(P, X)
    Z3 = F["Z3"]
    if y is None:
        y = conf_targets(Z3, T, tol)
    d = Z3[:, :3] - T
    z = Z3[:, 3]
    bce = np.logaddexp(0.0, z) - y * z
    loss = float(np.mean((d * d).sum(axis=1) + lam * bce))
    dZ3 = np.empty_like(Z3)
    dZ3[:, :3] = 2.0 * d / n
    dZ3[:, 3] = lam * (sigmoid(z) - y) / n
    G = {"W3": F["H2"].T @ dZ3, "b3": dZ3.sum(axis=0)}
    dZ2 = (dZ3 @ P["W3"].T) * gelu_grad(F["Z2"])
    G["W2"] = F["H1"].T @ dZ2
    G["b2"] = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ P["W2"].T) * gelu_grad(F["Z1"])
    G["W1"] = X.T @ dZ1
    G["b1"] = dZ1.sum(axis=0)
    return loss, G, y


def adam(P: dict, G: dict, M: dict, V: dict, t: int, lr: float, b1: float = 0.9, b2: float = 0.999,
         eps: float = 1e-8):
    """One Adam step (t counts from 1). Returns new (P, M, V)."""
    Pn, Mn, Vn = {}, {}, {}
    for k in P:
        Mn[k] = b1 * M[k] + (1.0 - b1) * G[k]
        Vn[k] = b2 * V[k] + (1.0 - b2) * G[k] * G[k]
        mh = Mn[k] / (1.0 - b1 ** t)
        vh = Vn[k] / (1.0 - b2 ** t)
        Pn[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return Pn, Mn, Vn


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64 (finite inputs)."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def _plane(re, im, desc):
    """First estimate x0 and the in-plane basis (e1, e2) of the refinement at x0 (Sec. 3.3.3): t is
    grad Re psi x grad Im psi of the trilinear patch; e1 = t x u / |t x u| with u the axis of the
    smallest |t_i|, e2 = t x e1. None when t is degenerate (the refinement then uses the face
    flux; the surrogate leaves such cells to it)."""
    from . import trilerp
    x0 = first_estimate(desc)
    _, g = trilerp(re, im, x0)
    gr, gi = g.real, g.imag
    t = np.cross(gr, gi)
    tn = np.linalg.norm(t)
    if not (tn > 1e-6 * np.linalg.norm(gr) * np.linalg.norm(gi)) or tn == 0.0:
        return None
    t = t / tn
    u = np.zeros(3)
    u[int(np.argmin(np.abs(t)))] = 1.0
    e1 = np.cross(t, u)
    e1 /= np.linalg.norm(e1)
    return x0, e1, np.cross(t, e1)


def inside(x) -> bool:
    return bool(np.all(x >= -1.0) and np.all(x <= 2.0))


def newton_step(re, im, e1, e2, x):
    """Length of the Newton step on (Re psi, Im psi) in the plane (e1, e2) from x: |J^-1 psi(x)| with
    J the 2x2 in-plane Jacobian (inf if J is singular). Near a simple zero it estimates |x - zero|."""
    from . import trilerp
    v, g = trilerp(re, im, x)
    J = np.array([[e1 @ g.real, e2 @ g.real], [e1 @ g.imag, e2 @ g.imag]])
    det = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
    if det == 0.0:
        return 0.0 if v == 0 else np.inf
    dy = np.array([J[1, 1] * v.real - J[0, 1] * v.imag, -J[1, 0] * v.real + J[0, 0] * v.imag]) / det
    return float(np.hypot(dy[0], dy[1]))


def polish(re, im, desc: int, x_start, max_step: float = 0.0, with_step: bool = False):
    """The surrogate's final step: x_start (the network's point) projected onto the refinement's
    plane through x0, then one Newton step on (Re psi, Im psi) in that plane (the refinement's
    polish, Sec. 3.3.3 reading). Returns (x, |psi(x)|^2) (plus the length of the Newton step that
    would follow, if with_step), or None where the refinement must run instead: degenerate tangent,
    singular Jacobian, a point outside the patch, or -- max_step > 0 -- a following Newton step
    longer than max_step cells (the estimate of the polished point's distance from the zero)."""
    from . import trilerp
    pl = _plane(re, im, desc)
    if pl is None:
        return None
    x0, e1, e2 = pl
    d = np.asarray(x_start, np.float64) - x0
    y = np.array([d @ e1, d @ e2])
    xp = x0 + y[0] * e1 + y[1] * e2
    if not inside(xp):
        return None
    v, g = trilerp(re, im, xp)
    J = np.array([[e1 @ g.real, e2 @ g.real], [e1 @ g.imag, e2 @ g.imag]])
    det = J[0, 0] * J[1, 1] - J[0, 1] * J[1, 0]
    if det == 0.0:
        return None
    dy = -np.array([J[1, 1] * v.real - J[0, 1] * v.imag, -J[1, 0] * v.real + J[0, 0] * v.imag]) / det
    y = y + dy
    x = x0 + y[0] * e1 + y[1] * e2
    if not inside(x):
        return None
    v, _ = trilerp(re, im, x)
    rho = float(abs(v) ** 2)
    nxt = newton_step(re, im, e1, e2, x)
    if max_step > 0.0 and rho != 0.0 and not nxt <= max_step:
        return None
    return (x, rho, nxt) if with_step else (x, rho)
