"""Pins of the FP64 surrogate network of the oracle (oracle.mlp) against what mathematics fixes:
central differences of the loss, textbook values of the normal CDF, the odd-part identity of GELU,
Adam's closed form under a constant gradient, the feature normalisation, and bfloat16 rounding
against an independent conversion."""
import numpy as np
import pytest

import vxinputs
from oracle import mlp as M


def small_problem(seed=0, n=12):
    rng = np.random.default_rng(seed)
    P = vxinputs.mlp_init(seed + 7)
    for k in ("b1", "b2", "b3"):
        P[k] = rng.normal(0, 0.3, P[k].shape)
    P["W3"] = P["W3"] * 10.0  # outputs of order 1 so that both confidence targets occur
    X = rng.normal(size=(n, 128))
    Z3 = M.forward(P, X)["Z3"]
    T = Z3[:, :3] + rng.normal(0, 0.2, (n, 3))
    T[: n // 2] = Z3[: n // 2, :3] + 0.005  # half the samples within the confidence tolerance
    return P, X, T


@pytest.mark.parametrize("lam", [0.0, 0.3])
def test_gradient_central_differences(lam):
    P, X, T = small_problem()
    loss, G, y = M.loss_grad(P, X, T, lam=lam, tol=0.02)
    assert 0 < y.sum() < len(y)
    rng = np.random.default_rng(3)
    h = 1e-6
    for name in M.NAMES:
        idx = [tuple(rng.integers(0, s) for s in P[name].shape) for _ in range(12)]
        fd, an = [], []
        for i in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[name][i] += h
            Pm[name][i] -= h
            lp = M.loss_grad(Pp, X, T, lam=lam, tol=0.02, y=y)[0]
            lm = M.loss_grad(Pm, X, T, lam=lam, tol=0.02, y=y)[0]
            fd.append((lp - lm) / (2 * h))
            an.append(G[name][i])
        fd, an = np.array(fd), np.array(an)
        rel = np.linalg.norm(fd - an) / max(np.linalg.norm(an), 1e-300)
        assert rel <= 1e-6, (name, rel)


def test_gelu_values_and_identities():
    # gelu(x) = x Phi(x); Phi(1) and Phi(2) from tables of the standard normal CDF
    assert M.gelu(np.float64(1.0)) == pytest.approx(0.8413447460685429, abs=1e-15)
    assert M.gelu(np.float64(2.0)) == pytest.approx(2 * 0.9772498680518208, abs=1e-15)
    assert M.gelu(np.float64(0.0)) == 0.0
    x = np.linspace(-6, 6, 241)
    # Phi(x) + Phi(-x) = 1  =>  gelu(x) - gelu(-x) = x
    assert np.abs(M.gelu(x) - M.gelu(-x) - x).max() < 1e-14
    assert M.gelu(np.float64(40.0)) == 40.0 and abs(M.gelu(np.float64(-40.0))) < 1e-300
    h = 1e-6
    fd = (M.gelu(x + h) - M.gelu(x - h)) / (2 * h)
    assert np.abs(fd - M.gelu_grad(x)).max() < 1e-8
    assert M.gelu_grad(np.float64(0.0)) == 0.5


def test_adam_closed_form():
    rng = np.random.default_rng(5)
    P = {"w": rng.normal(size=50)}
    g = {"w": rng.normal(size=50)}
    Mo = {"w": np.zeros(50)}
    V = {"w": np.zeros(50)}
    lr, eps = 1e-3, 1e-8
    w0 = P["w"].copy()
    for t in range(1, 6):
        P, Mo, V = M.adam(P, g, Mo, V, t, lr, eps=eps)
        # with a constant gradient the bias-corrected moments are exactly g and g^2
        step = lr * g["w"] / (np.abs(g["w"]) + eps)
        assert np.abs(P["w"] - (w0 - t * step)).max() < 1e-12


def test_features():
    rng = np.random.default_rng(8)
    re, im = rng.normal(size=(4, 4, 4)), rng.normal(size=(4, 4, 4))
    f = M.features(re, im)
    assert f.shape == (128,)
    assert (f * f).sum() == pytest.approx(64.0, rel=1e-12)  # mean |psi|^2 normalised to 1
    assert np.allclose(M.features(3.7 * re, 3.7 * im), f, rtol=0, atol=1e-14)
    th = 0.83  # a global phase rotates every (Re, Im) pair by the same angle
    c, s = np.cos(th), np.sin(th)
    g = M.features(c * re - s * im, s * re + c * im)
    assert np.allclose(g[0::2], c * f[0::2] - s * f[1::2], atol=1e-13)
    assert np.allclose(g[1::2], s * f[0::2] + c * f[1::2], atol=1e-13)
    assert f[2 * (1 + 4 * 2 + 16 * 3)] == pytest.approx(re[3, 2, 1] / np.sqrt(np.mean(re ** 2 + im ** 2)))
    assert not M.features(np.zeros(64), np.zeros(64)).any()


def test_first_estimate():
    assert np.allclose(M.first_estimate(0b01 | 0b11 << 2), [0.5, 0.5, 0.5])  # -x and +x pierced
    assert np.allclose(M.first_estimate(0b01 | 0b11 << 6), [0.25, 0.75, 0.5])  # -x and +y
    assert np.allclose(M.first_estimate(0b01 << 8 | 0b11 << 10), [0.5, 0.5, 0.5])  # -z and +z
    assert np.allclose(M.first_estimate(0), [0.5, 0.5, 0.5])


def test_bf16_rounding():
    import torch
    one = 1.0
    assert M.bf16(np.array([one + 2.0 ** -8]))[0] == 1.0  # tie to even
    assert M.bf16(np.array([one + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie to even, upwards
    assert M.bf16(np.array([one + 2.0 ** -8 + 2.0 ** -20]))[0] == 1.0 + 2.0 ** -7
    x = np.random.default_rng(9).normal(size=10000) * np.exp(np.random.default_rng(10).uniform(-20, 20, 10000))
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M.bf16(x), ref)


def test_polish_linear_field_lands_on_the_line():
    """For linear psi = a.(x-p) + i b.(x-p) the trilinear patch is exact and one Newton step from any
    point of the plane reaches the plane's intersection with the nodal line p + s (a x b)."""
    rng = np.random.default_rng(21)
    for trial in range(20):
        a, b = rng.normal(size=3), rng.normal(size=3)
        p = rng.uniform(0.2, 0.8, 3)
        idx = np.arange(4) - 1.0
        zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
        X = np.stack([xx, yy, zz], -1) - p
        re, im = X @ a, X @ b
        desc = 0b01 | 0b11 << 2  # -x and +x faces: x0 = cell centre
        start = np.array([0.5, 0.5, 0.5]) + rng.normal(0, 0.3, 3)
        res = M.polish(re, im, desc, start)
        assert res is not None
        x, rho = res
        t = np.cross(a, b)
        t /= np.linalg.norm(t)
        # on the nodal line, and in the plane through x0 normal to t
        assert abs(a @ (x - p)) < 1e-12 and abs(b @ (x - p)) < 1e-12
        assert abs((x - np.array([0.5, 0.5, 0.5])) @ t) < 1e-12
        assert rho < 1e-24


def test_polish_degenerate_cases():
    re = np.zeros((4, 4, 4))
    im = np.zeros((4, 4, 4))
    assert M.polish(re, im, 0b01 | 0b11 << 2, [0.5, 0.5, 0.5]) is None  # no pseudo-vorticity


def test_newton_step_estimates_the_distance_to_the_core():
    """For linear psi the Newton step from any point of the plane is exact, so its length is the
    distance to the core's point in the plane; the acceptance bound of the polish then rejects
    exactly the starts whose step is longer than max_step (here on a field with a bilinear term,
    where one Newton step does not land exactly and the following step is the remaining error)."""
    rng = np.random.default_rng(22)
    idx = np.arange(4) - 1.0
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    for trial in range(20):
        a, b = rng.normal(size=3), rng.normal(size=3)
        p = rng.uniform(0.3, 0.7, 3)
        X = np.stack([xx, yy, zz], -1) - p
        re, im = X @ a, X @ b
        x0 = np.array([0.5, 0.5, 0.5])
        t = np.cross(a, b)
        t /= np.linalg.norm(t)
        u = np.zeros(3)
        u[int(np.argmin(np.abs(t)))] = 1
        e1 = np.cross(t, u)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(t, e1)
        core = p + ((x0 - p) @ t) * t  # the nodal line's point in the plane through x0
        y = rng.normal(0, 0.3, 2)
        x = x0 + y[0] * e1 + y[1] * e2
        assert abs(M.newton_step(re, im, e1, e2, x) - np.linalg.norm(x - core)) < 1e-12
    # bilinear term: psi = (x - 1/2) + i (y - 1/2) + 0.4 (x - 1/2)(y - 1/2); z-line through the centre
    re = (xx - 0.5) + 0.4 * (xx - 0.5) * (yy - 0.5)
    im = (yy - 0.5) + 0 * zz
    desc = 0b01 << 8 | 0b01 << 10  # -z and +z faces pierced (winding +1): x0 = centre, plane z = 1/2
    start = np.array([0.8, 0.25, 0.5])
    x, rho, nxt = M.polish(re, im, desc, start, with_step=True)
    assert abs(x[2] - 0.5) < 1e-15 and nxt > 1e-4 and rho > 0
    assert M.polish(re, im, desc, start, max_step=0.5 * nxt) is None
    x2, rho2 = M.polish(re, im, desc, start, max_step=2 * nxt)
    assert np.array_equal(x2, x)
    # the step after the polish estimates the remaining distance to the core at (1/2, 1/2, 1/2)
    assert 0.5 < nxt / np.linalg.norm(x - 0.5) < 2.0
