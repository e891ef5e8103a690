"""Pins of the oracle's core-sample refinement (arXiv 1911.12070, Sec. 3.3.3).

The refinement minimises the density |psi|^2 -- zero on a vortex core -- in the plane through the
mean-position estimate x0 normal to the pseudo-vorticity direction, with psi linearly
interpolated between nodes (Sec. 5). Checks:
  * closed form: for psi linear in x, trilinear interpolation is exact, the core is the line
    through p along a x b, the pseudo-vorticity is a x b, so x* is the projection of x0 on it;
  * symmetry: a straight core through a cell centre is found exactly there;
  * metamorphic: invariance under psi -> c psi and psi -> conj(psi), covariance under the cube's
    axis permutations and reflections;
  * the paper's claims: |psi(x*)|^2 ~ 0 where |psi(x0)|^2 is not (Sec. 3.3.3), and x* lies within
    about one cell of x0 (the estimator's one-cell uncertainty, Sec. 3.3.1);
  * brute force: x* is the zero of psi in the plane nearest to x0 (the "nearest point on the
    core line" of Sec. 3.3.3) on nearly all samples.
"""
import itertools

import numpy as np
import pytest

import oracle
import vxinputs

IDX = np.arange(4) - 1.0  # local node coordinates of a patch


def patch_from_function(fn):
    z, y, x = np.meshgrid(IDX, IDX, IDX, indexing="ij")
    v = fn(x, y, z)
    return v.real.copy(), v.imag.copy()


def desc_of_patch(re, im):
    """Cell descriptor of the patch's central cell from the oracle's winding of its 8 corners."""
    sub = (re + 1j * im)[1:3, 1:3, 1:3].astype(np.complex64)
    _, _, cdesc = oracle.winding_box(sub, (1 << 20, 1 << 20, 1 << 20), (0, 0, 0), periodic=7)
    return int(cdesc[0, 0, 0])


def x0_of_desc(desc):
    ctr = np.array([[0, .5, .5], [1, .5, .5], [.5, 0, .5], [.5, 1, .5], [.5, .5, 0], [.5, .5, 1]])
    faces = [f for f in range(6) if (desc >> (2 * f)) & 3]
    return ctr[faces].mean(0)


def test_linear_field_closed_form():
    rng = np.random.default_rng(1)
    done = 0
    for _ in range(200):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        p = rng.uniform(0.3, 0.7, 3)
        scale = 10 ** rng.uniform(-3, 1)
        re, im = patch_from_function(lambda x, y, z: scale * (
            a[0] * (x - p[0]) + a[1] * (y - p[1]) + a[2] * (z - p[2]) +
            1j * (b[0] * (x - p[0]) + b[1] * (y - p[1]) + b[2] * (z - p[2]))))
        d = desc_of_patch(re, im)
        if d == 0:
            continue
        t = np.cross(a, b)
        t /= np.linalg.norm(t)
        x0 = x0_of_desc(d)
        expect = p + np.dot(x0 - p, t) * t
        x, rho, it, st = oracle.refine_patch(re, im, d)
        if st & oracle.BOUNDARY:
            continue
        assert np.abs(x - expect).max() < 1e-12, (x, expect, st)
        assert st & ~(oracle.MULTI | oracle.BOUNDARY) == 0
        assert rho < 1e-24 * max(scale, 1) ** 2
        done += 1
    assert done > 150


def test_core_through_cell_centre():
    for prof in (lambda d: d / np.sqrt(d * d + 2.0), lambda d: np.tanh(d), lambda d: d):
        def fn(x, y, z):
            dx, dy = x - 0.5, y - 0.5
            d = np.sqrt(dx * dx + dy * dy)
            with np.errstate(invalid="ignore", divide="ignore"):
                ph = np.where(d > 0, (dx + 1j * dy) / np.where(d > 0, d, 1), 0)
            return prof(d) * ph * np.exp(0.3j * z)
        re, im = patch_from_function(fn)
        d = desc_of_patch(re, im)
        x, rho, it, st = oracle.refine_patch(re, im, d)
        assert np.abs(x - 0.5).max() < 1e-14
        assert rho < 1e-28


def _tangle_samples(seed=3, dims=(48, 48, 48), nw=128, shell=(3, 7), limit=400):
    t = vxinputs.make_tangle(dims, nw, shell, seed)
    psi = vxinputs.eval_tangle(t)
    W = oracle.winding(psi)
    sel = np.arange(min(limit, len(W.cells)))
    return psi, W.cells[sel], W.cdesc[sel]


def test_paper_claims_density_and_distance():
    psi, cells, cdesc = _tangle_samples()
    S = oracle.refine(psi, cells, cdesc)
    ok = (S.status & (oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.NO_FACES)) == 0
    assert ok.mean() > 0.97
    assert (S.rho[ok] < 1e-10).all()
    # the density at the initial estimate is far from zero
    rho0 = []
    for c, d in zip(cells, cdesc):
        re, im = oracle.gather_patch(psi, int(c))
        v, _ = oracle.trilerp(re, im, x0_of_desc(int(d)))
        rho0.append(abs(v) ** 2)
    rho0 = np.array(rho0)
    assert np.median(rho0) > 1e4 * np.median(S.rho[ok] + 1e-300)
    # one-cell uncertainty of the mean estimate
    dist = np.array([np.linalg.norm(S.x[s] - x0_of_desc(int(cdesc[s]))) for s in range(len(cells))])
    assert np.percentile(dist[ok], 99) < 1.0


def _transform_patch(re, im, perm, flips):
    """Apply x_a -> x_perm[a] (then reflect about the cell centre where flips[a])."""
    v = re + 1j * im  # indexed [z][y][x]
    v = np.transpose(v, axes=[2 - perm[2 - q] for q in range(3)]) if perm != (0, 1, 2) else v
    for a in range(3):
        if flips[a]:
            v = np.flip(v, axis=2 - a)
    return v.real.copy(), v.imag.copy()


def _transform_point(x, perm, flips):
    y = np.empty(3)
    for a in range(3):
        y[a] = x[perm[a]]
    for a in range(3):
        if flips[a]:
            y[a] = 1.0 - y[a]
    return y


def test_metamorphic_invariance_and_covariance():
    psi, cells, cdesc = _tangle_samples(seed=4, limit=60)
    base_bad = oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.BOUNDARY | oracle.TANGENT_FALLBACK
    rng = np.random.default_rng(5)
    checked = 0
    for c, d in zip(cells, cdesc):
        re, im = oracle.gather_patch(psi, int(c))
        x, rho, it, st = oracle.refine_patch(re, im, int(d))
        if st & base_bad:
            continue
        # psi -> c psi, psi -> conj(psi)
        cc = complex(*rng.standard_normal(2)) * 10 ** rng.uniform(-2, 2)
        v = (re + 1j * im) * cc
        x2, *_ = oracle.refine_patch(v.real, v.imag, desc_of_patch(v.real, v.imag))
        assert np.abs(x2 - x).max() < 1e-9
        x3, *_ = oracle.refine_patch(re, -im, desc_of_patch(re, -im))
        assert np.abs(x3 - x).max() < 1e-9
        # axis permutations and reflections of the cube
        for perm in itertools.permutations(range(3)):
            flips = tuple(int(f) for f in rng.integers(0, 2, 3))
            r2, i2 = _transform_patch(re, im, perm, flips)
            x4, _, _, st4 = oracle.refine_patch(r2, i2, desc_of_patch(r2, i2))
            assert np.abs(x4 - _transform_point(x, perm, flips)).max() < 1e-9, (perm, flips)
        checked += 1
    assert checked > 30


def _plane(re, im, desc):
    """Plane of the sample (same construction as the oracle): x0, e1, e2."""
    x0 = x0_of_desc(desc)
    v, g = oracle.trilerp(re, im, x0)
    t = np.cross(g.real, g.imag)
    t /= np.linalg.norm(t)
    u = int(np.argmin(np.abs(t)))
    eu = np.zeros(3)
    eu[u] = 1
    e1 = np.cross(t, eu)
    e1 /= np.linalg.norm(e1)
    return x0, e1, np.cross(t, e1)


def test_bruteforce_nearest_zero():
    psi, cells, cdesc = _tangle_samples(seed=6, limit=120)
    agree = total = 0
    for c, d in zip(cells, cdesc):
        re, im = oracle.gather_patch(psi, int(c))
        x, rho, it, st = oracle.refine_patch(re, im, int(d))
        if st & (oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.TANGENT_FALLBACK | oracle.MULTI):
            continue
        x0, e1, e2 = _plane(re, im, int(d))
        zeros = []
        for s1 in np.linspace(-2.0, 2.0, 17):
            for s2 in np.linspace(-2.0, 2.0, 17):
                y = np.array([s1, s2])
                for _ in range(40):
                    p = x0 + y[0] * e1 + y[1] * e2
                    if not ((p >= -1).all() and (p <= 2).all()):
                        break
                    v, g = oracle.trilerp(re, im, p)
                    J = np.array([[e1 @ g.real, e2 @ g.real], [e1 @ g.imag, e2 @ g.imag]])
                    if abs(np.linalg.det(J)) < 1e-300:
                        break
                    y = y - np.linalg.solve(J, [v.real, v.imag])
                else:
                    p = x0 + y[0] * e1 + y[1] * e2
                    v, _ = oracle.trilerp(re, im, p)
                    if (p >= -1).all() and (p <= 2).all() and abs(v) < 1e-9:
                        if not any(np.linalg.norm(p - z) < 1e-6 for z in zeros):
                            zeros.append(p)
        if not zeros:
            continue
        nearest = min(zeros, key=lambda z: np.linalg.norm(z - x0))
        total += 1
        agree += np.linalg.norm(nearest - x) < 1e-6
    assert total > 60
    assert agree / total > 0.95, (agree, total)


# ---------------------------------------------------------------- tangent fallback (Sec. 3.3.3)
# The pseudo-vorticity grad Re psi x grad Im psi gives the line direction wherever it is not
# degenerate. The cases below are fields built from node values whose trilinear interpolation is
# the stated polynomial exactly (only products of distinct coordinates appear), chosen so that the
# pseudo-vorticity vanishes at x0 while the cell is pierced: the refinement then has to use the
# cell's face flux, or the first pierced face's normal when the flux cancels.

def _plain_trilerp(re, im, x):
    """Trilinear value of a 4x4x4 patch at x (independent of the oracle's evaluation)."""
    c = np.clip(np.floor(x), -1, 1).astype(int)
    u = x - c
    v = 0j
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                w = (u[0] if dx else 1 - u[0]) * (u[1] if dy else 1 - u[1]) * (u[2] if dz else 1 - u[2])
                q = (c[2] + 1 + dz, c[1] + 1 + dy, c[0] + 1 + dx)
                v += w * (re[q] + 1j * im[q])
    return v


def _faces_of(desc):
    out = []
    for f in range(6):
        v = (desc >> (2 * f)) & 3
        out.append(1 if v == 1 else (-1 if v == 3 else 0))
    return out


@pytest.mark.parametrize("px", [0.3125, 0.71875, 0.1])
def test_tangent_fallback_face_flux_plane(px):
    # Re psi = x - px, Im psi = (3/4)(x - 1/2)(y - 1/2): a straight core along z at (px, 1/2);
    # grad Im psi = 0 at the cell centre, so grad Re x grad Im = 0 there
    re, im = patch_from_function(lambda x, y, z: (x - px) + 0.75j * (x - 0.5) * (y - 0.5) + 0 * z)
    d = desc_of_patch(re, im)
    f6 = _faces_of(d)
    assert f6[:4] == [0, 0, 0, 0] and f6[4] == f6[5] != 0  # pierced through -z and +z only
    x0 = x0_of_desc(d)
    assert np.array_equal(x0, [0.5, 0.5, 0.5])
    _, g = oracle.trilerp(re, im, x0)
    assert np.linalg.norm(np.cross(g.real, g.imag)) == 0.0
    x, rho, it, st = oracle.refine_patch(re, im, d)
    assert st & oracle.TANGENT_FALLBACK
    assert not st & (oracle.NONZERO_MIN | oracle.NOT_CONVERGED)
    # face flux (w_z(n) + w_z(n+ez)) e_z: the plane z = 1/2, whose only zero is (px, 1/2, 1/2)
    assert it > 0 and abs(x[2] - 0.5) < 1e-15
    assert np.abs(x - [px, 0.5, 0.5]).max() < 1e-12
    assert rho < 1e-24 and abs(_plain_trilerp(re, im, x)) < 1e-12


@pytest.mark.parametrize("eta,fallback", [(1e-9, True), (1e-7, True), (1e-5, False), (1e-3, False)])
def test_tangent_fallback_threshold(eta, fallback):
    # grad Re = (1, 0, 0), grad Im = (1/2, eta, 0) at the centre: |t| = eta against
    # 1e-6 |grad Re| |grad Im| = 5e-7; both planes are z = 1/2, with the zero at (5/16, 1/2, 1/2)
    px = 0.3125
    re, im = patch_from_function(lambda x, y, z: (x - px) + 1j * (
        0.5 * (x - px) + 0.75 * (x - 0.5) * (y - 0.5) + eta * (y - 0.5)) + 0 * z)
    d = desc_of_patch(re, im)
    x, rho, it, st = oracle.refine_patch(re, im, d)
    assert bool(st & oracle.TANGENT_FALLBACK) == fallback
    assert np.abs(x - [px, 0.5, 0.5]).max() < 1e-12


@pytest.mark.parametrize("y1,gam,kap", [(0.55, 0.25, 2 ** -5), (0.45, 0.25, -2 ** -5), (0.5625, -0.5, 2 ** -4)])
def test_tangent_fallback_first_face_normal(y1, gam, kap):
    # Re psi = y - y1, Im psi = (x - 1/2)(z - 1/2) - kap + gam (y - 1/2): the zero set is a
    # hyperbola in the plane y = y1 that crosses the faces -x, +x, -z, +z; the x and z fluxes
    # cancel, grad Re || grad Im at the centre. The direction is then the first pierced face's
    # normal (-x): the plane x = 1/2, on which |psi|^2 depends on y alone and has no zero.
    re, im = patch_from_function(lambda x, y, z: (y - y1) + 1j * ((x - 0.5) * (z - 0.5) - kap + gam * (y - 0.5)))
    d = desc_of_patch(re, im)
    f6 = _faces_of(d)
    assert f6[0] != 0 and f6[1] != 0 and f6[4] != 0 and f6[5] != 0 and f6[2] == f6[3] == 0
    assert f6[0] + f6[1] == 0 and f6[4] + f6[5] == 0  # zero face flux on every axis
    x, rho, it, st = oracle.refine_patch(re, im, d)
    assert st & oracle.TANGENT_FALLBACK and st & oracle.MULTI and st & oracle.NONZERO_MIN
    assert x[0] == 0.5 and x[2] == 0.5  # stays in the plane x = 1/2 and on the line of steepest descent
    y_min = (y1 + gam * (kap + 0.5 * gam)) / (1 + gam * gam)  # minimiser of (y-y1)^2 + (gam(y-1/2)-kap)^2
    assert abs(x[1] - y_min) < 0.01
    ys = np.linspace(-1, 2, 3001)
    f_plane = [abs(_plain_trilerp(re, im, np.array([0.5, yy, 0.5]))) ** 2 for yy in ys]
    assert rho <= min(f_plane) + 1e-5


def test_seeded_refinement_closed_form_and_identity():
    """A caller's seed replaces the face-centre estimate: the face-centre estimate itself as seed gives
    the unseeded result bit for bit, and on a linear field (trilinear exact) the refined point from any
    seed is the seed's projection onto the nodal line along the pseudo-vorticity a x b."""
    rng = np.random.default_rng(31)
    psi, cells, cdesc = _tangle_samples(seed=8, limit=200)
    S = oracle.refine(psi, cells, cdesc)
    seeds = np.array([x0_of_desc(int(d)) for d in cdesc])
    T = oracle.refine(psi, cells, cdesc, seeds=seeds)
    assert np.array_equal(S.x, T.x) and np.array_equal(S.status, T.status)
    idx = np.arange(4) - 1.0
    zz, yy, xx = np.meshgrid(idx, idx, idx, indexing="ij")
    done = 0
    for _ in range(60):
        a, b = rng.standard_normal(3), rng.standard_normal(3)
        p = rng.uniform(0.3, 0.7, 3)
        X = np.stack([xx, yy, zz], -1) - p
        scale = 2.0 ** int(rng.integers(-3, 3))
        grid = (scale * (X @ a + 1j * (X @ b))).astype(np.complex128)
        # an open 4x4x4 grid holding just this patch: its cell (1, 1, 1) (id 21) is the patch's centre
        W = oracle.winding(grid.astype(np.complex64), 0)
        if 21 not in W.cells.tolist():
            continue
        i = W.cells.tolist().index(21)
        seed = rng.uniform(0.1, 0.9, 3)
        R = oracle.refine(grid.astype(np.complex64), W.cells[i:i + 1], W.cdesc[i:i + 1], periodic=0,
                          seeds=seed[None, :])
        if R.status[0] & (oracle.BOUNDARY | oracle.TANGENT_FALLBACK):
            continue
        # the FP32 node values are the exact linear field of the FP32-rounded coefficients: refit them
        vals = grid.astype(np.complex64).astype(np.complex128).reshape(-1)
        A = np.c_[xx.reshape(-1), yy.reshape(-1), zz.reshape(-1), np.ones(64)]
        cr = np.linalg.lstsq(A, vals.real, rcond=None)[0]
        ci = np.linalg.lstsq(A, vals.imag, rcond=None)[0]
        t = np.cross(cr[:3], ci[:3])
        t /= np.linalg.norm(t)
        # the nodal line: Re = Im = 0; its point closest to the seed along the plane normal to t
        M = np.array([cr[:3], ci[:3], t])
        expect = np.linalg.solve(M, [-cr[3], -ci[3], t @ seed])
        assert np.abs(R.x[0] - expect).max() < 1e-6, (R.x[0], expect)
        done += 1
    assert done > 20
