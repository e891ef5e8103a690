"""Pins of the oracle's winding pass against what the paper and the mathematics fix.

The paper (arXiv 1911.12070, Sec. 2.2) identifies vortices by the circulation of the phase
gradient around a small closed path: |C| = 2 pi when the path encloses a core, 0 otherwise, the
sign giving the direction (right-hand rule, Sec. 3.4). The oracle evaluates it on every unit face
of the grid with an exact crossing-number predicate. These tests check it against:
  * hand-derived single faces (tests/golden/face_cases.txt);
  * exact rational winding numbers about q = (-2^-10, 2^-30) by quadrant walking (brute force);
  * the principal-value phase-sum form of the circulation (atan2, FP64) on non-degenerate faces;
  * exact invariants (zero net flux per cell, even pierced faces, zero slab sums);
  * a straight line and a ring whose windings are known in closed form.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import vxinputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ------------------------------------------------------------------ independent exact winding
def _quadrant(x: Fraction, y: Fraction) -> int:
    if x > 0 and y >= 0:
        return 0
    if x <= 0 and y > 0:
        return 1
    if x < 0 and y <= 0:
        return 2
    return 3


def exact_winding(poly, q=(Fraction(-1, 2 ** 10), Fraction(1, 2 ** 30))) -> int:
    """Winding number of a closed polygon about q by exact quadrant walking (no float)."""
    qx, qy = q
    pts = [(Fraction(float(z.real)) - qx, Fraction(float(z.imag)) - qy) for z in poly]
    quarter = 0
    for s in range(len(pts)):
        ax, ay = pts[s]
        bx, by = pts[(s + 1) % len(pts)]
        da = (_quadrant(bx, by) - _quadrant(ax, ay)) % 4
        if da == 1:
            quarter += 1
        elif da == 3:
            quarter -= 1
        elif da == 2:
            cr = ax * by - ay * bx
            assert cr != 0
            quarter += 2 if cr > 0 else -2
    assert quarter % 4 == 0
    return quarter // 4


def face_corners(psi, i, j, k, a):
    nz, ny, nx = psi.shape
    P = lambda x, y, z: psi[z % nz, y % ny, x % nx]
    if a == 0:
        return [P(i, j, k), P(i, j + 1, k), P(i, j + 1, k + 1), P(i, j, k + 1)]
    if a == 1:
        return [P(i, j, k), P(i, j, k + 1), P(i + 1, j, k + 1), P(i + 1, j, k)]
    return [P(i, j, k), P(i + 1, j, k), P(i + 1, j + 1, k), P(i, j + 1, k)]


# ------------------------------------------------------------------ golden hand-derived faces
def test_golden_faces():
    rows = []
    with open(os.path.join(GOLDEN, "face_cases.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if line:
                rows.append([float(v) for v in line.split()])
    assert len(rows) >= 8
    for r in rows:
        v = [complex(r[2 * q], r[2 * q + 1]) for q in range(4)]
        assert oracle.polygon(v) == int(r[8]), r
        assert exact_winding(v) == int(r[8]), r


def test_edge_antisymmetry_and_range():
    rng = np.random.default_rng(0)
    vals = rng.integers(-2, 3, size=(4000, 2, 2)).astype(np.float32)
    for a, b in vals:
        ca = oracle.edge(complex(*a), complex(*b))
        cb = oracle.edge(complex(*b), complex(*a))
        assert ca in (-1, 0, 1) and ca == -cb


# ------------------------------------------------------------------ brute force on tiny grids
@pytest.mark.parametrize("dims,seed", [((2, 2, 2), 1), ((3, 2, 4), 2), ((4, 4, 4), 3), ((3, 3, 3), 4)])
def test_bruteforce_tiny_periodic(dims, seed):
    psi = vxinputs.random_small_int_field(dims, seed)
    W = oracle.winding(psi, periodic=7)
    nx, ny, nz = dims
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for a in range(3):
                    assert W.w[k, j, i, a] == exact_winding(face_corners(psi, i, j, k, a))


def test_bruteforce_tiny_nonperiodic():
    dims = (4, 3, 3)
    for periodic in range(8):
        psi = vxinputs.random_small_int_field(dims, 10 + periodic)
        W = oracle.winding(psi, periodic=periodic)
        nx, ny, nz = dims
        per = [(periodic >> a) & 1 for a in range(3)]
        n = (nx, ny, nz)
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    c = (i, j, k)
                    for a in range(3):
                        others = [b for b in range(3) if b != a]
                        exists = all(per[b] or c[b] + 1 < n[b] for b in others)
                        expect = exact_winding(face_corners(psi, i, j, k, a)) if exists else 0
                        assert W.w[k, j, i, a] == expect


# ------------------------------------------------------------------ principal-value circulation
def circulation_atan2(poly) -> float:
    ph = np.angle(np.array(poly, np.complex128))
    d = np.diff(np.concatenate([ph, ph[:1]]))
    d = (d + np.pi) % (2 * np.pi) - np.pi
    return float(d.sum())


def test_against_phase_sum_on_smooth_fields():
    t = vxinputs.make_tangle((24, 20, 16), 96, (2, 5), seed=7)
    fields = [vxinputs.eval_tangle(t), vxinputs.eval_line_ring(vxinputs.line_ring_32())]
    checked = 0
    for psi in fields:
        W = oracle.winding(psi)
        nz, ny, nx = psi.shape
        for k in range(nz):
            for j in range(ny):
                for i in range(nx):
                    for a in range(3):
                        poly = face_corners(psi, i, j, k, a)
                        if min(abs(complex(z)) for z in poly) < 1e-6:
                            continue
                        C = circulation_atan2(poly)
                        # Sec. 2.2: |C| = 2 pi around a core, 0 otherwise; threshold pi
                        assert abs(abs(C) - 2 * np.pi) < 1e-9 or abs(C) < 1e-9
                        assert W.w[k, j, i, a] == (0 if abs(C) < np.pi else int(np.sign(C)))
                        checked += 1
    assert checked > 30000


# ------------------------------------------------------------------ exact invariants
def invariants(W, periodic=7):
    w = W.w.astype(np.int64)
    wx, wy, wz = w[..., 0], w[..., 1], w[..., 2]
    assert np.abs(w).max() <= 1
    if periodic == 7:
        flux = (np.roll(wx, -1, 2) - wx) + (np.roll(wy, -1, 1) - wy) + (np.roll(wz, -1, 0) - wz)
        assert not flux.any(), "net winding through a closed cell surface must vanish"
        npierced = ((np.roll(wx, -1, 2) != 0).astype(int) + (wx != 0) + (np.roll(wy, -1, 1) != 0) +
                    (wy != 0) + (np.roll(wz, -1, 0) != 0) + (wz != 0))
        assert (npierced % 2 == 0).all()
        assert not wz.sum(axis=(1, 2)).any()
        assert not wx.sum(axis=(0, 1)).any()
        assert not wy.sum(axis=(0, 2)).any()
        # packed field agrees with the windings and the pierced flag with the cell faces
        enc = lambda v: (v & 3).astype(np.uint8)
        pk = enc(wx) | (enc(wy) << 2) | (enc(wz) << 4) | ((npierced > 0).astype(np.uint8) << 6)
        assert np.array_equal(pk, W.packed)
        nz_, ny_, nx_ = wx.shape
        ids = np.nonzero(w.reshape(-1))[0]
        assert np.array_equal(W.faces, ids.astype(np.uint64))
        assert np.array_equal(W.fsign, w.reshape(-1)[ids].astype(np.int8))
        cells = np.nonzero((npierced > 0).reshape(-1))[0]
        assert np.array_equal(W.cells, cells.astype(np.uint64))


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_invariants_random_integer(seed):
    invariants(oracle.winding(vxinputs.random_small_int_field((6, 5, 7), seed)))


def test_invariants_tangle_and_line_ring():
    t = vxinputs.make_tangle((32, 32, 32), 128, (3, 6), seed=11)
    invariants(oracle.winding(vxinputs.eval_tangle(t)))
    invariants(oracle.winding(vxinputs.eval_line_ring(vxinputs.line_ring_32())))


def test_conjugation_flips_windings():
    t = vxinputs.make_tangle((20, 20, 20), 64, (3, 6), seed=12)
    psi = vxinputs.eval_tangle(t)
    W1 = oracle.winding(psi)
    W2 = oracle.winding(np.conj(psi))
    assert np.array_equal(W1.w, -W2.w)


# ------------------------------------------------------------------ line and ring (Sec. 2.2 / 3.4)
WIN = (3, 28)  # cells whose nodes stay >= 2 cells from the min-image seams of the 32^3 field


def _in_window(i, j, k):
    return all(WIN[0] <= c <= WIN[1] for c in (i, j, k))


def test_straight_line_winding():
    lr = vxinputs.line_ring_32()
    W = oracle.winding(vxinputs.eval_line_ring(lr))
    i0, j0 = int(np.floor(lr.line[0])), int(np.floor(lr.line[1]))
    for k in range(WIN[0], WIN[1] + 1):
        assert W.w[k, j0, i0, 2] == 1, k  # +1 about +z
        # the ring is horizontal (z = 16.47), so the only pierced xy-face in the window is the line's
        ks = W.w[k, WIN[0]:WIN[1] + 1, WIN[0]:WIN[1] + 1, 2]
        assert np.count_nonzero(ks) == 1


def test_ring_closed_cycle_and_sign():
    lr = vxinputs.line_ring_32()
    psi = vxinputs.eval_line_ring(lr)
    W = oracle.winding(psi)
    cx, cy, cz = lr.ring_center
    i0, j0 = int(np.floor(lr.line[0])), int(np.floor(lr.line[1]))
    nx = ny = 32
    ring_cells = []
    for c, d in zip(W.cells, W.cdesc):
        c = int(c)
        i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
        if not _in_window(i, j, k) or (i, j) == (i0, j0):
            continue
        ring_cells.append((i, j, k, int(d)))
    assert len(ring_cells) == 64
    assert all(k == int(np.floor(cz)) for _, _, k, _ in ring_cells)
    cellset = {(i, j, k) for i, j, k, _ in ring_cells}
    # every ring cell has exactly two pierced faces, shared with ring neighbours: one cycle
    nbr = {}
    for i, j, k, d in ring_cells:
        faces = [f for f in range(6) if (d >> (2 * f)) & 3]
        assert len(faces) == 2
        step = {0: (-1, 0, 0), 1: (1, 0, 0), 2: (0, -1, 0), 3: (0, 1, 0), 4: (0, 0, -1), 5: (0, 0, 1)}
        nbr[(i, j, k)] = [(i + step[f][0], j + step[f][1], k + step[f][2]) for f in faces]
        for q in nbr[(i, j, k)]:
            assert q in cellset
    start = next(iter(cellset))
    seen, prev, cur = {start}, None, start
    while True:
        nxt = [q for q in nbr[cur] if q != prev][0]
        if nxt == start:
            break
        assert nxt not in seen
        seen.add(nxt)
        prev, cur = cur, nxt
    assert len(seen) == 64
    # sign: -1 about the azimuthal direction e_phi
    for i, j, k, d in ring_cells:
        for f in range(6):
            v = (d >> (2 * f)) & 3
            if not v:
                continue
            w = 1 if v == 1 else -1
            a = f // 2
            fc = np.array([i + 0.5, j + 0.5, k + 0.5])
            fc[a] = (i, j, k)[a] + (f % 2)
            r = fc[:2] - np.array([cx, cy])
            ephi = np.array([-r[1], r[0], 0.0]) / np.linalg.norm(r)
            assert np.sign(ephi[a]) == -w


# ------------------------------------------------------------------ box evaluation = whole-grid pass
def _box_sub(psi, origin, size, periodic, rng):
    """Values of the box plus one node in each positive direction, wrapped on periodic axes;
    nodes past the end of an open axis get random values (they must never be read)."""
    nz, ny, nx = psi.shape
    x0, y0, z0 = origin
    bx, by, bz = size
    out = np.empty((bz + 1, by + 1, bx + 1), np.complex64)
    for k in range(bz + 1):
        for j in range(by + 1):
            for i in range(bx + 1):
                g = [x0 + i, y0 + j, z0 + k]
                outside = False
                for a, n in enumerate((nx, ny, nz)):
                    if g[a] >= n:
                        if (periodic >> a) & 1:
                            g[a] %= n
                        else:
                            outside = True
                if outside:
                    out[k, j, i] = complex(*rng.standard_normal(2))
                else:
                    out[k, j, i] = psi[g[2], g[1], g[0]]
    return out


def _small_int_field(rng, shape):
    vals = rng.integers(-2, 3, size=shape + (2,)).astype(np.float32)
    return (vals[..., 0] + 1j * vals[..., 1]).astype(np.complex64)


@pytest.mark.parametrize("periodic", range(8))
def test_winding_box_equals_whole_grid(periodic):
    """The box evaluation used by sampled checks of large grids gives, node for node, the face
    windings, packed bytes and cell descriptors of the whole-grid pass: whole grids, boxes inside,
    boxes that wrap the seams of periodic axes, for every combination of periodic axes, on
    small-integer fields (zeros and collinear values) and on smooth tangles."""
    rng = np.random.default_rng(100 + periodic)
    fields = [_small_int_field(rng, (5, 4, 6)), _small_int_field(rng, (3, 7, 2)),
              vxinputs.eval_tangle(vxinputs.make_tangle((12, 10, 9), 24, (1, 3), seed=7 + periodic))]
    for psi in fields:
        nz, ny, nx = psi.shape
        W = oracle.winding(psi, periodic)
        cdesc_full = np.zeros(psi.shape, np.uint16)
        cz, cy, cx = np.unravel_index(W.cells.astype(np.int64), psi.shape)
        cdesc_full[cz, cy, cx] = W.cdesc
        boxes = [((0, 0, 0), (nx, ny, nz))]
        for _ in range(4):
            size = tuple(int(rng.integers(1, n + 1)) for n in (nx, ny, nz))
            origin = []
            for a, (n, s) in enumerate(zip((nx, ny, nz), size)):
                hi = n - 1 if (periodic >> a) & 1 else n - s  # periodic boxes may run past the seam
                origin.append(int(rng.integers(0, hi + 1)))
            boxes.append((tuple(origin), size))
        for origin, size in boxes:
            sub = _box_sub(psi, origin, size, periodic, rng)
            w, packed, cdesc = oracle.winding_box(sub, (nx, ny, nz), origin, periodic)
            bx, by, bz = size
            zi = (origin[2] + np.arange(bz)) % nz
            yi = (origin[1] + np.arange(by)) % ny
            xi = (origin[0] + np.arange(bx)) % nx
            sel = np.ix_(zi, yi, xi)
            assert np.array_equal(packed, W.packed[sel]), (periodic, origin, size)
            assert np.array_equal(w, W.w[sel]), (periodic, origin, size)
            assert np.array_equal(cdesc, cdesc_full[sel]), (periodic, origin, size)
