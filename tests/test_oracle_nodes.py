"""Pins of the oracle's node-centred circulation (Sec. 2.2: the circulation around a ring through a
grid node in each coordinate plane, the largest |C| kept, vortex node where |C| > pi).

  * the ring's circulation / 2 pi, computed directly as the winding of the ring's 8-edge image
    polygon (the exact crossing rule, and exact rational quadrant walking), equals the sum of the
    four face windings the oracle uses -- on small-integer fields with zeros and collinear values,
    for every combination of periodic axes;
  * a straight line: exactly the four nodes around its pierced face in each plane are vortex nodes,
    with C = +2 pi in the line's plane (the four circulation paths around a core, Sec. 3.3.1);
  * conjugating psi reverses every circulation.
"""
import numpy as np
import pytest

import oracle
import vxinputs
from test_oracle_winding import exact_winding


def ring_vertices(n, a):
    """Nodes of the ring of node n (i, j, k) in the plane normal to axis a, counter-clockwise about
    +e_a: the boundary of the 2 x 2 faces around n."""
    u, v = {0: (1, 2), 1: (2, 0), 2: (0, 1)}[a]

    def off(du, dv):
        p = list(n)
        p[u] += du
        p[v] += dv
        return tuple(p)
    return [off(-1, -1), off(0, -1), off(1, -1), off(1, 0), off(1, 1), off(0, 1), off(-1, 1), off(-1, 0)]


def ring_winding(psi, verts, exact=False):
    nz, ny, nx = psi.shape
    vals = [psi[k % nz, j % ny, i % nx] for (i, j, k) in verts]
    if exact:
        return exact_winding([complex(v) for v in vals])
    return sum(oracle.edge(complex(vals[q]), complex(vals[(q + 1) % 8])) for q in range(8))


@pytest.mark.parametrize("periodic", range(8))
def test_ring_equals_sum_of_faces(periodic):
    rng = np.random.default_rng(200 + periodic)
    vals = rng.integers(-2, 3, size=(5, 4, 6, 2)).astype(np.float32)
    psi = (vals[..., 0] + 1j * vals[..., 1]).astype(np.complex64)
    nz, ny, nx = psi.shape
    W = oracle.winding(psi, periodic)
    C, node = oracle.node_circulation(W.w, periodic)
    dims = (nx, ny, nz)
    checked = 0
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                for a in range(3):
                    verts = ring_vertices((i, j, k), a)
                    # the ring exists whole only where every vertex is inside (or wraps around) the grid
                    if any(not (periodic >> b) & 1 and not 0 <= p[b] < dims[b] for p in verts for b in range(3)):
                        continue
                    r = ring_winding(psi, verts)
                    assert C[k, j, i, a] == r, (i, j, k, a)
                    if checked % 7 == 0:
                        assert r == ring_winding(psi, verts, exact=True)
                    checked += 1
    assert checked > 100
    # node bytes from their definition
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = C[k, j, i]
                m = np.abs(c)
                if m.max() == 0:
                    assert node[k, j, i] == 0
                    continue
                b = int(np.argmax(m))
                assert node[k, j, i] & 3 == min(m[b], 3)
                assert bool(node[k, j, i] & 4) == (c[b] < 0)
                assert (node[k, j, i] >> 3) & 3 == b and node[k, j, i] & 0x40


def test_straight_line_four_vortex_nodes_per_plane():
    nx, ny, nz = 9, 8, 6
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    psi = ((x - 3.3) + 1j * (y - 4.6)).astype(np.complex64)
    W = oracle.winding(psi, 0)
    C, node = oracle.node_circulation(W.w, 0)
    vortex = (node & 0x40) != 0
    expect = np.zeros_like(vortex)
    expect[:, 4:6, 3:5] = True  # the corners of the face at (3, 4) in every plane
    assert np.array_equal(vortex, expect)
    assert (C[expect][:, 2] == 1).all() and (C[..., :2] == 0).all()
    assert (node[expect] == (1 | (2 << 3) | 0x40)).all()


def test_conjugation_reverses_circulation():
    t = vxinputs.make_tangle((24, 20, 16), 64, (1, 4), 9)
    psi = vxinputs.eval_tangle(t)
    C, _ = oracle.node_circulation(oracle.winding(psi).w)
    C2, _ = oracle.node_circulation(oracle.winding(np.conj(psi)).w)
    assert np.array_equal(C2, -C) and np.abs(C).max() >= 1
