"""Sample points by box means and iterative graph reduction (Sec. 3.3.1, 3.3.2): the oracle pinned
by what the paper and the geometry fix, and the library's host implementation (vx_reduce) equal to
the oracle bit for bit on the same lists (no GPU needed: the lists are the oracle's, which the GPU
reproduces exactly)."""
import numpy as np
import pytest

import oracle
import vxinputs
from oracle import graph as G


def mi(d, n):
    return d - n * np.round(d / n)


def reduced_degrees(m, edges):
    deg = np.zeros(m, np.int64)
    for u, v in edges:
        deg[u] += 1
        deg[v] += 1
    return deg


def test_reduction_preserves_components_and_members():
    for seed, per in ((3, 7), (4, 0), (5, 5)):
        psi = vxinputs.eval_tangle(vxinputs.make_tangle((64, 64, 64), 256, (3, 7), seed), (0, 0, 0, 48, 40, 36))
        W = oracle.winding(psi, per)
        comp, deg, types, st = G.graph_lines((48, 40, 36), per, W.cells, W.cdesc)
        for k in (3, 6):
            pos, edges, mem, rcomp, passes = G.reduce_graph((48, 40, 36), per, W.cells, W.cdesc, k, 5)
            assert sum(mem) == len(W.cells)  # every cell in exactly one sample node
            assert sorted(set(rcomp)) == list(range(st["ncomp"]))  # every line keeps at least one node
            for u, v in edges:
                assert rcomp[u] == rcomp[v]  # nodes join only within a line
            # connectivity is inherited: one reduced component per line
            parent = list(range(len(pos)))

            def find(a):
                while parent[a] != a:
                    parent[a] = parent[parent[a]]
                    a = parent[a]
                return a
            for u, v in edges:
                parent[find(u)] = find(v)
            assert len({find(a) for a in range(len(pos))}) == st["ncomp"]
            assert 1 <= passes <= 5


def test_box_size_sets_the_sample_spacing():
    """The box side approximately defines the distance between final sample points (Sec. 3.3.2)."""
    psi = vxinputs.eval_tangle(vxinputs.make_tangle((96, 96, 96), 512, (3, 6), 11))
    W = oracle.winding(psi)
    for k in (3, 5, 8):
        pos, edges, mem, rcomp, passes = G.reduce_graph((96, 96, 96), 7, W.cells, W.cdesc, k, 5)
        e = np.array(edges)
        d = mi(pos[e[:, 1]] - pos[e[:, 0]], 96.0)
        L = np.linalg.norm(d, axis=1)
        assert 0.5 * k < np.median(L) < 1.5 * k, (k, np.median(L))


def test_ring_stays_a_closed_loop_on_the_circle():
    lr = vxinputs.line_ring_32()
    psi = vxinputs.eval_line_ring(lr)
    W = oracle.winding(psi)
    comp, deg, types, st = G.graph_lines((32, 32, 32), 7, W.cells, W.cdesc)
    z = (W.cells // 1024).astype(int)
    x = (W.cells % 32).astype(int)
    ring_c = comp[np.flatnonzero((z == 16) & (x == 16))[0]]
    cx, cy, cz = lr.ring_center
    for k in (3, 4):
        pos, edges, mem, rcomp, passes = G.reduce_graph((32, 32, 32), 7, W.cells, W.cdesc, k, 5)
        nodes = [i for i, c in enumerate(rcomp) if c == ring_c]
        sub = [(u, v) for u, v in edges if rcomp[u] == ring_c]
        assert len(sub) == len(nodes) and (reduced_degrees(len(pos), sub)[nodes] == 2).all()  # a cycle
        assert 2 * np.pi * lr.radius / (1.6 * k) < len(nodes) < 2 * np.pi * lr.radius / (0.6 * k)
        p = pos[nodes]
        r = np.hypot(p[:, 0] - cx, p[:, 1] - cy)
        assert np.abs(r - lr.radius).max() < 0.75 and np.abs(p[:, 2] - (cz - 0.0)).max() < 1.0


def test_straight_periodic_line_samples_lie_on_the_line():
    nx, ny, nz = 9, 8, 24
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    psi = ((xx - 3.3) + 1j * (yy - 4.6)).astype(np.complex64)  # a z-line, periodic along z only
    W = oracle.winding(psi, 4)
    for k in (3, 4, 6):
        pos, edges, mem, rcomp, passes = G.reduce_graph((nx, ny, nz), 4, W.cells, W.cdesc, k, 5)
        assert (pos[:, 0] == 3.5).all() and (pos[:, 1] == 4.5).all()  # mean of the cells' face centres
        assert len(edges) == len(pos)  # the line closes through the periodic z-axis
        zs = np.sort(pos[:, 2])
        gaps = np.diff(np.r_[zs, zs[0] + nz])
        assert gaps.min() > 0.5 * k - 1 and gaps.max() < 1.5 * k + 1


CASES = [("ring", None, 7, 3), ("tangle", 3, 7, 3), ("tangle", 3, 7, 8), ("tangle", 4, 0, 5), ("tangle", 5, 5, 4),
         ("int", 6, 7, 3), ("int", 7, 2, 5)]


@pytest.mark.parametrize("kind,seed,periodic,k", CASES)
def test_library_reduction_equals_oracle(kind, seed, periodic, k):
    from paper_1911_12070_amd import dims, vx_reduce
    if kind == "ring":
        psi = vxinputs.eval_line_ring(vxinputs.line_ring_32())
    elif kind == "int":
        psi = vxinputs.random_small_int_field((9, 8, 7), seed)
    else:
        psi = vxinputs.eval_tangle(vxinputs.make_tangle((64, 64, 64), 256, (3, 7), seed), (0, 0, 0, 48, 40, 36))
    nz, ny, nx = psi.shape
    W = oracle.winding(psi, periodic)
    perm = np.random.default_rng(seed or 0).permutation(len(W.cells))
    R = vx_reduce(dims(nx, ny, nz, periodic), W.cells[perm], W.cdesc[perm], k, 5)
    pos, edges, mem, rcomp, passes = G.reduce_graph((nx, ny, nz), periodic, W.cells, W.cdesc, k, 5)
    assert np.array_equal(R["pos"], pos)  # bit for bit: the same sums in the same order
    assert np.array_equal(R["edges"], np.array(edges, np.int64).reshape(-1, 2))
    assert R["members"].tolist() == list(mem) and R["comp"].tolist() == list(rcomp) and R["passes"] == passes
    # refinement seeds: the cell holding each node and the node's offset in it
    cells = R["seed_cell"].astype(np.int64)
    c3 = np.stack([cells % nx, (cells // nx) % ny, cells // (nx * ny)], 1)
    assert np.abs(c3 + R["seed_off"].astype(np.float64) - pos).max() < 1e-5 + 1e-6 * max(nx, ny, nz)
    for q, n in enumerate((nx, ny, nz)):
        assert (c3[:, q] >= 0).all() and (c3[:, q] <= (n - 1 if (periodic >> q) & 1 else n - 2)).all()
    listed = dict(zip(W.cells.tolist(), W.cdesc.tolist()))
    assert R["seed_desc"].tolist() == [listed.get(int(c), 0) for c in cells]
