"""The dual graph of the vortex lines (Sec. 3.1), its components by depth-first traversal (Sec. 3.2),
line classes (Sec. 3.4) and branch points (Sec. 4.2): the oracle pinned against an independent
construction and closed forms, and the library's host implementation (vx_graph_lines) against the
oracle on the same lists. The lists come from the oracle's winding pass, which the GPU reproduces
bit for bit (the GPU tests compare the two); these tests run without a GPU."""
import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

import oracle
import vxinputs
from oracle import graph as G


def canonical_partition(cells, labels):
    """Labels renumbered by the smallest cell id of each class."""
    first = {}
    for c, l in sorted(zip(cells.tolist(), labels.tolist())):
        first.setdefault(l, len(first))
    return np.array([first[l] for l in labels.tolist()], np.int64)


def faces_graph(dims, periodic, W):
    """Components built from the pierced-face list alone: face (n, a) joins cell n and cell n - e_a
    (each where it exists); an independent construction of the same graph."""
    nx, ny, nz = dims
    idx = {int(c): i for i, c in enumerate(W.cells)}
    rows, cols = [], []
    nb = 0
    for f in W.faces.tolist():
        n, a = f // 3, f % 3
        co = [n % nx, (n // nx) % ny, n // (nx * ny)]
        q = list(co)
        q[a] -= 1
        if q[a] < 0:
            if not (periodic >> a) & 1:
                nb += 1
                continue
            q[a] += (nx, ny, nz)[a]
        m = q[0] + nx * (q[1] + ny * q[2])
        if n not in idx:  # cell n does not exist (the face lies on the far open boundary)
            nb += 1
            continue
        rows.append(idx[n])
        cols.append(idx[m])
    A = coo_matrix((np.ones(len(rows)), (rows, cols)), shape=(len(W.cells),) * 2)
    nc, lab = connected_components(A, directed=False)
    return nc, lab, len(rows), nb


FIELDS = [("tangle", (48, 40, 36), 7, 3), ("tangle", (48, 40, 36), 0, 4), ("tangle", (40, 44, 30), 5, 5),
          ("int", (9, 7, 6), 7, 6), ("int", (8, 6, 7), 2, 7), ("tangle", (2, 40, 32), 7, 8)]


def field(kind, dims, seed):
    if kind == "int":
        return vxinputs.random_small_int_field(dims, seed)
    t = vxinputs.make_tangle((64, 64, 64), 256, (3, 7), seed)
    return vxinputs.eval_tangle(t, (0, 0, 0, *dims))


@pytest.mark.parametrize("kind,dims,periodic,seed", FIELDS)
def test_oracle_graph_against_face_construction(kind, dims, periodic, seed):
    psi = field(kind, dims, seed)
    W = oracle.winding(psi, periodic)
    comp, deg, types, st = G.graph_lines(dims, periodic, W.cells, W.cdesc)
    nc, lab, nedge, nb = faces_graph(dims, periodic, W)
    assert st["ncomp"] == nc and st["nedge"] == nedge and st["nboundary"] == nb
    assert np.array_equal(canonical_partition(W.cells, comp), canonical_partition(W.cells, lab))
    assert st["nedge"] + st["nboundary"] == len(W.faces)  # every pierced face: an edge or a boundary face
    pierced = np.array([sum(1 for w in G.decode(d) if w) for d in W.cdesc])
    if periodic == 7:
        assert (deg == pierced).all() and (deg % 2 == 0).all()  # zero net flux: an even number of faces


def test_oracle_line_ring_components():
    psi = vxinputs.eval_line_ring(vxinputs.line_ring_32())
    W = oracle.winding(psi)
    comp, deg, types, st = G.graph_lines((32, 32, 32), 7, W.cells, W.cdesc)
    assert st["ntype"] == [0, st["ncomp"], 0] and st["nbranch"] == 0  # closed loops only
    z = (W.cells // 1024).astype(int)
    ring = comp == comp[np.flatnonzero((z == 16) & (W.cells % 32 == 16))[0]]
    assert ring.sum() == 64 and (z[ring] == 16).all()  # the ring: one closed loop of 64 cells
    x, y = (W.cells % 32).astype(int), ((W.cells // 32) % 32).astype(int)
    line = comp == comp[np.flatnonzero((x == 16) & (y == 15))[0]]
    assert line.sum() == 32 and (x[line] == 16).all() and (y[line] == 15).all()  # the z-line, closed by periodicity


def test_oracle_open_line_is_type_one():
    nx, ny, nz = 9, 8, 6
    zz, yy, xx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    psi = ((xx - 3.3) + 1j * (yy - 4.6)).astype(np.complex64)
    W = oracle.winding(psi, 0)
    comp, deg, types, st = G.graph_lines((nx, ny, nz), 0, W.cells, W.cdesc)
    assert st["ncomp"] == 1 and list(types) == [1] and st["nvert"] == nz - 1
    assert sorted(deg.tolist()) == [1, 1] + [2] * (nz - 3) and st["nboundary"] == 2


@pytest.mark.parametrize("kind,dims,periodic,seed", FIELDS + [("ring", (32, 32, 32), 7, 0)])
def test_library_graph_equals_oracle(kind, dims, periodic, seed):
    from paper_1911_12070_amd import dims as mkdims, vx_graph_lines
    psi = vxinputs.eval_line_ring(vxinputs.line_ring_32()) if kind == "ring" else field(kind, dims, seed)
    W = oracle.winding(psi, periodic)
    rng = np.random.default_rng(seed)
    perm = rng.permutation(len(W.cells))  # the library accepts any order (the GPU's is unspecified)
    cells, cdesc = W.cells[perm], W.cdesc[perm]
    comp, deg, types, st = vx_graph_lines(mkdims(*dims, periodic), cells, cdesc)
    ocomp, odeg, otypes, ost = G.graph_lines(dims, periodic, cells, cdesc)
    assert np.array_equal(comp, ocomp) and np.array_equal(deg, odeg) and np.array_equal(types, otypes)
    assert st == ost


def test_library_graph_rejects_incomplete_lists():
    from paper_1911_12070_amd import VxError, dims as mkdims, vx_graph_lines
    psi = field("tangle", (48, 40, 36), 3)
    W = oracle.winding(psi)
    with pytest.raises(VxError):
        vx_graph_lines(mkdims(48, 40, 36, 7), W.cells[1:], W.cdesc[1:])  # a neighbour is missing
    with pytest.raises(VxError):
        vx_graph_lines(mkdims(48, 40, 36, 7), np.r_[W.cells, W.cells[:1]], np.r_[W.cdesc, W.cdesc[:1]])
