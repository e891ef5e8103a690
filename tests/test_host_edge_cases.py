"""Degenerate inputs of the host consumers (dual graph, box reduction, curves): empty lists, isolated
and repeated nodes, self loops, two-node loops, a line ending on an open boundary, and argument
errors. The library is compared with the oracle where both define a result."""
import numpy as np
import pytest

import oracle
import vxinputs
from oracle import graph as G
from test_curves import assert_same, lib_curves, oracle_curves


def test_empty_lists():
    from paper_1911_12070_amd import dims, vx_graph_lines, vx_reduce
    d = dims(8, 8, 8, 7)
    e64, e16 = np.zeros(0, np.uint64), np.zeros(0, np.uint16)
    comp, deg, ctype, st = vx_graph_lines(d, e64, e16)
    assert len(comp) == len(deg) == len(ctype) == 0
    assert st == {"nvert": 0, "nedge": 0, "nboundary": 0, "ncomp": 0, "ntype": [0, 0, 0], "nbranch": 0}
    assert G.graph_lines((8, 8, 8), 7, [], [])[3] == st
    R = vx_reduce(d, e64, e16, 4, 5)
    assert R["pos"].shape == (0, 3) and R["edges"].shape == (0, 2) and len(R["seed_cell"]) == 0
    pos, edges, mem, comp, passes = G.reduce_graph((8, 8, 8), 7, [], [], 4, 5)
    assert len(pos) == 0 and len(edges) == 0
    C = lib_curves((8, 8, 8), 7, np.zeros((0, 3)), np.zeros((0, 2), np.int64))
    assert len(C["length"]) == 0 and len(C["points"]) == 0 and C["total_length"] == 0.0


@pytest.mark.parametrize("periodic", [0, 7])
def test_curves_of_degenerate_graphs(periodic):
    dims = (16, 16, 16)
    pos = np.array([[1.5, 2.5, 3.5], [2.5, 2.5, 3.5], [2.5, 3.5, 3.5], [9.0, 9.0, 9.0], [12.0, 1.0, 1.0]], float)
    cases = [
        [],                        # isolated nodes only: one single-node chain each
        [(0, 1)],                  # one segment, three isolated nodes
        [(0, 1), (1, 0)],          # the same edge twice
        [(0, 0), (1, 2)],          # a self loop (ignored) and a segment
        [(0, 1), (1, 2), (2, 0)],  # a triangle: one closed loop
        [(3, 4), (4, 3), (0, 1)],  # a repeated two-node edge beside a segment
    ]
    for edges in cases:
        e = np.array(edges, np.int64).reshape(-1, 2)
        assert_same(lib_curves(dims, periodic, pos, e), oracle_curves(dims, periodic, pos, e))


def test_line_ending_on_an_open_boundary_is_type_one():
    from paper_1911_12070_amd import dims, vx_graph_lines
    # a straight line along z through an open 12^3 grid: its cells form one open chain (Type I) whose
    # two end cells each have one pierced face on the boundary
    psi = vxinputs.eval_line_ring(vxinputs.line_ring_32())[:, 4:16, 4:16].copy()  # the z-line, no ring
    psi = psi[8:20]
    nz, ny, nx = psi.shape
    W = oracle.winding(psi, 0)
    comp, deg, ctype, st = vx_graph_lines(dims(nx, ny, nz, 0), W.cells, W.cdesc)
    Oc, Od, Ot, Ost = G.graph_lines((nx, ny, nz), 0, W.cells, W.cdesc)
    assert st == Ost and np.array_equal(comp, Oc) and np.array_equal(deg, Od) and np.array_equal(ctype, Ot)
    assert st["ncomp"] >= 1 and 1 in ctype.tolist()


def test_argument_errors():
    from paper_1911_12070_amd import VxError, dims, vx_curves, vx_graph_lines, vx_reduce
    d = dims(8, 8, 8, 7)
    cells = np.array([0], np.uint64)
    with pytest.raises(VxError):
        vx_reduce(d, cells, np.array([0x005], np.uint16), 0, 5)  # box below 1
    with pytest.raises(VxError):
        vx_reduce(d, cells, np.array([0x005], np.uint16), 4, 0)  # no pass
    with pytest.raises(VxError):
        vx_curves(d, np.zeros((2, 3)), np.array([[0, 2]], np.int64))  # edge to a node that does not exist
    with pytest.raises(VxError):
        vx_curves(d, np.zeros((2, 3)), np.array([[0, 1]], np.int64), 0)  # no point per segment
    with pytest.raises(VxError):
        vx_graph_lines(d, np.array([0, 0], np.uint64), np.array([0x005, 0x005], np.uint16))  # repeated cell
