"""CPU ORACLE -- test infrastructure only: the host consumers of the pierced-cell list, written
plainly in Python from the paper's description.

  dual graph   Sec. 3.1 (graph of vortex nodes linked to their neighbours), in dual form: vertices
               are pierced cells; a pierced face joins the two cells that share it. The face (n, a)
               is the -a face of cell n and the +a face of cell n - e_a.
  components   Sec. 3.2: depth-first traversal from an unvisited vertex until none is left; here
               started from the unvisited cell of lowest id.
  classes      Sec. 3.4: Type I (connectivity <= 2 everywhere, some vertex below 2), Type II (2
               everywhere), Type III (some vertex above 2); branch points: connectivity > 2
               (Sec. 4.2 reconnection events).

It shares no code with the GPU library and never imports it.
"""
from __future__ import annotations

import numpy as np


def decode(desc: int):
    """The six face windings (-x, +x, -y, +y, -z, +z) of a cell descriptor."""
    out = []
    for f in range(6):
        v = (int(desc) >> (2 * f)) & 3
        out.append(1 if v == 1 else (-1 if v == 3 else 0))
    return out


def dual_graph(dims, periodic: int, cells, cdesc):
    """Adjacency of the listed cells: adj[i] = list of (j, out) for input positions i, j, with out = +1
    if the line leaves cell i through the shared face (outward winding +1), -1 if it enters; and the
    number of pierced faces of each cell on a non-periodic boundary."""
    nx, ny, nz = dims
    where = {int(c): i for i, c in enumerate(cells)}
    assert len(where) == len(cells), "duplicate cell"
    adj = [[] for _ in cells]
    nbound = [0] * len(cells)
    n3 = (nx, ny, nz)
    for i, (c, d) in enumerate(zip(cells, cdesc)):
        c = int(c)
        co = [c % nx, (c // nx) % ny, c // (nx * ny)]
        for f, w in enumerate(decode(d)):
            if w == 0:
                continue
            a, side = f // 2, f % 2
            q = list(co)
            q[a] += 1 if side else -1
            if (periodic >> a) & 1:
                q[a] %= n3[a]
            elif not 0 <= q[a] <= n3[a] - 2:  # cells of an open axis: min corner 0 .. n - 2
                nbound[i] += 1
                continue
            j = where[q[0] + nx * (q[1] + ny * q[2])]
            adj[i].append((j, w if side else -w))
    return adj, nbound


def components(cells, adj):
    """Component label of every input position, by depth-first traversal from the unvisited cell of
    lowest id; labels in order of discovery."""
    comp = [-1] * len(cells)
    nc = 0
    for s in sorted(range(len(cells)), key=lambda i: int(cells[i])):
        if comp[s] >= 0:
            continue
        comp[s] = nc
        stack = [s]
        while stack:
            v = stack.pop()
            for u, _ in adj[v]:
                if comp[u] < 0:
                    comp[u] = nc
                    stack.append(u)
        nc += 1
    return np.array(comp, np.int64), nc


def classify(adj, comp, nc):
    deg = np.array([len(a) for a in adj], np.int64)
    types = []
    for c in range(nc):
        dc = deg[comp == c]
        types.append(3 if dc.max() > 2 else (2 if dc.min() == 2 else 1))
    return deg, np.array(types, np.int32)


def graph_lines(dims, periodic, cells, cdesc):
    """Everything the library's vx_graph_lines returns: (comp, degree, comp_type, stats dict)."""
    adj, nbound = dual_graph(dims, periodic, cells, cdesc)
    comp, nc = components(cells, adj)
    deg, types = classify(adj, comp, nc)
    stats = {"nvert": len(cells), "nedge": int(deg.sum()) // 2, "nboundary": int(sum(nbound)), "ncomp": nc,
             "ntype": [int((types == t).sum()) for t in (1, 2, 3)], "nbranch": int((deg > 2).sum())}
    return comp, deg.astype(np.int32), types, stats
