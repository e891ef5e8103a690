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
  samples      Sec. 3.3.1 / 3.3.2: the candidate sample around a vertex is the mean position of the
               connected sub-graph inside a box of side k around it; the sub-graph collapses into one
               node; the next vertex is an unprocessed neighbour of the collapsed ones; passes repeat
               on the reduced graph until nothing merges.

It shares no code with the GPU library and never imports it.
"""
from __future__ import annotations

import math

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


# ----------------------------------------------------------------------------------------------
# sample points by box means and iterative graph reduction (Sec. 3.3.1, 3.3.2)
# ----------------------------------------------------------------------------------------------

def first_estimate_point(dims, cell: int, desc: int):
    """Min corner of the cell plus the mean of its pierced-face centres (the mean-position estimator
    of Sec. 3.3.1 with a one-cell box)."""
    nx, ny, nz = dims
    co = [cell % nx, (cell // nx) % ny, cell // (nx * ny)]
    s = [0.0, 0.0, 0.0]
    k = 0
    for f, w in enumerate(decode(desc)):
        if w == 0:
            continue
        for a in range(3):
            s[a] += float(f % 2) if a == f // 2 else 0.5
        k += 1
    return [co[a] + (s[a] / k if k else 0.5) for a in range(3)]


def _disp(dims, periodic, a, b):
    """b - a with the minimum image on periodic axes (ties of the rounding to even)."""
    out = []
    for q in range(3):
        t = b[q] - a[q]
        if (periodic >> q) & 1:
            t -= dims[q] * round(t / dims[q])
        out.append(t)
    return out


def _wrap(dims, periodic, x, q):
    if (periodic >> q) & 1:
        return x - dims[q] * math.floor(x / dims[q])
    return x


def reduce_once(dims, periodic, pos, adj, members, comp, half):
    """One pass of the reduction. pos: list of [x, y, z]; adj: list of sets of neighbour ids.
    Returns the reduced (pos, adj, members, comp)."""
    n = len(pos)
    done = [False] * n
    owner = [-1] * n
    rpos, rmem, rcomp = [], [], []
    seed = None
    while True:
        if seed is None:
            rest = [v for v in range(n) if not done[v]]
            if not rest:
                break
            v = rest[0]
        else:
            v = seed
        # the connected unprocessed vertices inside the box around v (depth-first traversal)
        sub = []
        done[v] = True
        stack = [v]
        while stack:
            u = stack.pop()
            sub.append(u)
            for w in adj[u]:
                if not done[w] and all(abs(t) <= half for t in _disp(dims, periodic, pos[v], pos[w])):
                    done[w] = True
                    stack.append(w)
        sub.sort()
        acc = [0.0, 0.0, 0.0]
        for u in sub:
            d = _disp(dims, periodic, pos[v], pos[u])
            for q in range(3):
                acc[q] += d[q]
        rid = len(rpos)
        rpos.append([_wrap(dims, periodic, pos[v][q] + acc[q] / len(sub), q) for q in range(3)])
        rmem.append(sum(members[u] for u in sub))
        rcomp.append(comp[v])
        for u in sub:
            owner[u] = rid
        cand = [w for u in sub for w in adj[u] if not done[w]]
        seed = min(cand) if cand else None
    radj = [set() for _ in rpos]
    for u in range(n):
        for w in adj[u]:
            if owner[u] != owner[w]:
                radj[owner[u]].add(owner[w])
    return rpos, radj, rmem, rcomp


def reduce_graph(dims, periodic, cells, cdesc, box_k, max_passes):
    """The reduced graph: (pos [m][3], sorted edge list [(u, v), u < v], members, comp, passes)."""
    order = sorted(range(len(cells)), key=lambda i: int(cells[i]))
    scells = [int(cells[i]) for i in order]
    sdesc = [int(cdesc[i]) for i in order]
    adj_in, _ = dual_graph(dims, periodic, scells, sdesc)
    comp, _ = components(scells, adj_in)
    pos = [first_estimate_point(dims, c, d) for c, d in zip(scells, sdesc)]
    adj = [set(j for j, _ in a if j != i) for i, a in enumerate(adj_in)]
    members = [1] * len(pos)
    comp = comp.tolist()
    passes = 0
    for _ in range(max_passes):
        n0 = len(pos)
        pos, adj, members, comp = reduce_once(dims, periodic, pos, adj, members, comp, 0.5 * box_k)
        passes += 1
        if len(pos) == n0:
            break
    edges = sorted((u, w) for u in range(len(pos)) for w in adj[u] if u < w)
    return np.array(pos, np.float64).reshape(-1, 3), edges, members, comp, passes


# ----------------------------------------------------------------------------------------------
# vectorisation (Sec. 3.4): chains split at branch points and Catmull-Rom curves
# ----------------------------------------------------------------------------------------------

def chains(n, edges):
    """Ordered node chains of a sample graph: from every node of connectivity other than 2 (ascending),
    along each unused edge (ascending neighbour), through connectivity-2 nodes to the next such node;
    then the remaining loops, each from its lowest node towards its lower neighbour.
    Returns a list of (nodes, closed)."""
    adj = [set() for _ in range(n)]
    for u, v in edges:
        if u != v:
            adj[u].add(v)
            adj[v].add(u)
    adj = [sorted(a) for a in adj]
    used = set()
    out = []
    for v in range(n):
        if len(adj[v]) == 2:
            continue
        if not adj[v]:
            out.append(([v], False))
            continue
        for w in adj[v]:
            if (v, w) in used:
                continue
            ch = [v, w]
            used |= {(v, w), (w, v)}
            prev, cur = v, w
            while len(adj[cur]) == 2:
                nxt = adj[cur][0] if adj[cur][1] == prev else adj[cur][1]
                used |= {(cur, nxt), (nxt, cur)}
                ch.append(nxt)
                prev, cur = cur, nxt
            out.append((ch, False))
    for v in range(n):
        if len(adj[v]) != 2 or (v, adj[v][0]) in used:
            continue
        ch = [v]
        prev, cur = v, min(adj[v])
        used |= {(v, cur), (cur, v)}
        while cur != v:
            ch.append(cur)
            nxt = adj[cur][0] if adj[cur][1] == prev else adj[cur][1]
            used |= {(cur, nxt), (nxt, cur)}
            prev, cur = cur, nxt
        out.append((ch, True))
    return out


def catmull_rom_point(a, b, c, d, t):
    """Uniform Catmull-Rom: the cubic through b (t = 0) and c (t = 1) with tangents (c - a) / 2 and
    (d - b) / 2."""
    t2 = t * t
    t3 = t2 * t
    return [0.5 * ((2.0 * b[q]) + (c[q] - a[q]) * t + (2.0 * a[q] - 5.0 * b[q] + 4.0 * c[q] - d[q]) * t2 +
                   (3.0 * b[q] - a[q] - 3.0 * c[q] + d[q]) * t3) for q in range(3)]


def curve(dims, periodic, pos, nodes, closed, seg):
    """Catmull-Rom polyline of one chain and its length."""
    m = len(nodes)
    P = [list(pos[nodes[0]])]
    for i in range(1, m + 1):
        d = _disp(dims, periodic, pos[nodes[i - 1]], pos[nodes[i % m]])
        P.append([P[-1][q] + d[q] for q in range(3)])
    shift = [P[m][q] - P[0][q] for q in range(3)]

    def ctrl(i):
        if not closed:
            return P[min(max(i, 0), m - 1)]
        turns, j = divmod(i, m)
        return [P[j][q] + turns * shift[q] for q in range(3)]

    nseg = m if closed else m - 1
    pts = []
    for i in range(nseg):
        for j in range(seg):
            pts.append(catmull_rom_point(ctrl(i - 1), ctrl(i), ctrl(i + 1), ctrl(i + 2), j / seg))
    pts.append(list(ctrl(nseg)))
    length = 0.0
    for k in range(len(pts) - 1):
        dx, dy, dz = (pts[k + 1][q] - pts[k][q] for q in range(3))
        length += math.sqrt(dx * dx + dy * dy + dz * dz)
    return pts, length
