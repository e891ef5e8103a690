// Host consumers of the pierced-cell list (host C++, no device code):
//   * the dual graph of the vortex lines (Sec. 3.1 graph of vortex nodes, in dual form): vertices
//     are the pierced cells, and every pierced face joins the two cells that share it; the face's
//     winding orients the edge by the right-hand rule (Sec. 3.4, line direction);
//   * connected components by depth-first traversal (Sec. 3.2), started from the unvisited vertex
//     of lowest cell id, so that the labels are canonical;
//   * the class of each component (Sec. 3.4): Type I (simple open: every vertex of connectivity at
//     most 2, some below 2), Type II (simple closed: every vertex of connectivity 2), Type III
//     (complex: some vertex of connectivity above 2); vertices of connectivity above 2 are the
//     branch points, the reconnection candidates of Sec. 4.2.
// A face on a non-periodic grid boundary has no second cell: it is counted as a boundary face of its
// cell, and that cell's connectivity is its number of neighbour cells.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/vx.h"

namespace vxg {

inline int dec2(uint32_t d, int f) {
    const uint32_t v = (d >> (2 * f)) & 3u;
    return v == 1u ? 1 : (v == 3u ? -1 : 0);
}

// The dual graph of a list of pierced cells: vertices in ascending cell id.
struct Dual {
    int64_t n = 0;
    std::vector<uint64_t> cell;    // sorted cell ids
    std::vector<uint16_t> desc;    // their descriptors
    std::vector<int64_t> input;    // input position of each sorted vertex
    std::vector<int64_t> start;    // CSR: edges of vertex v are [start[v], start[v+1])
    std::vector<int64_t> nbr;      // neighbour vertex
    std::vector<int8_t> out;       // +1: the line leaves v along this edge, -1: it enters v
    std::vector<int32_t> nbound;   // pierced faces of v on a non-periodic boundary
    int64_t nboundary = 0;
};

// Builds the graph; returns VX_ERR_INVALID (with *bad = the offending input position) for duplicate
// cells, cells outside the grid, or a pierced face whose neighbour cell is not listed.
inline vx_status build_dual(const vx_dims &d, const uint64_t *cells, const uint16_t *desc, int64_t n, Dual &g,
                            int64_t *bad) {
    g.n = n;
    g.input.resize(n);
    for (int64_t i = 0; i < n; ++i) g.input[i] = i;
    std::sort(g.input.begin(), g.input.end(), [&](int64_t a, int64_t b) { return cells[a] < cells[b]; });
    g.cell.resize(n);
    g.desc.resize(n);
    const uint64_t N = (uint64_t)d.nx * (uint64_t)d.ny * (uint64_t)d.nz;
    for (int64_t v = 0; v < n; ++v) {
        g.cell[v] = cells[g.input[v]];
        g.desc[v] = desc[g.input[v]];
        if (g.cell[v] >= N || (v > 0 && g.cell[v] == g.cell[v - 1])) {
            *bad = g.input[v];
            return VX_ERR_INVALID;
        }
    }
    const int64_t dim[3] = {d.nx, d.ny, d.nz};
    const int per[3] = {(int)(d.periodic & 1u), (int)((d.periodic >> 1) & 1u), (int)((d.periodic >> 2) & 1u)};
    g.start.assign(n + 1, 0);
    g.nbound.assign(n, 0);
    g.nbr.clear();
    g.out.clear();
    g.nboundary = 0;
    for (int64_t v = 0; v < n; ++v) {
        const uint64_t c = g.cell[v];
        const int64_t co[3] = {(int64_t)(c % (uint64_t)d.nx), (int64_t)((c / (uint64_t)d.nx) % (uint64_t)d.ny),
                               (int64_t)(c / ((uint64_t)d.nx * (uint64_t)d.ny))};
        for (int f = 0; f < 6; ++f) {
            const int w = dec2(g.desc[v], f);
            if (w == 0) continue;
            const int a = f >> 1, side = f & 1;  // side 0: the face normal to -e_a, 1: to +e_a
            int64_t q[3] = {co[0], co[1], co[2]};
            q[a] += side ? 1 : -1;
            if (per[a]) {
                q[a] = (q[a] + dim[a]) % dim[a];
            } else if (q[a] < 0 || q[a] > dim[a] - 2) {  // cells of an open axis: min corner 0 .. n - 2
                ++g.nbound[v];
                ++g.nboundary;
                continue;
            }
            const uint64_t id = (uint64_t)q[0] + (uint64_t)d.nx * ((uint64_t)q[1] + (uint64_t)d.ny * (uint64_t)q[2]);
            const auto it = std::lower_bound(g.cell.begin(), g.cell.end(), id);
            if (it == g.cell.end() || *it != id) {
                *bad = g.input[v];
                return VX_ERR_INVALID;
            }
            g.nbr.push_back(it - g.cell.begin());
            // winding about +e_a; outward through the +a face it is w, through the -a face -w
            g.out.push_back((int8_t)(side ? w : -w));
        }
        g.start[v + 1] = (int64_t)g.nbr.size();
    }
    return VX_OK;
}

// Components by depth-first traversal from the unvisited vertex of lowest cell id; returns the count.
inline int64_t components(const Dual &g, std::vector<int64_t> &comp) {
    comp.assign(g.n, -1);
    std::vector<int64_t> stack;
    int64_t nc = 0;
    for (int64_t s = 0; s < g.n; ++s) {
        if (comp[s] >= 0) continue;
        comp[s] = nc;
        stack.push_back(s);
        while (!stack.empty()) {
            const int64_t v = stack.back();
            stack.pop_back();
            for (int64_t e = g.start[v]; e < g.start[v + 1]; ++e) {
                const int64_t u = g.nbr[e];
                if (comp[u] < 0) {
                    comp[u] = nc;
                    stack.push_back(u);
                }
            }
        }
        ++nc;
    }
    return nc;
}

// Class of each component from the connectivity of its vertices (1, 2 or 3 for Type I, II, III).
inline void classify(const Dual &g, const std::vector<int64_t> &comp, int64_t nc, std::vector<int32_t> &type) {
    std::vector<int32_t> maxdeg(nc, 0), mindeg(nc, 1 << 30);
    for (int64_t v = 0; v < g.n; ++v) {
        const int32_t deg = (int32_t)(g.start[v + 1] - g.start[v]);
        maxdeg[comp[v]] = std::max(maxdeg[comp[v]], deg);
        mindeg[comp[v]] = std::min(mindeg[comp[v]], deg);
    }
    type.resize(nc);
    for (int64_t c = 0; c < nc; ++c) type[c] = maxdeg[c] > 2 ? 3 : (mindeg[c] == 2 ? 2 : 1);
}

}  // namespace vxg

using namespace vxg;

extern "C" vx_status vx_graph_lines(vx_dims dims, const uint64_t *h_cells, const uint16_t *h_cell_desc, int64_t n,
                                    int64_t *h_comp, int32_t *h_degree, int32_t *h_comp_type, vx_graph_stats *stats) {
    if (n < 0 || (n > 0 && (!h_cells || !h_cell_desc || !h_comp)) || !stats) return VX_ERR_INVALID;
    if (dims.nx < 1 || dims.ny < 1 || dims.nz < 1 || dims.periodic > 7u) return VX_ERR_INVALID;
    try {
        Dual g;
        int64_t bad = -1;
        if (vx_status st = build_dual(dims, h_cells, h_cell_desc, n, g, &bad)) {
            std::memset(stats, 0, sizeof *stats);
            stats->bad_input = bad;
            return st;
        }
        std::vector<int64_t> comp;
        const int64_t nc = components(g, comp);
        std::vector<int32_t> type;
        classify(g, comp, nc, type);
        std::memset(stats, 0, sizeof *stats);
        stats->nvert = n;
        stats->nedge = (int64_t)g.nbr.size() / 2;
        stats->nboundary = g.nboundary;
        stats->ncomp = nc;
        stats->bad_input = -1;
        for (int64_t c = 0; c < nc; ++c) ++stats->ntype[type[c] - 1];
        for (int64_t v = 0; v < n; ++v) {
            const int32_t deg = (int32_t)(g.start[v + 1] - g.start[v]);
            if (deg > 2) ++stats->nbranch;
            h_comp[g.input[v]] = comp[v];
            if (h_degree) h_degree[g.input[v]] = deg;
        }
        if (h_comp_type)
            for (int64_t c = 0; c < nc; ++c) h_comp_type[c] = type[c];
        return VX_OK;
    } catch (const std::bad_alloc &) {
        return VX_ERR_NOMEM;
    }
}
