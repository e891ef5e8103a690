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
//   * sample points by box means and iterative graph reduction (Sec. 3.3.1, 3.3.2): the candidate
//     sample around a vertex is the mean position of the connected sub-graph inside a box of side
//     k cells centred on it; that sub-graph collapses into one node of a reduced graph; the next
//     vertex is an unprocessed neighbour of the collapsed ones; passes repeat on the reduced graph
//     until nothing merges (positions converged) or a pass limit is reached.
// A face on a non-periodic grid boundary has no second cell: it is counted as a boundary face of its
// cell, and that cell's connectivity is its number of neighbour cells.
// Every floating-point sum runs in ascending vertex order and nothing is contracted, so the results
// do not depend on traversal order and are reproducible bit for bit.
#include <algorithm>
#include <cmath>
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

// Index of the first entry >= id in the ascending array a (a.size() if none), for an id near a[v]:
// a galloping search outward from v, then a binary search in the last interval. Neighbours along x
// are the next entries, along y a few entries away, so most lookups touch a few nearby lines.
inline int64_t find_from(const std::vector<uint64_t> &a, int64_t v, uint64_t id) {
    const int64_t n = (int64_t)a.size();
    int64_t lo, hi;  // the answer lies in [lo + 1, hi]
    if (id > a[v]) {
        lo = v;
        hi = v + 1;
        for (int64_t step = 1; hi < n && a[hi] < id; step <<= 1) {
            lo = hi;
            hi = v + 2 * step;
        }
        hi = std::min(hi, n);
    } else {
        hi = v;
        lo = v - 1;
        for (int64_t step = 1; lo >= 0 && a[lo] >= id; step <<= 1) {
            hi = lo;
            lo = v - 2 * step;
        }
        lo = std::max(lo, (int64_t)-1);
    }
    return std::lower_bound(a.begin() + (lo + 1), a.begin() + hi, id) - a.begin();
}

// Builds the graph; returns VX_ERR_INVALID (with *bad = the offending input position: for a duplicate
// cell the later of the two) for duplicate cells, cells outside the grid, or a pierced face whose
// neighbour cell is not listed.
inline vx_status build_dual(const vx_dims &d, const uint64_t *cells, const uint16_t *desc, int64_t n, Dual &g,
                            int64_t *bad) {
    g.n = n;
    {
        std::vector<std::pair<uint64_t, int64_t>> key((size_t)n);
        for (int64_t i = 0; i < n; ++i) key[i] = {cells[i], i};
        std::sort(key.begin(), key.end());
        g.input.resize(n);
        g.cell.resize(n);
        for (int64_t v = 0; v < n; ++v) {
            g.cell[v] = key[v].first;
            g.input[v] = key[v].second;
        }
    }
    g.desc.resize(n);
    const uint64_t N = (uint64_t)d.nx * (uint64_t)d.ny * (uint64_t)d.nz;
    for (int64_t v = 0; v < n; ++v) {
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
            const int64_t at = find_from(g.cell, v, id);
            if (at == n || g.cell[at] != id) {
                *bad = g.input[v];
                return VX_ERR_INVALID;
            }
            g.nbr.push_back(at);
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

// ------------------------------------------------------------------------------------------------
// Sample points (Sec. 3.3.1, 3.3.2)

// Position of a pierced cell's first estimate: its min corner plus the mean of its pierced-face
// centres (the face normal to -e_a has centre 1/2 on the other axes and 0 on a, +e_a 1 on a).
inline void cell_point(const vx_dims &d, uint64_t c, uint32_t desc, double p[3]) {
    const uint64_t co[3] = {c % (uint64_t)d.nx, (c / (uint64_t)d.nx) % (uint64_t)d.ny,
                            c / ((uint64_t)d.nx * (uint64_t)d.ny)};
    double s[3] = {0.0, 0.0, 0.0};
    int np = 0;
    for (int f = 0; f < 6; ++f) {
        if (dec2(desc, f) == 0) continue;
        for (int a = 0; a < 3; ++a) s[a] += a == (f >> 1) ? (double)(f & 1) : 0.5;
        ++np;
    }
    for (int a = 0; a < 3; ++a) p[a] = (double)co[a] + (np ? s[a] / (double)np : 0.5);
}

struct Geom {
    double n[3];
    int per[3];
    // displacement b - a, minimum image on periodic axes
    void disp(const double *a, const double *b, double *o) const {
        for (int q = 0; q < 3; ++q) {
            double t = b[q] - a[q];
            if (per[q]) t -= n[q] * std::nearbyint(t / n[q]);
            o[q] = t;
        }
    }
    // position wrapped into [0, n) on periodic axes
    double wrap(double x, int q) const { return per[q] ? x - n[q] * std::floor(x / n[q]) : x; }
};

// A graph of points: positions, undirected adjacency (CSR, duplicates removed, no self loops).
struct PGraph {
    int64_t n = 0;
    std::vector<double> pos;      // [n][3]
    std::vector<int64_t> start;   // [n+1]
    std::vector<int64_t> nbr;
    std::vector<int64_t> members; // original vertices merged into each node
    std::vector<int64_t> comp;    // component (of the original graph) of each node
};

// Undirected adjacency from vertex pairs: each vertex's neighbours ascending, without duplicates or
// self loops (bucketed by vertex, then each short list sorted).
inline void csr_from_pairs(int64_t n, std::vector<std::pair<int64_t, int64_t>> &pairs, PGraph &g) {
    std::vector<int64_t> first(n + 1, 0);
    for (auto &e : pairs)
        if (e.first != e.second) {
            ++first[e.first + 1];
            ++first[e.second + 1];
        }
    for (int64_t v = 0; v < n; ++v) first[v + 1] += first[v];
    std::vector<int64_t> all((size_t)first[n]), fill(first.begin(), first.end() - 1);
    for (auto &e : pairs)
        if (e.first != e.second) {
            all[fill[e.first]++] = e.second;
            all[fill[e.second]++] = e.first;
        }
    g.start.assign(n + 1, 0);
    g.nbr.clear();
    g.nbr.reserve(all.size());
    for (int64_t v = 0; v < n; ++v) {
        const auto b = all.begin() + first[v], e = all.begin() + first[v + 1];
        std::sort(b, e);
        g.nbr.insert(g.nbr.end(), b, std::unique(b, e));
        g.start[v + 1] = (int64_t)g.nbr.size();
    }
}

// One reduction pass; returns the reduced graph.
inline PGraph reduce_pass(const PGraph &g, const Geom &geo, double half) {
    PGraph r;
    std::vector<char> done(g.n, 0);
    std::vector<int64_t> owner(g.n, -1), stack, sub, cand;
    int64_t lowest = 0, seed = -1;
    for (;;) {
        int64_t v = seed;
        if (v < 0) {
            while (lowest < g.n && done[lowest]) ++lowest;
            if (lowest == g.n) break;
            v = lowest;
        }
        // connected sub-graph of unprocessed vertices inside the box around v (depth-first)
        const double *pv = &g.pos[3 * v];
        sub.clear();
        stack.assign(1, v);
        done[v] = 1;
        while (!stack.empty()) {
            const int64_t u = stack.back();
            stack.pop_back();
            sub.push_back(u);
            for (int64_t e = g.start[u]; e < g.start[u + 1]; ++e) {
                const int64_t w = g.nbr[e];
                if (done[w]) continue;
                double dd[3];
                geo.disp(pv, &g.pos[3 * w], dd);
                if (std::fabs(dd[0]) <= half && std::fabs(dd[1]) <= half && std::fabs(dd[2]) <= half) {
                    done[w] = 1;
                    stack.push_back(w);
                }
            }
        }
        std::sort(sub.begin(), sub.end());
        // the mean position, summed in ascending vertex order relative to v
        double acc[3] = {0.0, 0.0, 0.0};
        int64_t nmem = 0;
        for (int64_t u : sub) {
            double dd[3];
            geo.disp(pv, &g.pos[3 * u], dd);
            for (int q = 0; q < 3; ++q) acc[q] += dd[q];
            nmem += g.members[u];
        }
        const int64_t id = r.n++;
        for (int q = 0; q < 3; ++q) r.pos.push_back(geo.wrap(pv[q] + acc[q] / (double)sub.size(), q));
        r.members.push_back(nmem);
        r.comp.push_back(g.comp[v]);
        for (int64_t u : sub) owner[u] = id;
        // next: the lowest unprocessed neighbour of the collapsed vertices
        seed = -1;
        for (int64_t u : sub)
            for (int64_t e = g.start[u]; e < g.start[u + 1]; ++e) {
                const int64_t w = g.nbr[e];
                if (!done[w] && (seed < 0 || w < seed)) seed = w;
            }
    }
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (int64_t u = 0; u < g.n; ++u)
        for (int64_t e = g.start[u]; e < g.start[u + 1]; ++e)
            if (u < g.nbr[e]) pairs.emplace_back(owner[u], owner[g.nbr[e]]);
    csr_from_pairs(r.n, pairs, r);
    return r;
}

}  // namespace vxg

using namespace vxg;

struct vx_reduced {
    vx_dims dims{};
    int passes = 0;
    PGraph g;
};

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

extern "C" vx_status vx_reduce(vx_dims dims, const uint64_t *h_cells, const uint16_t *h_cell_desc, int64_t n, int box_k,
                               int max_passes, vx_reduced **out) {
    if (!out) return VX_ERR_INVALID;
    *out = nullptr;
    if (n < 0 || (n > 0 && (!h_cells || !h_cell_desc)) || box_k < 1 || box_k > 64 || max_passes < 1 || max_passes > 64)
        return VX_ERR_INVALID;
    if (dims.nx < 1 || dims.ny < 1 || dims.nz < 1 || dims.periodic > 7u) return VX_ERR_INVALID;
    try {
        Dual dg;
        int64_t bad = -1;
        if (vx_status st = build_dual(dims, h_cells, h_cell_desc, n, dg, &bad)) return st;
        std::vector<int64_t> comp;
        components(dg, comp);
        PGraph g;
        g.n = n;
        g.pos.resize(3 * (size_t)n);
        for (int64_t v = 0; v < n; ++v) cell_point(dims, dg.cell[v], dg.desc[v], &g.pos[3 * v]);
        g.members.assign(n, 1);
        g.comp = comp;
        std::vector<std::pair<int64_t, int64_t>> pairs;
        for (int64_t v = 0; v < n; ++v)
            for (int64_t e = dg.start[v]; e < dg.start[v + 1]; ++e)
                if (v < dg.nbr[e]) pairs.emplace_back(v, dg.nbr[e]);
        csr_from_pairs(n, pairs, g);
        Geom geo{{(double)dims.nx, (double)dims.ny, (double)dims.nz},
                 {(int)(dims.periodic & 1u), (int)((dims.periodic >> 1) & 1u), (int)((dims.periodic >> 2) & 1u)}};
        vx_reduced *r = new vx_reduced();
        r->dims = dims;
        for (int p = 0; p < max_passes; ++p) {
            PGraph next = reduce_pass(g, geo, 0.5 * box_k);
            const bool merged = next.n < g.n;
            g = std::move(next);
            ++r->passes;
            if (!merged) break;
        }
        r->g = std::move(g);
        *out = r;
        return VX_OK;
    } catch (const std::bad_alloc &) {
        return VX_ERR_NOMEM;
    }
}

extern "C" vx_status vx_reduced_info(const vx_reduced *r, int64_t *nnode, int64_t *nedge, int32_t *passes) {
    if (!r) return VX_ERR_INVALID;
    if (nnode) *nnode = r->g.n;
    if (nedge) *nedge = (int64_t)r->g.nbr.size() / 2;
    if (passes) *passes = r->passes;
    return VX_OK;
}

extern "C" vx_status vx_reduced_get(const vx_reduced *r, double *h_pos, int64_t *h_edges, int64_t *h_members,
                                    int64_t *h_comp) {
    if (!r) return VX_ERR_INVALID;
    const PGraph &g = r->g;
    if (h_pos) std::memcpy(h_pos, g.pos.data(), g.pos.size() * sizeof(double));
    if (h_edges) {
        int64_t k = 0;
        for (int64_t u = 0; u < g.n; ++u)
            for (int64_t e = g.start[u]; e < g.start[u + 1]; ++e)
                if (u < g.nbr[e]) {
                    h_edges[2 * k] = u;
                    h_edges[2 * k + 1] = g.nbr[e];
                    ++k;
                }
    }
    if (h_members) std::memcpy(h_members, g.members.data(), g.members.size() * sizeof(int64_t));
    if (h_comp) std::memcpy(h_comp, g.comp.data(), g.comp.size() * sizeof(int64_t));
    return VX_OK;
}

extern "C" vx_status vx_reduced_seeds(const vx_reduced *r, const uint64_t *h_cells, const uint16_t *h_cell_desc,
                                      int64_t n, uint64_t *h_seed_cell, uint16_t *h_seed_desc, float *h_seed_off) {
    if (!r || !h_seed_cell || !h_seed_desc || !h_seed_off || n < 0 || (n > 0 && (!h_cells || !h_cell_desc)))
        return VX_ERR_INVALID;
    try {
        const vx_dims &d = r->dims;
        std::vector<std::pair<uint64_t, uint16_t>> listed(n);
        for (int64_t i = 0; i < n; ++i) listed[i] = {h_cells[i], h_cell_desc[i]};
        std::sort(listed.begin(), listed.end());
        const int64_t dim[3] = {d.nx, d.ny, d.nz};
        for (int64_t v = 0; v < r->g.n; ++v) {
            int64_t c[3];
            for (int q = 0; q < 3; ++q) {
                const double x = r->g.pos[3 * v + q], fl = std::floor(x);
                double off;
                if ((d.periodic >> q) & 1u) {  // the cell that holds x, wrapped
                    c[q] = (((int64_t)fl % dim[q]) + dim[q]) % dim[q];
                    off = x - fl;
                } else {  // cells of an open axis: min corner 0 .. n - 2
                    c[q] = std::min<int64_t>(std::max<int64_t>((int64_t)fl, 0), std::max<int64_t>(dim[q] - 2, 0));
                    off = x - (double)c[q];
                }
                h_seed_off[3 * v + q] = (float)off;
            }
            const uint64_t id = (uint64_t)c[0] + (uint64_t)d.nx * ((uint64_t)c[1] + (uint64_t)d.ny * (uint64_t)c[2]);
            h_seed_cell[v] = id;
            const auto it = std::lower_bound(listed.begin(), listed.end(), std::make_pair(id, (uint16_t)0));
            h_seed_desc[v] = (it != listed.end() && it->first == id) ? it->second : 0;
        }
        return VX_OK;
    } catch (const std::bad_alloc &) {
        return VX_ERR_NOMEM;
    }
}

extern "C" vx_status vx_reduced_destroy(vx_reduced *r) {
    delete r;
    return VX_OK;
}

// ------------------------------------------------------------------------------------------------
// Vectorisation (Sec. 3.4): chains split at branch points, re-ordered from their starting points,
// and uniform Catmull-Rom curves through the ordered samples.

namespace vxg {

struct Curves {
    std::vector<int64_t> node_start{0};  // chain c: nodes[node_start[c] .. node_start[c+1])
    std::vector<int64_t> nodes;
    std::vector<int32_t> closed;
    std::vector<int64_t> pt_start{0};    // curve c: pts[pt_start[c] .. pt_start[c+1]) (3 doubles each)
    std::vector<double> pts;
    std::vector<double> len;
    double total = 0.0;
};

// Point at parameter t of the uniform Catmull-Rom segment from b to c (neighbours a and d).
inline void catmull_rom(const double *a, const double *b, const double *c, const double *d, double t, double *o) {
    const double t2 = t * t, t3 = t2 * t;
    for (int q = 0; q < 3; ++q)
        o[q] = 0.5 * ((2.0 * b[q]) + (c[q] - a[q]) * t + (2.0 * a[q] - 5.0 * b[q] + 4.0 * c[q] - d[q]) * t2 +
                      (3.0 * b[q] - a[q] - 3.0 * c[q] + d[q]) * t3);
}

// The curve of one chain: its control points unwrapped along the chain (each one the previous plus
// the minimum-image displacement), end points repeated for an open chain, wrapped around (shifted by
// the loop's lattice displacement) for a closed one; `seg` points per segment, then the last point.
inline void chain_curve(const Geom &geo, const std::vector<double> &pos, const int64_t *nodes, int64_t m, bool closed,
                        int seg, Curves &cv) {
    std::vector<double> P(3 * (size_t)(m + 1));
    for (int q = 0; q < 3; ++q) P[q] = pos[3 * nodes[0] + q];
    for (int64_t i = 1; i <= m; ++i) {
        const int64_t prev = nodes[i - 1], cur = nodes[i % m];
        double dd[3];
        geo.disp(&pos[3 * prev], &pos[3 * cur], dd);
        for (int q = 0; q < 3; ++q) P[3 * i + q] = P[3 * (i - 1) + q] + dd[q];
    }
    // P[m] is the closing point of a loop (node 0 after one turn)
    const double shift[3] = {P[3 * m] - P[0], P[3 * m + 1] - P[1], P[3 * m + 2] - P[2]};
    auto ctrl = [&](int64_t i, double *o) {  // control point i of the chain, any integer i
        if (!closed) {
            const int64_t j = std::min<int64_t>(std::max<int64_t>(i, 0), m - 1);
            for (int q = 0; q < 3; ++q) o[q] = P[3 * j + q];
            return;
        }
        int64_t turns = 0, j = i;
        while (j < 0) {
            j += m;
            --turns;
        }
        while (j >= m) {
            j -= m;
            ++turns;
        }
        for (int q = 0; q < 3; ++q) o[q] = P[3 * j + q] + (double)turns * shift[q];
    };
    const int64_t nseg = closed ? m : m - 1;
    double length = 0.0, last[3] = {0, 0, 0};
    bool have = false;
    auto emit = [&](const double *o) {
        if (have) {
            const double dx = o[0] - last[0], dy = o[1] - last[1], dz = o[2] - last[2];
            length += std::sqrt(dx * dx + dy * dy + dz * dz);
        }
        for (int q = 0; q < 3; ++q) {
            cv.pts.push_back(o[q]);
            last[q] = o[q];
        }
        have = true;
    };
    double a[3], b[3], c[3], d[3], o[3];
    for (int64_t i = 0; i < nseg; ++i) {
        ctrl(i - 1, a);
        ctrl(i, b);
        ctrl(i + 1, c);
        ctrl(i + 2, d);
        for (int j = 0; j < seg; ++j) {
            catmull_rom(a, b, c, d, (double)j / (double)seg, o);
            emit(o);
        }
    }
    ctrl(nseg, o);  // the end of the last segment (a loop's closing point; a single node's only point)
    emit(o);
    cv.pt_start.push_back((int64_t)cv.pts.size() / 3);
    cv.len.push_back(length);
    cv.total += length;
}

inline void build_curves(const Geom &geo, const std::vector<double> &pos, int64_t n, const std::vector<int64_t> &start,
                         const std::vector<int64_t> &nbr, int seg, Curves &cv) {
    std::vector<int64_t> deg(n);
    for (int64_t v = 0; v < n; ++v) deg[v] = start[v + 1] - start[v];
    std::vector<char> used(nbr.size(), 0);
    auto mark = [&](int64_t u, int64_t w) {  // mark edge u-w used in both directions
        for (int64_t e = start[u]; e < start[u + 1]; ++e)
            if (nbr[e] == w) used[e] = 1;
        for (int64_t e = start[w]; e < start[w + 1]; ++e)
            if (nbr[e] == u) used[e] = 1;
    };
    std::vector<int64_t> chain;
    auto finish = [&](bool closed) {
        cv.nodes.insert(cv.nodes.end(), chain.begin(), chain.end());
        cv.node_start.push_back((int64_t)cv.nodes.size());
        cv.closed.push_back(closed ? 1 : 0);
        chain_curve(geo, pos, chain.data(), (int64_t)chain.size(), closed, seg, cv);
    };
    // chains between ends (connectivity other than 2), from the lowest end, edges in neighbour order
    for (int64_t v = 0; v < n; ++v) {
        if (deg[v] == 2) continue;
        if (deg[v] == 0) {
            chain.assign(1, v);
            finish(false);
            continue;
        }
        for (int64_t e = start[v]; e < start[v + 1]; ++e) {
            if (used[e]) continue;
            chain.assign(1, v);
            int64_t prev = v, cur = nbr[e];
            mark(prev, cur);
            chain.push_back(cur);
            while (deg[cur] == 2) {
                const int64_t a = nbr[start[cur]], b = nbr[start[cur] + 1];
                const int64_t nxt = a == prev ? b : a;
                mark(cur, nxt);
                prev = cur;
                cur = nxt;
                chain.push_back(cur);
            }
            finish(false);
        }
    }
    // what is left are loops of connectivity-2 nodes: from the lowest node towards its lower neighbour
    for (int64_t v = 0; v < n; ++v) {
        if (deg[v] != 2 || used[start[v]]) continue;
        chain.assign(1, v);
        int64_t prev = v, cur = std::min(nbr[start[v]], nbr[start[v] + 1]);
        mark(prev, cur);
        while (cur != v) {
            chain.push_back(cur);
            const int64_t a = nbr[start[cur]], b = nbr[start[cur] + 1];
            const int64_t nxt = a == prev ? b : a;
            mark(cur, nxt);
            prev = cur;
            cur = nxt;
        }
        finish(true);
    }
}

}  // namespace vxg

struct vx_curves {
    Curves c;
};

extern "C" vx_status vx_curves_build(vx_dims dims, const double *h_pos, int64_t n, const int64_t *h_edges,
                                     int64_t nedge, int seg_points, vx_curves **out) {
    if (!out) return VX_ERR_INVALID;
    *out = nullptr;
    if (n < 0 || nedge < 0 || (n > 0 && !h_pos) || (nedge > 0 && !h_edges) || seg_points < 1 || seg_points > 1024)
        return VX_ERR_INVALID;
    if (dims.nx < 1 || dims.ny < 1 || dims.nz < 1 || dims.periodic > 7u) return VX_ERR_INVALID;
    try {
        std::vector<std::pair<int64_t, int64_t>> pairs;
        for (int64_t e = 0; e < nedge; ++e) {
            const int64_t u = h_edges[2 * e], v = h_edges[2 * e + 1];
            if (u < 0 || u >= n || v < 0 || v >= n) return VX_ERR_INVALID;
            pairs.emplace_back(u, v);
        }
        PGraph g;
        g.n = n;
        csr_from_pairs(n, pairs, g);
        std::vector<double> pos(h_pos, h_pos + 3 * n);
        Geom geo{{(double)dims.nx, (double)dims.ny, (double)dims.nz},
                 {(int)(dims.periodic & 1u), (int)((dims.periodic >> 1) & 1u), (int)((dims.periodic >> 2) & 1u)}};
        vx_curves *cv = new vx_curves();
        build_curves(geo, pos, n, g.start, g.nbr, seg_points, cv->c);
        *out = cv;
        return VX_OK;
    } catch (const std::bad_alloc &) {
        return VX_ERR_NOMEM;
    }
}

extern "C" vx_status vx_curves_info(const vx_curves *cv, int64_t *ncurve, int64_t *npoint, int64_t *nnode,
                                    double *total_length) {
    if (!cv) return VX_ERR_INVALID;
    if (ncurve) *ncurve = (int64_t)cv->c.len.size();
    if (npoint) *npoint = (int64_t)cv->c.pts.size() / 3;
    if (nnode) *nnode = (int64_t)cv->c.nodes.size();
    if (total_length) *total_length = cv->c.total;
    return VX_OK;
}

extern "C" vx_status vx_curves_get(const vx_curves *cv, int64_t *h_pt_start, double *h_points, double *h_length,
                                   int32_t *h_closed, int64_t *h_node_start, int64_t *h_nodes) {
    if (!cv) return VX_ERR_INVALID;
    const Curves &c = cv->c;
    if (h_pt_start) std::memcpy(h_pt_start, c.pt_start.data(), c.pt_start.size() * sizeof(int64_t));
    if (h_points) std::memcpy(h_points, c.pts.data(), c.pts.size() * sizeof(double));
    if (h_length) std::memcpy(h_length, c.len.data(), c.len.size() * sizeof(double));
    if (h_closed) std::memcpy(h_closed, c.closed.data(), c.closed.size() * sizeof(int32_t));
    if (h_node_start) std::memcpy(h_node_start, c.node_start.data(), c.node_start.size() * sizeof(int64_t));
    if (h_nodes) std::memcpy(h_nodes, c.nodes.data(), c.nodes.size() * sizeof(int64_t));
    return VX_OK;
}

extern "C" vx_status vx_curves_destroy(vx_curves *cv) {
    delete cv;
    return VX_OK;
}
