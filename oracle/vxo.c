/*
 * CPU ORACLE -- test infrastructure only.
 *
 * A plain, slow, obviously correct implementation of the vortex-core hot path described in
 * Liu, Xiong & Liu, "Vectorizing Quantum Turbulence Vortex-Core Lines for Real-Time
 * Visualization" (arXiv 1911.12070):
 *   - circulation-based identification (Sec. 2.2, circulation equation): the phase winding of
 *     psi around every unit face of the grid, one face per node and axis;
 *   - the pierced faces and pierced cells (the vortex-node graph of Sec. 3.1 in dual form);
 *   - the mean-position estimate of a core sample (Sec. 3.3.1) and its density-guided
 *     refinement (Sec. 3.3.3): minimise |psi|^2 in the plane through the estimate that is normal
 *     to the pseudo-vorticity direction, psi linearly interpolated between nodes (Sec. 5).
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg load this library. It
 * shares no code with the GPU library. FP64 throughout except where the winding predicate works
 * on the FP32 input values themselves.
 *
 * Grid layout: node (i,j,k) has linear id n = i + nx*(j + ny*k) (x fastest, the scan order of
 * Sec. 3.1); psi is complex64 interleaved (re, im).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------------------------
 * Winding of one face.
 *
 * The circulation of grad(phase) around a closed path is 2*pi times the winding number of the
 * path's image in the complex plane about the origin (Sec. 2.2). For a unit face with psi
 * interpolated linearly along its edges (Sec. 5 assumes linear interpolation between nodes), the
 * image is a quadrilateral with straight edges. Its winding number is counted with the
 * crossing-number rule: an edge that crosses the ray from the origin along +Re upwards counts +1,
 * downwards -1. To give every degenerate configuration (a vertex at 0, an edge through 0) exactly
 * one answer, the point is taken at q = (-delta, +eps) with 0 < eps << delta << 1: an edge a->b
 * crosses upwards iff Im a <= 0 < Im b, and then counts iff cross(a, b) >= 0; downwards iff
 * Im a > 0 >= Im b, and then counts iff cross(a, b) <= 0, where cross(a,b) = Re a Im b - Im a Re b.
 * The two products are exact in FP64 (24-bit significands), so the comparison is exact.
 * ------------------------------------------------------------------------------------------- */
static int edge_count(const float *a, const float *b) {
    int up = (a[1] <= 0.0f) && (b[1] > 0.0f);
    int down = (a[1] > 0.0f) && (b[1] <= 0.0f);
    if (!up && !down) return 0;
    double p1 = (double)a[0] * (double)b[1];
    double p2 = (double)a[1] * (double)b[0];
    if (up) return p1 >= p2 ? 1 : 0;
    return p1 <= p2 ? -1 : 0;
}

int vxo_edge(const float *a, const float *b) { return edge_count(a, b); }

/* Winding number of the closed polygon v0->v1->v2->v3->v0 about q. */
static int polygon_winding(const float *v0, const float *v1, const float *v2, const float *v3) {
    return edge_count(v0, v1) + edge_count(v1, v2) + edge_count(v2, v3) + edge_count(v3, v0);
}

int vxo_polygon(const float *v0, const float *v1, const float *v2, const float *v3) {
    return polygon_winding(v0, v1, v2, v3);
}

typedef struct {
    int64_t n[3];
    int periodic[3];
} grid_t;

/* Index of node (i,j,k) after periodic wrap; -1 if an index is outside a non-periodic axis. */
static int64_t node_index(const grid_t *g, int64_t i, int64_t j, int64_t k) {
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= g->n[a]) {
            if (!g->periodic[a]) return -1;
            c[a] = ((c[a] % g->n[a]) + g->n[a]) % g->n[a];
        }
    }
    return c[0] + g->n[0] * (c[1] + g->n[1] * c[2]);
}

/*
 * Winding of face (node (i,j,k), normal axis a), counted by the right-hand rule about +e_a
 * (Sec. 3.4: line direction from the circulation path by the right-hand rule). The corners are
 * visited counter-clockwise seen from +e_a:
 *   a = x (yz-face): n, n+ey, n+ey+ez, n+ez
 *   a = y (zx-face): n, n+ez, n+ez+ex, n+ex
 *   a = z (xy-face): n, n+ex, n+ex+ey, n+ey
 * Returns 0 for a face that needs a node outside a non-periodic axis (the face does not exist).
 */
static int face_winding(const grid_t *g, const float *psi, int64_t i, int64_t j, int64_t k, int a) {
    int64_t c[4];
    if (a == 0) {
        c[0] = node_index(g, i, j, k);     c[1] = node_index(g, i, j + 1, k);
        c[2] = node_index(g, i, j + 1, k + 1); c[3] = node_index(g, i, j, k + 1);
    } else if (a == 1) {
        c[0] = node_index(g, i, j, k);     c[1] = node_index(g, i, j, k + 1);
        c[2] = node_index(g, i + 1, j, k + 1); c[3] = node_index(g, i + 1, j, k);
    } else {
        c[0] = node_index(g, i, j, k);     c[1] = node_index(g, i + 1, j, k);
        c[2] = node_index(g, i + 1, j + 1, k); c[3] = node_index(g, i, j + 1, k);
    }
    for (int q = 0; q < 4; ++q)
        if (c[q] < 0) return 0;
    return polygon_winding(psi + 2 * c[0], psi + 2 * c[1], psi + 2 * c[2], psi + 2 * c[3]);
}

static int cell_exists(const grid_t *g, int64_t i, int64_t j, int64_t k) {
    int64_t c[3] = {i, j, k};
    for (int a = 0; a < 3; ++a)
        if (!g->periodic[a] && c[a] + 1 >= g->n[a]) return 0;
    return 1;
}

static unsigned enc2(int w) { return (unsigned)w & 3u; } /* 2-bit two's complement */

/*
 * Whole-grid winding pass.
 *   w       : int8[3*N] (nullable) face windings, w[3n+a]
 *   packed  : uint8[N]  (nullable) bits 1:0 w_x, 3:2 w_y, 5:4 w_z, bit 6 = cell n pierced
 *   faces   : pierced faces in ascending id = 3n+a, with their sign (fsign)
 *   cells   : pierced cells in ascending id = n, with their 12-bit descriptor: 2-bit windings of
 *             the faces (-x, +x, -y, +y, -z, +z) = (w_x(n), w_x(n+ex), w_y(n), w_y(n+ey),
 *             w_z(n), w_z(n+ez)), each about +e_axis, lowest bits first
 *   counts  : [0] pierced faces, [1] pierced cells (true counts; arrays hold at most cap entries)
 */
void vxo_winding(int nx, int ny, int nz, unsigned periodic, const float *psi, int8_t *w,
                 uint8_t *packed, uint64_t *faces, int8_t *fsign, int64_t face_cap,
                 uint64_t *cells, uint16_t *cdesc, int64_t cell_cap, int64_t *counts) {
    grid_t g = {{nx, ny, nz}, {(int)(periodic & 1u), (int)((periodic >> 1) & 1u), (int)((periodic >> 2) & 1u)}};
    int64_t nf = 0, nc = 0;
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                int64_t n = i + (int64_t)nx * (j + (int64_t)ny * k);
                int wn[3];
                for (int a = 0; a < 3; ++a) {
                    wn[a] = face_winding(&g, psi, i, j, k, a);
                    if (w) w[3 * n + a] = (int8_t)wn[a];
                    if (wn[a] != 0) {
                        if (nf < face_cap) {
                            faces[nf] = (uint64_t)(3 * n + a);
                            fsign[nf] = (int8_t)wn[a];
                        }
                        ++nf;
                    }
                }
                int pierced = 0;
                unsigned desc = 0;
                if (cell_exists(&g, i, j, k)) {
                    int f6[6] = {wn[0], face_winding(&g, psi, i + 1, j, k, 0),
                                 wn[1], face_winding(&g, psi, i, j + 1, k, 1),
                                 wn[2], face_winding(&g, psi, i, j, k + 1, 2)};
                    for (int f = 0; f < 6; ++f) {
                        desc |= enc2(f6[f]) << (2 * f);
                        if (f6[f] != 0) pierced = 1;
                    }
                    if (pierced) {
                        if (nc < cell_cap) {
                            cells[nc] = (uint64_t)n;
                            cdesc[nc] = (uint16_t)desc;
                        }
                        ++nc;
                    }
                }
                if (packed)
                    packed[n] = (uint8_t)(enc2(wn[0]) | (enc2(wn[1]) << 2) | (enc2(wn[2]) << 4) |
                                          ((unsigned)pierced << 6));
            }
    if (counts) {
        counts[0] = nf;
        counts[1] = nc;
    }
}

/* Windings and packed bytes for the nodes of a box (x0,y0,z0, bx,by,bz) of a grid whose values are
 * given only on the box plus one node in each positive direction (sub = (bz+1)*(by+1)*(bx+1)
 * complex values, x fastest). Used for sampled checks of large grids: the face windings and the
 * cell flag of node n depend only on the 2x2x2 nodes n + {0,1}^3. Periodicity is that of the
 * full grid; the caller supplies wrapped values. Faces and cells that would need a node outside a
 * non-periodic axis of the full grid are zero, as in vxo_winding. */
void vxo_winding_box(int nx, int ny, int nz, unsigned periodic, int x0, int y0, int z0, int bx,
                     int by, int bz, const float *sub, int8_t *w, uint8_t *packed, uint16_t *cdesc) {
    int64_t sx = bx + 1, sy = by + 1;
    for (int64_t k = 0; k < bz; ++k)
        for (int64_t j = 0; j < by; ++j)
            for (int64_t i = 0; i < bx; ++i) {
                int64_t gi = x0 + i, gj = y0 + j, gk = z0 + k;
                int exists[3];
                /* face a exists iff the two in-plane axes can step +1 */
                int step[3] = {(periodic & 1u) || gi + 1 < nx, ((periodic >> 1) & 1u) || gj + 1 < ny,
                               ((periodic >> 2) & 1u) || gk + 1 < nz};
                exists[0] = step[1] && step[2];
                exists[1] = step[2] && step[0];
                exists[2] = step[0] && step[1];
#define S(di, dj, dk) (sub + 2 * ((i + (di)) + sx * ((j + (dj)) + sy * (k + (dk)))))
                int wn[3];
                wn[0] = exists[0] ? polygon_winding(S(0, 0, 0), S(0, 1, 0), S(0, 1, 1), S(0, 0, 1)) : 0;
                wn[1] = exists[1] ? polygon_winding(S(0, 0, 0), S(0, 0, 1), S(1, 0, 1), S(1, 0, 0)) : 0;
                wn[2] = exists[2] ? polygon_winding(S(0, 0, 0), S(1, 0, 0), S(1, 1, 0), S(0, 1, 0)) : 0;
                int cell = step[0] && step[1] && step[2];
                int pierced = 0;
                unsigned desc = 0;
                if (cell) {
                    int f6[6] = {wn[0], polygon_winding(S(1, 0, 0), S(1, 1, 0), S(1, 1, 1), S(1, 0, 1)),
                                 wn[1], polygon_winding(S(0, 1, 0), S(0, 1, 1), S(1, 1, 1), S(1, 1, 0)),
                                 wn[2], polygon_winding(S(0, 0, 1), S(1, 0, 1), S(1, 1, 1), S(0, 1, 1))};
                    for (int f = 0; f < 6; ++f) {
                        desc |= enc2(f6[f]) << (2 * f);
                        if (f6[f] != 0) pierced = 1;
                    }
                }
#undef S
                int64_t q = i + bx * (j + (int64_t)by * k);
                if (w)
                    for (int a = 0; a < 3; ++a) w[3 * q + a] = (int8_t)wn[a];
                if (packed)
                    packed[q] = (uint8_t)(enc2(wn[0]) | (enc2(wn[1]) << 2) | (enc2(wn[2]) << 4) |
                                          ((unsigned)pierced << 6));
                if (cdesc) cdesc[q] = (uint16_t)(pierced ? desc : 0);
            }
}

/* ---------------------------------------------------------------------------------------------
 * Core-sample refinement (Sec. 3.3.3).
 * ------------------------------------------------------------------------------------------- */

enum {
    ST_MULTI = 1,            /* four or six pierced faces: a branch / reconnection cell */
    ST_TANGENT_FALLBACK = 2, /* pseudo-vorticity degenerate; face-flux direction used */
    ST_BOUNDARY = 4,         /* a trial point was rejected because it left the patch */
    ST_NONZERO_MIN = 8,      /* |psi|^2 above rho_tol at the end */
    ST_NOT_CONVERGED = 16,   /* Newton polish ended without a short step and rho above rho_tol */
    ST_NO_FACES = 32         /* the listed cell has no pierced face */
};

typedef struct {
    int32_t max_descent, max_newton, max_halvings;
    double step0, step_max, armijo, descent_tol, newton_tol, rho_tol;
} vxo_refine_params;

/* A 4x4x4 patch of nodes around cell n: local node (a,b,c), a,b,c in 0..3, is grid node
 * n + (a-1, b-1, c-1). lo/hi bound the cell-local coordinates that the patch covers on each axis
 * ([-1, 2] inside the grid; narrower next to a non-periodic boundary). */
typedef struct {
    double re[64], im[64];
    int lo[3], hi[3];
} patch_t;

static int pidx(int a, int b, int c) { return a + 4 * (b + 4 * c); }

/* psi linearly interpolated between nodes (Sec. 5): trilinear on the unit cell that holds x,
 * cell = clamp(floor(x), lo, hi-1) per axis. Returns value and gradient in cell units. */
static void trilerp(const patch_t *p, const double x[3], double *vr, double *vi, double gr[3],
                    double gi[3]) {
    int c[3];
    double u[3];
    for (int a = 0; a < 3; ++a) {
        int f = (int)floor(x[a]);
        if (f < p->lo[a]) f = p->lo[a];
        if (f > p->hi[a] - 1) f = p->hi[a] - 1;
        c[a] = f;
        u[a] = x[a] - f;
    }
    *vr = *vi = 0.0;
    for (int a = 0; a < 3; ++a) gr[a] = gi[a] = 0.0;
    for (int d = 0; d < 8; ++d) {
        int dx = d & 1, dy = (d >> 1) & 1, dz = (d >> 2) & 1;
        int q = pidx(c[0] + 1 + dx, c[1] + 1 + dy, c[2] + 1 + dz);
        double wx = dx ? u[0] : 1.0 - u[0];
        double wy = dy ? u[1] : 1.0 - u[1];
        double wz = dz ? u[2] : 1.0 - u[2];
        double sx = dx ? 1.0 : -1.0, sy = dy ? 1.0 : -1.0, sz = dz ? 1.0 : -1.0;
        *vr += wx * wy * wz * p->re[q];
        *vi += wx * wy * wz * p->im[q];
        gr[0] += sx * wy * wz * p->re[q];
        gi[0] += sx * wy * wz * p->im[q];
        gr[1] += wx * sy * wz * p->re[q];
        gi[1] += wx * sy * wz * p->im[q];
        gr[2] += wx * wy * sz * p->re[q];
        gi[2] += wx * wy * sz * p->im[q];
    }
}

static int inside(const patch_t *p, const double x[3]) {
    for (int a = 0; a < 3; ++a)
        if (!(x[a] >= p->lo[a] && x[a] <= p->hi[a])) return 0;
    return 1;
}

static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]); }
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

static int dec2(unsigned desc, int f) {
    unsigned v = (desc >> (2 * f)) & 3u;
    return v == 1 ? 1 : (v == 3 ? -1 : 0);
}

/*
 * Refine one core sample of a pierced cell.
 *  1. x0 = mean of the centres of the cell's pierced faces: the mean-position estimator of
 *     Sec. 3.3.1, applied to the dual graph with a one-cell box.
 *  2. t = grad Re psi x grad Im psi at x0, normalised: the pseudo-vorticity direction of the
 *     line (Sec. 3.3.3). If it is degenerate (|t| <= 1e-6 |grad Re| |grad Im|), t is the face
 *     flux (w(-a) + w(+a))_a of the cell; if that is zero too, the first pierced face's normal
 *     times its winding.
 *  3. The plane through x0 normal to t, with basis e1 = normalize(t x e_u) (u = axis of the
 *     smallest |t_u|, lowest index first) and e2 = t x e1.
 *  4. Gradient descent of f(y) = |psi(x0 + y1 e1 + y2 e2)|^2 from y = 0 (the paper's in-plane
 *     minimisation): steepest-descent direction, trial step length
 *     s = min(2 s_prev, step_max) (the first is step0), halved until the Armijo condition
 *     f(y + s d) <= f(y) - armijo * s * |g| holds; at most max_descent accepted steps; stop
 *     once an accepted step is shorter than descent_tol.
 *  5. Newton polish on r(y) = (Re psi, Im psi) with the 2x2 in-plane Jacobian, which has the
 *     same fixed point as the descent when it reaches a zero of psi: a step is halved until
 *     f decreases strictly; at most max_newton steps; stop once a step is shorter than
 *     newton_tol.
 *  Trial points outside the patch count as rejected trials (status BOUNDARY).
 */
void vxo_refine_patch(const patch_t *p, unsigned desc, const double *seed, const vxo_refine_params *prm,
                      double xout[3], double *rho_out, int *iters_out, int *status_out, double *cond_out) {
    static const double ctr[6][3] = {{0, .5, .5}, {1, .5, .5}, {.5, 0, .5},
                                     {.5, 1, .5}, {.5, .5, 0}, {.5, .5, 1}};
    int status = 0, npierced = 0;
    double x0[3] = {0, 0, 0};
    for (int f = 0; f < 6; ++f)
        if (dec2(desc, f) != 0) {
            for (int a = 0; a < 3; ++a) x0[a] += ctr[f][a];
            ++npierced;
        }
    if (npierced == 0) {
        x0[0] = x0[1] = x0[2] = 0.5;
        status |= ST_NO_FACES;
    } else {
        for (int a = 0; a < 3; ++a) x0[a] /= npierced;
    }
    if (npierced >= 4) status |= ST_MULTI;
    /* a caller's seed (a sample point of the box reduction, Sec. 3.3.2) replaces the estimate */
    if (seed)
        for (int a = 0; a < 3; ++a) x0[a] = seed[a];

    double vr, vi, gr[3], gi[3];
    trilerp(p, x0, &vr, &vi, gr, gi);

    double t[3];
    cross3(gr, gi, t);
    double tn = norm3(t);
    if (!(tn > 1e-6 * norm3(gr) * norm3(gi)) || tn == 0.0) {
        status |= ST_TANGENT_FALLBACK;
        for (int a = 0; a < 3; ++a) t[a] = (double)(dec2(desc, 2 * a) + dec2(desc, 2 * a + 1));
        if (norm3(t) == 0.0) {
            t[0] = 0.0; t[1] = 0.0; t[2] = 1.0;
            for (int f = 0; f < 6; ++f)
                if (dec2(desc, f) != 0) {
                    t[0] = t[1] = t[2] = 0.0;
                    t[f / 2] = (double)dec2(desc, f);
                    break;
                }
        }
        tn = norm3(t);
    }
    for (int a = 0; a < 3; ++a) t[a] /= tn;

    int u = 0;
    for (int a = 1; a < 3; ++a)
        if (fabs(t[a]) < fabs(t[u])) u = a;
    double eu[3] = {0, 0, 0};
    eu[u] = 1.0;
    double e1[3], e2[3];
    cross3(t, eu, e1);
    double n1 = norm3(e1);
    for (int a = 0; a < 3; ++a) e1[a] /= n1;
    cross3(t, e1, e2);

    double y[2] = {0.0, 0.0}, x[3];
    for (int a = 0; a < 3; ++a) x[a] = x0[a];
    double f = vr * vr + vi * vi;
    int iters = 0;

    /* gradient descent */
    double s_prev = 0.5 * prm->step0;
    for (int it = 0; it < prm->max_descent; ++it) {
        if (f == 0.0) break;
        double G[3];
        for (int a = 0; a < 3; ++a) G[a] = 2.0 * (vr * gr[a] + vi * gi[a]);
        double g1 = dot3(e1, G), g2 = dot3(e2, G);
        double gn = sqrt(g1 * g1 + g2 * g2);
        if (gn == 0.0) break;
        double d1 = -g1 / gn, d2 = -g2 / gn;
        double s = 2.0 * s_prev;
        if (s > prm->step_max) s = prm->step_max;
        int accepted = 0;
        double yt[2], xt[3], tr, ti, tgr[3], tgi[3], ft = 0.0;
        for (int h = 0; h < prm->max_halvings; ++h) {
            yt[0] = y[0] + s * d1;
            yt[1] = y[1] + s * d2;
            for (int a = 0; a < 3; ++a) xt[a] = x0[a] + yt[0] * e1[a] + yt[1] * e2[a];
            if (!inside(p, xt)) {
                status |= ST_BOUNDARY;
                s *= 0.5;
                continue;
            }
            trilerp(p, xt, &tr, &ti, tgr, tgi);
            ft = tr * tr + ti * ti;
            if (ft <= f - prm->armijo * s * gn) {
                accepted = 1;
                break;
            }
            s *= 0.5;
        }
        if (!accepted) break;
        y[0] = yt[0];
        y[1] = yt[1];
        for (int a = 0; a < 3; ++a) {
            x[a] = xt[a];
            gr[a] = tgr[a];
            gi[a] = tgi[a];
        }
        vr = tr;
        vi = ti;
        f = ft;
        s_prev = s;
        ++iters;
        if (s < prm->descent_tol) break;
    }

    /* Newton polish */
    int converged = 0;
    for (int it = 0; it < prm->max_newton; ++it) {
        if (f == 0.0) {
            converged = 1;
            break;
        }
        double j00 = dot3(e1, gr), j01 = dot3(e2, gr);
        double j10 = dot3(e1, gi), j11 = dot3(e2, gi);
        double det = j00 * j11 - j01 * j10;
        if (det == 0.0) break;
        double dy0 = -(j11 * vr - j01 * vi) / det;
        double dy1 = -(-j10 * vr + j00 * vi) / det;
        double lam = 1.0;
        int accepted = 0;
        double yt[2], xt[3], tr, ti, tgr[3], tgi[3], ft = 0.0;
        for (int h = 0; h < prm->max_halvings; ++h) {
            yt[0] = y[0] + lam * dy0;
            yt[1] = y[1] + lam * dy1;
            for (int a = 0; a < 3; ++a) xt[a] = x0[a] + yt[0] * e1[a] + yt[1] * e2[a];
            if (!inside(p, xt)) {
                status |= ST_BOUNDARY;
                lam *= 0.5;
                continue;
            }
            trilerp(p, xt, &tr, &ti, tgr, tgi);
            ft = tr * tr + ti * ti;
            if (ft < f) {
                accepted = 1;
                break;
            }
            lam *= 0.5;
        }
        if (!accepted) break;
        double step = lam * sqrt(dy0 * dy0 + dy1 * dy1);
        y[0] = yt[0];
        y[1] = yt[1];
        for (int a = 0; a < 3; ++a) {
            x[a] = xt[a];
            gr[a] = tgr[a];
            gi[a] = tgi[a];
        }
        vr = tr;
        vi = ti;
        f = ft;
        ++iters;
        if (step < prm->newton_tol) {
            converged = 1;
            break;
        }
    }
    if (f > prm->rho_tol) status |= ST_NONZERO_MIN;
    if (!converged && f > prm->rho_tol) status |= ST_NOT_CONVERGED;
    if (cond_out) {
        /* diagnostic only: 2-norm condition number of the in-plane Jacobian of (Re psi, Im psi) at the
         * result, sigma_max / sigma_min from the 2x2 singular values (inf when singular) */
        double j00 = dot3(e1, gr), j01 = dot3(e2, gr), j10 = dot3(e1, gi), j11 = dot3(e2, gi);
        double fro2 = j00 * j00 + j01 * j01 + j10 * j10 + j11 * j11;
        double det = fabs(j00 * j11 - j01 * j10);
        double disc = sqrt(fmax(fro2 * fro2 - 4.0 * det * det, 0.0));
        double smax2 = 0.5 * (fro2 + disc), smin2 = 0.5 * (fro2 - disc);
        *cond_out = (det == 0.0 || smin2 <= 0.0) ? INFINITY : sqrt(smax2 / smin2);
    }
    for (int a = 0; a < 3; ++a) xout[a] = x[a];
    *rho_out = f;
    *iters_out = iters;
    *status_out = status;
}

/* Gather the patch of cell (i,j,k) from the grid. Nodes outside a non-periodic axis are absent:
 * the patch bounds shrink so that no point outside the grid is ever evaluated. */
static void gather_patch(const grid_t *g, const float *psi, int64_t i, int64_t j, int64_t k, patch_t *p) {
    int64_t c0[3] = {i, j, k};
    for (int a = 0; a < 3; ++a) {
        p->lo[a] = (g->periodic[a] || c0[a] - 1 >= 0) ? -1 : 0;
        p->hi[a] = (g->periodic[a] || c0[a] + 2 < g->n[a]) ? 2 : 1;
    }
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                int64_t q = node_index(g, i + a - 1, j + b - 1, k + c - 1);
                int idx = pidx(a, b, c);
                if (q < 0) {
                    p->re[idx] = p->im[idx] = 0.0;
                } else {
                    p->re[idx] = (double)psi[2 * q];
                    p->im[idx] = (double)psi[2 * q + 1];
                }
            }
}

/* Refine the listed cells of a grid. out_x: double[3*ncell] cell-local position of the sample;
 * rho: |psi|^2 there; iters, status per sample; cond (nullable): the condition number of the
 * in-plane Jacobian at the sample. seeds (nullable, double[3*ncell], cell-local): starting points that
 * replace the face-centre estimate. */
void vxo_refine(int nx, int ny, int nz, unsigned periodic, const float *psi, int64_t ncell,
                const uint64_t *cells, const uint16_t *cdesc, const double *seeds, const vxo_refine_params *prm,
                double *out_x, double *rho, int32_t *iters, int32_t *status, double *cond) {
    grid_t g = {{nx, ny, nz}, {(int)(periodic & 1u), (int)((periodic >> 1) & 1u), (int)((periodic >> 2) & 1u)}};
    patch_t p;
    for (int64_t s = 0; s < ncell; ++s) {
        int64_t n = (int64_t)cells[s];
        int64_t i = n % nx, j = (n / nx) % ny, k = n / ((int64_t)nx * ny);
        gather_patch(&g, psi, i, j, k, &p);
        int it, st;
        vxo_refine_patch(&p, cdesc[s], seeds ? seeds + 3 * s : NULL, prm, out_x + 3 * s, rho + s, &it, &st,
                         cond ? cond + s : NULL);
        iters[s] = it;
        status[s] = st;
    }
}

/* Refine one sample from an explicit patch (re/im arrays of 64, local node (a,b,c) at a+4b+16c)
 * and patch bounds lo[3], hi[3]. */
void vxo_refine_one(const double *re, const double *im, const int *lo, const int *hi, unsigned desc,
                    const vxo_refine_params *prm, double *xout, double *rho, int32_t *iters,
                    int32_t *status) {
    patch_t p;
    memcpy(p.re, re, sizeof p.re);
    memcpy(p.im, im, sizeof p.im);
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = lo[a];
        p.hi[a] = hi[a];
    }
    int it, st;
    vxo_refine_patch(&p, desc, NULL, prm, xout, rho, &it, &st, NULL);
    *iters = it;
    *status = st;
}

/* Trilinear value and gradient on an explicit patch (exposed for the tests). */
void vxo_trilerp(const double *re, const double *im, const int *lo, const int *hi, const double *x,
                 double *out /* vr, vi, gr[3], gi[3] */) {
    patch_t p;
    memcpy(p.re, re, sizeof p.re);
    memcpy(p.im, im, sizeof p.im);
    for (int a = 0; a < 3; ++a) {
        p.lo[a] = lo[a];
        p.hi[a] = hi[a];
    }
    trilerp(&p, x, out, out + 1, out + 2, out + 5);
}
