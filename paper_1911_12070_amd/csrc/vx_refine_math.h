// Device arithmetic of the core-sample refinement (Sec. 3.3.1 mean-position estimate, Sec. 3.3.3
// in-plane minimisation of |psi|^2 with psi linearly interpolated between nodes, Sec. 5), shared by
// every kernel that evaluates or steps a sample: the refinement kernels and the surrogate's polish.
// Each function contracts products into sums within its own expressions only (the pragma at the top
// of each body), so that it rounds alike in every translation unit and whatever the surrounding
// control flow: the refinement kernels rely on this to be bit-identical to one another.
#pragma once

#include "vx_internal.h"

#define VX_CONTRACT_ON _Pragma("clang fp contract(on)")

namespace vxr {

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float a, float b, float c) {
    VX_CONTRACT_ON
    return V3{a, b, c};
}
__device__ __forceinline__ float dot(const V3 &a, const V3 &b) {
    VX_CONTRACT_ON
    return a.x * b.x + a.y * b.y + a.z * b.z;
}
__device__ __forceinline__ V3 crs(const V3 &a, const V3 &b) {
    VX_CONTRACT_ON
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// hardware reciprocal square root and reciprocal (about 1 ulp): the normalisations and step
// directions they feed are search directions, whose last-bit rounding does not move the minimum
__device__ __forceinline__ float rsq(float a) {
    VX_CONTRACT_ON
    return __builtin_amdgcn_rsqf(a);
}
__device__ __forceinline__ float rcp(float a) {
    VX_CONTRACT_ON
    return __builtin_amdgcn_rcpf(a);
}
__device__ __forceinline__ float comp(const V3 &a, int i) {
    VX_CONTRACT_ON
    return i == 0 ? a.x : (i == 1 ? a.y : a.z);
}

__device__ __forceinline__ int dec2(uint32_t d, int f) {
    VX_CONTRACT_ON
    const uint32_t v = (d >> (2 * f)) & 3u;
    return v == 1u ? 1 : (v == 3u ? -1 : 0);
}

// node g + c of an axis of n nodes (g in [0, n), c in [-1, 2]): wrapped if the axis is periodic,
// else clamped. In 32-bit unsigned arithmetic, where g + c = -1 is the only value above 2^31.
__device__ __forceinline__ uint32_t wrap(int g, int c, int n, int per) {
    VX_CONTRACT_ON
    const uint32_t q = (uint32_t)g + (uint32_t)c, un = (uint32_t)n;
    const uint32_t below = per ? un - 1u : 0u, above = per ? q - un : un - 1u;
    return q == 0xffffffffu ? below : (q >= un ? above : q);
}

// quotient and remainder of n by d for n < 2^53 (every cell id of a grid that fits in memory):
// an FP64 estimate off by at most one, then an integer correction
__device__ __forceinline__ uint64_t divmod53(uint64_t n, uint64_t d, double rd, uint64_t &r) {
    VX_CONTRACT_ON
    uint64_t q = (uint64_t)((double)n * rd);
    int64_t rem = (int64_t)(n - q * d);
    if (rem < 0) {
        --q;
        rem += (int64_t)d;
    } else if (rem >= (int64_t)d) {
        ++q;
        rem -= (int64_t)d;
    }
    r = (uint64_t)rem;
    return q;
}

// ---- arithmetic shared by the refinement kernels (each a forced-inline function, so that every
// kernel computes the same FP32 expressions and reaches the same bits)

// first estimate (Sec. 3.3.1): mean of the centres of the pierced faces (-x,+x,-y,+y,-z,+z)
__device__ __forceinline__ V3 first_estimate(uint32_t desc, uint32_t &status) {
    VX_CONTRACT_ON
    float sx = 0.f, sy = 0.f, sz = 0.f;
    int npierced = 0;
#pragma unroll
    for (int fc = 0; fc < 6; ++fc) {
        if (dec2(desc, fc) == 0) continue;
        const int a = fc >> 1;
        const float side = (float)(fc & 1);
        sx += a == 0 ? side : 0.5f;
        sy += a == 1 ? side : 0.5f;
        sz += a == 2 ? side : 0.5f;
        ++npierced;
    }
    if (npierced >= 4) status |= VX_SAMPLE_MULTI;
    if (npierced == 0) {
        status |= VX_SAMPLE_NO_FACES;
        return v3(0.5f, 0.5f, 0.5f);
    }
    const float inv = 1.0f / (float)npierced;
    return v3(sx * inv, sy * inv, sz * inv);
}

// The node patch of a sample, in the cell's local coordinates: [lo, hc + 1] per axis, where lo is
// -1 if the patch reaches one node below the cell (else 0) and hc is 1 if it reaches two nodes above
// (else 0) -- the cells of the patch are lo .. hc. Kept as floats so that the per-pass tests need no
// decoding.
struct Box {
    V3 lo, hc;
};

__device__ __forceinline__ Box patch_box(int gi, int gj, int gk, int nx, int ny, int nz, int px, int py, int pz) {
    VX_CONTRACT_ON
    const int g3[3] = {gi, gj, gk};
    const int n3[3] = {nx, ny, nz};
    const int p3[3] = {px, py, pz};
    float lo[3], hc[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[a] = (p3[a] || g3[a] - 1 >= 0) ? -1.f : 0.f;
        hc[a] = (p3[a] || g3[a] + 2 < n3[a]) ? 1.f : 0.f;
    }
    return Box{v3(lo[0], lo[1], lo[2]), v3(hc[0], hc[1], hc[2])};
}

// the patch cell that holds point x (clamped to the patch) and the local coordinates in it;
// returns the cell's code (cx+1) + 4 (cy+1) + 16 (cz+1)
__device__ __forceinline__ int locate(const V3 &x, const Box &b, int c[3], float u[3]) {
    VX_CONTRACT_ON
    const float xs[3] = {x.x, x.y, x.z}, lo[3] = {b.lo.x, b.lo.y, b.lo.z}, hc[3] = {b.hc.x, b.hc.y, b.hc.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const float fl = fminf(fmaxf(floorf(xs[a]), lo[a]), hc[a]);
        c[a] = (int)fl;
        u[a] = xs[a] - fl;
    }
    return (c[0] + 1) + 4 * (c[1] + 1) + 16 * (c[2] + 1);
}

// the 8 nodes of patch cell c of the sample cell at node (gi, gj, gk); corner d = dx + 2 dy + 4 dz
__device__ __forceinline__ void fetch_corners(const float2 *psi_p, int fnx, int fny, int fnz, int fpx, int fpy,
                                              int fpz, int gi, int gj, int gk, const int c[3], float2 v[8]) {
    VX_CONTRACT_ON
    const uint64_t nx64 = (uint64_t)fnx, nxy = (uint64_t)fnx * (uint64_t)fny;
    const uint32_t i0 = wrap(gi, c[0], fnx, fpx), i1 = wrap(gi, c[0] + 1, fnx, fpx);
    const uint32_t j0 = wrap(gj, c[1], fny, fpy), j1 = wrap(gj, c[1] + 1, fny, fpy);
    const uint32_t k0 = wrap(gk, c[2], fnz, fpz), k1 = wrap(gk, c[2] + 1, fnz, fpz);
    const float2 *r00 = psi_p + nx64 * (uint64_t)j0 + nxy * (uint64_t)k0;
    const float2 *r10 = psi_p + nx64 * (uint64_t)j1 + nxy * (uint64_t)k0;
    const float2 *r01 = psi_p + nx64 * (uint64_t)j0 + nxy * (uint64_t)k1;
    const float2 *r11 = psi_p + nx64 * (uint64_t)j1 + nxy * (uint64_t)k1;
    v[0] = r00[i0];
    v[1] = r00[i1];
    v[2] = r10[i0];
    v[3] = r10[i1];
    v[4] = r01[i0];
    v[5] = r01[i1];
    v[6] = r11[i0];
    v[7] = r11[i1];
}

// The trilinear interpolant of a cell as a polynomial in the local coordinates (u, v, w):
// f = c0 + c1 u + c2 v + c3 w + c4 uv + c5 uw + c6 vw + c7 uvw, from the corners d = dx + 2 dy + 4 dz
// (computed once per cell change, then cached)
__device__ __forceinline__ void tri_coeffs(const float2 v[8], float2 c[8]) {
    VX_CONTRACT_ON
    auto sub = [](float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); };
    c[0] = v[0];
    c[1] = sub(v[1], v[0]);
    c[2] = sub(v[2], v[0]);
    c[3] = sub(v[4], v[0]);
    const float2 d32 = sub(v[3], v[2]), d54 = sub(v[5], v[4]), d64 = sub(v[6], v[4]), d76 = sub(v[7], v[6]);
    c[4] = sub(d32, c[1]);
    c[5] = sub(d54, c[1]);
    c[6] = sub(d64, c[2]);
    c[7] = sub(sub(d76, d54), c[4]);
}

// trilinear psi and its gradient (cell units) at local coordinates u of a cell with coefficients c
// (nested: 11 multiply-adds per component)
__device__ __forceinline__ void trilinear(const float2 c[8], const float u[3], float &tr, float &ti, V3 &tgr,
                                          V3 &tgi) {
    VX_CONTRACT_ON
    const float x = u[0], y = u[1], z = u[2];
    float r[2], gx[2], gy[2], gz[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const float c0 = k ? c[0].y : c[0].x, c1 = k ? c[1].y : c[1].x, c2 = k ? c[2].y : c[2].x;
        const float c3 = k ? c[3].y : c[3].x, c4 = k ? c[4].y : c[4].x, c5 = k ? c[5].y : c[5].x;
        const float c6 = k ? c[6].y : c[6].x, c7 = k ? c[7].y : c[7].x;
        const float A = fmaf(c7, z, c4), B = fmaf(c5, z, c1), C = fmaf(c6, z, c2), D = fmaf(c3, z, c0);
        const float E = fmaf(x, A, C);  // d/dy
        r[k] = fmaf(y, E, fmaf(x, B, D));
        gx[k] = fmaf(y, A, B);
        gy[k] = E;
        gz[k] = fmaf(x, fmaf(c7, y, c5), fmaf(c6, y, c3));
    }
    tr = r[0];
    ti = r[1];
    tgr = v3(gx[0], gy[0], gz[0]);
    tgi = v3(gx[1], gy[1], gz[1]);
}

// orthonormal basis (e1, e2) of the plane normal to the pseudo-vorticity Re grad psi x Im grad psi
// at x0; a degenerate cross product falls back to the net face flux, then to one pierced face
__device__ __forceinline__ void plane_basis(const V3 &tgr, const V3 &tgi, uint32_t desc, V3 &e1, V3 &e2,
                                            uint32_t &status) {
    VX_CONTRACT_ON
    V3 t = crs(tgr, tgi);
    // |t| > 1e-6 |grad Re| |grad Im|, compared squared
    float tt = dot(t, t);
    if (!(tt > 1e-12f * dot(tgr, tgr) * dot(tgi, tgi)) || tt == 0.f) {
        status |= VX_SAMPLE_TANGENT_FALLBACK;
        t = v3((float)(dec2(desc, 0) + dec2(desc, 1)), (float)(dec2(desc, 2) + dec2(desc, 3)),
               (float)(dec2(desc, 4) + dec2(desc, 5)));
        if (dot(t, t) == 0.f) {
            t = v3(0.f, 0.f, 1.f);
            for (int fc = 0; fc < 6; ++fc) {
                const int w = dec2(desc, fc);
                if (w != 0) {
                    const int a = fc >> 1;
                    t = v3(a == 0 ? (float)w : 0.f, a == 1 ? (float)w : 0.f, a == 2 ? (float)w : 0.f);
                    break;
                }
            }
        }
        tt = dot(t, t);
    }
    const float itn = rsq(tt);
    t = v3(t.x * itn, t.y * itn, t.z * itn);
    int ax = 0;
    if (fabsf(t.y) < fabsf(comp(t, ax))) ax = 1;
    if (fabsf(t.z) < fabsf(comp(t, ax))) ax = 2;
    e1 = crs(t, v3(ax == 0 ? 1.f : 0.f, ax == 1 ? 1.f : 0.f, ax == 2 ? 1.f : 0.f));
    const float in1 = rsq(dot(e1, e1));
    e1 = v3(e1.x * in1, e1.y * in1, e1.z * in1);
    e2 = crs(t, e1);
}

// |psi|^2 from (Re psi, Im psi), one fused multiply-add in a fixed order: every kernel that compares
// densities forms them through this function, so that equal values compare equal whatever the
// compiler contracts elsewhere
__device__ __forceinline__ float rho2(float re, float im) { return fmaf(re, re, im * im); }

// the point x0 + y1 e1 + y2 e2
__device__ __forceinline__ V3 plane_point(const V3 &x0, const V3 &e1, const V3 &e2, float y1, float y2) {
    VX_CONTRACT_ON
    return v3(x0.x + y1 * e1.x + y2 * e2.x, x0.y + y1 * e1.y + y2 * e2.y, x0.z + y1 * e1.z + y2 * e2.z);
}

__device__ __forceinline__ bool in_patch(const V3 &x, const Box &b) {
    VX_CONTRACT_ON
    return x.x >= b.lo.x && x.x <= b.hc.x + 1.f && x.y >= b.lo.y && x.y <= b.hc.y + 1.f && x.z >= b.lo.z &&
           x.z <= b.hc.z + 1.f;
}

// the accepted Newton step alpha (p1, p2) is shorter than tol (compared squared: no square root)
__device__ __forceinline__ bool newton_short(float alpha, float p1, float p2, float tol) {
    VX_CONTRACT_ON
    return alpha * alpha * (p1 * p1 + p2 * p2) < tol * tol;
}

// the gradients of Re psi and Im psi in the plane: J = [[e1.gr, e2.gr], [e1.gim, e2.gim]], the
// Jacobian of (Re psi, Im psi) with respect to the in-plane coordinates (y1, y2); both step kinds
// start from it
struct PlaneJ {
    float j00, j01, j10, j11;
};
__device__ __forceinline__ PlaneJ plane_jac(const V3 &gr, const V3 &gim, const V3 &e1, const V3 &e2) {
    VX_CONTRACT_ON
    return PlaneJ{dot(e1, gr), dot(e2, gr), dot(e1, gim), dot(e2, gim)};
}

// steepest descent of |psi|^2 in the plane: gradient g = 2 J^T psi, direction (n1, n2) * den = -g / |g|,
// gn = |g|
__device__ __forceinline__ bool descent_dir(float vr, float vi, const PlaneJ &J, float &n1, float &n2, float &den,
                                            float &gn) {
    VX_CONTRACT_ON
    const float g1 = 2.f * (vr * J.j00 + vi * J.j10), g2 = 2.f * (vr * J.j01 + vi * J.j11);
    const float gg = g1 * g1 + g2 * g2;
    const float ig = rsq(gg);
    gn = gg * ig;
    n1 = -g1;
    n2 = -g2;
    den = ig;
    return gg > 0.f && ig < INFINITY;
}

// Newton step for (Re psi, Im psi) = 0 in the plane: direction (n1, n2) * den = -J^-1 psi
__device__ __forceinline__ bool newton_dir(float vr, float vi, const PlaneJ &J, float &n1, float &n2, float &den) {
    VX_CONTRACT_ON
    const float j00 = J.j00, j01 = J.j01, j10 = J.j10, j11 = J.j11;
    const float det = j00 * j11 - j01 * j10;
    const float idet = rcp(det);
    n1 = -(j11 * vr - j01 * vi);
    n2 = -(-j10 * vr + j00 * vi);
    den = idet;
    return det != 0.f && fabsf(idet) < INFINITY;
}

}  // namespace vxr
