// Core-sample refinement (Sec. 3.3.1 mean-position estimate, Sec. 3.3.3 density-guided minimisation
// in the plane normal to the pseudo-vorticity, psi linearly interpolated between nodes as in Sec. 5).
//
// One lane per listed cell, grid-stride over min(*count, cap) read on the device, so the launch
// needs no host synchronisation. The iterate only ever needs the 8 corners of the unit cell that
// holds it; they are fetched from global memory (L1/L2-resident: neighbouring samples share nodes)
// when the iterate changes cell, and kept in registers otherwise. FP32 arithmetic throughout.
#include "vx_internal.h"

namespace {

constexpr int REF_THREADS = 256;

struct RefArgs {
    const float2 *psi;
    const uint64_t *cells;
    const uint16_t *desc;
    const float *seed;
    const int64_t *count;
    int64_t cap;
    vx_sample *out;
    int nx, ny, nz;
    int px, py, pz;
    vx_refine_params p;
};

struct V3 {
    float x, y, z;
};
__device__ __forceinline__ V3 v3(float a, float b, float c) { return V3{a, b, c}; }
__device__ __forceinline__ float dot(const V3 &a, const V3 &b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 crs(const V3 &a, const V3 &b) {
    return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float nrm(const V3 &a) { return sqrtf(dot(a, a)); }
__device__ __forceinline__ float comp(const V3 &a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

__device__ __forceinline__ int dec2(uint32_t d, int f) {
    const uint32_t v = (d >> (2 * f)) & 3u;
    return v == 1u ? 1 : (v == 3u ? -1 : 0);
}

// Trilinear psi on the patch of one sample, with a one-cell cache of corner values.
struct Patch {
    const float2 *psi;
    int64_t gi, gj, gk;  // grid node of the sample cell's min corner
    int nx, ny, nz, px, py, pz;
    int lo[3], hi[3];    // cell-local extent of the patch on each axis
    int cc[3];           // cached cell
    float2 v[8];         // its corners, index dx + 2 dy + 4 dz

    __device__ int64_t wrap(int64_t q, int n, int per) const {
        if (q < 0) return per ? q + n : 0;
        if (q >= n) return per ? q - n : n - 1;
        return q;
    }
    __device__ void load(int cx, int cy, int cz) {
        cc[0] = cx;
        cc[1] = cy;
        cc[2] = cz;
#pragma unroll
        for (int d = 0; d < 8; ++d) {
            const int64_t i = wrap(gi + cx + (d & 1), nx, px);
            const int64_t j = wrap(gj + cy + ((d >> 1) & 1), ny, py);
            const int64_t k = wrap(gk + cz + ((d >> 2) & 1), nz, pz);
            v[d] = psi[i + (int64_t)nx * (j + (int64_t)ny * k)];
        }
    }
    __device__ bool inside(const V3 &x) const {
        return x.x >= lo[0] && x.x <= hi[0] && x.y >= lo[1] && x.y <= hi[1] && x.z >= lo[2] && x.z <= hi[2];
    }
    // value and gradient (cell units) at x
    __device__ void eval(const V3 &x, float &vr, float &vi, V3 &gr, V3 &gi) {
        int c[3];
        float u[3];
        const float xs[3] = {x.x, x.y, x.z};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int f = (int)floorf(xs[a]);
            f = max(lo[a], min(f, hi[a] - 1));
            c[a] = f;
            u[a] = xs[a] - (float)f;
        }
        if (c[0] != cc[0] || c[1] != cc[1] || c[2] != cc[2]) load(c[0], c[1], c[2]);
        const float ux = u[0], uy = u[1], uz = u[2];
        const float mx = 1.f - ux, my = 1.f - uy, mz = 1.f - uz;
        // along x
        const float2 a00 = make_float2(mx * v[0].x + ux * v[1].x, mx * v[0].y + ux * v[1].y);
        const float2 a10 = make_float2(mx * v[2].x + ux * v[3].x, mx * v[2].y + ux * v[3].y);
        const float2 a01 = make_float2(mx * v[4].x + ux * v[5].x, mx * v[4].y + ux * v[5].y);
        const float2 a11 = make_float2(mx * v[6].x + ux * v[7].x, mx * v[6].y + ux * v[7].y);
        const float2 d00 = make_float2(v[1].x - v[0].x, v[1].y - v[0].y);
        const float2 d10 = make_float2(v[3].x - v[2].x, v[3].y - v[2].y);
        const float2 d01 = make_float2(v[5].x - v[4].x, v[5].y - v[4].y);
        const float2 d11 = make_float2(v[7].x - v[6].x, v[7].y - v[6].y);
        // along y
        const float2 b0 = make_float2(my * a00.x + uy * a10.x, my * a00.y + uy * a10.y);
        const float2 b1 = make_float2(my * a01.x + uy * a11.x, my * a01.y + uy * a11.y);
        vr = mz * b0.x + uz * b1.x;
        vi = mz * b0.y + uz * b1.y;
        gr.z = b1.x - b0.x;
        gi.z = b1.y - b0.y;
        const float2 ey0 = make_float2(a10.x - a00.x, a10.y - a00.y);
        const float2 ey1 = make_float2(a11.x - a01.x, a11.y - a01.y);
        gr.y = mz * ey0.x + uz * ey1.x;
        gi.y = mz * ey0.y + uz * ey1.y;
        const float2 ex0 = make_float2(my * d00.x + uy * d10.x, my * d00.y + uy * d10.y);
        const float2 ex1 = make_float2(my * d01.x + uy * d11.x, my * d01.y + uy * d11.y);
        gr.x = mz * ex0.x + uz * ex1.x;
        gi.x = mz * ex0.y + uz * ex1.y;
    }
};

__global__ __launch_bounds__(REF_THREADS) void refine_k(RefArgs A) {
    const int64_t n_items = min(*A.count, A.cap);
    const vx_refine_params &P = A.p;
    for (int64_t s = (int64_t)blockIdx.x * REF_THREADS + threadIdx.x; s < n_items;
         s += (int64_t)gridDim.x * REF_THREADS) {
        const uint64_t cell = A.cells[s];
        const uint32_t desc = A.desc[s];
        Patch pt;
        pt.psi = A.psi;
        pt.nx = A.nx;
        pt.ny = A.ny;
        pt.nz = A.nz;
        pt.px = A.px;
        pt.py = A.py;
        pt.pz = A.pz;
        pt.gi = (int64_t)(cell % (uint64_t)A.nx);
        pt.gj = (int64_t)((cell / (uint64_t)A.nx) % (uint64_t)A.ny);
        pt.gk = (int64_t)(cell / ((uint64_t)A.nx * (uint64_t)A.ny));
        const int64_t g3[3] = {pt.gi, pt.gj, pt.gk};
        const int n3[3] = {A.nx, A.ny, A.nz};
        const int p3[3] = {A.px, A.py, A.pz};
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            pt.lo[a] = (p3[a] || g3[a] - 1 >= 0) ? -1 : 0;
            pt.hi[a] = (p3[a] || g3[a] + 2 < n3[a]) ? 2 : 1;
        }
        pt.load(0, 0, 0);

        uint32_t status = 0;
        int npierced = 0;
        V3 x0 = v3(0.f, 0.f, 0.f);
        {
            // face centres in order -x, +x, -y, +y, -z, +z
            float sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
            for (int f = 0; f < 6; ++f) {
                if (dec2(desc, f) == 0) continue;
                const int a = f >> 1;
                const float side = (float)(f & 1);
                sx += a == 0 ? side : 0.5f;
                sy += a == 1 ? side : 0.5f;
                sz += a == 2 ? side : 0.5f;
                ++npierced;
            }
            if (npierced == 0) {
                x0 = v3(0.5f, 0.5f, 0.5f);
                status |= VX_SAMPLE_NO_FACES;
            } else {
                const float inv = 1.0f / (float)npierced;
                x0 = v3(sx * inv, sy * inv, sz * inv);
            }
        }
        if (npierced >= 4) status |= VX_SAMPLE_MULTI;
        if (A.seed) x0 = v3(A.seed[3 * s], A.seed[3 * s + 1], A.seed[3 * s + 2]);

        float vr, vi;
        V3 gr, gi;
        pt.eval(x0, vr, vi, gr, gi);

        V3 t = crs(gr, gi);
        float tn = nrm(t);
        if (!(tn > 1e-6f * nrm(gr) * nrm(gi)) || tn == 0.f) {
            status |= VX_SAMPLE_TANGENT_FALLBACK;
            t = v3((float)(dec2(desc, 0) + dec2(desc, 1)), (float)(dec2(desc, 2) + dec2(desc, 3)),
                   (float)(dec2(desc, 4) + dec2(desc, 5)));
            if (nrm(t) == 0.f) {
                t = v3(0.f, 0.f, 1.f);
                for (int f = 0; f < 6; ++f) {
                    const int w = dec2(desc, f);
                    if (w != 0) {
                        const int a = f >> 1;
                        t = v3(a == 0 ? (float)w : 0.f, a == 1 ? (float)w : 0.f, a == 2 ? (float)w : 0.f);
                        break;
                    }
                }
            }
            tn = nrm(t);
        }
        t = v3(t.x / tn, t.y / tn, t.z / tn);
        int u = 0;
        if (fabsf(t.y) < fabsf(comp(t, u))) u = 1;
        if (fabsf(t.z) < fabsf(comp(t, u))) u = 2;
        V3 e1 = crs(t, v3(u == 0 ? 1.f : 0.f, u == 1 ? 1.f : 0.f, u == 2 ? 1.f : 0.f));
        const float n1 = nrm(e1);
        e1 = v3(e1.x / n1, e1.y / n1, e1.z / n1);
        const V3 e2 = crs(t, e1);

        float y1 = 0.f, y2 = 0.f;
        V3 x = x0;
        float f = vr * vr + vi * vi;
        int iters = 0;

        // gradient descent with a halving step rule
        float s_prev = 0.5f * P.step0;
        for (int it = 0; it < P.max_descent; ++it) {
            if (f == 0.f) break;
            const V3 G = v3(2.f * (vr * gr.x + vi * gi.x), 2.f * (vr * gr.y + vi * gi.y),
                            2.f * (vr * gr.z + vi * gi.z));
            const float g1 = dot(e1, G), g2 = dot(e2, G);
            const float gn = sqrtf(g1 * g1 + g2 * g2);
            if (gn == 0.f) break;
            const float d1 = -g1 / gn, d2 = -g2 / gn;
            float st = fminf(2.f * s_prev, P.step_max);
            bool accepted = false;
            float ty1 = 0.f, ty2 = 0.f, tr = 0.f, ti = 0.f, ft = 0.f;
            V3 xt, tgr, tgi;
            for (int hv = 0; hv < P.max_halvings; ++hv) {
                ty1 = y1 + st * d1;
                ty2 = y2 + st * d2;
                xt = v3(x0.x + ty1 * e1.x + ty2 * e2.x, x0.y + ty1 * e1.y + ty2 * e2.y,
                        x0.z + ty1 * e1.z + ty2 * e2.z);
                if (!pt.inside(xt)) {
                    status |= VX_SAMPLE_BOUNDARY;
                    st *= 0.5f;
                    continue;
                }
                pt.eval(xt, tr, ti, tgr, tgi);
                ft = tr * tr + ti * ti;
                if (ft <= f - P.armijo * st * gn) {
                    accepted = true;
                    break;
                }
                st *= 0.5f;
            }
            if (!accepted) break;
            y1 = ty1;
            y2 = ty2;
            x = xt;
            gr = tgr;
            gi = tgi;
            vr = tr;
            vi = ti;
            f = ft;
            s_prev = st;
            ++iters;
            if (st < P.descent_tol) break;
        }

        // Newton polish on (Re psi, Im psi) in the plane
        bool converged = false;
        for (int it = 0; it < P.max_newton; ++it) {
            if (f == 0.f) {
                converged = true;
                break;
            }
            const float j00 = dot(e1, gr), j01 = dot(e2, gr);
            const float j10 = dot(e1, gi), j11 = dot(e2, gi);
            const float det = j00 * j11 - j01 * j10;
            if (det == 0.f) break;
            const float dy1 = -(j11 * vr - j01 * vi) / det;
            const float dy2 = -(-j10 * vr + j00 * vi) / det;
            float lam = 1.f;
            bool accepted = false;
            float ty1 = 0.f, ty2 = 0.f, tr = 0.f, ti = 0.f, ft = 0.f;
            V3 xt, tgr, tgi;
            for (int hv = 0; hv < P.max_halvings; ++hv) {
                ty1 = y1 + lam * dy1;
                ty2 = y2 + lam * dy2;
                xt = v3(x0.x + ty1 * e1.x + ty2 * e2.x, x0.y + ty1 * e1.y + ty2 * e2.y,
                        x0.z + ty1 * e1.z + ty2 * e2.z);
                if (!pt.inside(xt)) {
                    status |= VX_SAMPLE_BOUNDARY;
                    lam *= 0.5f;
                    continue;
                }
                pt.eval(xt, tr, ti, tgr, tgi);
                ft = tr * tr + ti * ti;
                if (ft < f) {
                    accepted = true;
                    break;
                }
                lam *= 0.5f;
            }
            if (!accepted) break;
            const float step = lam * sqrtf(dy1 * dy1 + dy2 * dy2);
            y1 = ty1;
            y2 = ty2;
            x = xt;
            gr = tgr;
            gi = tgi;
            vr = tr;
            vi = ti;
            f = ft;
            ++iters;
            if (step < P.newton_tol) {
                converged = true;
                break;
            }
        }
        if (f > P.rho_tol) status |= VX_SAMPLE_NONZERO_MIN;
        if (!converged && f > P.rho_tol) status |= VX_SAMPLE_NOT_CONVERGED;

        vx_sample o;
        o.cell = cell;
        o.off[0] = x.x;
        o.off[1] = x.y;
        o.off[2] = x.z;
        o.rho = f;
        o.iters = (uint16_t)min(iters, 65535);
        o.status = (uint16_t)status;
        o.reserved = 0;
        A.out[s] = o;
    }
}

}  // namespace

vx_status vx_refine_launch(vx_handle *h, const vx_dims &d, const void *psi, const uint64_t *cells,
                           const uint16_t *desc, const float *seed, const int64_t *count, int64_t cap,
                           const vx_refine_params &p, vx_sample *out, hipStream_t s) {
    RefArgs A;
    A.psi = (const float2 *)psi;
    A.cells = cells;
    A.desc = desc;
    A.seed = seed;
    A.count = count;
    A.cap = cap;
    A.out = out;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    A.px = (int)(d.periodic & 1u);
    A.py = (int)((d.periodic >> 1) & 1u);
    A.pz = (int)((d.periodic >> 2) & 1u);
    A.p = p;
    // enough lanes for the capacity, capped at a few resident workgroups per CU
    const int64_t need = (cap + REF_THREADS - 1) / REF_THREADS;
    const int64_t maxb = 16LL * (h->num_cu > 0 ? h->num_cu : 256);
    const int64_t blocks = std::max<int64_t>(1, std::min(need, maxb));
    vx_timer tm(h, s, VX_KIND_REFINE);
    hipLaunchKernelGGL(refine_k, dim3((unsigned)blocks), dim3(REF_THREADS), 0, s, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "refine_k launch");
}
