// Surrogate of the core-sample refinement: a 128-NH-NH-4 GELU network (NH = VX_MLP_NHID) that maps the 4x4x4
// psi patch of a pierced cell to the offset of its refined core sample from the first estimate (the mean of
// the pierced-face centres, Sec. 3.3.1) plus a confidence. Training data are produced by the plain refinement
// (Sec. 3.3.3); below the confidence threshold the plain refinement runs.
//
// Matrix cores. The two hidden layers are BF16 products with FP32 accumulation on
// v_mfma_f32_16x16x32_bf16: lane l of a wavefront holds row (l % 16) of a 16x32 A block and column
// (l % 16) of a 32x16 B block, k = 8 (l / 16) .. +7 as eight BF16 values; the 16x16 FP32 result
// holds rows 4 (l / 16) + i, column l % 16 in its four registers. A training workgroup (4 wavefronts) owns a
// tile of 64 rows; wavefront w computes columns NH/4 w .. NH/4 (w+1) - 1 of a layer for all 64 rows (4 x
// NH/64 blocks). A operands come from LDS (row pitch padded by 8 values so that the 16 rows of a block fall
// on different banks), B operands are read as 16-byte vectors from transposed BF16 weight copies (k
// contiguous), which stay in L2. The 4-wide head runs on the matrix cores too (N padded to 16); its
// gradients, the bias gradients and the loss are small reductions done on the vector ALUs.
//
// Training on a minibatch of n rows (all on the device, no host synchronisation):
//   fwd_train_k   per 64-row tile: layers, H1/H2 and gelu'(Z1)/gelu'(Z2) to global scratch (BF16),
//                 head, loss terms, dZ3 (FP32)
//   bwd_rows_k    per tile: dZ2 = (dZ3 W3^T) * gelu'(Z2), dZ1 = (dZ2 W2^T) * gelu'(Z1) (MFMA), the
//                 gradients of W3 and of every bias (atomics into the FP32 gradient buffer)
//   wgrad_k       dW1 = X^T dZ1 and dW2 = H1^T dZ2: split over row chunks; each 32-row step is
//                 staged transposed in LDS so that both operands are read as 16-byte vectors;
//                 partial 128x128 blocks are added atomically
//   adam_k        Adam update of the FP32 master weights, refreshed BF16 copies, gradient zeroed
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "vx_refine_math.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

constexpr int NIN = VX_MLP_NIN, NH = VX_MLP_NHID, NOUT = VX_MLP_NOUT;
constexpr int OFF_W1 = 0, OFF_B1 = OFF_W1 + NIN * NH, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NH * NH;
constexpr int OFF_W3 = OFF_B2 + NH, OFF_B3 = OFF_W3 + NH * NOUT, NPARAM = OFF_B3 + NOUT;
static_assert(NPARAM == VX_MLP_NPARAMS, "parameter count");

constexpr int TM = 64;           // rows per tile
constexpr int NT = 256;          // threads per workgroup
constexpr int WFT = NH / 4;      // hidden features per wavefront in the training kernels (4 wavefronts)
constexpr int NCB = WFT / 16;    // their 16-column blocks
static_assert(NH == 128 || NH == 256,
              "hidden width 128 or 256: 128-column weight-gradient blocks, one bwd_rows_k thread per column");
constexpr int POLISH_WG_PER_CU = 5;  // polish workgroups per CU (what fits at its 87 VGPRs)
constexpr int XP = NIN + 8;      // LDS row pitch (values) of the input tile
constexpr int HP = NH + 8;       // LDS row pitch of a hidden tile
constexpr int GT = 1024;         // table intervals on [-8, 8]
constexpr float GLO = -8.f, GSC = 64.f;   // table on [GLO, GLO + GT / GSC] = [-8, 8]
constexpr int WCH = 512;         // rows per chunk of the weight-gradient kernel

__device__ __forceinline__ f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 ld8(const __bf16 *p) { return *(const bf16x8 *)p; }
// two floats as bfloat16 (round to nearest even) in one word, the first in the low half; one
// v_cvt_pk_bf16_f32
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    typedef float f2v __attribute__((ext_vector_type(2)));
    typedef __bf16 h2v __attribute__((ext_vector_type(2)));
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((f2v){a, b}, h2v));
}

// gelu or its derivative, piecewise linear in the table coordinate u = (x - GLO) GSC: segment i
// (u in [i, i + 1]) is stored as (intercept, slope), f = intercept + u slope. No conditionals, so
// that the lookups of a whole epilogue can be in flight together. Outside [-8, 8] the end segments
// continue linearly; their slopes are those of gelu (0 and 1) and of gelu' (0 and 0) there to FP32
// precision, so gelu(x) = x above 8 and gelu' stays 0 or 1. (x - GLO) GSC is one rounding either
// way, GSC being a power of two.
__device__ __forceinline__ float tab(const float2 *t, float x) {
    const float u = fmaf(x, GSC, -GLO * GSC);
    const float2 e = t[(int)fminf(fmaxf(u, 0.f), (float)(GT - 1))];
    return fmaf(u, e.y, e.x);
}

// gelu for the inference kernel without a table: Phi(x) ~ sigmoid(x (a + b x^2 + c x^4)) with a = 1.5950158,
// b = 0.0740113, c = -7.0303e-4 (fitted for the least maximum of |x sigmoid(..) - x Phi(x)| over all x, which
// is 2.6e-5 here, as small as the table's error), evaluated as x / (1 + 2^(xc q(xc^2))) with q = -(a + b t +
// c t^2) log2(e) and xc = x clamped to [-8, 8] (beyond, the x^4 term would turn the sign; there the result is
// x or 0 to FP32 precision). One exp2 and one reciprocal, hardware approximations within an ulp or two; no
// LDS traffic, which the table's scattered lookups cost the network kernel.
__device__ __forceinline__ float gelu_fit(float x) {
    const float xc = __builtin_amdgcn_fmed3f(x, -8.f, 8.f);
    const float t = xc * xc;
    const float q = fmaf(fmaf(t, 1.014263020e-03f, -1.067757234e-01f), t, -2.301121235e+00f);
    return x * __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(xc * q));
}

struct Geo {
    const float2 *psi;
    int nx, ny, nz, px, py, pz;
    double rnx, rnxy;  // 1 / nx and 1 / (nx ny), for the cell-id split
};

__device__ __forceinline__ int wrapc(int q, int n, int per) {
    const int below = per ? q + n : 0, above = per ? q - n : n - 1;
    return q < 0 ? below : (q >= n ? above : q);
}

// cell id -> node coordinates (cells of any grid that fits in memory, < 2^53)
__device__ __forceinline__ void cell_xyz(uint64_t cell, const Geo &g, int &i, int &j, int &k) {
    // quotients by multiplication with the FP64 reciprocals, corrected by one (exact below 2^53)
    uint64_t rxy, ri;
    k = (int)vxr::divmod53(cell, (uint64_t)g.nx * (uint64_t)g.ny, g.rnxy, rxy);
    j = (int)vxr::divmod53(rxy, (uint64_t)g.nx, g.rnx, ri);
    i = (int)ri;
}

// the patch lies inside the grid (always on periodic axes)
__device__ __forceinline__ bool interior(const Geo &g, int i, int j, int k) {
    return (g.px || (i >= 1 && i + 2 < g.nx)) && (g.py || (j >= 1 && j + 2 < g.ny)) &&
           (g.pz || (k >= 1 && k + 2 < g.nz));
}

// Four consecutive lanes gather one patch: lane quarter c loads the 16 nodes of patch plane c and
// the group reduces the sum of |psi|^2 with two xor shuffles (all four lanes must be active).
// Writes the 32 BF16 features of plane c to dst[32 c .. 32 c + 31] if `write`.
__device__ __forceinline__ void gather_features(const Geo &g, int i, int j, int k, int c, __bf16 *dst,
                                                bool write = true) {
    float2 v[16];
    const int kk = wrapc(k + c - 1, g.nz, g.pz);
    const uint64_t nx = (uint64_t)g.nx;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int jj = wrapc(j + b - 1, g.ny, g.py);
        const float2 *row = g.psi + nx * ((uint64_t)jj + (uint64_t)g.ny * (uint64_t)kk);
#pragma unroll
        for (int a = 0; a < 4; ++a) v[4 * b + a] = row[wrapc(i + a - 1, g.nx, g.px)];
    }
    float ss = 0.f;
#pragma unroll
    for (int q = 0; q < 16; ++q) ss += v[q].x * v[q].x + v[q].y * v[q].y;
    ss += __shfl_xor(ss, 1);
    ss += __shfl_xor(ss, 2);
    const float s = ss > 0.f ? sqrtf(ss * (1.f / 64.f)) : 1.f;
    const float is = 1.f / s;
    if (!write) return;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        dst[32 * c + 2 * q] = (__bf16)(v[q].x * is);
        dst[32 * c + 2 * q + 1] = (__bf16)(v[q].y * is);
    }
}

// The surrogate's final step, in the refinement's own arithmetic (the functions of vx_refine_math.h, Sec.
// 3.3.3 reading): the network's point xs projected onto the plane through x0 normal to t = grad Re psi x grad
// Im psi at x0, then one Newton step on (Re psi, Im psi) in that plane. False where the plain refinement must
// run: degenerate t, singular Jacobian, a point outside the patch, or -- when max_step > 0 -- a Newton step
// from the polished point that would be longer than max_step cells (that step estimates the polished point's
// distance from the zero of psi in the plane, so a confident but wrong prediction goes to the plain method
// instead of being reported). The corners of the cell itself come in ctr (64 contiguous bytes written by the
// network kernel, loaded by the caller together with its other inputs), the others from the field; those of
// x0's cell and of xs's cell are requested together: the projected point and the Newton point mostly lie in
// one of the two, so that the evaluations usually wait for one round of loads.
__device__ bool polish(const Geo &g, int i, int j, int k, uint32_t desc, const float4 ctr[4], const vxr::V3 &x0,
                       const vxr::V3 &xs, float max_step, vxr::V3 &out, float &rho) {
    using namespace vxr;
    constexpr int CENTRE = 21;  // locate()'s code of the cell itself: (0+1) + 4 (0+1) + 16 (0+1)
    const Box box = patch_box(i, j, k, g.nx, g.ny, g.nz, g.px, g.py, g.pz);
    int c0[3], cs[3], cp[3];
    float u0[3], us[3], up[3];
    const int k0 = locate(x0, box, c0, u0), ks = locate(xs, box, cs, us);
    float2 Z[8], A[8], B[8], C[8], cf[8];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 e = ctr[q];
        Z[2 * q] = make_float2(e.x, e.y);
        Z[2 * q + 1] = make_float2(e.z, e.w);
    }
    if (k0 == CENTRE) {
#pragma unroll
        for (int q = 0; q < 8; ++q) A[q] = Z[q];
    } else {
        fetch_corners(g.psi, g.nx, g.ny, g.nz, g.px, g.py, g.pz, i, j, k, c0, A);
    }
    if (ks == CENTRE) {
#pragma unroll
        for (int q = 0; q < 8; ++q) B[q] = Z[q];
    } else {
        fetch_corners(g.psi, g.nx, g.ny, g.nz, g.px, g.py, g.pz, i, j, k, cs, B);
    }
    float vr, vi;
    V3 gr, gi, e1, e2;
    tri_coeffs(A, cf);
    trilinear(cf, u0, vr, vi, gr, gi);
    uint32_t status = 0;
    plane_basis(gr, gi, desc, e1, e2, status);
    if (status & VX_SAMPLE_TANGENT_FALLBACK) return false;
    const V3 d = v3(xs.x - x0.x, xs.y - x0.y, xs.z - x0.z);
    float y1 = dot(d, e1), y2 = dot(d, e2);
    const V3 xp = plane_point(x0, e1, e2, y1, y2);
    if (!in_patch(xp, box)) return false;
    const int kp = locate(xp, box, cp, up);
    if (kp == ks || kp == k0) {
#pragma unroll
        for (int q = 0; q < 8; ++q) C[q] = kp == ks ? B[q] : A[q];
    } else {
        fetch_corners(g.psi, g.nx, g.ny, g.nz, g.px, g.py, g.pz, i, j, k, cp, C);
    }
    tri_coeffs(C, cf);
    trilinear(cf, up, vr, vi, gr, gi);
    float n1, n2, den;
    if (!newton_dir(vr, vi, plane_jac(gr, gi, e1, e2), n1, n2, den)) return false;
    const float p1 = n1 * den, p2 = n2 * den;
    y1 = y1 + p1;
    y2 = y2 + p2;
    out = plane_point(x0, e1, e2, y1, y2);
    if (!in_patch(out, box)) return false;
    int co[3];
    float uo[3];
    if (locate(out, box, co, uo) != kp) {
        fetch_corners(g.psi, g.nx, g.ny, g.nz, g.px, g.py, g.pz, i, j, k, co, C);
        tri_coeffs(C, cf);
    }
    trilinear(cf, uo, vr, vi, gr, gi);
    rho = vxr::rho2(vr, vi);
    if (max_step > 0.f && rho != 0.f) {
        if (!newton_dir(vr, vi, plane_jac(gr, gi, e1, e2), n1, n2, den)) return false;
        const float q1 = n1 * den, q2 = n2 * den;
        if (!(q1 * q1 + q2 * q2 <= max_step * max_step)) return false;
    }
    return true;
}

// ---------------------------------------------------------------------------- layer building blocks

// acc = A (64 x K, LDS, pitch AP) times B (K x 16 NC: columns n0 .. n0 + 16 NC - 1 of a K-contiguous
// weight copy Wt[col][k]) for this wavefront
template <int K, int AP, int NC>
__device__ __forceinline__ void layer(const __bf16 *sA, const __bf16 *__restrict__ Wt, int n0, f32x4 acc[4][NC]) {
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 b[NC], a[4];
#pragma unroll
        for (int c = 0; c < NC; ++c) b[c] = ld8(Wt + (size_t)(n0 + 16 * c + (l & 15)) * K + k0 + 8 * (l >> 4));
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = ld8(sA + (16 * r + (l & 15)) * AP + k0 + 8 * (l >> 4));
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < NC; ++c) acc[r][c] = mfma(a[r], b[c], acc[r][c]);
    }
}

// head: rows 16w .. 16w+15 of H (LDS) times W3 (16 x 256 padded copy); returns this lane's column
// (l % 16) for rows 16w + 4 (l / 16) + i
__device__ __forceinline__ f32x4 head(const __bf16 *sH, const __bf16 *__restrict__ W3t) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < NH; k0 += 32) {
        const bf16x8 a = ld8(sH + (16 * w + (l & 15)) * HP + k0 + 8 * (l >> 4));
        const bf16x8 b = ld8(W3t + (l & 15) * NH + k0 + 8 * (l >> 4));
        acc = mfma(a, b, acc);
    }
    return acc;
}

struct Net {  // device copies used by the kernels
    const float *master;  // FP32 parameters (host layout)
    const __bf16 *w1t;    // [NH][NIN]  W1 transposed
    const __bf16 *w2t;    // [NH][NH]   W2 transposed
    const __bf16 *w2c;    // [NH][NH]   W2 as is (rows = inputs): B operand of dH1 = dZ2 W2^T
    const __bf16 *w3t;    // [16][NH]   W3 transposed, rows 4..15 zero
    const float2 *gelu;   // [GT] (value, step)
    const float2 *dgelu;  // [GT] (derivative, step)
};

// copy the two tables into LDS (all threads)
__device__ __forceinline__ void load_tables(const Net &N, float2 *sg, float2 *sd) {
    for (int i = threadIdx.x; i < GT; i += NT) {
        sg[i] = N.gelu[i];
        if (sd) sd[i] = N.dgelu[i];
    }
}

// both hidden layers for the input tile sX; H2 ends in sH. Optionally stores H1/H2 and the gelu
// derivatives of the valid rows to global memory (training).
__device__ __forceinline__ void hidden(const Net &N, const __bf16 *sX, __bf16 *sH, const float2 *sg, const float2 *sd,
                                       int64_t row0, int64_t nrows, __bf16 *H1, __bf16 *G1, __bf16 *H2, __bf16 *G2) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n0 = WFT * w;
    f32x4 acc[4][NCB];
    layer<NIN, XP, NCB>(sX, N.w1t, n0, acc);
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        const int col = n0 + 16 * c + (l & 15);
        const float bias = N.master[OFF_B1 + col];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * r + 4 * (l >> 4) + i;
                const float z = acc[r][c][i] + bias;
                const __bf16 hv = (__bf16)tab(sg, z);
                sH[row * HP + col] = hv;
                if (H1 && row0 + row < nrows) {
                    H1[(row0 + row) * NH + col] = hv;
                    G1[(row0 + row) * NH + col] = (__bf16)tab(sd, z);
                }
            }
    }
    __syncthreads();
    layer<NH, HP, NCB>(sH, N.w2t, n0, acc);
    __syncthreads();  // every wavefront has read H1
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        const int col = n0 + 16 * c + (l & 15);
        const float bias = N.master[OFF_B2 + col];
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * r + 4 * (l >> 4) + i;
                const float z = acc[r][c][i] + bias;
                const __bf16 hv = (__bf16)tab(sg, z);
                sH[row * HP + col] = hv;
                if (H2 && row0 + row < nrows) {
                    H2[(row0 + row) * NH + col] = hv;
                    G2[(row0 + row) * NH + col] = (__bf16)tab(sd, z);
                }
            }
    }
    __syncthreads();
}

// network outputs of the 64 rows into sOut[64][4] (Z3 with the bias; column 3 is the logit)
__device__ __forceinline__ void outputs(const Net &N, const __bf16 *sH, float *sOut) {
    const int l = threadIdx.x & 63, w = threadIdx.x >> 6;
    const f32x4 z = head(sH, N.w3t);
    const int col = l & 15;
    if (col < NOUT) {
#pragma unroll
        for (int i = 0; i < 4; ++i) sOut[(16 * w + 4 * (l >> 4) + i) * NOUT + col] = z[i] + N.master[OFF_B3 + col];
    }
    __syncthreads();
}

// load rows of BF16 features (optionally through an index list) into sX; rows past n are zero
__device__ __forceinline__ void load_x(const __bf16 *__restrict__ feat, const int32_t *__restrict__ idx, int64_t row0,
                                       int64_t n, __bf16 *sX) {
    for (int e = threadIdx.x; e < TM * (NIN / 8); e += NT) {
        const int r = e / (NIN / 8), q = e % (NIN / 8);
        bf16x8 v;
        if (row0 + r < n) {
            const int64_t src = idx ? (int64_t)idx[row0 + r] : row0 + r;
            v = ld8(feat + src * NIN + 8 * q);
        } else {
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = (__bf16)0.f;
        }
        *(bf16x8 *)(sX + r * XP + 8 * q) = v;
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------- kernels

__global__ void tables_k(float2 *gelu, float2 *dgelu) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= GT) return;
    auto g = [](double x) { return x * 0.5 * (1.0 + erf(x / sqrt(2.0))); };
    auto dg = [](double x) { return 0.5 * (1.0 + erf(x / sqrt(2.0))) + x * exp(-0.5 * x * x) / sqrt(2.0 * M_PI); };
    const double x0 = GLO + (double)i / GSC, x1 = GLO + (double)(i + 1) / GSC;
    const double sg = g(x1) - g(x0), sd = dg(x1) - dg(x0);  // slopes per unit of u
    gelu[i] = make_float2((float)(g(x0) - i * sg), (float)sg);
    dgelu[i] = make_float2((float)(dg(x0) - i * sd), (float)sd);
}

// host-layout FP32 parameters -> BF16 operand copies
__global__ void refresh_k(const float *__restrict__ p, __bf16 *w1t, __bf16 *w2t, __bf16 *w2c, __bf16 *w3t) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < OFF_B3; e += gridDim.x * blockDim.x) {
        const __bf16 v = (__bf16)p[e];
        if (e < OFF_B1) {
            const int i = e / NH, o = e % NH;
            w1t[o * NIN + i] = v;
        } else if (e >= OFF_W2 && e < OFF_B2) {
            const int q = e - OFF_W2, i = q / NH, o = q % NH;
            w2t[o * NH + i] = v;
            w2c[q] = v;
        } else if (e >= OFF_W3) {
            const int q = e - OFF_W3, i = q / NOUT, o = q % NOUT;
            w3t[o * NH + i] = v;
        }
    }
}

// forward of a minibatch with everything the backward pass needs; loss terms and dZ3
__global__ __launch_bounds__(NT) void fwd_train_k(Net N, const __bf16 *__restrict__ feat, const float *__restrict__ target,
                                                  const int32_t *__restrict__ idx, int64_t n, float lam, float tol,
                                                  __bf16 *H1, __bf16 *G1, __bf16 *H2, __bf16 *G2, float *dZ3,
                                                  float *loss) {
    __shared__ __attribute__((aligned(16))) __bf16 sX[TM * XP];
    __shared__ __attribute__((aligned(16))) __bf16 sH[TM * HP];
    __shared__ float2 sg[GT], sd[GT];
    __shared__ float sOut[TM * NOUT];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    load_tables(N, sg, sd);
    load_x(feat, idx, row0, n, sX);
    hidden(N, sX, sH, sg, sd, row0, n, H1, G1, H2, G2);
    outputs(N, sH, sOut);
    // loss terms of the tile's rows (one thread per row), reduced over the wavefront
    const int t = threadIdx.x;
    float mse = 0.f, bce = 0.f;
    if (t < TM && row0 + t < n) {
        const int64_t r = row0 + t;
        const int64_t src = idx ? (int64_t)idx[r] : r;
        const float inv_n = 1.f / (float)n;
        float d[3], dm = 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            d[a] = sOut[t * NOUT + a] - target[src * 3 + a];
            mse += d[a] * d[a];
            dm = fmaxf(dm, fabsf(d[a]));
        }
        const float z = sOut[t * NOUT + 3];
        const float y = dm < tol ? 1.f : 0.f;
        bce = fmaxf(z, 0.f) + log1pf(expf(-fabsf(z))) - y * z;
        const float sg_ = 1.f / (1.f + expf(-z));
#pragma unroll
        for (int a = 0; a < 3; ++a) dZ3[r * NOUT + a] = 2.f * d[a] * inv_n;
        dZ3[r * NOUT + 3] = lam * (sg_ - y) * inv_n;
    }
    if (t < 64) {
        for (int o = 32; o > 0; o >>= 1) {
            mse += __shfl_xor(mse, o);
            bce += __shfl_xor(bce, o);
        }
        if (t == 0 && loss) {
            atomicAdd(&loss[0], mse / (float)n);
            atomicAdd(&loss[1], bce / (float)n);
        }
    }
}

// backward through the layers for a 64-row tile: dZ2, dZ1 (global), gradients of W3 and the biases
__global__ __launch_bounds__(NT) void bwd_rows_k(Net N, int64_t n, const float *__restrict__ dZ3,
                                                 const __bf16 *__restrict__ H2, const __bf16 *__restrict__ G1,
                                                 const __bf16 *__restrict__ G2, __bf16 *dZ2g, __bf16 *dZ1g,
                                                 float *grad) {
    __shared__ __attribute__((aligned(16))) __bf16 sD[TM * HP];  // dZ2 tile (A operand)
    __shared__ float sZ3[TM * NOUT];
    __shared__ float sW3[NH * NOUT];
    const int t = threadIdx.x;
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    for (int e = t; e < TM * NOUT; e += NT) sZ3[e] = row0 + e / NOUT < n ? dZ3[row0 * NOUT + e] : 0.f;
    for (int e = t; e < NH * NOUT; e += NT) sW3[e] = N.master[OFF_W3 + e];
    __syncthreads();
    // column t: dH2 = dZ3 W3^T, dZ2 = dH2 gelu'(Z2); gradients of b2, W3 row t; b3
    if (t < NH) {
        const int o = t;
        float db2 = 0.f, gw[NOUT] = {0.f, 0.f, 0.f, 0.f};
        for (int r = 0; r < TM; ++r) {
            float v = 0.f;
            if (row0 + r < n) {
                float dh = 0.f;
#pragma unroll
                for (int j = 0; j < NOUT; ++j) dh += sZ3[r * NOUT + j] * sW3[o * NOUT + j];
                v = dh * (float)G2[(row0 + r) * NH + o];
                const float h2 = (float)H2[(row0 + r) * NH + o];
#pragma unroll
                for (int j = 0; j < NOUT; ++j) gw[j] += h2 * sZ3[r * NOUT + j];
            }
            const __bf16 vb = (__bf16)v;
            sD[r * HP + o] = vb;
            if (row0 + r < n) dZ2g[(row0 + r) * NH + o] = vb;
            db2 += (float)vb;
        }
        atomicAdd(&grad[OFF_B2 + o], db2);
#pragma unroll
        for (int j = 0; j < NOUT; ++j) atomicAdd(&grad[OFF_W3 + o * NOUT + j], gw[j]);
        if (t < NOUT) {
            float s = 0.f;
            for (int r = 0; r < TM; ++r) s += sZ3[r * NOUT + t];
            atomicAdd(&grad[OFF_B3 + t], s);
        }
    }
    __syncthreads();
    // dH1 = dZ2 W2^T on the matrix cores; dZ1 = dH1 gelu'(Z1); gradient of b1
    const int l = t & 63, w = t >> 6, n0 = WFT * w;
    f32x4 acc[4][NCB];
    layer<NH, HP, NCB>(sD, N.w2c, n0, acc);
#pragma unroll
    for (int c = 0; c < NCB; ++c) {
        const int col = n0 + 16 * c + (l & 15);
        float db1 = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * r + 4 * (l >> 4) + i;
                if (row0 + row < n) {
                    const __bf16 v = (__bf16)(acc[r][c][i] * (float)G1[(row0 + row) * NH + col]);
                    dZ1g[(row0 + row) * NH + col] = v;
                    db1 += (float)v;
                }
            }
        db1 += __shfl_xor(db1, 16);
        db1 += __shfl_xor(db1, 32);
        if (l < 16) atomicAdd(&grad[OFF_B1 + col], db1);
    }
}

// C[M][N] += sum over rows r of A[r][M] B[r][N]: A, B row-major BF16 with leading dimensions MA,
// NB (A rows optionally through idx); block (chunk, mt, nt) covers rows [chunk*WCH, +WCH) and the
// 128x128 output block (mt, nt); each 32-row step is staged transposed in LDS.
__global__ __launch_bounds__(NT) void wgrad_k(const __bf16 *__restrict__ A, int MA, const int32_t *__restrict__ idx,
                                              const __bf16 *__restrict__ B, int NB, int64_t n, float *C) {
    constexpr int KP = 40;  // LDS pitch of a transposed 32-row step
    __shared__ __attribute__((aligned(16))) __bf16 sA[128 * KP];
    __shared__ __attribute__((aligned(16))) __bf16 sB[128 * KP];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int m0 = 128 * blockIdx.y, nb0 = 128 * blockIdx.z;
    const int64_t r0 = (int64_t)blockIdx.x * WCH;
    const int64_t r1 = min(n, r0 + WCH);
    const int wm = 64 * (w & 1), wn = 64 * (w >> 1);
    f32x4 acc[4][4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t k0 = r0; k0 < r1; k0 += 32) {
        // thread t stages row (t / 8) of the step, 16 columns (t % 8) * 16 .. +15 of each operand
        {
            const int rr = t >> 3, cc = (t & 7) * 16;
            const int64_t r = k0 + rr;
            bf16x8 a0, a1, b0, b1;
            if (r < r1) {
                const int64_t ra = idx ? (int64_t)idx[r] : r;
                a0 = ld8(A + ra * MA + m0 + cc);
                a1 = ld8(A + ra * MA + m0 + cc + 8);
                b0 = ld8(B + r * NB + nb0 + cc);
                b1 = ld8(B + r * NB + nb0 + cc + 8);
            } else {
#pragma unroll
                for (int j = 0; j < 8; ++j) a0[j] = a1[j] = b0[j] = b1[j] = (__bf16)0.f;
            }
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sA[(cc + j) * KP + rr] = a0[j];
                sA[(cc + 8 + j) * KP + rr] = a1[j];
                sB[(cc + j) * KP + rr] = b0[j];
                sB[(cc + 8 + j) * KP + rr] = b1[j];
            }
        }
        __syncthreads();
        bf16x8 a[4], b[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r] = ld8(sA + (wm + 16 * r + (l & 15)) * KP + 8 * (l >> 4));
#pragma unroll
        for (int c = 0; c < 4; ++c) b[c] = ld8(sB + (wn + 16 * c + (l & 15)) * KP + 8 * (l >> 4));
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) acc[r][c] = mfma(a[r], b[c], acc[r][c]);
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int m = m0 + wm + 16 * r + 4 * (l >> 4) + i;
                const int nn = nb0 + wn + 16 * c + (l & 15);
                atomicAdd(&C[(size_t)m * NB + nn], acc[r][c][i]);
            }
}

__global__ void adam_k(float *p, float *m, float *v, float *g, float lr, float b1, float b2, float eps, float c1,
                       float c2) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPARAM; e += gridDim.x * blockDim.x) {
        const float ge = g[e];
        const float me = b1 * m[e] + (1.f - b1) * ge;
        const float ve = b2 * v[e] + (1.f - b2) * ge * ge;
        m[e] = me;
        v[e] = ve;
        p[e] -= lr * (me * c1) / (sqrtf(ve * c2) + eps);
        g[e] = 0.f;
    }
}

__global__ void copy_zero_k(float *g, float *out) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NPARAM; e += gridDim.x * blockDim.x) {
        out[e] = g[e];
        g[e] = 0.f;
    }
}

__global__ void zero_f_k(float *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0.f;
}

// plain forward: outputs (Z3[0..2], conf) of feature rows
__global__ __launch_bounds__(NT) void fwd_k(Net N, const __bf16 *__restrict__ feat, int64_t n, float *out) {
    __shared__ __attribute__((aligned(16))) __bf16 sX[TM * XP];
    __shared__ __attribute__((aligned(16))) __bf16 sH[TM * HP];
    __shared__ float2 sg[GT];
    __shared__ float sOut[TM * NOUT];
    const int64_t row0 = (int64_t)blockIdx.x * TM;
    load_tables(N, sg, nullptr);
    load_x(feat, nullptr, row0, n, sX);
    hidden(N, sX, sH, sg, nullptr, row0, n, nullptr, nullptr, nullptr, nullptr);
    outputs(N, sH, sOut);
    const int t = threadIdx.x;
    if (t < TM && row0 + t < n) {
        out[(row0 + t) * 4 + 0] = sOut[t * NOUT + 0];
        out[(row0 + t) * 4 + 1] = sOut[t * NOUT + 1];
        out[(row0 + t) * 4 + 2] = sOut[t * NOUT + 2];
        out[(row0 + t) * 4 + 3] = 1.f / (1.f + expf(-sOut[t * NOUT + 3]));
    }
}

// features of listed cells, four lanes per cell (64 cells per workgroup)
__global__ __launch_bounds__(NT) void features_k(Geo g, const uint64_t *__restrict__ cells,
                                                 const int64_t *__restrict__ count, int64_t cap, __bf16 *feat) {
    const int64_t n = min(*count, cap);
    if ((int64_t)blockIdx.x * TM >= n) return;  // uniform per workgroup
    const int64_t s = (int64_t)blockIdx.x * TM + (threadIdx.x >> 2);
    const int c = threadIdx.x & 3;
    const bool ok = s < n;
    const uint64_t cell = ok ? cells[s] : 0;
    const uint64_t ncell = (uint64_t)g.nx * g.ny * g.nz;
    int i = 0, j = 0, k = 0;
    if (cell < ncell) cell_xyz(cell, g, i, j, k);
    gather_features(g, i, j, k, c, feat + (ok ? s : 0) * NIN, ok);
}

// training rows from refined samples (see vx_mlp_dataset)
__global__ __launch_bounds__(NT) void dataset_k(Geo g, const uint64_t *__restrict__ cells, const uint16_t *__restrict__ desc,
                                                const vx_sample *__restrict__ smp, const int64_t *__restrict__ count,
                                                int64_t cap, __bf16 *feat, float *target, unsigned long long *d_n,
                                                int64_t n_cap, unsigned long long *flag) {
    const int64_t n = min(*count, cap);
    if ((int64_t)blockIdx.x * TM >= n) return;  // uniform per workgroup
    const int64_t s = (int64_t)blockIdx.x * TM + (threadIdx.x >> 2);
    const int c = threadIdx.x & 3;
    const uint32_t bad = VX_SAMPLE_MULTI | VX_SAMPLE_NO_FACES | VX_SAMPLE_NONZERO_MIN | VX_SAMPLE_NOT_CONVERGED |
                         VX_SAMPLE_BOUNDARY | VX_SAMPLE_BAD_CELL;
    bool keep = false;
    uint64_t cell = 0;
    int i = 0, j = 0, k = 0;
    if (s < n) {
        cell = cells[s];
        keep = (smp[s].status & bad) == 0 && smp[s].cell == cell && cell < (uint64_t)g.nx * g.ny * g.nz;
        if (keep) {
            cell_xyz(cell, g, i, j, k);
            keep = interior(g, i, j, k);
        }
    }
    // one slot per kept cell: the group's first lane reserves it, the others read it by shuffle
    unsigned long long slot = 0;
    if (keep && c == 0) slot = atomicAdd(d_n, 1ull);
    const int lead = (int)(threadIdx.x & ~3u) & 63;
    slot = ((unsigned long long)(uint32_t)__shfl((int)(slot >> 32), lead) << 32) | (uint32_t)__shfl((int)slot, lead);
    const bool store = keep && (int64_t)slot < n_cap;
    if (keep && c == 0 && (int64_t)slot >= n_cap) atomicOr(flag, (unsigned long long)VX_OVERFLOW_DATASET);
    gather_features(g, i, j, k, c, feat + (store ? (int64_t)slot : 0) * NIN, store);
    if (store) {
        if (c == 0) {
            uint32_t st0 = 0;
            const vxr::V3 x0 = vxr::first_estimate(desc[s], st0);
            target[slot * 3 + 0] = smp[s].off[0] - x0.x;
            target[slot * 3 + 1] = smp[s].off[1] - x0.y;
            target[slot * 3 + 2] = smp[s].off[2] - x0.z;
        }
    }
}

constexpr int NK1 = NIN / 32, NK2 = NH / 32;  // k-steps of the two hidden layers
constexpr int NTI = 2 * NH;                     // inference workgroup: NH / 32 wavefronts of 32 features
constexpr int GPC = NTI / TM;                   // gather threads per cell
constexpr int RPT = 16 / GPC;                   // patch rows (4 nodes each) per gather thread

// Workgroup barrier for LDS traffic only: this wavefront's LDS operations are complete, global loads
// may still be in flight (they land in registers that are not read before their own wait).
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// Inference, part 1: the network for every listed cell. Persistent: workgroups of NH / 32 wavefronts, as many
// per CU as fit, walk the 64-cell tiles; wavefront w owns features 32w .. 32w+31 of both hidden layers and
// keeps their B operands in registers for the whole run (NIN / 16 + NH / 16 + 1 16-byte fragments) instead of
// loading them per tile. The layers are computed transposed, (X W)^T = W^T X^T, so that a lane ends with four
// consecutive features of one cell: they go to LDS as one 8-byte word (first layer) or, after the second
// layer, straight into a B operand of the head, whose k index is permuted to match (k = 8q + j holds feature
// 32w + 4q + j for j < 4 and 32w + 16 + 4q + j - 4 otherwise, q = lane / 16). Each wavefront thus multiplies
// its own 32 features by the matching rows of W3 and the NH / 32 partial heads of a cell are summed in LDS,
// by wavefront 0 after the next tile's first barrier: two barriers per tile (features, first layer). The
// barriers wait for LDS traffic only, so that the patch nodes of the next tile (and the cell ids of the one
// after) stay in flight across them. Each layer runs block by block of 16 cells (all k-steps of a block,
// then its gelu epilogue), so that a block's epilogue can issue beside the next block's matrix products and
// only one A fragment is live at a time; gelu is the fitted closed form (gelu_fit), so the CU's LDS carries
// operands only. Registers are held to what three workgroups per CU allow (168). Output per cell: (Z3[0],
// Z3[1], Z3[2], conf).
__global__ __launch_bounds__(NTI) __attribute__((amdgpu_waves_per_eu(3, 3))) void infer_net_k(
    Net N, Geo g, const uint64_t *__restrict__ cells, const int64_t *__restrict__ count, int64_t cap,
    float4 *net_out, float4 *centre, int64_t *fb_count, unsigned long long *flag) {
    constexpr int NW = NTI / 64;
    static_assert(NW * 32 == NH && (GPC == 4 || GPC == 8), "one wavefront per 32 hidden features");
    __shared__ __attribute__((aligned(16))) __bf16 sX[TM * XP];
    __shared__ __attribute__((aligned(16))) __bf16 sH[TM * HP];
    __shared__ __attribute__((aligned(16))) float sB[2 * NH];          // b1 then b2
    __shared__ __attribute__((aligned(16))) float sP[NW * TM * NOUT];  // partial heads [wavefront][cell][4]
    const int64_t cnt = *count;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *fb_count = 0;  // the fallback queue of polish_k, launched next
        if (cnt > cap) atomicOr(flag, (unsigned long long)VX_OVERFLOW_REFINE);
    }
    const int64_t n = min(cnt, cap);
    const int64_t ntiles = (n + TM - 1) / TM;
    if ((int64_t)blockIdx.x >= ntiles) return;  // uniform per workgroup
    const int t = threadIdx.x, l = t & 63, w = t >> 6, n0 = 32 * w, q4 = 4 * (l >> 4);
    const int64_t G = gridDim.x;
    sB[t] = N.master[t < NH ? OFF_B1 + t : OFF_B2 + t - NH];
    bf16x8 b1[2][NK1], b2[2][NK2], a3;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        const int col = n0 + 16 * c + (l & 15);
#pragma unroll
        for (int kk = 0; kk < NK1; ++kk) b1[c][kk] = ld8(N.w1t + col * NIN + 32 * kk + 8 * (l >> 4));
#pragma unroll
        for (int kk = 0; kk < NK2; ++kk) b2[c][kk] = ld8(N.w2t + col * NH + 32 * kk + 8 * (l >> 4));
    }
    {   // head A operand: row l % 16 of W3^T (rows 4..15 are zero), the permuted k of this wavefront
        const __bf16 *p = N.w3t + (l & 15) * NH + n0 + q4;
        const uint2 lo = *(const uint2 *)p, hi = *(const uint2 *)(p + 16);
        a3 = __builtin_bit_cast(bf16x8, make_uint4(lo.x, lo.y, hi.x, hi.y));
    }
    const float4 bias3 = make_float4(N.master[OFF_B3], N.master[OFF_B3 + 1], N.master[OFF_B3 + 2], N.master[OFF_B3 + 3]);

    // gather role: GPC threads per cell; thread (r, q) loads patch rows q RPT .. q RPT + RPT - 1 (row R:
    // row R % 4 of patch plane R / 4), i.e. features 8 RPT q .. 8 RPT (q + 1) - 1
    const int r = t / GPC, q = t % GPC;
    const uint64_t ncell = (uint64_t)g.nx * g.ny * g.nz;
    auto cell_of = [&](int64_t tile) -> uint64_t {
        const int64_t s = tile * TM + r;
        const uint64_t c = (tile < ntiles && s < n) ? cells[s] : 0;
        return c < ncell ? c : 0;
    };
    float2 v[4 * RPT];
    auto fetch = [&](uint64_t cell) {
        int i, j, k;
        cell_xyz(cell, g, i, j, k);
        const uint64_t nx = (uint64_t)g.nx;
        // away from the x seams a row's four nodes are contiguous: two 16-byte loads (8-byte aligned)
        const bool xin = i >= 1 && i + 2 < g.nx;
#pragma unroll
        for (int b = 0; b < RPT; ++b) {
            const int R = q * RPT + b;
            const int kk = wrapc(k + (R >> 2) - 1, g.nz, g.pz);
            const int jj = wrapc(j + (R & 3) - 1, g.ny, g.py);
            const float2 *row = g.psi + nx * ((uint64_t)jj + (uint64_t)g.ny * (uint64_t)kk);
            if (xin) {
                typedef float f4a8 __attribute__((ext_vector_type(4), aligned(8)));
                const f4a8 lo = *(const f4a8 *)(row + i - 1), hi = *(const f4a8 *)(row + i + 1);
                v[4 * b + 0] = make_float2(lo.x, lo.y);
                v[4 * b + 1] = make_float2(lo.z, lo.w);
                v[4 * b + 2] = make_float2(hi.x, hi.y);
                v[4 * b + 3] = make_float2(hi.z, hi.w);
            } else {
#pragma unroll
                for (int a = 0; a < 4; ++a) v[4 * b + a] = row[wrapc(i + a - 1, g.nx, g.px)];
            }
        }
    };
    // output of tile tt (if it is one of this workgroup's tiles): bias + the NW partial heads
    auto head_out = [&](int64_t tt) {
        if (tt >= (int64_t)blockIdx.x && t < TM && tt * TM + t < n) {
            float4 o = bias3;
#pragma unroll
            for (int u = 0; u < NW; ++u) {
                const float4 p = *(const float4 *)(sP + (u * TM + t) * NOUT);
                o.x += p.x;
                o.y += p.y;
                o.z += p.z;
                o.w += p.w;
            }
            net_out[tt * TM + t] = make_float4(o.x, o.y, o.z, 1.f / (1.f + expf(-o.w)));
        }
    };
    int64_t tile = blockIdx.x;
    fetch(cell_of(tile));
    uint64_t cell_next = cell_of(tile + G);
    for (; tile < ntiles; tile += G) {
        // features -> sX (free: the previous tile's first layer ended before its second barrier)
        {
            float ss = 0.f;
#pragma unroll
            for (int e = 0; e < 4 * RPT; ++e) ss += v[e].x * v[e].x + v[e].y * v[e].y;
#pragma unroll
            for (int o = 1; o < GPC; o <<= 1) ss += __shfl_xor(ss, o);
            const float is = 1.f / (ss > 0.f ? sqrtf(ss * (1.f / 64.f)) : 1.f);
            uint32_t *dst = (uint32_t *)(sX + r * XP + 8 * RPT * q);
#pragma unroll
            for (int e = 0; e < 4 * RPT; ++e) dst[e] = pack2(v[e].x * is, v[e].y * is);
            // the cell's own corners d = dx + 2 dy + 4 dz (nodes 1, 2 of rows 1, 2 of planes 1, 2) for the
            // polish, from the threads that hold those rows: corners 2 (dy + 2 dz) and 2 (dy + 2 dz) + 1 as
            // one float4 (streaming stores: read once, by the next kernel)
            const int64_t s = tile * TM + r;
            if (s < n) {
                typedef float f4v __attribute__((ext_vector_type(4)));
#pragma unroll
                for (int b = 0; b < RPT; ++b) {
                    const int R = q * RPT + b, pz = R >> 2, py = R & 3;
                    if (pz >= 1 && pz <= 2 && py >= 1 && py <= 2)
                        __builtin_nontemporal_store((f4v){v[4 * b + 1].x, v[4 * b + 1].y, v[4 * b + 2].x, v[4 * b + 2].y},
                                                    (f4v *)(centre + 4 * s + 2 * (pz - 1) + (py - 1)));
                }
            }
        }
        // next tile's nodes and the ids of the one after, in flight while this tile's layers run
        fetch(cell_next);
        cell_next = cell_of(tile + 2 * G);
        lds_barrier();  // sX complete (and, at the first tile, the table and the biases)
        // the previous tile's partial heads were complete at this barrier; wavefront 0 sums them
        // (they are overwritten only after the next barrier, which it reaches after reading them)
        head_out(tile - G);
        // this lane accumulates features n0 + 16c + q4 + 0..3 of cell 16rr + l % 16, from their biases
        f32x4 acc[4][2];
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const f32x4 b = *(const f32x4 *)(sB + n0 + 16 * c + q4);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) acc[rr][c] = b;
        }
        // sH is free: the previous tile's second layer ended before this tile's first barrier
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
#pragma unroll
            for (int kk = 0; kk < NK1; ++kk) {
                const bf16x8 a = ld8(sX + (16 * rr + (l & 15)) * XP + 32 * kk + 8 * (l >> 4));
#pragma unroll
                for (int c = 0; c < 2; ++c) acc[rr][c] = mfma(b1[c][kk], a, acc[rr][c]);
            }
#pragma unroll
            for (int c = 0; c < 2; ++c)
                *(uint2 *)(sH + (16 * rr + (l & 15)) * HP + n0 + 16 * c + q4) =
                    make_uint2(pack2(gelu_fit(acc[rr][c][0]), gelu_fit(acc[rr][c][1])),
                               pack2(gelu_fit(acc[rr][c][2]), gelu_fit(acc[rr][c][3])));
        }
        lds_barrier();  // H1 complete
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const f32x4 b = *(const f32x4 *)(sB + NH + n0 + 16 * c + q4);
#pragma unroll
            for (int rr = 0; rr < 4; ++rr) acc[rr][c] = b;
        }
        // H2 never leaves registers: partial head of this wavefront's 32 features; lanes 0..15 end
        // with outputs 0..3 of cell 16rr + l (the rows of the other lanes are the zero padding)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
#pragma unroll
            for (int kk = 0; kk < NK2; ++kk) {
                const bf16x8 a = ld8(sH + (16 * rr + (l & 15)) * HP + 32 * kk + 8 * (l >> 4));
#pragma unroll
                for (int c = 0; c < 2; ++c) acc[rr][c] = mfma(b2[c][kk], a, acc[rr][c]);
            }
            const uint4 hv = make_uint4(pack2(gelu_fit(acc[rr][0][0]), gelu_fit(acc[rr][0][1])),
                                        pack2(gelu_fit(acc[rr][0][2]), gelu_fit(acc[rr][0][3])),
                                        pack2(gelu_fit(acc[rr][1][0]), gelu_fit(acc[rr][1][1])),
                                        pack2(gelu_fit(acc[rr][1][2]), gelu_fit(acc[rr][1][3])));
            const f32x4 z = mfma(a3, __builtin_bit_cast(bf16x8, hv), f32x4{0.f, 0.f, 0.f, 0.f});
            if (l < 16) *(f32x4 *)(sP + (w * TM + 16 * rr + l) * NOUT) = z;
        }
    }
    lds_barrier();  // the last tile's partial heads complete
    head_out(tile - G);
}

// Inference, part 2: one thread per listed cell. Confident single-core interior cells get the network's point
// polished by one Newton step; the others, and cells whose polish fails, are queued (cell, descriptor,
// position in the list) for the plain refinement, with one atomic per workgroup and pass.
__global__ __launch_bounds__(NT) void polish_k(Geo g, const uint64_t *__restrict__ cells,
                                               const uint16_t *__restrict__ desc, const int64_t *__restrict__ count,
                                               int64_t cap, const float4 *__restrict__ net_out,
                                               const float4 *__restrict__ centre, float thr, float max_step,
                                               vx_sample *out, uint64_t *fb_cell, uint16_t *fb_desc, int64_t *fb_index,
                                               int64_t *fb_count) {
    __shared__ uint32_t s_cnt;
    __shared__ int64_t s_base;
    const int64_t n = min(*count, cap);
    // grid-stride over the listed cells: the grid is sized for the capacity only up to what the chip
    // holds at once, so that a short list does not pay for thousands of workgroups that find nothing
    // to do (each would wait for the count before returning)
    const int64_t stride = (int64_t)gridDim.x * NT;
    for (int64_t s0 = (int64_t)blockIdx.x * NT; s0 < n; s0 += stride) {  // uniform per workgroup
        const int64_t s = s0 + threadIdx.x;
        bool queue = false;
        uint64_t cell = 0;
        uint32_t d = 0;
        if (s < n) {
            cell = cells[s];
            d = desc[s];
            // requested with the other inputs (one round of loads), whether the cell is polished or not
            float4 ctr[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) ctr[q] = centre[4 * s + q];
            uint32_t st0 = 0;
            const vxr::V3 x0 = vxr::first_estimate(d, st0);
            const int np = __popc((d | (d >> 1)) & 0x555u);  // pierced faces: nonzero 2-bit fields
            const float4 o = net_out[s];
            bool mine = np == 2 && o.w >= thr && cell < (uint64_t)g.nx * g.ny * g.nz;
            int i = 0, j = 0, k = 0;
            if (mine) {
                cell_xyz(cell, g, i, j, k);
                mine = interior(g, i, j, k);
            }
            if (mine) {
                const vxr::V3 xs = vxr::v3(x0.x + o.x, x0.y + o.y, x0.z + o.z);
                vxr::V3 x;
                float rho = 0.f;
                mine = polish(g, i, j, k, d, ctr, x0, xs, max_step, x, rho);
                if (mine) {
                    vx_sample r{};
                    r.cell = cell;
                    r.off[0] = x.x;
                    r.off[1] = x.y;
                    r.off[2] = x.z;
                    r.rho = rho;
                    r.iters = 1;
                    r.status = (uint16_t)VX_SAMPLE_SURROGATE;
                    out[s] = r;
                }
            }
            queue = !mine;
        }
        // the workgroup's queued cells take one block of the queue: the wavefronts count theirs in LDS
        // and one thread reserves the block with a single atomic (device-scope atomics on one counter
        // are serialised; one per wavefront made the queue the bottleneck of this kernel)
        const uint64_t qm = __ballot(queue);
        const int lane = (int)(threadIdx.x & 63);
        if (threadIdx.x == 0) s_cnt = 0;
        __syncthreads();
        uint32_t woff = 0;
        if (qm) {
            const int lead = __builtin_ctzll(qm);
            if (lane == lead) woff = atomicAdd(&s_cnt, (uint32_t)__popcll(qm));
            woff = (uint32_t)__shfl((int)woff, lead);
        }
        __syncthreads();
        if (threadIdx.x == 0 && s_cnt)
            s_base = (int64_t)atomicAdd((unsigned long long *)fb_count, (unsigned long long)s_cnt);
        __syncthreads();
        if (queue) {
            const uint32_t rank =
                __builtin_amdgcn_mbcnt_hi((uint32_t)(qm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)qm, 0u));
            const int64_t k = s_base + woff + rank;
            fb_cell[k] = cell;
            fb_desc[k] = (uint16_t)d;
            fb_index[k] = s;
        }
        __syncthreads();  // s_cnt and s_base are reset and rewritten by the next iteration
    }
}

}  // namespace

// ---------------------------------------------------------------------------- host side

struct vx_mlp {
    vx_handle *h = nullptr;
    int64_t max_batch = 0;
    int64_t step = 0;
    float *master = nullptr, *mom1 = nullptr, *mom2 = nullptr, *grad = nullptr;
    __bf16 *w1t = nullptr, *w2t = nullptr, *w2c = nullptr, *w3t = nullptr;
    float2 *gelu = nullptr, *dgelu = nullptr;
    // training scratch
    __bf16 *H1 = nullptr, *G1 = nullptr, *H2 = nullptr, *G2 = nullptr, *dZ2 = nullptr, *dZ1 = nullptr;
    float *dZ3 = nullptr, *loss = nullptr;
    // inference buffers, sized by vx_mlp_reserve for lists of up to fb_cap cells
    int64_t fb_cap = 0;
    float4 *net_out = nullptr;
    float4 *centre = nullptr;  // [cap][4]: the 8 corners of each listed cell, for the polish
    uint64_t *fb_cell = nullptr;
    uint16_t *fb_desc = nullptr;
    int64_t *fb_index = nullptr;
    int64_t *fb_count = nullptr;
    int infer_per_cu = 1;  // resident infer_net_k workgroups per CU
    std::vector<void *> allocs;
};

namespace {

Net net_of(const vx_mlp *m) {
    Net N;
    N.master = m->master;
    N.w1t = m->w1t;
    N.w2t = m->w2t;
    N.w2c = m->w2c;
    N.w3t = m->w3t;
    N.gelu = m->gelu;
    N.dgelu = m->dgelu;
    return N;
}

vx_status dalloc(vx_mlp *m, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return vx_hip_check(m->h, e, "vx_mlp: hipMalloc");
    m->allocs.push_back(*p);
    return VX_OK;
}

Geo geo_of(const vx_dims &d, const void *psi) {
    Geo g;
    g.psi = (const float2 *)psi;
    g.nx = d.nx;
    g.ny = d.ny;
    g.nz = d.nz;
    g.px = (int)(d.periodic & 1u);
    g.py = (int)((d.periodic >> 1) & 1u);
    g.pz = (int)((d.periodic >> 2) & 1u);
    g.rnx = 1.0 / (double)d.nx;
    g.rnxy = 1.0 / ((double)d.nx * (double)d.ny);
    return g;
}

vx_status refresh(vx_mlp *m, hipStream_t s) {
    hipLaunchKernelGGL(refresh_k, dim3(256), dim3(256), 0, s, m->master, m->w1t, m->w2t, m->w2c, m->w3t);
    return vx_hip_check(m->h, hipGetLastError(), "vx_mlp: refresh");
}

// forward (training) + backward into m->grad
vx_status grad_pass(vx_mlp *m, const uint16_t *feat, const float *target, const int32_t *idx, int64_t n, float lam,
                    float tol, hipStream_t s) {
    const Net N = net_of(m);
    const unsigned tiles = (unsigned)((n + TM - 1) / TM);
    const __bf16 *X = (const __bf16 *)feat;
    hipLaunchKernelGGL(zero_f_k, dim3(1), dim3(64), 0, s, m->loss, 2);
    hipLaunchKernelGGL(fwd_train_k, dim3(tiles), dim3(NT), 0, s, N, X, target, idx, n, lam, tol, m->H1, m->G1, m->H2,
                       m->G2, m->dZ3, m->loss);
    hipLaunchKernelGGL(bwd_rows_k, dim3(tiles), dim3(NT), 0, s, N, n, m->dZ3, m->H2, m->G1, m->G2, m->dZ2, m->dZ1,
                       m->grad);
    const unsigned chunks = (unsigned)((n + WCH - 1) / WCH);
    hipLaunchKernelGGL(wgrad_k, dim3(chunks, NH / 128, NH / 128), dim3(NT), 0, s, (const __bf16 *)m->H1, NH,
                       (const int32_t *)nullptr, (const __bf16 *)m->dZ2, NH, n, m->grad + OFF_W2);
    hipLaunchKernelGGL(wgrad_k, dim3(chunks, NIN / 128, NH / 128), dim3(NT), 0, s, X, NIN, idx,
                       (const __bf16 *)m->dZ1, NH, n, m->grad + OFF_W1);
    return vx_hip_check(m->h, hipGetLastError(), "vx_mlp: gradient kernels");
}

vx_status check_n(vx_mlp *m, int64_t n) {
    if (n < 1 || n > m->max_batch)
        return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp: batch of %lld rows (1..%lld)", (long long)n,
                       (long long)m->max_batch);
    return VX_OK;
}

}  // namespace

extern "C" vx_status vx_mlp_create(vx_handle *h, const float *h_params, int64_t max_batch, vx_mlp **out) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (!out || !h_params) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_create: null argument");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (1LL << 26)) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_create: max_batch");
    if (vx_status st = vx_bind(h)) return st;
    vx_mlp *m = new (std::nothrow) vx_mlp();
    if (!m) return VX_ERR_NOMEM;
    m->h = h;
    m->max_batch = max_batch;
    const size_t P4 = (size_t)NPARAM * 4;
    const size_t act = (size_t)max_batch * NH * 2;
    vx_status st = VX_OK;
    void **fl[] = {(void **)&m->master, (void **)&m->mom1, (void **)&m->mom2, (void **)&m->grad};
    for (void **p : fl)
        if (st == VX_OK) st = dalloc(m, p, P4);
    if (st == VX_OK) st = dalloc(m, (void **)&m->w1t, (size_t)NIN * NH * 2);
    if (st == VX_OK) st = dalloc(m, (void **)&m->w2t, (size_t)NH * NH * 2);
    if (st == VX_OK) st = dalloc(m, (void **)&m->w2c, (size_t)NH * NH * 2);
    if (st == VX_OK) st = dalloc(m, (void **)&m->w3t, (size_t)16 * NH * 2);
    if (st == VX_OK) st = dalloc(m, (void **)&m->gelu, GT * sizeof(float2));
    if (st == VX_OK) st = dalloc(m, (void **)&m->dgelu, GT * sizeof(float2));
    void **ac[] = {(void **)&m->H1, (void **)&m->G1, (void **)&m->H2, (void **)&m->G2, (void **)&m->dZ2, (void **)&m->dZ1};
    for (void **p : ac)
        if (st == VX_OK) st = dalloc(m, p, act);
    if (st == VX_OK) st = dalloc(m, (void **)&m->dZ3, (size_t)max_batch * NOUT * 4);
    if (st == VX_OK) st = dalloc(m, (void **)&m->loss, 64);
    if (st == VX_OK) st = dalloc(m, (void **)&m->fb_count, 64);
    if (st == VX_OK) st = vx_hip_check(h, hipMemcpy(m->master, h_params, P4, hipMemcpyHostToDevice), "vx_mlp_create");
    if (st == VX_OK) st = vx_hip_check(h, hipMemset(m->mom1, 0, P4), "hipMemset");
    if (st == VX_OK) st = vx_hip_check(h, hipMemset(m->mom2, 0, P4), "hipMemset");
    if (st == VX_OK) st = vx_hip_check(h, hipMemset(m->grad, 0, P4), "hipMemset");
    if (st == VX_OK) st = vx_hip_check(h, hipMemset(m->w3t, 0, (size_t)16 * NH * 2), "hipMemset");
    if (st == VX_OK) {
        hipLaunchKernelGGL(tables_k, dim3((GT + 255) / 256), dim3(256), 0, 0, m->gelu, m->dgelu);
        st = refresh(m, 0);
    }
    if (st == VX_OK) st = vx_hip_check(h, hipDeviceSynchronize(), "vx_mlp_create");
    if (st == VX_OK) {
        int nb = 0;
        st = vx_hip_check(h, hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, infer_net_k, NTI, 0), "vx_mlp_create");
        m->infer_per_cu = nb > 0 ? nb : 1;
    }
    if (st) {
        vx_mlp_destroy(m);
        return st;
    }
    *out = m;
    return VX_OK;
}

extern "C" vx_status vx_mlp_destroy(vx_mlp *m) {
    if (!m) return VX_OK;
    (void)vx_bind(m->h);
    for (void *p : m->allocs) (void)hipFree(p);
    delete m;
    return VX_OK;
}

extern "C" vx_status vx_mlp_reserve(vx_mlp *m, int64_t max_cells) {
    if (!m) return VX_ERR_INVALID;
    vx_handle *h = m->h;
    h->err.clear();
    if (max_cells < 0 || max_cells > (1LL << 36)) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_reserve: max_cells");
    if (max_cells <= m->fb_cap) return VX_OK;
    if (vx_status st = vx_bind(h)) return st;
    // the old buffers may still be read by work in flight on any stream
    if (vx_status st = vx_hip_check(h, hipDeviceSynchronize(), "vx_mlp_reserve")) return st;
    for (void *q : {(void *)m->fb_cell, (void *)m->fb_desc, (void *)m->fb_index, (void *)m->net_out, (void *)m->centre}) {
        if (!q) continue;
        (void)hipFree(q);
        for (auto &a : m->allocs)
            if (a == q) a = nullptr;
    }
    m->fb_cell = nullptr;
    m->fb_desc = nullptr;
    m->fb_index = nullptr;
    m->net_out = nullptr;
    m->centre = nullptr;
    m->fb_cap = 0;
    const size_t c = (size_t)max_cells;
    vx_status st = dalloc(m, (void **)&m->fb_cell, c * 8);
    if (st == VX_OK) st = dalloc(m, (void **)&m->net_out, c * sizeof(float4));
    if (st == VX_OK) st = dalloc(m, (void **)&m->centre, c * 4 * sizeof(float4));
    if (st == VX_OK) st = dalloc(m, (void **)&m->fb_desc, c * 2);
    if (st == VX_OK) st = dalloc(m, (void **)&m->fb_index, c * 8);
    if (st) return st;
    m->fb_cap = max_cells;
    return VX_OK;
}

extern "C" vx_status vx_mlp_get_params(vx_mlp *m, float *h_params) {
    if (!m || !h_params) return VX_ERR_INVALID;
    if (vx_status st = vx_bind(m->h)) return st;
    return vx_hip_check(m->h, hipMemcpy(h_params, m->master, (size_t)NPARAM * 4, hipMemcpyDeviceToHost),
                        "vx_mlp_get_params");
}

extern "C" vx_status vx_mlp_set_params(vx_mlp *m, const float *h_params) {
    if (!m || !h_params) return VX_ERR_INVALID;
    if (vx_status st = vx_bind(m->h)) return st;
    vx_status st = vx_hip_check(m->h, hipMemcpy(m->master, h_params, (size_t)NPARAM * 4, hipMemcpyHostToDevice),
                                "vx_mlp_set_params");
    if (st == VX_OK) st = refresh(m, 0);
    if (st == VX_OK) st = vx_hip_check(m->h, hipDeviceSynchronize(), "vx_mlp_set_params");
    return st;
}

extern "C" vx_status vx_mlp_save(vx_mlp *m, const char *path) {
    if (!m || !path) return VX_ERR_INVALID;
    std::vector<float> p(NPARAM);
    if (vx_status st = vx_mlp_get_params(m, p.data())) return st;
    FILE *f = std::fopen(path, "wb");
    if (!f) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_save: cannot open %s", path);
    const char magic[8] = {'V', 'X', 'M', 'L', 'P', '1', 0, 0};
    const int64_t cnt = NPARAM;
    bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&cnt, 8, 1, f) == 1 &&
              std::fwrite(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? VX_OK : vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_save: write failed");
}

extern "C" vx_status vx_mlp_load(vx_mlp *m, const char *path) {
    if (!m || !path) return VX_ERR_INVALID;
    FILE *f = std::fopen(path, "rb");
    if (!f) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_load: cannot open %s", path);
    char magic[8];
    int64_t cnt = 0;
    std::vector<float> p(NPARAM);
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "VXMLP1", 6) == 0 && std::fread(&cnt, 8, 1, f) == 1 &&
              cnt == NPARAM && std::fread(p.data(), 4, NPARAM, f) == (size_t)NPARAM;
    std::fclose(f);
    if (!ok) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_load: %s is not a parameter file of this network", path);
    return vx_mlp_set_params(m, p.data());
}

extern "C" vx_status vx_mlp_dataset(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                                    const uint16_t *d_cell_desc, const vx_sample *d_samples, const int64_t *d_count,
                                    int64_t cap, uint16_t *d_feat, float *d_target, int64_t *d_n, int64_t n_cap,
                                    vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (!d_psi || !d_cells || !d_cell_desc || !d_samples || !d_count || !d_feat || !d_target || !d_n)
        return vx_fail(h, VX_ERR_INVALID, "vx_mlp_dataset: null pointer argument");
    if (((uintptr_t)d_feat & 15u) != 0) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_dataset: d_feat must be 16-byte aligned");
    if (cap < 0 || n_cap < 0) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_dataset: negative capacity");
    if (cap == 0) return VX_OK;
    if (vx_status st = vx_bind(h)) return st;
    const unsigned blocks = (unsigned)((cap + TM - 1) / TM);
    hipLaunchKernelGGL(dataset_k, dim3(blocks), dim3(NT), 0, (hipStream_t)s, geo_of(dims, d_psi), d_cells, d_cell_desc,
                       d_samples, d_count, cap, (__bf16 *)d_feat, d_target, (unsigned long long *)d_n, n_cap,
                       vx_overflow_flag(h));
    return vx_hip_check(h, hipGetLastError(), "dataset_k launch");
}

extern "C" vx_status vx_mlp_features(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                                     const int64_t *d_count, int64_t cap, uint16_t *d_feat, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (!d_psi || !d_cells || !d_count || !d_feat) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_features: null pointer");
    if (cap < 0) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_features: negative capacity");
    if (cap == 0) return VX_OK;
    if (vx_status st = vx_bind(h)) return st;
    hipLaunchKernelGGL(features_k, dim3((unsigned)((cap + TM - 1) / TM)), dim3(NT), 0, (hipStream_t)s,
                       geo_of(dims, d_psi), d_cells, d_count, cap, (__bf16 *)d_feat);
    return vx_hip_check(h, hipGetLastError(), "features_k launch");
}

extern "C" vx_status vx_mlp_train_step(vx_mlp *m, const uint16_t *d_feat, const float *d_target, const int32_t *d_idx,
                                       int64_t n, const vx_adam_params *p, float *d_loss, vx_stream s) {
    if (!m) return VX_ERR_INVALID;
    m->h->err.clear();
    if (!d_feat || !d_target || !p) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_train_step: null argument");
    if (vx_status st = check_n(m, n)) return st;
    if (!(p->lr > 0.f) || !(p->beta1 >= 0.f && p->beta1 < 1.f) || !(p->beta2 >= 0.f && p->beta2 < 1.f) || !(p->eps > 0.f))
        return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_train_step: bad Adam parameters");
    if (vx_status st = vx_bind(m->h)) return st;
    hipStream_t hs = (hipStream_t)s;
    vx_timer tm(m->h, hs, VX_KIND_MLP);
    vx_status st = grad_pass(m, d_feat, d_target, d_idx, n, p->conf_lambda, p->conf_tol, hs);
    if (st == VX_OK) {
        ++m->step;
        const float c1 = (float)(1.0 / (1.0 - std::pow((double)p->beta1, (double)m->step)));
        const float c2 = (float)(1.0 / (1.0 - std::pow((double)p->beta2, (double)m->step)));
        hipLaunchKernelGGL(adam_k, dim3(128), dim3(256), 0, hs, m->master, m->mom1, m->mom2, m->grad, p->lr, p->beta1,
                           p->beta2, p->eps, c1, c2);
        st = refresh(m, hs);
        if (st == VX_OK && d_loss)
            st = vx_hip_check(m->h, hipMemcpyAsync(d_loss, m->loss, 8, hipMemcpyDeviceToDevice, hs), "loss copy");
    }
    tm.stop();
    return st;
}

extern "C" vx_status vx_mlp_grad(vx_mlp *m, const uint16_t *d_feat, const float *d_target, int64_t n, float conf_lambda,
                                 float conf_tol, float *d_grad, float *d_loss, vx_stream s) {
    if (!m) return VX_ERR_INVALID;
    m->h->err.clear();
    if (!d_feat || !d_target || !d_grad) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_grad: null argument");
    if (vx_status st = check_n(m, n)) return st;
    if (vx_status st = vx_bind(m->h)) return st;
    hipStream_t hs = (hipStream_t)s;
    vx_status st = grad_pass(m, d_feat, d_target, nullptr, n, conf_lambda, conf_tol, hs);
    if (st == VX_OK) {
        hipLaunchKernelGGL(copy_zero_k, dim3(128), dim3(256), 0, hs, m->grad, d_grad);
        st = vx_hip_check(m->h, hipGetLastError(), "copy_zero_k");
    }
    if (st == VX_OK && d_loss)
        st = vx_hip_check(m->h, hipMemcpyAsync(d_loss, m->loss, 8, hipMemcpyDeviceToDevice, hs), "loss copy");
    return st;
}

extern "C" vx_status vx_mlp_forward(vx_mlp *m, const uint16_t *d_feat, int64_t n, float *d_out, vx_stream s) {
    if (!m) return VX_ERR_INVALID;
    m->h->err.clear();
    if (!d_feat || !d_out) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_forward: null argument");
    if (n < 0) return vx_fail(m->h, VX_ERR_INVALID, "vx_mlp_forward: negative n");
    if (n == 0) return VX_OK;
    if (vx_status st = vx_bind(m->h)) return st;
    hipLaunchKernelGGL(fwd_k, dim3((unsigned)((n + TM - 1) / TM)), dim3(NT), 0, (hipStream_t)s, net_of(m),
                       (const __bf16 *)d_feat, n, d_out);
    return vx_hip_check(m->h, hipGetLastError(), "fwd_k launch");
}

// the network kernel over a listed-cell capacity (persistent grid: the resident workgroups, at most one
// per 64-cell tile); its outputs go to net_out
static void launch_net(vx_mlp *m, vx_dims dims, const void *d_psi, const uint64_t *d_cells, const int64_t *d_count,
                       int64_t cap, float4 *net_out, hipStream_t hs) {
    vx_handle *h = m->h;
    vx_timer tm(h, hs, VX_KIND_MLP);
    const int64_t num_cu = h->num_cu > 0 ? h->num_cu : 256;
    const int64_t tiles = (cap + TM - 1) / TM;
    const int64_t grid = std::max<int64_t>(1, std::min<int64_t>(tiles, num_cu * m->infer_per_cu));
    hipLaunchKernelGGL(infer_net_k, dim3((unsigned)grid), dim3(NTI), 0, hs, net_of(m), geo_of(dims, d_psi), d_cells,
                       d_count, cap, net_out, m->centre, m->fb_count, vx_overflow_flag(h));
    tm.stop();
}

extern "C" vx_status vx_mlp_predict(vx_mlp *m, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                                    const int64_t *d_count, int64_t cap, float *d_out, vx_stream s) {
    if (!m) return VX_ERR_INVALID;
    vx_handle *h = m->h;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (cap < 0) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_predict: negative capacity");
    if (cap == 0) return VX_OK;
    if (!d_psi || !d_cells || !d_count || !d_out)
        return vx_fail(h, VX_ERR_INVALID, "vx_mlp_predict: null pointer argument");
    if ((reinterpret_cast<uintptr_t>(d_out) & 15u) != 0)
        return vx_fail(h, VX_ERR_INVALID, "vx_mlp_predict: d_out must be 16-byte aligned");
    if (vx_status st = vx_bind(h)) return st;
    if (cap > m->fb_cap)
        return vx_fail(h, VX_ERR_INVALID,
                       "vx_mlp_predict: capacity %lld exceeds the %lld cells reserved by vx_mlp_reserve",
                       (long long)cap, (long long)m->fb_cap);
    launch_net(m, dims, d_psi, d_cells, d_count, cap, reinterpret_cast<float4 *>(d_out), (hipStream_t)s);
    return vx_hip_check(h, hipGetLastError(), "vx_mlp_predict launch");
}

extern "C" vx_status vx_mlp_infer(vx_mlp *m, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                                  const uint16_t *d_cell_desc, const int64_t *d_count, int64_t cap, float conf_threshold,
                                  float max_step, const vx_refine_params *p, vx_sample *d_out, vx_stream s) {
    if (!m) return VX_ERR_INVALID;
    vx_handle *h = m->h;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (cap < 0) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_infer: negative capacity");
    if (cap == 0) return VX_OK;
    if (!d_psi || !d_cells || !d_cell_desc || !d_count || !d_out)
        return vx_fail(h, VX_ERR_INVALID, "vx_mlp_infer: null pointer argument");
    const vx_refine_params prm = p ? *p : vx_refine_defaults();
    if (vx_status st = vx_check_refine_params(h, prm)) return st;
    if (vx_status st = vx_bind(h)) return st;
    if (cap > m->fb_cap)
        return vx_fail(h, VX_ERR_INVALID, "vx_mlp_infer: capacity %lld exceeds the %lld cells reserved by vx_mlp_reserve",
                       (long long)cap, (long long)m->fb_cap);
    if (!(max_step >= 0.f)) return vx_fail(h, VX_ERR_INVALID, "vx_mlp_infer: max_step must be >= 0");
    hipStream_t hs = (hipStream_t)s;
    const int64_t num_cu = h->num_cu > 0 ? h->num_cu : 256;
    launch_net(m, dims, d_psi, d_cells, d_count, cap, m->net_out, hs);
    vx_timer tp(h, hs, VX_KIND_POLISH);
    const int64_t pgrid = std::max<int64_t>(1, std::min<int64_t>((cap + NT - 1) / NT, (int64_t)POLISH_WG_PER_CU * num_cu));
    hipLaunchKernelGGL(polish_k, dim3((unsigned)pgrid), dim3(NT), 0, hs, geo_of(dims, d_psi), d_cells,
                       d_cell_desc, d_count, cap, (const float4 *)m->net_out, (const float4 *)m->centre, conf_threshold,
                       max_step, d_out, m->fb_cell,
                       m->fb_desc, m->fb_index, m->fb_count);
    tp.stop();
    vx_status st = vx_hip_check(h, hipGetLastError(), "surrogate inference launch");
    if (st) return st;
    return vx_refine_launch(h, dims, d_psi, m->fb_cell, m->fb_desc, nullptr, m->fb_count, cap, prm, d_out, hs,
                            m->fb_index);
}
