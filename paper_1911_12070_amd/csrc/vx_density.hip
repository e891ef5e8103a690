// Density rho = |psi|^2 for the error metric of the vectorised lines (Sec. 5: e = sum_i rho(x_i) /
// (mean rho * N) over points x_i of the visualised lines; rho = 0 on a true core):
//   density_k       rho at arbitrary points, psi linearly interpolated between nodes (Sec. 5) with
//                   the refinement's own arithmetic (vx_refine_math.h), one thread per point;
//   mean_density_k  the mean of |psi|^2 over every node, accumulated in FP64 (one pass over psi).
#include "vx_refine_math.h"

namespace {

using namespace vxr;

struct DensArgs {
    const float2 *psi;
    int nx, ny, nz, px, py, pz;
};

__global__ __launch_bounds__(256) void density_k(DensArgs A, const double *__restrict__ pts, int64_t n,
                                                 float *__restrict__ rho) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int dim[3] = {A.nx, A.ny, A.nz}, per[3] = {A.px, A.py, A.pz};
    int g[3];
    float u[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double x = pts[3 * i + q];
        if (per[q]) x -= (double)dim[q] * floor(x / (double)dim[q]);
        const double fl = floor(x);
        int c = (int)fl;
        if (per[q]) c = ((c % dim[q]) + dim[q]) % dim[q];
        else c = min(max(c, 0), dim[q] - 2);  // cells of an open axis: min corner 0 .. n - 2
        g[q] = c;
        u[q] = (float)(per[q] ? x - fl : x - (double)c);
    }
    const int c0[3] = {0, 0, 0};
    float2 v[8], cf[8];
    fetch_corners(A.psi, A.nx, A.ny, A.nz, A.px, A.py, A.pz, g[0], g[1], g[2], c0, v);
    tri_coeffs(v, cf);
    float tr, ti;
    V3 tgr, tgi;
    trilinear(cf, u, tr, ti, tgr, tgi);
    rho[i] = vxr::rho2(tr, ti);
}

__global__ void zero_d_k(double *p) {
    if (threadIdx.x == 0) *p = 0.0;
}

__global__ __launch_bounds__(256) void mean_density_k(const float2 *__restrict__ psi, uint64_t nodes,
                                                      double *__restrict__ sum) {
    double acc = 0.0;
    for (uint64_t q = (uint64_t)blockIdx.x * 256 + threadIdx.x; q < nodes; q += (uint64_t)gridDim.x * 256) {
        const float2 p = psi[q];
        acc += (double)p.x * (double)p.x + (double)p.y * (double)p.y;
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if ((threadIdx.x & 63) == 0) atomicAdd(sum, acc);
}

__global__ void finish_mean_k(double *sum, double nodes) {
    if (threadIdx.x == 0) *sum = *sum / nodes;
}

DensArgs dens_args(const vx_dims &d, const void *psi) {
    return DensArgs{(const float2 *)psi, d.nx, d.ny, d.nz, (int)(d.periodic & 1u), (int)((d.periodic >> 1) & 1u),
                    (int)((d.periodic >> 2) & 1u)};
}

}  // namespace

extern "C" vx_status vx_density(vx_handle *h, vx_dims dims, const void *d_psi, const double *d_points, int64_t n,
                                float *d_rho, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    const int32_t nd[3] = {dims.nx, dims.ny, dims.nz};
    for (int a = 0; a < 3; ++a)
        if (nd[a] < 2) return vx_fail(h, VX_ERR_INVALID, "vx_density: every axis needs at least 2 nodes");
    if (n < 0) return vx_fail(h, VX_ERR_INVALID, "vx_density: negative count");
    if (n == 0) return VX_OK;
    if (!d_psi || !d_points || !d_rho) return vx_fail(h, VX_ERR_INVALID, "vx_density: null pointer argument");
    if (vx_status st = vx_bind(h)) return st;
    hipLaunchKernelGGL(density_k, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, (hipStream_t)s,
                       dens_args(dims, d_psi), d_points, n, d_rho);
    return vx_hip_check(h, hipGetLastError(), "density_k launch");
}

extern "C" vx_status vx_mean_density(vx_handle *h, vx_dims dims, const void *d_psi, double *d_out, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (!d_psi || !d_out) return vx_fail(h, VX_ERR_INVALID, "vx_mean_density: null pointer argument");
    if (vx_status st = vx_bind(h)) return st;
    const uint64_t nodes = (uint64_t)dims.nx * dims.ny * dims.nz;
    hipStream_t hs = (hipStream_t)s;
    const uint64_t want = (nodes + 255) / 256;
    const unsigned blocks = (unsigned)std::min<uint64_t>(want, (uint64_t)(h->num_cu > 0 ? h->num_cu : 256) * 16);
    hipLaunchKernelGGL(zero_d_k, dim3(1), dim3(64), 0, hs, d_out);
    hipLaunchKernelGGL(mean_density_k, dim3(blocks), dim3(256), 0, hs, (const float2 *)d_psi, nodes, d_out);
    hipLaunchKernelGGL(finish_mean_k, dim3(1), dim3(64), 0, hs, d_out, (double)nodes);
    return vx_hip_check(h, hipGetLastError(), "mean_density_k launch");
}
