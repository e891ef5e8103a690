// Synthetic wavefunction generators (support for the benchmark and tests; not on the timed path).
//
// Both kernels use FP64 with one rounding per operation (this file is compiled with
// -ffp-contract=off and the kernels also forbid contraction), so a host evaluation that performs
// the same operations in the same order produces the same complex64 bytes.
#include "vx_internal.h"

namespace {

constexpr int GEN_THREADS = 256;
constexpr int GEN_WCHUNK = 256;   // waves staged in LDS per pass
constexpr int GEN_LDS_TABLE = 2048;  // largest table kept in LDS (32 KiB)

// v mod M for v < 2^32, M <= 46340, via an FP64 quotient estimate and one correction.
__device__ inline uint32_t mod_u32(uint32_t v, uint32_t M, double invM) {
    uint32_t q = (uint32_t)((double)v * invM);
    int64_t r = (int64_t)v - (int64_t)q * (int64_t)M;
    if (r < 0) r += M;
    if (r >= (int64_t)M) r -= M;
    return (uint32_t)r;
}

// One workgroup per grid row (y, z); each thread accumulates up to 4 nodes of the row in wave order.
template <bool TABLE_IN_LDS>
__global__ __launch_bounds__(GEN_THREADS) void gen_tangle_k(int nx, int ny, int nz, int nwaves, uint32_t M,
                                                           const uint32_t *__restrict__ ax,
                                                           const uint32_t *__restrict__ ay,
                                                           const uint32_t *__restrict__ az,
                                                           const double2 *__restrict__ coef,
                                                           const double2 *__restrict__ table,
                                                           float2 *__restrict__ psi) {
#pragma clang fp contract(off)
    __shared__ uint32_t s_ax[GEN_WCHUNK];
    __shared__ uint32_t s_base[GEN_WCHUNK];
    __shared__ double2 s_coef[GEN_WCHUNK];
    __shared__ double2 s_table[TABLE_IN_LDS ? GEN_LDS_TABLE : 1];

    const int64_t row = blockIdx.x;  // row = y + ny * z
    const uint32_t y = (uint32_t)(row % ny);
    const uint32_t z = (uint32_t)(row / ny);
    const double invM = 1.0 / (double)M;
    if (TABLE_IN_LDS)
        for (uint32_t m = threadIdx.x; m < M; m += GEN_THREADS) s_table[m] = table[m];

    for (int x0 = 0; x0 < nx; x0 += 4 * GEN_THREADS) {
        double re[4] = {0.0, 0.0, 0.0, 0.0}, im[4] = {0.0, 0.0, 0.0, 0.0};
        for (int w0 = 0; w0 < nwaves; w0 += GEN_WCHUNK) {
            __syncthreads();
            const int wk = w0 + threadIdx.x;
            if (wk < nwaves) {
                s_ax[threadIdx.x] = ax[wk];
                s_base[threadIdx.x] = mod_u32(ay[wk] * y + az[wk] * z, M, invM);
                s_coef[threadIdx.x] = coef[wk];
            }
            __syncthreads();
            const int nk = min(GEN_WCHUNK, nwaves - w0);
            for (int q = 0; q < 4; ++q) {
                const int x = x0 + q * GEN_THREADS + threadIdx.x;
                if (x >= nx) break;
                double r = re[q], i = im[q];
                for (int k = 0; k < nk; ++k) {
                    const uint32_t m = mod_u32(s_base[k] + s_ax[k] * (uint32_t)x, M, invM);
                    const double2 t = TABLE_IN_LDS ? s_table[m] : table[m];
                    const double2 c = s_coef[k];
                    const double p1 = c.x * t.x;
                    const double p2 = c.y * t.y;
                    const double d = p1 - p2;
                    r = r + d;
                    const double q1 = c.x * t.y;
                    const double q2 = c.y * t.x;
                    const double sm = q1 + q2;
                    i = i + sm;
                }
                re[q] = r;
                im[q] = i;
            }
        }
        for (int q = 0; q < 4; ++q) {
            const int x = x0 + q * GEN_THREADS + threadIdx.x;
            if (x < nx) psi[row * nx + x] = make_float2((float)re[q], (float)im[q]);
        }
    }
}

__device__ inline double minimg(double d, double n) { return d - n * rint(d / n); }

__global__ __launch_bounds__(GEN_THREADS) void gen_line_ring_k(int nx, int ny, int nz, vx_line_ring p,
                                                              const float2 *__restrict__ noise,
                                                              float2 *__restrict__ psi) {
#pragma clang fp contract(off)
    const int64_t total = (int64_t)nx * ny * nz;
    const double two_xi2 = 2.0 * p.xi * p.xi;
    for (int64_t q = (int64_t)blockIdx.x * GEN_THREADS + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * GEN_THREADS) {
        const double x = (double)(q % nx), y = (double)((q / nx) % ny), z = (double)(q / ((int64_t)nx * ny));
        const double dx = minimg(x - p.line_x, nx), dy = minimg(y - p.line_y, ny);
        const double sl = sqrt(dx * dx + dy * dy + two_xi2);
        const double lr = dx / sl, li = dy / sl;
        const double rx = minimg(x - p.ring_cx, nx), ry = minimg(y - p.ring_cy, ny), rz = minimg(z - p.ring_cz, nz);
        const double u = sqrt(rx * rx + ry * ry) - p.radius, v = rz;
        const double sr = sqrt(u * u + v * v + two_xi2);
        const double rr = u / sr, ri = v / sr;
        double pr = lr * rr - li * ri;
        double pi = lr * ri + li * rr;
        if (noise) {
            const float2 e = noise[q];
            pr += (double)e.x;
            pi += (double)e.y;
        }
        psi[q] = make_float2((float)pr, (float)pi);
    }
}

}  // namespace

extern "C" vx_status vx_gen_tangle(vx_handle *h, vx_dims d, const vx_tangle *t, void *d_psi, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, d)) return st;
    if (!t || !d_psi || !t->d_ax || !t->d_ay || !t->d_az || !t->d_coef || !t->d_table)
        return vx_fail(h, VX_ERR_INVALID, "vx_gen_tangle: null pointer argument");
    if (t->nwaves < 1 || t->table_size < 1 || t->table_size > 46340u)
        return vx_fail(h, VX_ERR_INVALID, "vx_gen_tangle: nwaves %d, table_size %u out of range", t->nwaves,
                       t->table_size);
    const int64_t rows = (int64_t)d.ny * d.nz;
    if (rows > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_gen_tangle: too many rows");
    if (vx_status st = vx_bind(h)) return st;
    hipStream_t st = (hipStream_t)s;
    if (t->table_size <= (uint32_t)GEN_LDS_TABLE)
        hipLaunchKernelGGL(gen_tangle_k<true>, dim3((unsigned)rows), dim3(GEN_THREADS), 0, st, d.nx, d.ny, d.nz,
                           t->nwaves, t->table_size, t->d_ax, t->d_ay, t->d_az, (const double2 *)t->d_coef,
                           (const double2 *)t->d_table, (float2 *)d_psi);
    else
        hipLaunchKernelGGL(gen_tangle_k<false>, dim3((unsigned)rows), dim3(GEN_THREADS), 0, st, d.nx, d.ny, d.nz,
                           t->nwaves, t->table_size, t->d_ax, t->d_ay, t->d_az, (const double2 *)t->d_coef,
                           (const double2 *)t->d_table, (float2 *)d_psi);
    return vx_hip_check(h, hipGetLastError(), "gen_tangle_k launch");
}

extern "C" vx_status vx_gen_line_ring(vx_handle *h, vx_dims d, const vx_line_ring *p, const float *d_noise,
                                      void *d_psi, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, d)) return st;
    if (!p || !d_psi) return vx_fail(h, VX_ERR_INVALID, "vx_gen_line_ring: null pointer argument");
    if (!(p->xi > 0.0)) return vx_fail(h, VX_ERR_INVALID, "vx_gen_line_ring: xi must be positive");
    if (vx_status st = vx_bind(h)) return st;
    const int64_t total = (int64_t)d.nx * d.ny * d.nz;
    const int64_t blocks = std::min<int64_t>((total + GEN_THREADS - 1) / GEN_THREADS, 65536);
    hipLaunchKernelGGL(gen_line_ring_k, dim3((unsigned)blocks), dim3(GEN_THREADS), 0, (hipStream_t)s, d.nx, d.ny,
                       d.nz, *p, (const float2 *)d_noise, (float2 *)d_psi);
    return vx_hip_check(h, hipGetLastError(), "gen_line_ring_k launch");
}
