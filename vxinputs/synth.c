/*
 * Seeded synthetic wavefunction fields: host-side evaluation.
 *
 * This module only builds inputs. It holds none of the vortex-identification or refinement
 * arithmetic; it is shared by the tests, the benchmark and the smoke check so that the CPU
 * oracle and the GPU library see the same complex64 bytes.
 *
 * Random-wave tangle: psi(x) = sum_k c_k * T[m_k(x)], with
 *   m_k(x) = (ax_k*x + ay_k*y + az_k*z) mod M,  T[m] = exp(2*pi*i*m/M)  (FP64 table),
 * accumulated in FP64 in wave order, one rounding per operation (no contraction), then rounded
 * to FP32. The integer phase index is exact, so any implementation that performs the same FP64
 * operations in the same order reproduces these bytes exactly.
 *
 * Line + ring field: product of two ideal vortex factors (d / sqrt(d^2 + 2 xi^2) core profile)
 * plus caller-supplied noise.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -shared -fPIC (no -ffast-math).
 */
#include <math.h>
#include <stdint.h>

static inline int64_t wrapi(int64_t v, int64_t n) {
    int64_t r = v % n;
    return r < 0 ? r + n : r;
}

void vxs_tangle(int nx, int ny, int nz, int bx0, int by0, int bz0, int bnx, int bny, int bnz,
                int nw, const uint32_t *ax, const uint32_t *ay, const uint32_t *az,
                const double *coef, uint32_t M, const double *table, float *out) {
    int64_t total = (int64_t)bnx * bny * bnz;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < total; ++q) {
        int64_t dx = q % bnx, dy = (q / bnx) % bny, dz = q / ((int64_t)bnx * bny);
        uint64_t x = (uint64_t)wrapi(bx0 + dx, nx);
        uint64_t y = (uint64_t)wrapi(by0 + dy, ny);
        uint64_t z = (uint64_t)wrapi(bz0 + dz, nz);
        double re = 0.0, im = 0.0;
        for (int k = 0; k < nw; ++k) {
            uint64_t m = ((uint64_t)ay[k] * y + (uint64_t)az[k] * z) % M;
            m = (m + (uint64_t)ax[k] * x) % M;
            double tr = table[2 * m], ti = table[2 * m + 1];
            double cr = coef[2 * k], ci = coef[2 * k + 1];
            double p1 = cr * tr;
            double p2 = ci * ti;
            double d = p1 - p2;
            re = re + d;
            double q1 = cr * ti;
            double q2 = ci * tr;
            double s = q1 + q2;
            im = im + s;
        }
        out[2 * q] = (float)re;
        out[2 * q + 1] = (float)im;
    }
}

static inline double minimg(double d, double n) { return d - n * nearbyint(d / n); }

/* prm: [line_x, line_y, ring_cx, ring_cy, ring_cz, ring_radius, xi] */
void vxs_line_ring(int nx, int ny, int nz, const double *prm, const float *noise, float *out) {
    double lx = prm[0], ly = prm[1], cx = prm[2], cy = prm[3], cz = prm[4], R = prm[5], xi = prm[6];
    double two_xi2 = 2.0 * xi * xi;
    int64_t total = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < total; ++q) {
        double x = (double)(q % nx), y = (double)((q / nx) % ny), z = (double)(q / ((int64_t)nx * ny));
        double dx = minimg(x - lx, nx), dy = minimg(y - ly, ny);
        double sl = sqrt(dx * dx + dy * dy + two_xi2);
        double lr = dx / sl, li = dy / sl;
        double rx = minimg(x - cx, nx), ry = minimg(y - cy, ny), rz = minimg(z - cz, nz);
        double u = sqrt(rx * rx + ry * ry) - R, v = rz;
        double sr = sqrt(u * u + v * v + two_xi2);
        double rr = u / sr, ri = v / sr;
        double pr = lr * rr - li * ri;
        double pi = lr * ri + li * rr;
        if (noise) {
            pr += (double)noise[2 * q];
            pi += (double)noise[2 * q + 1];
        }
        out[2 * q] = (float)pr;
        out[2 * q + 1] = (float)pi;
    }
}
