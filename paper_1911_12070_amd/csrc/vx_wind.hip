// Winding + compaction: phase winding of every grid face (Sec. 2.2 circulation, as an exact winding
// number), the packed per-node field, and the lists of pierced faces and cells (Sec. 3.1 vortex-node
// graph in dual form), in one pass over psi.
//
// Layout of the work
//   * A wavefront owns a column tile: 256 consecutive x-nodes (4 per lane, two 16-byte loads) by TY
//     rows, and marches along z over a chunk of planes. Each psi value is loaded once per chunk plus
//     one halo row (y), one halo plane (z, at the chunk start) and one halo node per row (x, a
//     uniform scalar load); the halos of neighbouring tiles are read back from L2.
//   * The x-neighbour of a lane's last node is the next lane's first node (cross-lane shuffle).
//   * All windings of plane k, the cell flags and the packed byte are formed from planes k and k+1;
//     the in-plane edge values of k+1 are kept for the next step.
//   * Pierced faces and cells are appended per wavefront: ballot + mbcnt give each lane its slot in
//     a wavefront-private LDS buffer; a full buffer is flushed with one global atomic per list.
//   * Workgroups (4 wavefronts stacked in y) are renumbered so that each XCD receives a contiguous
//     range of tiles, keeping the y/z halo re-reads inside one XCD's L2.
#include "vx_internal.h"

namespace {

constexpr int WAVES = 4;         // wavefronts per workgroup (stacked in y)
constexpr int NPL = 4;           // nodes per lane (x)
constexpr int XT = 64 * NPL;     // x-extent of a tile
constexpr int LBUF = 256;        // LDS list entries per wavefront and list

struct WindArgs {
    const float *psi;
    uint8_t *wind;
    uint64_t *faces;
    int8_t *fsign;
    int64_t fcap;
    uint64_t *cells;
    uint16_t *cdesc;
    int64_t ccap;
    int64_t *counts;
    int nx, ny, nz;
    int px, py, pz;
    int ntx, nty, ntz, zc;
};

// Contribution of the directed edge a->b to the winding about q = (-delta, +eps): +1 if it crosses
// Im = 0 upwards with cross(a,b) >= 0, -1 if downwards with cross(a,b) <= 0, else 0. When Re a and
// Re b have the same sign the answer follows from the signs alone; otherwise the 2x2 determinant is
// formed from the FP32 values in FP64, where both products are exact, so its sign is exact.
__device__ __forceinline__ int edge_c(float2 a, float2 b) {
    const bool pa = a.y > 0.0f, pb = b.y > 0.0f;
    const bool na = a.x < 0.0f, nb = b.x < 0.0f;
    bool cnt = !na && !nb;
    if ((pa != pb) && (na != nb)) {
        const double d = fma((double)a.x, (double)b.y, -((double)a.y * (double)b.x));
        cnt = pb ? (d >= 0.0) : (d <= 0.0);
    }
    const int s = (int)pb - (int)pa;
    return cnt ? s : 0;
}

__device__ __forceinline__ uint32_t enc2(int w) { return (uint32_t)w & 3u; }

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd * per + min(xcd, rem) + slot;
}

__device__ __forceinline__ float2 shfl_down1(float2 v) {
    return make_float2(__shfl_down(v.x, 1), __shfl_down(v.y, 1));
}

template <int TY>
struct Raw {
    float4 a[TY + 1], b[TY + 1];
    float2 h[TY + 1];
};

template <int TY>
__global__ __launch_bounds__(64 * WAVES) void wind_compact_k(WindArgs A) {
    __shared__ uint64_t s_fbuf[WAVES][LBUF];
    __shared__ uint64_t s_cbuf[WAVES][LBUF];

    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % A.ntx;
    const int t2 = tile / A.ntx;
    const int ty = t2 % A.nty;
    const int tz = t2 / A.nty;
    const int nx = A.nx, ny = A.ny, nz = A.nz;

    const int j0 = (ty * WAVES + wave) * TY;
    if (j0 >= ny) return;  // no barrier follows: idle wavefronts may leave
    const int xw = tx * XT;
    const int z0 = tz * A.zc;
    const int z1 = min(z0 + A.zc, nz);

    const int nvalid = min(XT, nx - xw);
    const int l_last = nvalid / NPL - 1;
    const bool lane_ok = lane <= l_last;
    const int xl = lane_ok ? xw + NPL * lane : xw;
    const int x_end = xw + nvalid;
    const int hx = x_end < nx ? x_end : (A.px ? 0 : nx - 1);
    // x-step of a lane's last node (the only node whose +x neighbour can fall off the grid)
    const bool xok3 = A.px || (xl + NPL < nx);

    int yload[TY + 1];
    bool row_ok[TY], yok[TY + 1];
#pragma unroll
    for (int r = 0; r <= TY; ++r) {
        const int y = j0 + r;
        yload[r] = y < ny ? y : (A.py ? y % ny : ny - 1);
        yok[r] = A.py || (y + 1 < ny);
        if (r < TY) row_ok[r] = y < ny;
    }

    const float4 *psi4 = reinterpret_cast<const float4 *>(A.psi);
    const float2 *psi2 = reinterpret_cast<const float2 *>(A.psi);

    auto issue = [&](int k, Raw<TY> &raw) {
        const int zz = k < nz ? k : (A.pz ? k % nz : nz - 1);
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            const int64_t base = ((int64_t)zz * ny + yload[r]) * nx;
            const int64_t q = (base + xl) >> 1;
            raw.a[r] = psi4[q];
            raw.b[r] = psi4[q + 1];
            raw.h[r] = psi2[base + hx];
        }
    };
    auto finish = [&](const Raw<TY> &raw, float2 (&v)[TY + 1][NPL + 1]) {
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
            v[r][0] = make_float2(raw.a[r].x, raw.a[r].y);
            v[r][1] = make_float2(raw.a[r].z, raw.a[r].w);
            v[r][2] = make_float2(raw.b[r].x, raw.b[r].y);
            v[r][3] = make_float2(raw.b[r].z, raw.b[r].w);
            const float2 nb = shfl_down1(v[r][0]);
            v[r][4] = lane == l_last ? raw.h[r] : nb;
        }
    };

    float2 P0[TY + 1][NPL + 1], P1[TY + 1][NPL + 1];
    int cx0[TY + 1][NPL], cy0[TY][NPL + 1], wz0[TY][NPL];

    Raw<TY> raw;
    issue(z0, raw);
    finish(raw, P0);
    issue(z0 + 1, raw);
#pragma unroll
    for (int r = 0; r <= TY; ++r)
#pragma unroll
        for (int s = 0; s < NPL; ++s) cx0[r][s] = edge_c(P0[r][s], P0[r][s + 1]);
#pragma unroll
    for (int r = 0; r < TY; ++r)
#pragma unroll
        for (int s = 0; s <= NPL; ++s) cy0[r][s] = edge_c(P0[r][s], P0[r + 1][s]);
#pragma unroll
    for (int r = 0; r < TY; ++r)
#pragma unroll
        for (int s = 0; s < NPL; ++s) {
            const bool ex = (s < NPL - 1 || xok3) && yok[r];
            wz0[r][s] = ex ? cx0[r][s] + cy0[r][s + 1] - cx0[r + 1][s] - cy0[r][s] : 0;
        }

    int fcnt = 0, ccnt = 0;
    uint64_t *fbuf = s_fbuf[wave];
    uint64_t *cbuf = s_cbuf[wave];

    auto flush_faces = [&]() {
        if (fcnt == 0) return;
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(&A.counts[0]),
                                        (unsigned long long)fcnt);
        base = __shfl(base, 0);
        for (int i = lane; i < fcnt; i += 64) {
            const uint64_t e = fbuf[i];
            const int64_t idx = (int64_t)base + i;
            if (idx < A.fcap) {
                A.faces[idx] = e >> 1;
                A.fsign[idx] = (e & 1) ? (int8_t)-1 : (int8_t)1;
            }
        }
        __builtin_amdgcn_wave_barrier();
        fcnt = 0;
    };
    auto flush_cells = [&]() {
        if (ccnt == 0) return;
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0) base = atomicAdd(reinterpret_cast<unsigned long long *>(&A.counts[1]),
                                        (unsigned long long)ccnt);
        base = __shfl(base, 0);
        for (int i = lane; i < ccnt; i += 64) {
            const uint64_t e = cbuf[i];
            const int64_t idx = (int64_t)base + i;
            if (idx < A.ccap) {
                A.cells[idx] = e >> 12;
                A.cdesc[idx] = (uint16_t)(e & 0xfffu);
            }
        }
        __builtin_amdgcn_wave_barrier();
        ccnt = 0;
    };
    auto append = [&](bool pred, uint64_t entry, uint64_t *buf, int &cnt, bool faces) {
        const uint64_t m = __ballot(pred);
        if (m == 0) return;
        const int c = __popcll(m);
        if (cnt + c > LBUF) {
            if (faces) flush_faces(); else flush_cells();
        }
        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (pred) buf[pos] = entry;
        cnt += c;
    };

    for (int k = z0; k < z1; ++k) {
        finish(raw, P1);
        if (k + 1 < z1) issue(k + 2, raw);
        const bool zok = A.pz || (k + 1 < nz);

        int cx1[TY + 1][NPL], cy1[TY][NPL + 1], cz[TY + 1][NPL + 1];
#pragma unroll
        for (int r = 0; r <= TY; ++r)
#pragma unroll
            for (int s = 0; s < NPL; ++s) cx1[r][s] = edge_c(P1[r][s], P1[r][s + 1]);
#pragma unroll
        for (int r = 0; r < TY; ++r)
#pragma unroll
            for (int s = 0; s <= NPL; ++s) cy1[r][s] = edge_c(P1[r][s], P1[r + 1][s]);
#pragma unroll
        for (int r = 0; r <= TY; ++r)
#pragma unroll
            for (int s = 0; s <= NPL; ++s) cz[r][s] = edge_c(P0[r][s], P1[r][s]);

        int wz1[TY][NPL], wx[TY][NPL + 1], wy[TY + 1][NPL];
#pragma unroll
        for (int r = 0; r < TY; ++r)
#pragma unroll
            for (int s = 0; s < NPL; ++s) {
                const bool ex = (s < NPL - 1 || xok3) && yok[r];
                wz1[r][s] = ex ? cx1[r][s] + cy1[r][s + 1] - cx1[r + 1][s] - cy1[r][s] : 0;
            }
#pragma unroll
        for (int r = 0; r < TY; ++r)
#pragma unroll
            for (int s = 0; s <= NPL; ++s) {
                const bool ex = yok[r] && zok;
                wx[r][s] = ex ? cy0[r][s] + cz[r + 1][s] - cy1[r][s] - cz[r][s] : 0;
            }
#pragma unroll
        for (int r = 0; r <= TY; ++r)
#pragma unroll
            for (int s = 0; s < NPL; ++s) {
                const bool ex = zok && (s < NPL - 1 || xok3);
                wy[r][s] = ex ? cz[r][s] + cx1[r][s] - cz[r][s + 1] - cx0[r][s] : 0;
            }

        // packed bytes and the cell flags of plane k
        uint32_t word[TY];
        bool any = false;
#pragma unroll
        for (int r = 0; r < TY; ++r) {
            uint32_t wd = 0;
#pragma unroll
            for (int s = 0; s < NPL; ++s) {
                const bool cell_ok = (s < NPL - 1 || xok3) && yok[r] && zok;
                const int orv = wx[r][s] | wx[r][s + 1] | wy[r][s] | wy[r + 1][s] | wz0[r][s] | wz1[r][s];
                const uint32_t pierced = (cell_ok && orv != 0) ? 1u : 0u;
                const uint32_t byte = enc2(wx[r][s]) | (enc2(wy[r][s]) << 2) | (enc2(wz0[r][s]) << 4) |
                                      (pierced << 6);
                wd |= byte << (8 * s);
            }
            const bool ok = lane_ok && row_ok[r];
            word[r] = ok ? wd : 0u;
            any |= word[r] != 0u;
            if (A.wind && ok) {
                const int64_t n0 = (int64_t)xl + (int64_t)nx * (j0 + r + (int64_t)ny * k);
                __builtin_nontemporal_store(wd, reinterpret_cast<uint32_t *>(A.wind + n0));
            }
        }

        if (__ballot(any) != 0) {
#pragma unroll
            for (int r = 0; r < TY; ++r) {
                if (__ballot(word[r] != 0u) == 0) continue;
#pragma unroll
                for (int s = 0; s < NPL; ++s) {
                    const uint32_t byte = (word[r] >> (8 * s)) & 0xffu;
                    if (__ballot(byte != 0u) == 0) continue;
                    const int64_t n = (int64_t)xl + s + (int64_t)nx * (j0 + r + (int64_t)ny * k);
                    append((byte & 0x03u) != 0, (uint64_t)(3 * n) << 1 | (uint64_t)((byte >> 1) & 1u), fbuf,
                           fcnt, true);
                    append((byte & 0x0cu) != 0, (uint64_t)(3 * n + 1) << 1 | (uint64_t)((byte >> 3) & 1u),
                           fbuf, fcnt, true);
                    append((byte & 0x30u) != 0, (uint64_t)(3 * n + 2) << 1 | (uint64_t)((byte >> 5) & 1u),
                           fbuf, fcnt, true);
                    const uint32_t desc = enc2(wx[r][s]) | (enc2(wx[r][s + 1]) << 2) | (enc2(wy[r][s]) << 4) |
                                          (enc2(wy[r + 1][s]) << 6) | (enc2(wz0[r][s]) << 8) |
                                          (enc2(wz1[r][s]) << 10);
                    append((byte & 0x40u) != 0, (uint64_t)n << 12 | desc, cbuf, ccnt, false);
                }
            }
        }

        // advance: plane k+1 becomes plane k
#pragma unroll
        for (int r = 0; r <= TY; ++r) {
#pragma unroll
            for (int s = 0; s <= NPL; ++s) P0[r][s] = P1[r][s];
#pragma unroll
            for (int s = 0; s < NPL; ++s) cx0[r][s] = cx1[r][s];
        }
#pragma unroll
        for (int r = 0; r < TY; ++r) {
#pragma unroll
            for (int s = 0; s <= NPL; ++s) cy0[r][s] = cy1[r][s];
#pragma unroll
            for (int s = 0; s < NPL; ++s) wz0[r][s] = wz1[r][s];
        }
    }
    flush_faces();
    flush_cells();
}

__global__ void zero_counts_k(int64_t *c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

template <int TY>
vx_status launch_ty(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o, hipStream_t s,
                    int zc) {
    WindArgs A;
    A.psi = (const float *)psi;
    A.wind = o.d_wind;
    A.faces = o.d_faces;
    A.fsign = o.d_face_sign;
    A.fcap = o.face_cap;
    A.cells = o.d_cells;
    A.cdesc = o.d_cell_desc;
    A.ccap = o.cell_cap;
    A.counts = o.d_counts;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    A.px = (int)(d.periodic & 1u);
    A.py = (int)((d.periodic >> 1) & 1u);
    A.pz = (int)((d.periodic >> 2) & 1u);
    A.zc = zc;
    A.ntx = (d.nx + XT - 1) / XT;
    A.nty = (d.ny + WAVES * TY - 1) / (WAVES * TY);
    A.ntz = (d.nz + zc - 1) / zc;
    const int64_t nblocks = (int64_t)A.ntx * A.nty * A.ntz;
    if (nblocks > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_winding: too many tiles");
    hipLaunchKernelGGL(zero_counts_k, dim3(1), dim3(64), 0, s, o.d_counts);
    vx_timer tm(h, s, VX_KIND_WIND);
    hipLaunchKernelGGL(wind_compact_k<TY>, dim3((unsigned)nblocks), dim3(64 * WAVES), 0, s, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "wind_compact_k launch");
}

}  // namespace

vx_status vx_wind_launch(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o,
                         hipStream_t s) {
    if (d.nx % NPL != 0)
        return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_winding: nx = %d must be a multiple of %d", d.nx, NPL);
    const int ty = h->wind_ty > 0 ? h->wind_ty : 1;
    int zc = h->wind_zc;
    if (zc <= 0) {
        // z-chunk: enough workgroups to fill the chip several times over
        const int64_t cols = (int64_t)((d.nx + XT - 1) / XT) * ((d.ny + WAVES * ty - 1) / (WAVES * ty));
        const int64_t want = 8LL * (h->num_cu > 0 ? h->num_cu : 256);
        zc = d.nz;
        while (zc > 16 && cols * ((d.nz + zc - 1) / zc) < want) zc = (zc + 1) / 2;
    }
    switch (ty) {
        case 1: return launch_ty<1>(h, d, psi, o, s, zc);
        case 2: return launch_ty<2>(h, d, psi, o, s, zc);
        case 4: return launch_ty<4>(h, d, psi, o, s, zc);
        default: return vx_fail(h, VX_ERR_INVALID, "vx_winding: rows per wavefront %d not built (1, 2, 4)", ty);
    }
}
