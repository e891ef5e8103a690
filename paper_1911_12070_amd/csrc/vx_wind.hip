// Winding + compaction: phase winding of every grid face (Sec. 2.2 circulation, as an exact winding
// number), the packed per-node field, and the lists of pierced faces and cells (Sec. 3.1 vortex-node
// graph in dual form), in one pass over psi.
//
// Bit-sliced formulation
//   A wavefront owns a tile of 64 x-columns (one per lane) by 32 rows and marches along z over a
//   chunk of planes. For each plane a lane packs, for its column, one bit per row into 32-bit words:
//   "Im psi > 0" and "Re psi < 0". Everything after that is bitwise logic on words, 32 nodes at a time:
//     * an edge a->b crosses Im = 0 where the Im bits differ (upwards if b's bit is set);
//     * if Re a and Re b are both >= 0 the crossing counts (+1 up, -1 down); if both are < 0 it does
//       not; only when Re also changes sign is the determinant Re a Im b - Im a Re b needed, and it is
//       formed from the FP32 values in FP64 (both products exact), for those few edges only;
//     * the winding of a face is the sum of four edge terms in {-1,0,1}; with |w| <= 1 it is nonzero
//       iff an odd number of terms are nonzero, and +1 iff some term is +1 and fewer than two are -1;
//     * neighbours: x+1 is the next lane (cross-lane move of a whole word), y+1 is the next bit,
//       z+1 is the next plane of the march.
//   Lane 63 and row 31 are halo: a tile outputs 63 columns x 31 rows, so every neighbour an output
//   needs lies inside the tile; neighbouring tiles overlap by one column and one row (re-read from
//   L2). The first plane of a chunk is the z halo of the previous chunk.
//   Pierced faces and cells are appended per wavefront into LDS (ballot + mbcnt) and flushed with one
//   global atomic per list when the buffer fills. Workgroups are renumbered so that each XCD gets a
//   contiguous range of tiles, keeping halo re-reads inside one XCD's L2.
#include "vx_internal.h"

namespace {

constexpr int TXO = 63;   // output columns per tile (64 loaded)
constexpr int TYO = 31;   // output rows per tile (32 loaded)
constexpr int LBUF = 512; // LDS list entries per wavefront and list

struct WindArgs {
    const float2 *psi;
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

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd * per + min(xcd, rem) + slot;
}

// word of lane+1 (lane 63 receives 0; it is a halo lane whose neighbour is never used)
__device__ __forceinline__ uint32_t next_lane(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}

struct WT {  // a ternary value per bit: +1 where p is set, -1 where n is set
    uint32_t p, n;
};

// t1 + t2 - t3 - t4 for four terms in {-1,0,1} whose sum is known to lie in {-1,0,1}
__device__ __forceinline__ WT sum4(WT t1, WT t2, WT t3, WT t4) {
    const uint32_t P1 = t1.p, N1 = t1.n, P2 = t2.p, N2 = t2.n;
    const uint32_t P3 = t3.n, N3 = t3.p, P4 = t4.n, N4 = t4.p;  // negated terms
    const uint32_t nz = (P1 | N1) ^ (P2 | N2) ^ (P3 | N3) ^ (P4 | N4);
    const uint32_t pany = P1 | P2 | P3 | P4;
    const uint32_t n2 = (N1 & N2) | (N3 & N4) | ((N1 | N2) & (N3 | N4));
    const uint32_t wp = nz & pany & ~n2;
    return WT{wp, nz & ~wp};
}

__device__ __forceinline__ WT shr1(WT a) { return WT{a.p >> 1, a.n >> 1}; }
__device__ __forceinline__ WT lane_next(WT a) { return WT{next_lane(a.p), next_lane(a.n)}; }
__device__ __forceinline__ WT mask(WT a, uint32_t m) { return WT{a.p & m, a.n & m}; }

// edge values from the sign words of the two end points; `ex` holds, for edges where both Re and Im
// change sign, whether the exact determinant test says the crossing counts
__device__ __forceinline__ WT edges(uint32_t pia, uint32_t pib, uint32_t nra, uint32_t nrb, uint32_t ex) {
    const uint32_t up = ~pia & pib, dn = pia & ~pib;
    const uint32_t cnt = ~(nra | nrb) | ((nra ^ nrb) & ex);
    return WT{up & cnt, dn & cnt};
}

__device__ __forceinline__ uint32_t needs_exact(uint32_t pia, uint32_t pib, uint32_t nra, uint32_t nrb) {
    return (pia ^ pib) & (nra ^ nrb);
}

// exact count decision of the edge a->b (called only when Im and Re both change sign along it)
__device__ __forceinline__ bool exact_count(float2 a, float2 b) {
    const double d = fma((double)a.x, (double)b.y, -((double)a.y * (double)b.x));
    return b.y > 0.0f ? (d >= 0.0) : (d <= 0.0);
}

__global__ __launch_bounds__(64) void wind_bits_k(WindArgs A) {
    __shared__ uint64_t s_fbuf[LBUF];
    __shared__ uint64_t s_cbuf[LBUF];

    const int lane = threadIdx.x;
    const int tile = xcd_tile(blockIdx.x, gridDim.x);
    const int tx = tile % A.ntx;
    const int t2 = tile / A.ntx;
    const int ty = t2 % A.nty;
    const int tz = t2 / A.nty;
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int x0 = tx * TXO, y0 = ty * TYO, z0 = tz * A.zc;
    const int z1 = min(z0 + A.zc, nz);

    // this lane's column and its +x neighbour's column (load indices, wrapped or clamped)
    const int xg = x0 + lane;
    const int xc = xg < nx ? xg : (A.px ? xg % nx : nx - 1);
    const int xg1 = xg + 1;
    const int xc1 = xg1 < nx ? xg1 : (A.px ? xg1 % nx : nx - 1);
    const bool lane_out = lane < TXO && xg < nx;
    const bool xstep = A.px || (xg + 1 < nx);

    // row words: valid output rows and rows whose +y step exists
    uint32_t rvalid = 0, ystep = 0;
    for (int r = 0; r < 32; ++r) {
        const int y = y0 + r;
        if (r < TYO && y < ny) rvalid |= 1u << r;
        if (A.py || y + 1 < ny) ystep |= 1u << r;
    }
    const bool wrap_rows = y0 + 32 > ny;
    auto row_of = [&](int r) -> int {
        const int y = y0 + r;
        return y < ny ? y : (A.py ? y % ny : ny - 1);
    };
    auto plane_of = [&](int k) -> int { return k < nz ? k : (A.pz ? k % nz : nz - 1); };

    const float2 *psi = A.psi;
    float2 raw[32];
    auto issue = [&](int k) {
        const int64_t pbase = (int64_t)plane_of(k) * ny;
        if (!wrap_rows) {
            const float2 *p = psi + (pbase + y0) * nx + xc;
#pragma unroll
            for (int r = 0; r < 32; ++r) raw[r] = p[(int64_t)r * nx];
        } else {
#pragma unroll
            for (int r = 0; r < 32; ++r) raw[r] = psi[(pbase + row_of(r)) * nx + xc];
        }
    };
    auto sign_words = [&](uint32_t &pi, uint32_t &nr) {
        uint32_t a = 0, b = 0;
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            a |= raw[r].y > 0.0f ? (1u << r) : 0u;
            b |= raw[r].x < 0.0f ? (1u << r) : 0u;
        }
        pi = a;
        nr = b;
    };
    auto node_ptr = [&](int col, int r, int k) -> const float2 * {
        return psi + ((int64_t)plane_of(k) * ny + row_of(r)) * nx + col;
    };

    // Resolve the pending exact edges of the in-plane (x, y) edges of plane k and, if qz is given,
    // of the z edges k -> k+1. Returns the count-decision words.
    auto resolve = [&](uint32_t qx, uint32_t qy, uint32_t qz, int k, uint32_t &ex, uint32_t &ey, uint32_t &ez) {
        ex = ey = ez = 0;
        while (__ballot((qx | qy | qz) != 0u) != 0) {
            if ((qx | qy | qz) != 0u) {
                int dir, r;
                if (qx) {
                    dir = 0;
                    r = __builtin_ctz(qx);
                } else if (qy) {
                    dir = 1;
                    r = __builtin_ctz(qy);
                } else {
                    dir = 2;
                    r = __builtin_ctz(qz);
                }
                const float2 a = *node_ptr(xc, r, dir == 2 ? k - 1 : k);
                const float2 b = dir == 0 ? *node_ptr(xc1, r, k) : (dir == 1 ? *node_ptr(xc, r + 1, k) : *node_ptr(xc, r, k));
                const uint32_t bit = 1u << r;
                const uint32_t c = exact_count(a, b) ? bit : 0u;
                if (dir == 0) {
                    ex |= c;
                    qx &= ~bit;
                } else if (dir == 1) {
                    ey |= c;
                    qy &= ~bit;
                } else {
                    ez |= c;
                    qz &= ~bit;
                }
            }
        }
    };

    // ---- LDS list buffers -----------------------------------------------------------------------
    int fcnt = 0, ccnt = 0;
    auto flush = [&](bool faces) {
        int &cnt = faces ? fcnt : ccnt;
        if (cnt == 0) return;
        __builtin_amdgcn_wave_barrier();
        unsigned long long base = 0;
        if (lane == 0)
            base = atomicAdd(reinterpret_cast<unsigned long long *>(&A.counts[faces ? 0 : 1]), (unsigned long long)cnt);
        base = __shfl(base, 0);
        for (int i = lane; i < cnt; i += 64) {
            const int64_t idx = (int64_t)base + i;
            if (faces) {
                const uint64_t e = s_fbuf[i];
                if (idx < A.fcap) {
                    A.faces[idx] = e >> 1;
                    A.fsign[idx] = (e & 1) ? (int8_t)-1 : (int8_t)1;
                }
            } else {
                const uint64_t e = s_cbuf[i];
                if (idx < A.ccap) {
                    A.cells[idx] = e >> 12;
                    A.cdesc[idx] = (uint16_t)(e & 0xfffu);
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        cnt = 0;
    };
    auto append = [&](bool pred, uint64_t entry, bool faces) {
        const uint64_t m = __ballot(pred);
        if (m == 0) return;
        const int c = __popcll(m);
        if ((faces ? fcnt : ccnt) + c > LBUF) flush(faces);
        int &cnt = faces ? fcnt : ccnt;
        const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (pred) (faces ? s_fbuf : s_cbuf)[pos] = entry;
        cnt += c;
    };

    // ---- prologue: plane z0 ----------------------------------------------------------------------
    uint32_t pi0, nr0;
    issue(z0);
    sign_words(pi0, nr0);
    issue(z0 + 1);
    WT cx0, cy0, wz0;
    {
        const uint32_t pin = next_lane(pi0), nrn = next_lane(nr0);
        const uint32_t piy = pi0 >> 1, nry = nr0 >> 1;
        uint32_t ex, ey, ez;
        resolve(lane < 63 ? needs_exact(pi0, pin, nr0, nrn) : 0u, needs_exact(pi0, piy, nr0, nry) & 0x7fffffffu, 0u, z0,
                ex, ey, ez);
        cx0 = edges(pi0, pin, nr0, nrn, ex);
        cy0 = edges(pi0, piy, nr0, nry, ey);
        wz0 = mask(sum4(cx0, lane_next(cy0), shr1(cx0), cy0), xstep ? ystep : 0u);
    }

    const uint64_t plane_nodes = (uint64_t)nx * (uint64_t)ny;
    for (int k = z0; k < z1; ++k) {
        uint32_t pi1, nr1;
        sign_words(pi1, nr1);
        if (k + 1 < z1) issue(k + 2);
        const bool zstep = A.pz || (k + 1 < nz);

        const uint32_t pin = next_lane(pi1), nrn = next_lane(nr1);
        const uint32_t piy = pi1 >> 1, nry = nr1 >> 1;
        uint32_t ex, ey, ez;
        resolve(lane < 63 ? needs_exact(pi1, pin, nr1, nrn) : 0u, needs_exact(pi1, piy, nr1, nry) & 0x7fffffffu,
                needs_exact(pi0, pi1, nr0, nr1), k + 1, ex, ey, ez);
        const WT cx1 = edges(pi1, pin, nr1, nrn, ex);
        const WT cy1 = edges(pi1, piy, nr1, nry, ey);
        const WT cz = edges(pi0, pi1, nr0, nr1, ez);

        // faces of plane k+1 (w_z) and plane k (w_x, w_y)
        const WT wz1 = mask(sum4(cx1, lane_next(cy1), shr1(cx1), cy1), xstep ? ystep : 0u);
        const WT wx = mask(sum4(cy0, shr1(cz), cy1, cz), zstep ? ystep : 0u);
        const WT wy = mask(sum4(cz, cx1, lane_next(cz), cx0), (zstep && xstep) ? 0xffffffffu : 0u);

        const WT wxn = lane_next(wx);
        const uint32_t nzx = wx.p | wx.n, nzy = wy.p | wy.n, nz0 = wz0.p | wz0.n, nz1 = wz1.p | wz1.n;
        const uint32_t outm = lane_out ? rvalid : 0u;
        const uint32_t cellm = (xstep && zstep) ? (ystep & outm) : 0u;
        const uint32_t pc = (nzx | wxn.p | wxn.n | nzy | (nzy >> 1) | nz0 | nz1) & cellm;

        // packed bytes: bit0 w_x != 0, bit1 w_x < 0, bit2/3 w_y, bit4/5 w_z, bit6 pierced cell
        if (A.wind && lane_out) {
            const uint32_t wrd[7] = {nzx, wx.n, nzy, wy.n, nz0, wz0.n, pc};
            uint8_t *wbase = A.wind + (uint64_t)k * plane_nodes + (uint64_t)xg;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                uint32_t d = 0;
#pragma unroll
                for (int b = 0; b < 7; ++b) {
                    const uint32_t nib = (wrd[b] >> (4 * g)) & 0xfu;
                    d |= (__umul24(nib, 0x204081u) & 0x01010101u) << b;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int r = 4 * g + i;
                    if (r < TYO && ((rvalid >> r) & 1u))
                        __builtin_nontemporal_store((uint8_t)(d >> (8 * i)), wbase + (uint64_t)row_of(r) * nx);
                }
            }
        }

        // pierced faces and cells of plane k
        uint32_t fx = nzx & outm, fy = nzy & outm, fz = nz0 & outm, fc = pc;
        if (__ballot((fx | fy | fz | fc) != 0u) != 0) {
            const WT wyu = shr1(wy);
            while (__ballot((fx | fy | fz | fc) != 0u) != 0) {
                bool hf = (fx | fy | fz) != 0u;
                uint64_t fe = 0;
                if (hf) {
                    int a, r;
                    uint32_t neg;
                    if (fx) {
                        a = 0;
                        r = __builtin_ctz(fx);
                        fx &= fx - 1;
                        neg = wx.n;
                    } else if (fy) {
                        a = 1;
                        r = __builtin_ctz(fy);
                        fy &= fy - 1;
                        neg = wy.n;
                    } else {
                        a = 2;
                        r = __builtin_ctz(fz);
                        fz &= fz - 1;
                        neg = wz0.n;
                    }
                    const uint64_t n = (uint64_t)k * plane_nodes + (uint64_t)(y0 + r) * nx + (uint64_t)xg;
                    fe = ((3 * n + a) << 1) | ((neg >> r) & 1u);
                }
                append(hf, fe, true);
                const bool hc = fc != 0u;
                uint64_t ce = 0;
                if (hc) {
                    const int r = __builtin_ctz(fc);
                    fc &= fc - 1;
                    auto e2 = [&](const WT &w) -> uint32_t {
                        return ((w.p >> r) & 1u) | (((w.n >> r) & 1u) ? 3u : 0u);
                    };
                    const uint32_t desc = e2(wx) | (e2(wxn) << 2) | (e2(wy) << 4) | (e2(wyu) << 6) | (e2(wz0) << 8) |
                                          (e2(wz1) << 10);
                    const uint64_t n = (uint64_t)k * plane_nodes + (uint64_t)(y0 + r) * nx + (uint64_t)xg;
                    ce = (n << 12) | desc;
                }
                append(hc, ce, false);
            }
        }

        pi0 = pi1;
        nr0 = nr1;
        cx0 = cx1;
        cy0 = cy1;
        wz0 = wz1;
    }
    flush(true);
    flush(false);
}

__global__ void zero_counts_k(int64_t *c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

}  // namespace

vx_status vx_wind_launch(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o,
                         hipStream_t s) {
    WindArgs A;
    A.psi = (const float2 *)psi;
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
    A.ntx = (d.nx + TXO - 1) / TXO;
    A.nty = (d.ny + TYO - 1) / TYO;
    int zc = h->wind_zc;
    if (zc <= 0) {
        // planes per chunk: enough tiles to keep every CU busy several times over
        const int64_t cols = (int64_t)A.ntx * A.nty;
        const int64_t want = 16LL * (h->num_cu > 0 ? h->num_cu : 256);
        zc = d.nz;
        while (zc > 32 && cols * ((d.nz + zc - 1) / zc) < want) zc = (zc + 1) / 2;
    }
    A.zc = zc;
    A.ntz = (d.nz + zc - 1) / zc;
    const int64_t nblocks = (int64_t)A.ntx * A.nty * A.ntz;
    if (nblocks > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_winding: too many tiles");
    hipLaunchKernelGGL(zero_counts_k, dim3(1), dim3(64), 0, s, o.d_counts);
    vx_timer tm(h, s, VX_KIND_WIND);
    hipLaunchKernelGGL(wind_bits_k, dim3((unsigned)nblocks), dim3(64), 0, s, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "wind_bits_k launch");
}
