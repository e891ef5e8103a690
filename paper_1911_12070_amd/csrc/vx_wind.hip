// Winding + compaction: phase winding of every grid face (Sec. 2.2 circulation, as an exact winding
// number), the packed per-node field, and the lists of pierced faces and cells (Sec. 3.1 vortex-node
// graph in dual form), in one pass over psi.
//
// Bit-sliced formulation
//   A wavefront owns a tile of 16 rows by 128 x-columns and marches along z over a chunk of planes.
//   Lane (r, c) = (lane / 4, lane % 4) holds row r, columns 32c .. 32c+31 of the tile. For each plane
//   a lane packs, for its 32 nodes, one bit per node into 32-bit words: "Im psi > 0" and
//   "Re psi < 0". Everything after that is bitwise logic on words, 32 nodes at a time:
//     * an edge a->b crosses Im = 0 where the Im bits differ (upwards if b's bit is set);
//     * if Re a and Re b are both >= 0 the crossing counts (+1 up, -1 down); if both are < 0 it does
//       not; only when Re also changes sign is the determinant Re a Im b - Im a Re b needed, and it is
//       formed from the FP32 values in FP64 (both products exact), for those few edges only;
//     * the winding of a face is the sum of four edge terms in {-1,0,1}; with |w| <= 1 it is nonzero
//       iff an odd number of terms are nonzero, and +1 iff some term is +1 and fewer than two are -1;
//     * neighbours: x+1 is the next bit (the word's last bit takes bit 0 of the next lane of the quad),
//       y+1 is four lanes on, z+1 is the next plane of the march.
//   Row 15 (lanes 60-63) is halo: a tile outputs 15 rows; neighbouring tiles overlap by one row.
//   Column 128 is halo too: the quad's last lane keeps it as one extra bit and forms only the
//   quantities the tile's last column needs from it. The first plane of a chunk is the z halo of the
//   previous chunk.
//
// Memory
//   psi for the next plane is requested a whole march step ahead with direct global->LDS loads:
//   each instruction fetches one full 1 KiB row of the tile. Inside LDS each row's 16-byte pieces are
//   rotated per row and chunk so that the per-lane reads that follow spread over all banks. Exact
//   determinants read their operands from LDS (or, for the previous plane, from L2). The packed byte
//   field of a tile row is one whole 128-byte line written by the row's four lanes, so the writes
//   reach memory as full lines. Pierced faces and cells are appended per wavefront into LDS
//   (ballot + mbcnt) and flushed with one global atomic per list when the buffer fills. Workgroups
//   are renumbered so that each XCD gets a contiguous range of tiles, keeping halo re-reads inside
//   one XCD's L2.
#include "vx_internal.h"

namespace {

constexpr int TXO = 128;   // output columns per tile (plus one halo column)
constexpr int TYO = 15;    // output rows per tile (16 loaded)
constexpr int LBUF = 256;  // LDS list entries per list
constexpr int PLANE_LDS = 16 * 1024;  // bytes of one plane tile in LDS (halo column follows)

using WindArgs = vx_wind_args;

__device__ __forceinline__ int xcd_tile(int b, int nb) {
    const int per = nb / 8, rem = nb % 8;
    const int xcd = b % 8, slot = b / 8;
    return xcd * per + min(xcd, rem) + slot;
}

// Cross-lane moves read other lanes' registers, which only works while those lanes are active. The
// empty volatile asm pins each move where it is written (outside any divergent branch), so the
// compiler cannot sink it into a branch whose exec mask would hide the source lane.
__device__ __forceinline__ uint32_t pin(uint32_t v) {
    asm volatile("" : "+v"(v));
    return v;
}
// word of the next row (lane + 4); the halo row's lanes get their own word, which is never used
__device__ __forceinline__ uint32_t next_lane(uint32_t v) { return pin((uint32_t)__shfl_down((int)v, 4)); }
// word of the next lane of the quad (lane + 1 within each group of four; the last keeps its own)
__device__ __forceinline__ uint32_t quad_next(uint32_t v) {
    return pin((uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xF9 /* quad_perm:[1,2,3,3] */, 0xf, 0xf, false));
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

__device__ __forceinline__ WT lane_next(WT a) { return WT{next_lane(a.p), next_lane(a.n)}; }
__device__ __forceinline__ WT mask(WT a, uint32_t m) { return WT{a.p & m, a.n & m}; }
// word of column+1: shift down one column; bit 31 takes bit 0 of the quad's next lane, or, in the
// quad's last lane (m4 all ones), the halo column's bit h
__device__ __forceinline__ uint32_t colnext(uint32_t w, uint32_t h, uint32_t m4) {
    const uint32_t nb = (quad_next(w) & ~m4) | (h & m4);
    return (w >> 1) | (nb << 31);
}
__device__ __forceinline__ WT colnext(WT w, WT h, uint32_t m4) {
    return WT{colnext(w.p, h.p, m4), colnext(w.n, h.n, m4)};
}

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

// exact count decision of the edge a->b (used only when Im and Re both change sign along it)
__device__ __forceinline__ bool exact_count(float2 a, float2 b) {
    const double d = fma((double)a.x, (double)b.y, -((double)a.y * (double)b.x));
    return b.y > 0.0f ? (d >= 0.0) : (d <= 0.0);
}

// LDS byte offset of the 16-byte piece q (columns 2q, 2q+1) of tile row r: inside the row's 1 KiB,
// chunk q/16 keeps its 16 pieces rotated by r + 4 (q/16), so lanes that read piece i of their own
// (row, chunk) at the same time spread over all banks.
__device__ __forceinline__ uint32_t piece_off(int r, int q) {
    const int cc = q >> 4;
    return (uint32_t)(r * 1024 + (cc * 16 + ((q + r + 4 * cc) & 15)) * 16);
}

// 4x4 byte transpose: t[j] = byte j of w0, w1, w2, w3 (in bytes 0..3), eight v_perm_b32
__device__ __forceinline__ void byte_transpose4(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3, uint32_t t[4]) {
    const uint32_t a0 = __builtin_amdgcn_perm(w1, w0, 0x06020400u), a1 = __builtin_amdgcn_perm(w1, w0, 0x07030501u);
    const uint32_t a2 = __builtin_amdgcn_perm(w3, w2, 0x06020400u), a3 = __builtin_amdgcn_perm(w3, w2, 0x07030501u);
    t[0] = __builtin_amdgcn_perm(a2, a0, 0x05040100u);
    t[1] = __builtin_amdgcn_perm(a3, a1, 0x05040100u);
    t[2] = __builtin_amdgcn_perm(a2, a0, 0x07060302u);
    t[3] = __builtin_amdgcn_perm(a3, a1, 0x07060302u);
}

// transpose of the 8x8 bit matrix held in (lo, hi) with row r in byte r and column c in bit c of
// that byte: three exchange rounds (bit pairs, 2x2 blocks, 4x4 blocks)
__device__ __forceinline__ void bit_transpose8(uint32_t &lo, uint32_t &hi) {
    uint32_t t0, t1;
    t0 = (lo ^ ((lo >> 7) | (hi << 25))) & 0x00AA00AAu;
    t1 = (hi ^ (hi >> 7)) & 0x00AA00AAu;
    lo ^= t0 ^ (t0 << 7);
    hi ^= t1 ^ ((t1 << 7) | (t0 >> 25));
    t0 = (lo ^ ((lo >> 14) | (hi << 18))) & 0x0000CCCCu;
    t1 = (hi ^ (hi >> 14)) & 0x0000CCCCu;
    lo ^= t0 ^ (t0 << 14);
    hi ^= t1 ^ ((t1 << 14) | (t0 >> 18));
    t0 = (lo ^ (hi << 4)) & 0xF0F0F0F0u;
    lo ^= t0;
    hi ^= t0 >> 4;
}

__device__ __forceinline__ void wait_vm() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
__device__ __forceinline__ void wait_lds() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// One tile (16 rows x 128 columns x one z-chunk) of one grid, run by one wavefront.
__device__ __forceinline__ void wind_tile(const WindArgs &A, int tile) {
    __shared__ __attribute__((aligned(16))) uint8_t s_plane[PLANE_LDS + 512];
    __shared__ uint64_t s_fbuf[LBUF];
    __shared__ uint64_t s_cbuf[LBUF];

    const int lane = threadIdx.x;
    const int tx = tile % A.ntx;
    const int t2 = tile / A.ntx;
    const int ty = t2 % A.nty;
    const int tz = t2 / A.nty;
    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int x0 = tx * TXO, y0 = ty * TYO, z0 = tz * A.zc;
    const int z1 = min(z0 + A.zc, nz);

    // this lane's row and column chunk
    const int r = lane >> 2, c = lane & 3;
    const bool last4 = c == 3;
    // lane masks kept opaque to the compiler (see pin): quad's last lane, rows with a row below
    const uint32_t m4 = pin(last4 ? 0xffffffffu : 0u);
    const uint32_t minner = pin(r < 15 ? 0xffffffffu : 0u);
    const int yg = y0 + r;
    const int yl = yg < ny ? yg : (A.py ? yg % ny : ny - 1);
    const bool row_out = r < TYO && yg < ny;
    const bool ystep = A.py || (yg + 1 < ny);
    // columns of this lane: valid outputs and +x steps; the halo column's load index
    const int xl0 = x0 + 32 * c;
    const int ncol = max(0, min(32, nx - xl0));
    const uint32_t cvalid = ncol >= 32 ? 0xffffffffu : ((1u << ncol) - 1u);
    uint32_t xstep = cvalid;
    if (!A.px && ncol > 0 && xl0 + ncol == nx) xstep &= ~(1u << (ncol - 1));
    const int xh = x0 + TXO < nx ? x0 + TXO : (A.px ? (x0 + TXO) % nx : nx - 1);
    // even rows use 16-byte loads of whole tile rows (in a ragged last column tile, the pieces past
    // the grid's end are the wrapped ones on a periodic axis, any valid one otherwise, as those
    // columns are never used); odd nx loads per node
    const bool xin = x0 + TXO <= nx;
    const bool fast = A.psi_a16 && ((nx & 1) == 0) && (xin || nx >= TXO);
    const bool yin = y0 + 16 <= ny;

    const float2 *psi = A.psi;
    const uint64_t plane_nodes = (uint64_t)nx * (uint64_t)ny;
    auto plane_of = [&](int k) -> int { return k < nz ? k : (A.pz ? k % nz : nz - 1); };
    auto row_of = [&](int r) -> int {
        const int y = y0 + r;
        return y < ny ? y : (A.py ? y % ny : ny - 1);
    };
    auto col_of = [&](int x) -> int { return x < nx ? x : (A.px ? x % nx : nx - 1); };

    // request plane k of the tile into LDS
    auto issue = [&](int k) {
        const float2 *pl = psi + (uint64_t)plane_of(k) * plane_nodes;
        if (fast) {
            const int cc = lane >> 4, xx = lane & 15;
            auto lds_row = [&](int j) { return (void __attribute__((address_space(3))) *)(s_plane + j * 1024); };
            if (xin && yin) {  // rows y0 .. y0+15 of the grid: one pointer stepped by a row (uniform branch)
                // row j: lane L lands at slot L; it fetches the piece whose rotated slot is L
                const float2 *row = pl + (uint64_t)y0 * nx + x0;
#pragma unroll
                for (int j = 0; j < 16; ++j, row += nx) {
                    const int q = 16 * cc + ((xx - j - 4 * cc) & 15);
                    __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(row + 2 * q),
                                                     lds_row(j), 16, 0, 0);
                }
            } else {  // the tile reaches past the last grid row or column: wrapped or clamped rows, and
                      // pieces past the last column wrapped (periodic; nx >= 128, so once) or clamped
                      // (their columns are never used); a loop, so that no row pointer stays live across
                      // the march, and pinned lane coordinates, so that no per-row column does
                const int ccr = (int)pin((uint32_t)cc), xxr = (int)pin((uint32_t)xx);
#pragma unroll 1
                for (int j = 0; j < 16; ++j) {
                    int col = x0 + 2 * (16 * ccr + ((xxr - j - 4 * ccr) & 15));
                    if (col >= nx) col = A.px ? col - nx : nx - 2;
                    __builtin_amdgcn_global_load_lds(
                        (const void __attribute__((address_space(1))) *)(pl + (uint64_t)row_of(j) * nx + col), lds_row(j),
                        16, 0, 0);
                }
            }
        } else {
            const float2 *rowp = pl + (uint64_t)yl * nx;
#pragma unroll 4
            for (int i = 0; i < 16; ++i) {
                const int q = 16 * c + i;
                const float2 a = rowp[col_of(x0 + 2 * q)], b = rowp[col_of(x0 + 2 * q + 1)];
                *reinterpret_cast<float4 *>(s_plane + piece_off(r, q)) = make_float4(a.x, a.y, b.x, b.y);
            }
        }
        // halo column of each row: Re and Im land in two 256-byte arrays (4 bytes per lane each)
        const float *hsrc = reinterpret_cast<const float *>(pl + (uint64_t)yl * nx + xh);
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)hsrc,
                                         (void __attribute__((address_space(3))) *)(s_plane + PLANE_LDS), 4, 0, 0);
        __builtin_amdgcn_global_load_lds((const void __attribute__((address_space(1))) *)(hsrc + 1),
                                         (void __attribute__((address_space(3))) *)(s_plane + PLANE_LDS + 256), 4, 0, 0);
    };
    auto lds_node = [&](int rr, int col) -> float2 {  // tile row, tile column (128 = halo column)
        if (col == TXO)
            return make_float2(*reinterpret_cast<const float *>(s_plane + PLANE_LDS + (4 * rr + 3) * 4),
                               *reinterpret_cast<const float *>(s_plane + PLANE_LDS + 256 + (4 * rr + 3) * 4));
        return *reinterpret_cast<const float2 *>(s_plane + piece_off(rr, col >> 1) + (col & 1) * 8);
    };
    // sign words of this lane's row from the plane in LDS
    auto sign_words = [&](uint32_t &pi, uint32_t &nr, uint32_t &pih, uint32_t &nrh) {
        uint32_t a = 0, b = 0;
        // the 16 read offsets are recomputed per plane rather than kept in registers: at <= 192
        // VGPRs two winding wavefronts per SIMD leave room for a refinement wavefront of another
        // frame to run beside them
        const int rr = (int)pin((uint32_t)r), cq = (int)pin((uint32_t)c);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const float4 v = *reinterpret_cast<const float4 *>(s_plane + piece_off(rr, 16 * cq + i));
            a |= (v.y > 0.0f ? 1u : 0u) << (2 * i);
            a |= (v.w > 0.0f ? 1u : 0u) << (2 * i + 1);
            b |= (v.x < 0.0f ? 1u : 0u) << (2 * i);
            b |= (v.z < 0.0f ? 1u : 0u) << (2 * i + 1);
        }
        const float2 h = make_float2(*reinterpret_cast<const float *>(s_plane + PLANE_LDS + lane * 4),
                                     *reinterpret_cast<const float *>(s_plane + PLANE_LDS + 256 + lane * 4));
        pi = a;
        nr = b;
        pih = h.y > 0.0f ? 1u : 0u;
        nrh = h.x < 0.0f ? 1u : 0u;
    };

    // Exact decisions for the pending edges of the plane in LDS (x: bit b -> b+1, y: row r -> r+1)
    // and of the z edges from plane kprev (read from L2) to the plane in LDS. Bit 0 of hy/hz: the halo
    // column (quad's last lane only).
    auto resolve = [&](uint32_t qx, uint32_t qy, uint32_t qz, uint32_t hy, uint32_t hz, int kprev,
                       uint32_t &ex, uint32_t &ey, uint32_t &ez, uint32_t &ehy, uint32_t &ehz) {
        ex = ey = ez = ehy = ehz = 0;
        const float2 *prev = psi + (uint64_t)plane_of(kprev) * plane_nodes + (uint64_t)yl * nx;
        while (__ballot((qx | qy | qz | hy | hz) != 0u) != 0) {
            if ((qx | qy | qz | hy | hz) != 0u) {
                int dir, b;
                if (qx) {
                    dir = 0;
                    b = __builtin_ctz(qx);
                } else if (qy) {
                    dir = 1;
                    b = __builtin_ctz(qy);
                } else if (qz) {
                    dir = 2;
                    b = __builtin_ctz(qz);
                } else if (hy) {
                    dir = 1;
                    b = 32;
                } else {
                    dir = 2;
                    b = 32;
                }
                const int col = b == 32 ? TXO : 32 * c + b;  // tile column
                float2 a, v;
                if (dir == 0) {
                    a = lds_node(r, col);
                    v = lds_node(r, col + 1);
                } else if (dir == 1) {
                    a = lds_node(r, col);
                    v = lds_node(r + 1, col);
                } else {
                    a = prev[col == TXO ? xh : col_of(x0 + col)];
                    v = lds_node(r, col);
                }
                const bool cnt = exact_count(a, v);
                if (b == 32) {
                    if (dir == 1) {
                        ehy = cnt ? 1u : 0u;
                        hy = 0;
                    } else {
                        ehz = cnt ? 1u : 0u;
                        hz = 0;
                    }
                } else {
                    const uint32_t bit = 1u << b;
                    const uint32_t m = cnt ? bit : 0u;
                    if (dir == 0) {
                        ex |= m;
                        qx &= ~bit;
                    } else if (dir == 1) {
                        ey |= m;
                        qy &= ~bit;
                    } else {
                        ez |= m;
                        qz &= ~bit;
                    }
                }
            }
        }
    };

    // ---- LDS list buffers -----------------------------------------------------------------------
    int fcnt = 0, ccnt = 0;
    auto flush = [&](bool faces) {
        int &cnt = faces ? fcnt : ccnt;
        if (cnt == 0) return;
        wait_lds();
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(reinterpret_cast<unsigned long long *>(&A.counts[faces ? 0 : 1]), (unsigned long long)cnt);
            if ((int64_t)base + cnt > (faces ? A.fcap : A.ccap)) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_WIND);
        }
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
        wait_lds();
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

    // ---- deferred packed-byte stores ----------------------------------------------------------------
    uint32_t pend[8];
    int pend_k = -1;
    auto store_pending = [&]() {
        if (pend_k < 0 || !row_out || ncol == 0) return;
        uint8_t *dst = A.wind + (uint64_t)pend_k * plane_nodes + (uint64_t)yg * nx + xl0;
        if (ncol == 32 && (nx & 15) == 0 && A.wind_a16) {
            // streaming stores: the field is not read again by this kernel
            typedef unsigned int u4v __attribute__((ext_vector_type(4)));
            __builtin_nontemporal_store((u4v){pend[0], pend[1], pend[2], pend[3]}, reinterpret_cast<u4v *>(dst));
            __builtin_nontemporal_store((u4v){pend[4], pend[5], pend[6], pend[7]}, reinterpret_cast<u4v *>(dst) + 1);
        } else if (ncol == 32 && (nx & 3) == 0 && A.wind_a4) {
#pragma unroll
            for (int g = 0; g < 8; ++g) reinterpret_cast<uint32_t *>(dst)[g] = pend[g];
        } else {
            for (int cc = 0; cc < ncol; ++cc) dst[cc] = (uint8_t)(pend[cc >> 2] >> (8 * (cc & 3)));
        }
    };

    // ---- prologue: plane z0 ----------------------------------------------------------------------
    uint32_t pi0, nr0, pih0, nrh0;
    WT cx0, cy0, cy0h, wz0;
    issue(z0);
    wait_vm();
    sign_words(pi0, nr0, pih0, nrh0);
    {
        const uint32_t pix = colnext(pi0, pih0, m4), nrx = colnext(nr0, nrh0, m4);
        const uint32_t piy = next_lane(pi0), nry = next_lane(nr0);
        const uint32_t pihy = next_lane(pih0), nrhy = next_lane(nrh0);
        uint32_t ex, ey, ez, ehy, ehz;
        resolve(needs_exact(pi0, pix, nr0, nrx), needs_exact(pi0, piy, nr0, nry) & minner, 0u,
                needs_exact(pih0, pihy, nrh0, nrhy) & minner & m4 & 1u, 0u, z0, ex, ey, ez, ehy, ehz);
        cx0 = edges(pi0, pix, nr0, nrx, ex);
        cy0 = edges(pi0, piy, nr0, nry, ey);
        cy0h = mask(edges(pih0, pihy, nrh0, nrhy, ehy), 1u);
        wz0 = mask(sum4(cx0, colnext(cy0, cy0h, m4), lane_next(cx0), cy0), ystep ? xstep : 0u);
    }
    wait_lds();
    issue(z0 + 1);

    for (int k = z0; k < z1; ++k) {
        const bool zstep = A.pz || (k + 1 < nz);
        wait_vm();
        uint32_t pi1, nr1, pih1, nrh1;
        sign_words(pi1, nr1, pih1, nrh1);

        const uint32_t pix = colnext(pi1, pih1, m4), nrx = colnext(nr1, nrh1, m4);
        const uint32_t piy = next_lane(pi1), nry = next_lane(nr1);
        const uint32_t pihy = next_lane(pih1), nrhy = next_lane(nrh1);
        uint32_t ex, ey, ez, ehy, ehz;
        resolve(needs_exact(pi1, pix, nr1, nrx), needs_exact(pi1, piy, nr1, nry) & minner,
                needs_exact(pi0, pi1, nr0, nr1), needs_exact(pih1, pihy, nrh1, nrhy) & minner & m4 & 1u,
                needs_exact(pih0, pih1, nrh0, nrh1) & m4 & 1u, k, ex, ey, ez, ehy, ehz);
        // previous plane's packed bytes, then (every LDS read of plane k+1 being done) request plane
        // k+2 into the same buffer
        store_pending();
        wait_lds();
        if (k + 1 < z1) issue(k + 2);

        const WT cx1 = edges(pi1, pix, nr1, nrx, ex);
        const WT cy1 = edges(pi1, piy, nr1, nry, ey);
        const WT cz = edges(pi0, pi1, nr0, nr1, ez);
        const WT cy1h = mask(edges(pih1, pihy, nrh1, nrhy, ehy), 1u);
        const WT czh = mask(edges(pih0, pih1, nrh0, nrh1, ehz), 1u);

        // faces of plane k+1 (w_z) and plane k (w_x, w_y); halo column's w_x for the last cell
        const WT wz1 = mask(sum4(cx1, colnext(cy1, cy1h, m4), lane_next(cx1), cy1), ystep ? xstep : 0u);
        const uint32_t yzm = (ystep && zstep) ? 0xffffffffu : 0u;
        const WT wx = mask(sum4(cy0, lane_next(cz), cy1, cz), yzm);
        const WT wxh = mask(sum4(cy0h, lane_next(czh), cy1h, czh), yzm & 1u);
        const WT wy = mask(sum4(cz, cx1, colnext(cz, czh, m4), cx0), zstep ? xstep : 0u);

        const WT wxr = colnext(wx, wxh, m4);  // w_x at x+1
        const WT wyu = lane_next(wy);     // w_y at y+1
        const uint32_t nzx = wx.p | wx.n, nzy = wy.p | wy.n, nz0 = wz0.p | wz0.n, nz1 = wz1.p | wz1.n;
        const uint32_t outm = row_out ? cvalid : 0u;
        const uint32_t cellm = (ystep && zstep) ? (xstep & outm) : 0u;
        const uint32_t pc = (nzx | wxr.p | wxr.n | nzy | wyu.p | wyu.n | nz0 | nz1) & cellm;

        // packed bytes of this row: bit0 w_x != 0, bit1 w_x < 0, bit2/3 w_y, bit4/5 w_z, bit6 cell.
        // They are written at the start of the next step, before that step's prefetch, so that the
        // wait for the prefetch never waits on these stores.
        // (bit b of node i's byte is bit i of word b: per 8 nodes an 8x8 bit transpose)
        if (A.wind) {
            uint32_t lo[4], hi[4];
            byte_transpose4(nzx, wx.n, nzy, wy.n, lo);
            byte_transpose4(nz0, wz0.n, pc, 0u, hi);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                bit_transpose8(lo[j], hi[j]);
                pend[2 * j] = lo[j];
                pend[2 * j + 1] = hi[j];
            }
            pend_k = k;
        }

        // pierced faces and cells of plane k
        uint32_t fx = nzx & outm, fy = nzy & outm, fz = nz0 & outm, fc = pc;
        if (__ballot((fx | fy | fz | fc) != 0u) != 0) {
            const uint64_t rowbase = (uint64_t)k * plane_nodes + (uint64_t)yg * nx + (uint64_t)xl0;
            while (__ballot((fx | fy | fz | fc) != 0u) != 0) {
                const bool hf = (fx | fy | fz) != 0u;
                uint64_t fe = 0;
                if (hf) {
                    int a, c;
                    uint32_t neg;
                    if (fx) {
                        a = 0;
                        c = __builtin_ctz(fx);
                        fx &= fx - 1;
                        neg = wx.n;
                    } else if (fy) {
                        a = 1;
                        c = __builtin_ctz(fy);
                        fy &= fy - 1;
                        neg = wy.n;
                    } else {
                        a = 2;
                        c = __builtin_ctz(fz);
                        fz &= fz - 1;
                        neg = wz0.n;
                    }
                    const uint64_t n = rowbase + (uint64_t)c;
                    fe = ((3 * n + a) << 1) | ((neg >> c) & 1u);
                }
                append(hf, fe, true);
                const bool hc = fc != 0u;
                uint64_t ce = 0;
                if (hc) {
                    const int c = __builtin_ctz(fc);
                    fc &= fc - 1;
                    auto e2 = [&](const WT &w) -> uint32_t {
                        return ((w.p >> c) & 1u) | (((w.n >> c) & 1u) ? 3u : 0u);
                    };
                    const uint32_t desc = e2(wx) | (e2(wxr) << 2) | (e2(wy) << 4) | (e2(wyu) << 6) | (e2(wz0) << 8) |
                                          (e2(wz1) << 10);
                    ce = ((rowbase + (uint64_t)c) << 12) | desc;
                }
                append(hc, ce, false);
            }
        }

        pi0 = pi1;
        nr0 = nr1;
        pih0 = pih1;
        nrh0 = nrh1;
        cx0 = cx1;
        cy0 = cy1;
        cy0h = cy1h;
        wz0 = wz1;
    }
    store_pending();
    flush(true);
    flush(false);
}

__global__ __launch_bounds__(64) void wind_bits_k(WindArgs A) { wind_tile(A, xcd_tile(blockIdx.x, gridDim.x)); }

// Several grids in one launch: the tiles of frame f are numbers tile_start[f] .. tile_start[f+1]-1
// of one combined range (renumbered per XCD as for a single grid); each workgroup finds its frame by
// binary search and reads that frame's arguments from the device table.
__global__ __launch_bounds__(64) void wind_batch_k(const WindArgs *__restrict__ frames,
                                                   const int *__restrict__ tile_start, int nframes) {
    const int t = xcd_tile(blockIdx.x, gridDim.x);
    int lo = 0, hi = nframes;  // invariant: tile_start[lo] <= t < tile_start[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (tile_start[mid] <= t) lo = mid;
        else hi = mid;
    }
    const WindArgs A = frames[lo];
    wind_tile(A, t - tile_start[lo]);
}

__global__ void zero_counts_k(int64_t *c) {
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

// zero the two counts of every frame of a batch
__global__ void zero_batch_counts_k(const WindArgs *__restrict__ frames, int nframes) {
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < nframes) {
        frames[f].counts[0] = 0;
        frames[f].counts[1] = 0;
    }
}

}  // namespace

int vx_wind_zc_for(vx_handle *h, const vx_dims &d) {
    if (h->wind_zc > 0) return h->wind_zc;
    const auto it = h->tuned_zc.find({d.nx, d.ny, d.nz, (int)d.periodic});
    if (it != h->tuned_zc.end()) return it->second;
    // planes per chunk: enough tiles to keep every CU busy several times over
    const int64_t cols = (int64_t)((d.nx + TXO - 1) / TXO) * ((d.ny + TYO - 1) / TYO);
    const int64_t want = 128LL * (h->num_cu > 0 ? h->num_cu : 256);
    int zc = d.nz;
    while (zc > 16 && cols * ((d.nz + zc - 1) / zc) < want) zc = (zc + 1) / 2;
    return zc;
}

vx_status vx_wind_make_args(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o, int zc,
                            vx_wind_args *out, int64_t *ntiles) {
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
    A.flag = vx_overflow_flag(h);
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    A.px = (int)(d.periodic & 1u);
    A.py = (int)((d.periodic >> 1) & 1u);
    A.pz = (int)((d.periodic >> 2) & 1u);
    A.ntx = (d.nx + TXO - 1) / TXO;
    A.nty = (d.ny + TYO - 1) / TYO;
    A.psi_a16 = ((uintptr_t)psi & 15u) == 0;
    A.wind_a16 = ((uintptr_t)o.d_wind & 15u) == 0;
    A.wind_a4 = ((uintptr_t)o.d_wind & 3u) == 0;
    if (zc <= 0) zc = vx_wind_zc_for(h, d);
    A.zc = zc;
    A.ntz = (d.nz + zc - 1) / zc;
    const int64_t nblocks = (int64_t)A.ntx * A.nty * A.ntz;
    if (nblocks > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "winding: too many tiles");
    *out = A;
    *ntiles = nblocks;
    return VX_OK;
}

// Resident workgroups per CU of the single-grid winding kernel. LDS alone would allow 7; capping
// them at 6 (unused dynamic LDS on each workgroup) keeps more of the halo rows and columns that
// neighbouring tiles share in L2 (1.4% faster at 1024^3), and the LDS left over still takes one
// refinement workgroup beside them, which the frame pipeline relies on. The batch kernel, whose
// small frames have fewer tiles to spread, keeps 7.
constexpr int WIND_WG_PER_CU = 6;

int wind_lds_pad(vx_handle *h) {
    if (h->wind_lds_pad < 0) {
        h->wind_lds_pad = 0;
        hipFuncAttributes fa;
        if (h->lds_per_cu > 0 && hipFuncGetAttributes(&fa, (const void *)wind_bits_k) == hipSuccess) {
            // per-workgroup LDS just above 1/(N+1) of the CU's: N fit, N+1 do not
            const int target = h->lds_per_cu / (WIND_WG_PER_CU + 1) + 512;
            h->wind_lds_pad = std::max(0, target - (int)fa.sharedSizeBytes);
        }
    }
    return h->wind_lds_pad;
}

vx_status vx_wind_enqueue(vx_handle *h, const vx_wind_args &A, int64_t ntiles, hipStream_t s) {
    hipLaunchKernelGGL(zero_counts_k, dim3(1), dim3(64), 0, s, A.counts);
    vx_timer tm(h, s, VX_KIND_WIND);
    const int pad = wind_lds_pad(h);
    if (ntiles > 0) hipLaunchKernelGGL(wind_bits_k, dim3((unsigned)ntiles), dim3(64), pad, s, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "wind_bits_k launch");
}

vx_status vx_wind_launch(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o,
                         hipStream_t s) {
    WindArgs A;
    int64_t nblocks = 0;
    if (vx_status st = vx_wind_make_args(h, d, psi, o, 0, &A, &nblocks)) return st;
    return vx_wind_enqueue(h, A, nblocks, s);
}

int vx_wind_batch_max_wg(vx_handle *h) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, wind_batch_k, 64, 0) != hipSuccess || nb < 1) return -1;
    return nb;
}

int vx_wind_batch_pad(vx_handle *h, int wg_per_cu) {
    hipFuncAttributes fa;
    if (wg_per_cu <= 0 || h->lds_per_cu <= 0 || hipFuncGetAttributes(&fa, (const void *)wind_batch_k) != hipSuccess)
        return 0;
    // per-workgroup LDS just above 1/(N+1) of the CU's: N fit, N+1 do not (no pad where LDS allows only N)
    return std::max(0, h->lds_per_cu / (wg_per_cu + 1) + 512 - (int)fa.sharedSizeBytes);
}

vx_status vx_wind_batch_enqueue(vx_handle *h, const vx_wind_args *d_frames, const int *d_tile_start, int nframes,
                                int64_t total_tiles, int lds_pad, hipStream_t s) {
    if (total_tiles > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "winding batch: too many tiles");
    hipLaunchKernelGGL(zero_batch_counts_k, dim3((nframes + 63) / 64), dim3(64), 0, s, d_frames, nframes);
    if (total_tiles > 0)
        hipLaunchKernelGGL(wind_batch_k, dim3((unsigned)total_tiles), dim3(64), lds_pad, s, d_frames, d_tile_start,
                           nframes);
    return vx_hip_check(h, hipGetLastError(), "wind_batch_k launch");
}
