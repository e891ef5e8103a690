// Node-centred circulation (Sec. 2.2): the circulation of the phase around a small ring in each of the
// three coordinate planes through a grid node, the largest of the three in magnitude, and the vortex
// nodes where it exceeds pi -- derived here from the exact face windings of the packed field.
//
// The ring of node n in the plane normal to axis a is the boundary of the 2 x 2 faces around n in that
// plane (corners n +- e_u +- e_v). Windings add over faces: the circulation / 2 pi around the ring is
// the sum of the windings of those four faces (shared inner edges cancel), e.g. for a = z
//   C_z(n) / 2 pi = w_z(n) + w_z(n - ex) + w_z(n - ey) + w_z(n - ex - ey),
// and likewise C_x from w_x(n), w_x(n - ey), w_x(n - ez), w_x(n - ey - ez) and C_y from w_y(n),
// w_y(n - ez), w_y(n - ex), w_y(n - ez - ex). Faces that would need nodes outside a non-periodic axis
// do not exist (winding 0).
//
// Work layout. A wavefront owns 256 consecutive nodes of one x-row (4 per lane, one 32-bit word of
// the packed field) and marches along z over a chunk of planes, keeping the previous plane's words
// in registers; x - 1 is the previous lane's word shifted by one byte. The four windings of a plane
// sum are added as biased 2-bit fields, four nodes per word (w + 1 in {0, 1, 2}, the sum of four in
// 0..8 fits a byte), and the three sums of a node index a 729-entry table in LDS that gives the
// output byte. Vortex nodes are appended per wavefront into LDS (ballot + mbcnt) and flushed with one
// atomic per 256 entries.
#include "vx_internal.h"

namespace {

constexpr int NODE_ZC = 64;   // planes per wavefront
constexpr int NBUF = 256;     // LDS list entries per wavefront
constexpr int LUT = 9 * 9 * 9;

struct NodeArgs {
    const uint8_t *wind;
    uint8_t *node;          // nullable
    uint64_t *list;         // nullable if cap == 0
    int64_t cap;
    int64_t *count;
    unsigned long long *flag;
    int nx, ny, nz;
    int px, py, pz;
    int aligned;            // nx % 4 == 0 and both fields 4-byte aligned: rows are whole words
};

// Output byte of a node from its three biased ring sums (each 0..8, 4 = zero circulation):
// bits 1:0 |C| / 2 pi of the plane with the largest |C| (ties: lowest axis), bit 2 its sign
// (1 = negative), bits 4:3 that plane's normal axis, bit 6 = vortex node (|C| > pi). 0 if all zero.
__device__ uint8_t node_byte(int sx, int sy, int sz) {
    const int s[3] = {sx - 4, sy - 4, sz - 4};
    int best = 0;
    for (int a = 1; a < 3; ++a)
        if (abs(s[a]) > abs(s[best])) best = a;
    const int v = s[best], mag = min(abs(v), 3);
    if (mag == 0) return 0;
    return (uint8_t)(mag | (v < 0 ? 4 : 0) | (best << 3) | 0x40);
}
// the table of node_circ_k: index Sx + 9 Sy + 81 Sz
__device__ uint8_t lut_entry(int e) { return node_byte(e % 9, (e / 9) % 9, e / 81); }

// The same byte for the wide kernel's index Sx | Sz << 4 | Sy << 8 (index values with a sum above 8
// never occur; their entries are 0)
constexpr int LUTW = 9 << 8;
__device__ uint8_t lutw_entry(int e) {
    const int sx = e & 15, sz = (e >> 4) & 15, sy = e >> 8;
    if (sx > 8 || sz > 8 || sy > 8) return 0;
    return node_byte(sx, sy, sz);
}

// biased windings w + 1 of field a (bits 2a+1:2a of each byte) of four packed bytes
__device__ __forceinline__ uint32_t biased(uint32_t w, int a) {
    return (((w >> (2 * a)) & 0x03030303u) + 0x01010101u) & 0x03030303u;
}

__global__ __launch_bounds__(64) void node_circ_k(NodeArgs A) {
    __shared__ uint8_t s_lut[LUT];
    __shared__ uint64_t s_buf[NBUF];
    const int lane = threadIdx.x;
    for (int e = lane; e < LUT; e += 64) s_lut[e] = lut_entry(e);
    __syncthreads();

    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int xw = blockIdx.x * 256;  // first node of the wavefront's row segment
    const int i0 = xw + 4 * lane;     // first of this lane's four nodes
    const int j = blockIdx.y;
    const int z0 = blockIdx.z * NODE_ZC, z1 = min(z0 + NODE_ZC, nz);
    const int jm = j > 0 ? j - 1 : (A.py ? ny - 1 : -1);   // row j - 1 (-1: absent)
    const int im = xw > 0 ? xw - 1 : (A.px ? nx - 1 : -1);  // node x - 1 of the segment's first node

    auto byte_at = [&](int jj, int kk, int ii) -> uint32_t {
        return A.wind[(uint64_t)ii + (uint64_t)nx * ((uint64_t)jj + (uint64_t)ny * (uint64_t)kk)];
    };
    // this lane's four bytes of row (jj, kk); zero for absent rows and past the row's end
    auto load4 = [&](int jj, int kk) -> uint32_t {
        if (jj < 0 || kk < 0 || i0 >= nx) return 0u;
        const uint64_t base = (uint64_t)nx * ((uint64_t)jj + (uint64_t)ny * (uint64_t)kk);
        if (A.aligned && i0 + 3 < nx) return *(const uint32_t *)(A.wind + base + i0);
        uint32_t w = 0;
        for (int b = 0; b < 4 && i0 + b < nx; ++b) w |= (uint32_t)A.wind[base + i0 + b] << (8 * b);
        return w;
    };
    // the bytes of nodes x - 1: the previous lane's last byte; lane 0 reads node im. The empty asm
    // keeps the cross-lane move where it is written, with every lane active (moved into the branch
    // below it would read lane 0 while lane 0 is inactive)
    auto xshift = [&](uint32_t w, int jj, int kk) -> uint32_t {
        uint32_t prev = (uint32_t)__shfl_up((int)w, 1);
        asm volatile("" : "+v"(prev));
        if (lane == 0) prev = (im >= 0 && jj >= 0 && kk >= 0) ? byte_at(jj, kk, im) << 24 : 0u;
        return (w << 8) | (prev >> 24);
    };

    int cnt = 0;
    auto flush = [&]() {
        if (cnt == 0) return;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(reinterpret_cast<unsigned long long *>(A.count), (unsigned long long)cnt);
            if ((int64_t)base + cnt > A.cap) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_WIND);
        }
        base = ((unsigned long long)(uint32_t)__shfl((int)(base >> 32), 0) << 32) | (uint32_t)__shfl((int)base, 0);
        for (int q = lane; q < cnt; q += 64) {
            const int64_t idx = (int64_t)base + q;
            if (idx < A.cap) A.list[idx] = s_buf[q];
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        cnt = 0;
    };

    const int kp = z0 > 0 ? z0 - 1 : (A.pz ? nz - 1 : -1);  // the plane before the chunk (-1: absent)
    uint32_t Wp = load4(j, kp), Wpm = load4(jm, kp);
    uint32_t Wpx = xshift(Wp, j, kp);
    for (int k = z0; k < z1; ++k) {
        const uint32_t W = load4(j, k), Wm = load4(jm, k);
        const uint32_t Wx = xshift(W, j, k), Wmx = xshift(Wm, jm, k);
        const uint32_t Sx = biased(W, 0) + biased(Wm, 0) + biased(Wp, 0) + biased(Wpm, 0);
        const uint32_t Sy = biased(W, 1) + biased(Wp, 1) + biased(Wx, 1) + biased(Wpx, 1);
        const uint32_t Sz = biased(W, 2) + biased(Wx, 2) + biased(Wm, 2) + biased(Wmx, 2);
        uint32_t o = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const uint32_t e = ((Sx >> (8 * b)) & 0xffu) + 9u * ((Sy >> (8 * b)) & 0xffu) + 81u * ((Sz >> (8 * b)) & 0xffu);
            o |= (uint32_t)s_lut[e] << (8 * b);
        }
        if (i0 + 4 > nx) o = i0 >= nx ? 0u : o & ((1u << (8 * (nx - i0))) - 1u);  // nodes past the row's end
        const uint64_t rowbase = (uint64_t)nx * ((uint64_t)j + (uint64_t)ny * (uint64_t)k);
        if (A.node && i0 < nx) {
            if (A.aligned && i0 + 3 < nx) {
                *(uint32_t *)(A.node + rowbase + i0) = o;
            } else {
                for (int b = 0; b < 4 && i0 + b < nx; ++b) A.node[rowbase + i0 + b] = (uint8_t)(o >> (8 * b));
            }
        }
        // vortex nodes of this plane (bit 6 of each byte)
        if (__ballot((o & 0x40404040u) != 0) != 0) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                const bool pred = ((o >> (8 * b)) & 0x40u) != 0;
                const uint64_t m = __ballot(pred);
                if (m == 0) continue;
                const int c = __popcll(m);
                if (cnt + c > NBUF) flush();
                const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                if (pred) s_buf[pos] = rowbase + (uint64_t)(i0 + b);
                __builtin_amdgcn_wave_barrier();
                cnt += c;
            }
        }
        Wp = W;
        Wpm = Wm;
        Wpx = Wx;
    }
    flush();
}

// Wide rows: rows whose length is a multiple of 16 nodes and 16-byte aligned fields. A wavefront owns
// WROWS consecutive rows of a 1024-node segment (16 nodes per lane, one 16-byte word per row) plus the
// row below them, and marches along z. Per row and plane it forms B (the biased x and z fields,
// bits 0-1 and 4-5 of each byte, in one mask-add-mask) and Y (the biased y field); the ring sums then
// reuse pair sums across rows and planes:
//   T = B(row) + B(row - 1):  Sx = T + T(previous plane) (low nibbles), Sz = T + T(x - 1) (high nibbles)
//   U = Y + Y(previous plane): Sy = U + U(x - 1).
// The neighbour x - 1 of a lane's first node is the previous lane's last byte; lane 0 reads the
// segment's neighbour bytes itself and keeps their y fields for the next plane. The three sums of a
// node (each 0..8) index the table as Sx | Sz << 4 | Sy << 8: one bit-field insert keeps Sx's low
// nibbles and Sz's high ones (no sum carries out of its nibble), and one byte permute per pair of
// nodes places the y sums above them in 16-bit halves.
// Vortex nodes are counted per lane, placed by a wavefront prefix sum into LDS and flushed as in
// node_circ_k. The results are node_circ_k's bit for bit.
constexpr int WROWS = 4;  // output rows per wavefront

__device__ __forceinline__ uint32_t bxz(uint32_t w) {  // biased x and z fields (w + 1 per 2-bit field)
    return ((w & 0x33333333u) + 0x11111111u) & 0x33333333u;
}
__device__ __forceinline__ uint32_t byf(uint32_t w) {  // biased y field
    return (((w >> 2) & 0x03030303u) + 0x01010101u) & 0x03030303u;
}
// per-node values of nodes x - 1: byte i of word t -> byte i + 1; `in` holds the value of the node
// before the lane's first in its top byte
__device__ __forceinline__ void xshift4(const uint32_t v[4], uint32_t in, uint32_t o[4]) {
    o[0] = __builtin_amdgcn_alignbyte(v[0], in, 3);
    o[1] = __builtin_amdgcn_alignbyte(v[1], v[0], 3);
    o[2] = __builtin_amdgcn_alignbyte(v[2], v[1], 3);
    o[3] = __builtin_amdgcn_alignbyte(v[3], v[2], 3);
}
// the previous lane's v (all lanes active; the empty asm keeps the move outside any branch)
__device__ __forceinline__ uint32_t from_prev_lane(uint32_t v) {
    uint32_t p = (uint32_t)__shfl_up((int)v, 1);
    asm volatile("" : "+v"(p));
    return p;
}

__global__ __launch_bounds__(64) void node_circ_wide_k(NodeArgs A) {
    __shared__ uint8_t s_lut[LUTW];
    __shared__ uint64_t s_buf[NBUF];
    const int lane = threadIdx.x;
    for (int e = lane; e < LUTW; e += 64) s_lut[e] = lutw_entry(e);
    __syncthreads();

    const int nx = A.nx, ny = A.ny, nz = A.nz;
    const int xw = blockIdx.x * 1024;  // first node of the wavefront's segment
    const int i0 = xw + 16 * lane;     // first of this lane's 16 nodes
    const bool active = i0 < nx;       // nx is a multiple of 16: a lane is wholly inside or outside
    const int j0 = blockIdx.y * WROWS;
    const int z0 = blockIdx.z * NODE_ZC, z1 = min(z0 + NODE_ZC, nz);
    const int im = xw > 0 ? xw - 1 : (A.px ? nx - 1 : -1);  // node x - 1 of the segment's first node

    // grid row of wavefront row q (q = 0: the row below j0; q >= 1: j0 + q - 1); -1 if absent
    int rows[WROWS + 1];
#pragma unroll
    for (int q = 0; q <= WROWS; ++q) {
        const int j = j0 + q - 1;
        rows[q] = j < 0 ? (A.py ? ny - 1 : -1) : (j < ny ? j : -1);
    }
    auto rowbase = [&](int j, int k) -> uint64_t {
        return (uint64_t)nx * ((uint64_t)j + (uint64_t)ny * (uint64_t)k);
    };
    auto load_row = [&](int j, int k, uint32_t w[4]) {
        w[0] = w[1] = w[2] = w[3] = 0u;
        if (j < 0 || k < 0 || !active) return;
        const uint4 v = *(const uint4 *)(A.wind + rowbase(j, k) + i0);
        w[0] = v.x;
        w[1] = v.y;
        w[2] = v.z;
        w[3] = v.w;
    };
    auto edge_byte = [&](int j, int k) -> uint32_t {  // node im of row j (lane 0's neighbour)
        return (lane == 0 && im >= 0 && j >= 0 && k >= 0) ? (uint32_t)A.wind[rowbase(j, k) + (uint64_t)im] : 0u;
    };

    int cnt = 0;
    auto flush = [&]() {
        if (cnt == 0) return;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        unsigned long long base = 0;
        if (lane == 0) {
            base = atomicAdd(reinterpret_cast<unsigned long long *>(A.count), (unsigned long long)cnt);
            if ((int64_t)base + cnt > A.cap) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_WIND);
        }
        base = ((unsigned long long)(uint32_t)__shfl((int)(base >> 32), 0) << 32) | (uint32_t)__shfl((int)base, 0);
        for (int q = lane; q < cnt; q += 64) {
            const int64_t idx = (int64_t)base + q;
            if (idx < A.cap) A.list[idx] = s_buf[q];
        }
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
        __builtin_amdgcn_wave_barrier();
        cnt = 0;
    };

    // state carried from the previous plane, per output row: T, Y (and lane 0's neighbour y field)
    uint32_t Tp[WROWS][4], Yp[WROWS][4], yim[WROWS];
    {
        const int kp = z0 > 0 ? z0 - 1 : (A.pz ? nz - 1 : -1);
        uint32_t w[4], Bb[4];
        load_row(rows[0], kp, w);
#pragma unroll
        for (int t = 0; t < 4; ++t) Bb[t] = bxz(w[t]);
#pragma unroll
        for (int q = 1; q <= WROWS; ++q) {
            load_row(rows[q], kp, w);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t b = bxz(w[t]);
                Tp[q - 1][t] = b + Bb[t];
                Bb[t] = b;
                Yp[q - 1][t] = byf(w[t]);
            }
            yim[q - 1] = byf(edge_byte(rows[q], kp));
        }
    }
    for (int k = z0; k < z1; ++k) {
        uint32_t w[4], Bb[4];
        load_row(rows[0], k, w);
        uint32_t eb = edge_byte(rows[0], k);
#pragma unroll
        for (int t = 0; t < 4; ++t) Bb[t] = bxz(w[t]);
        uint32_t Bbe = bxz(eb);  // lane 0: B of the neighbour node of the row below
        int nv = 0;              // vortex nodes of this lane in this plane
        uint32_t out[WROWS][4];
#pragma unroll
        for (int q = 1; q <= WROWS; ++q) {
            load_row(rows[q], k, w);
            const uint32_t e = edge_byte(rows[q], k);
            uint32_t T[4], U[4], Tx[4], Ux[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const uint32_t b = bxz(w[t]), y = byf(w[t]);
                T[t] = b + Bb[t];
                Bb[t] = b;
                U[t] = y + Yp[q - 1][t];
                Yp[q - 1][t] = y;
            }
            // values of the node before the lane's first: the previous lane's last, or lane 0's own
            const uint32_t be = bxz(e), ye = byf(e);
            uint32_t tin = from_prev_lane(T[3]), uin = from_prev_lane(U[3]);
            if (lane == 0) {
                tin = (be + Bbe) << 24;
                uin = (ye + yim[q - 1]) << 24;
            }
            Bbe = be;
            yim[q - 1] = ye;
            xshift4(T, tin, Tx);
            xshift4(U, uin, Ux);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                // per byte: Sx in the low nibble, Sz in the high one; Sy beside
                const uint32_t XZ = ((T[t] + Tp[q - 1][t]) & 0x0F0F0F0Fu) | ((T[t] + Tx[t]) & 0xF0F0F0F0u);
                const uint32_t Sy = U[t] + Ux[t];
                Tp[q - 1][t] = T[t];
                const uint32_t ie = __builtin_amdgcn_perm(Sy, XZ, 0x06020400u);  // nodes 0, 2
                const uint32_t io = __builtin_amdgcn_perm(Sy, XZ, 0x07030501u);  // nodes 1, 3
                const uint32_t o = (uint32_t)s_lut[ie & 0xffffu] | ((uint32_t)s_lut[io & 0xffffu] << 8) |
                                   ((uint32_t)s_lut[ie >> 16] << 16) | ((uint32_t)s_lut[io >> 16] << 24);
                out[q - 1][t] = (active && rows[q] >= 0) ? o : 0u;
                nv += __popc(out[q - 1][t] & 0x40404040u);
            }
        }
        if (A.node) {
#pragma unroll
            for (int q = 1; q <= WROWS; ++q)
                if (active && rows[q] >= 0)
                    *(uint4 *)(A.node + rowbase(rows[q], k) + i0) =
                        make_uint4(out[q - 1][0], out[q - 1][1], out[q - 1][2], out[q - 1][3]);
        }
        // vortex nodes: per-lane counts, a wavefront prefix sum, entries into LDS
        if (__ballot(nv != 0) != 0) {
            int incl = nv;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off);
                if (lane >= off) incl += v;
            }
            const int total = __shfl(incl, 63);
            if (cnt + total > NBUF) flush();
            int64_t pos = cnt + incl - nv;  // LDS slot of this lane's first entry
            unsigned long long gbase = 0;
            if (total > NBUF) {  // more than the buffer holds: every lane reserves its own slots
                if (nv) {
                    gbase = atomicAdd(reinterpret_cast<unsigned long long *>(A.count), (unsigned long long)nv);
                    if ((int64_t)gbase + nv > A.cap) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_WIND);
                }
            }
#pragma unroll
            for (int q = 1; q <= WROWS; ++q)
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    uint32_t m = out[q - 1][t] & 0x40404040u;
                    while (m) {
                        const int bb = __builtin_ctz(m) >> 3;
                        m &= m - 1;
                        const uint64_t id = rowbase(rows[q], k) + (uint64_t)(i0 + 4 * t + bb);
                        if (total > NBUF) {
                            if ((int64_t)gbase < A.cap) A.list[gbase] = id;
                            ++gbase;
                        } else {
                            s_buf[pos++] = id;
                        }
                    }
                }
            __builtin_amdgcn_wave_barrier();
            if (total <= NBUF) cnt += total;
        }
    }
    flush();
}

__global__ void zero_count_k(int64_t *c) {
    if (threadIdx.x == 0) *c = 0;
}

}  // namespace

extern "C" vx_status vx_node_circulation(vx_handle *h, vx_dims dims, const uint8_t *d_wind, uint8_t *d_node,
                                         uint64_t *d_nodes, int64_t node_cap, int64_t *d_count, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (!d_wind || !d_count) return vx_fail(h, VX_ERR_INVALID, "vx_node_circulation: null d_wind or d_count");
    if (node_cap < 0 || (node_cap > 0 && !d_nodes))
        return vx_fail(h, VX_ERR_INVALID, "vx_node_circulation: node_cap > 0 needs d_nodes");
    if (((uintptr_t)d_count & 7u) != 0) return vx_fail(h, VX_ERR_INVALID, "vx_node_circulation: d_count alignment");
    if (dims.ny > 65535 || (int64_t)(dims.nz + NODE_ZC - 1) / NODE_ZC > 65535)
        return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_node_circulation: grid too tall for the launch");
    if (vx_status st = vx_bind(h)) return st;
    NodeArgs A;
    A.wind = d_wind;
    A.node = d_node;
    A.list = d_nodes;
    A.cap = node_cap;
    A.count = d_count;
    A.flag = vx_overflow_flag(h);
    A.nx = dims.nx;
    A.ny = dims.ny;
    A.nz = dims.nz;
    A.px = (int)(dims.periodic & 1u);
    A.py = (int)((dims.periodic >> 1) & 1u);
    A.pz = (int)((dims.periodic >> 2) & 1u);
    A.aligned = (dims.nx % 4 == 0) && ((uintptr_t)d_wind & 3u) == 0 && ((uintptr_t)d_node & 3u) == 0;
    hipStream_t hs = (hipStream_t)s;
    hipLaunchKernelGGL(zero_count_k, dim3(1), dim3(64), 0, hs, d_count);
    // whole 16-node words per lane when rows allow it (node_circ_wide_k), else 4 nodes per lane
    const bool wide = dims.nx % 16 == 0 && ((uintptr_t)d_wind & 15u) == 0 && ((uintptr_t)d_node & 15u) == 0;
    const unsigned gz = (unsigned)((dims.nz + NODE_ZC - 1) / NODE_ZC);
    vx_timer tm(h, hs, VX_KIND_NODE);
    if (wide)
        hipLaunchKernelGGL(node_circ_wide_k, dim3((unsigned)((dims.nx + 1023) / 1024), (unsigned)((dims.ny + WROWS - 1) / WROWS), gz),
                           dim3(64), 0, hs, A);
    else
        hipLaunchKernelGGL(node_circ_k, dim3((unsigned)((dims.nx + 255) / 256), (unsigned)dims.ny, gz), dim3(64), 0, hs, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "node_circ_k launch");
}
