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
__device__ uint8_t lut_entry(int e) {
    const int s[3] = {e % 9 - 4, (e / 9) % 9 - 4, e / 81 - 4};
    int best = 0;
    for (int a = 1; a < 3; ++a)
        if (abs(s[a]) > abs(s[best])) best = a;
    const int v = s[best], mag = min(abs(v), 3);
    if (mag == 0) return 0;
    return (uint8_t)(mag | (v < 0 ? 4 : 0) | (best << 3) | 0x40);
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
    const dim3 grid((unsigned)((dims.nx + 255) / 256), (unsigned)dims.ny, (unsigned)((dims.nz + NODE_ZC - 1) / NODE_ZC));
    vx_timer tm(h, hs, VX_KIND_NODE);
    hipLaunchKernelGGL(node_circ_k, grid, dim3(64), 0, hs, A);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "node_circ_k launch");
}
