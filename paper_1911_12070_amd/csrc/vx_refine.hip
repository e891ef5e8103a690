// Core-sample refinement (Sec. 3.3.1 mean-position estimate, Sec. 3.3.3 density-guided minimisation
// in the plane normal to the pseudo-vorticity, psi linearly interpolated between nodes as in Sec. 5).
//
// Work layout. The number of listed cells is read on the device (no host synchronisation); the
// list is cut into chunks of REF_CHUNK samples that wavefronts claim from a device counter (zeroed
// by a one-thread kernel on the same stream before each launch). The iteration count per sample
// varies a lot (median about 9 accepted steps, a long tail past 30), so lanes do not take one
// sample each in lockstep: every lane runs its own sample as a state machine that performs one trilinear
// evaluation per pass of the wave's loop, and a lane whose sample is done writes it and takes the
// next unclaimed sample of the wave's chunk (ballot + mbcnt, the claim cursor is wave-uniform).
// The wave thus pays for the mean iteration count of its samples, not for the maximum over 64.
//
// The iterate only needs the 8 corners of the unit cell that holds it; they are cached per lane in
// LDS and fetched from global memory (L1/L2-resident: neighbouring samples share nodes) when the
// iterate changes cell. The state machine's bookkeeping after each evaluation is written as selects:
// loop-carried state updated under divergent branches costs register copies at every merge.
// FP32 arithmetic throughout.
#include "vx_internal.h"

namespace {

constexpr int REF_THREADS = 256;  // four wavefronts per workgroup
constexpr int REF_CHUNK = 64;     // samples a wavefront claims at a time

struct RefArgs {
    const float2 *psi;
    const uint64_t *cells;
    const uint16_t *desc;
    const float *seed;
    const int64_t *count;
    int64_t cap;
    vx_sample *out;
    const int64_t *out_index;    // nullable: sample s is written to out[out_index[s]]
    unsigned long long *chunks;  // chunk counter, zero at launch
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
// hardware reciprocal square root and reciprocal (about 1 ulp): the normalisations and step
// directions they feed are search directions, whose last-bit rounding does not move the minimum
__device__ __forceinline__ float rsq(float a) { return __builtin_amdgcn_rsqf(a); }
__device__ __forceinline__ float rcp(float a) { return __builtin_amdgcn_rcpf(a); }
__device__ __forceinline__ float comp(const V3 &a, int i) { return i == 0 ? a.x : (i == 1 ? a.y : a.z); }

__device__ __forceinline__ int dec2(uint32_t d, int f) {
    const uint32_t v = (d >> (2 * f)) & 3u;
    return v == 1u ? 1 : (v == 3u ? -1 : 0);
}

__device__ __forceinline__ int64_t wrap(int64_t q, int n, int per) {
    if (q < 0) return per ? q + n : 0;
    if (q >= n) return per ? q - n : n - 1;
    return q;
}

// quotient and remainder of n by d for n < 2^53 (every cell id of a grid that fits in memory):
// an FP64 estimate off by at most one, then an integer correction
__device__ __forceinline__ uint64_t divmod53(uint64_t n, uint64_t d, double rd, uint64_t &r) {
    uint64_t q = (uint64_t)((double)n * rd);
    int64_t rem = (int64_t)(n - q * d);
    if (rem < 0) {
        --q;
        rem += (int64_t)d;
    } else if (rem >= (int64_t)d) {
        ++q;
        rem -= (int64_t)d;
    }
    r = (uint64_t)rem;
    return q;
}

// lane phases
constexpr int PH_IDLE = 0;     // no sample
constexpr int PH_INIT = 1;     // pending evaluation at the first estimate x0
constexpr int PH_TRIAL = 2;    // pending evaluation of a trial point of the current step
constexpr int PH_BEGIN = 3;    // a step of the current kind starts at the next pass (no evaluation)
// step kinds
constexpr int MODE_DESCENT = 0;  // gradient descent of |psi|^2, halving step rule
constexpr int MODE_NEWTON = 1;   // Newton on (Re psi, Im psi), halving until |psi|^2 decreases

// BATCH = false: one grid, described by the kernel arguments. BATCH = true: the frames of a batch,
// described by a device table copied to LDS; work chunks never straddle frames, and each lane
// looks up its own sample's frame where the frame matters (corner fetch, output).
template <bool BATCH>
__global__ __launch_bounds__(REF_THREADS) void refine_k(RefArgs A, const vx_ref_frame *frames, int nframes,
                                                        int refill_min) {
    // corner cache: corner d (index dx + 2 dy + 4 dz) of the cell cached by thread t at [d][t]
    __shared__ float2 s_corner[8][REF_THREADS];
    constexpr int NF = BATCH ? VX_BATCH_MAX_FRAMES : 1;
    __shared__ vx_ref_frame s_fr[NF];
    __shared__ double s_rnx[NF], s_rnxy[NF];
    __shared__ int64_t s_items[NF], s_cstart[NF + 1];
    const vx_refine_params &P = A.p;
    const int tid = threadIdx.x;
    const int64_t nwaves = (int64_t)gridDim.x * (REF_THREADS / 64);
    const int64_t wave = (int64_t)blockIdx.x * (REF_THREADS / 64) + (tid >> 6);
    int64_t n_items = 0;  // single grid: number of samples
    if constexpr (BATCH) {
        // frame table, samples per frame and the prefix of chunks per frame
        if (tid < nframes) {
            const vx_ref_frame F = frames[tid];
            s_fr[tid] = F;
            const int64_t n = min(*F.count, F.cap);
            s_items[tid] = n;
            s_cstart[tid + 1] = (n + REF_CHUNK - 1) / REF_CHUNK;
            s_rnx[tid] = 1.0 / (double)F.nx;
            s_rnxy[tid] = 1.0 / ((double)F.nx * (double)F.ny);
        }
        if (tid == 0) s_cstart[0] = 0;
        __syncthreads();
        for (int off = 1; off < nframes; off <<= 1) {  // inclusive scan of s_cstart[1..nframes]
            const int64_t add = (tid < nframes && tid >= off) ? s_cstart[tid + 1 - off] : 0;
            __syncthreads();
            if (tid < nframes) s_cstart[tid + 1] += add;
            __syncthreads();
        }
    } else {
        n_items = min(*A.count, A.cap);
    }
    // chunk size: REF_CHUNK, or down to one sample when the list is short for the grid, so that a
    // short list (a surrogate's fallback cells, say) spreads over as many wavefronts as it can: its
    // time is then the latency of its slowest sample, and a wavefront with few live lanes runs the
    // code paths of those lanes only
    const int64_t chunk = BATCH ? REF_CHUNK : max((int64_t)1, min((int64_t)REF_CHUNK, (n_items + nwaves - 1) / nwaves));
    // samples [next, end) of frame cf are this wave's unclaimed ones (uniform); chunk w is wave w's
    // first, the rest are handed out in order by the chunk counter
    int cf = 0;
    int64_t next = 0, end = 0;
    bool more = true;  // unclaimed chunks may remain
    auto claim = [&](int64_t ci) {
        if constexpr (BATCH) {
            if (ci >= s_cstart[nframes]) {
                more = false;
                next = end = 0;
                return;
            }
            int lo = 0, hi = nframes;  // last frame whose first chunk is <= ci
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_cstart[mid] <= ci) lo = mid;
                else hi = mid;
            }
            cf = lo;
            next = (ci - s_cstart[lo]) * REF_CHUNK;
            end = min(s_items[lo], next + REF_CHUNK);
        } else {
            next = min(n_items, ci * chunk);
            end = min(n_items, next + chunk);
            more = next < end;
        }
    };
    claim(wave);
    // chunks beyond the first one per wavefront exist only if the list has more chunks than there
    // are wavefronts; otherwise nobody touches the counter
    if constexpr (BATCH) more = more && s_cstart[nframes] > nwaves;
    else more = more && (n_items + chunk - 1) / chunk > nwaves;

    int phase = PH_IDLE, mode = MODE_DESCENT;
    int fr = 0;  // frame of this lane's sample
    int64_t s = 0;
    uint64_t cell = 0;
    uint32_t desc = 0;
    int gi = 0, gj = 0, gk = 0;  // grid node of the sample cell's min corner
    uint32_t ext = 0;            // patch extent: bit a set if the patch reaches -1 on axis a,
                                 // bit 3 + a set if it reaches +2 (else it stops at 0 / +1)
    int ccode = -1;              // cached cell: (cx+1) + 4 (cy+1) + 16 (cz+1)
    V3 x0 = v3(0.f, 0.f, 0.f), e1 = x0, e2 = x0, xt = x0;
    float y1 = 0.f, y2 = 0.f, ty1 = 0.f, ty2 = 0.f;
    float vr = 0.f, vi = 0.f, f = 0.f;
    V3 gr = x0, gim = x0;
    float s_prev = 0.f, gn = 0.f;           // descent: last accepted length, gradient norm
    float alpha = 0.f, p1 = 0.f, p2 = 0.f;  // current step: length factor and direction
    int dit = 0, nit = 0, hv = 0, iters = 0;
    uint32_t status = 0;
    bool converged = false;

    while (true) {
        // ---- idle lanes claim the next samples of the wave's range, once enough of them are idle
        const uint64_t idle = __ballot(phase == PH_IDLE);
        const int n_idle = __popcll(idle);
        if (next >= end && more && (n_idle >= refill_min || n_idle == 64)) {
            unsigned long long c = 0;
            if ((tid & 63) == 0) c = atomicAdd(A.chunks, 1ull);
            claim((int64_t)nwaves + (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(c >> 32)) << 32) |
                                              __builtin_amdgcn_readfirstlane((uint32_t)c)));
        }
        if (next < end && (n_idle >= refill_min || n_idle == 64)) {
            if (phase == PH_IDLE) {
                const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(idle >> 32),
                                                                __builtin_amdgcn_mbcnt_lo((uint32_t)idle, 0u));
                const int64_t mine = next + (int64_t)rank;
                if (mine < end) {
                    // the claimed chunk's frame (uniform)
                    const uint64_t *cells_p = A.cells;
                    const uint16_t *desc_p = A.desc;
                    vx_sample *out_p = A.out;
                    int fnx = A.nx, fny = A.ny, fnz = A.nz, fpx = A.px, fpy = A.py, fpz = A.pz;
                    double rnx, rnxy;
                    if constexpr (BATCH) {
                        const vx_ref_frame &F = s_fr[cf];
                        cells_p = F.cells;
                        desc_p = F.desc;
                        out_p = F.out;
                        fnx = F.nx;
                        fny = F.ny;
                        fnz = F.nz;
                        fpx = (int)(F.periodic & 1u);
                        fpy = (int)((F.periodic >> 1) & 1u);
                        fpz = (int)((F.periodic >> 2) & 1u);
                        rnx = s_rnx[cf];
                        rnxy = s_rnxy[cf];
                    } else {
                        rnx = 1.0 / (double)A.nx;
                        rnxy = 1.0 / ((double)A.nx * (double)A.ny);
                    }
                    const uint64_t nx64 = (uint64_t)fnx, nxy = (uint64_t)fnx * (uint64_t)fny;
                    s = mine;
                    fr = cf;
                    cell = cells_p[s];
                    desc = desc_p[s];
                    if (cell >= nxy * (uint64_t)fnz) {
                        vx_sample o{};
                        o.cell = cell;
                        o.rho = -1.f;
                        o.status = (uint16_t)VX_SAMPLE_BAD_CELL;
                        out_p[(!BATCH && A.out_index) ? A.out_index[s] : s] = o;
                    } else {
                        uint64_t rxy, ri;
                        gk = (int)divmod53(cell, nxy, rnxy, rxy);
                        gj = (int)divmod53(rxy, nx64, rnx, ri);
                        gi = (int)ri;
                        const int g3[3] = {gi, gj, gk};
                        const int n3[3] = {fnx, fny, fnz};
                        const int p3[3] = {fpx, fpy, fpz};
                        ext = 0;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            if (p3[a] || g3[a] - 1 >= 0) ext |= 1u << a;
                            if (p3[a] || g3[a] + 2 < n3[a]) ext |= 8u << a;
                        }
                        ccode = -1;  // force a corner fetch at the first evaluation
                        status = 0;
                        iters = 0;
                        dit = 0;
                        nit = 0;
                        converged = false;
                        // first estimate: mean of the centres of the pierced faces (-x,+x,-y,+y,-z,+z)
                        float sx = 0.f, sy = 0.f, sz = 0.f;
                        int npierced = 0;
#pragma unroll
                        for (int fc = 0; fc < 6; ++fc) {
                            if (dec2(desc, fc) == 0) continue;
                            const int a = fc >> 1;
                            const float side = (float)(fc & 1);
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
                        if (npierced >= 4) status |= VX_SAMPLE_MULTI;
                        if (A.seed) x0 = v3(A.seed[3 * s], A.seed[3 * s + 1], A.seed[3 * s + 2]);
                        xt = x0;
                        phase = PH_INIT;
                    }
                }
            }
            next += (int64_t)n_idle;
        }
        if (__ballot(phase != PH_IDLE) == 0) {
            if (next >= end && !more) break;
            continue;  // nothing claimed yet, or every claimed id was out of range: claim again
        }

        // ---- one trilinear evaluation at the pending point (value and gradient, cell units); lanes
        // waiting to begin a step evaluate too (a point of their patch) and ignore the result
        float tr = 0.f, ti = 0.f;
        V3 tgr = v3(0.f, 0.f, 0.f), tgi = tgr;
        if (phase != PH_IDLE) {
            int c[3];
            float u[3];
            const float xs[3] = {xt.x, xt.y, xt.z};
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int lo = (ext >> a) & 1u ? -1 : 0, hi = (ext >> (3 + a)) & 1u ? 1 : 0;
                int fl = (int)floorf(xs[a]);
                fl = max(lo, min(fl, hi));
                c[a] = fl;
                u[a] = xs[a] - (float)fl;
            }
            const int code = (c[0] + 1) + 4 * (c[1] + 1) + 16 * (c[2] + 1);
            if (code != ccode) {
                ccode = code;
                const float2 *psi_p = A.psi;
                int fnx = A.nx, fny = A.ny, fnz = A.nz, fpx = A.px, fpy = A.py, fpz = A.pz;
                if constexpr (BATCH) {
                    const vx_ref_frame &F = s_fr[fr];
                    psi_p = F.psi;
                    fnx = F.nx;
                    fny = F.ny;
                    fnz = F.nz;
                    fpx = (int)(F.periodic & 1u);
                    fpy = (int)((F.periodic >> 1) & 1u);
                    fpz = (int)((F.periodic >> 2) & 1u);
                }
                const uint64_t nx64 = (uint64_t)fnx, nxy = (uint64_t)fnx * (uint64_t)fny;
                const int64_t i0 = wrap((int64_t)gi + c[0], fnx, fpx);
                const int64_t i1 = wrap((int64_t)gi + c[0] + 1, fnx, fpx);
                const int64_t j0 = wrap((int64_t)gj + c[1], fny, fpy);
                const int64_t j1 = wrap((int64_t)gj + c[1] + 1, fny, fpy);
                const int64_t k0 = wrap((int64_t)gk + c[2], fnz, fpz);
                const int64_t k1 = wrap((int64_t)gk + c[2] + 1, fnz, fpz);
                const float2 *r00 = psi_p + nx64 * (uint64_t)j0 + nxy * (uint64_t)k0;
                const float2 *r10 = psi_p + nx64 * (uint64_t)j1 + nxy * (uint64_t)k0;
                const float2 *r01 = psi_p + nx64 * (uint64_t)j0 + nxy * (uint64_t)k1;
                const float2 *r11 = psi_p + nx64 * (uint64_t)j1 + nxy * (uint64_t)k1;
                const float2 c0 = r00[i0], c1 = r00[i1], c2 = r10[i0], c3 = r10[i1];
                const float2 c4 = r01[i0], c5 = r01[i1], c6 = r11[i0], c7 = r11[i1];
                s_corner[0][tid] = c0;
                s_corner[1][tid] = c1;
                s_corner[2][tid] = c2;
                s_corner[3][tid] = c3;
                s_corner[4][tid] = c4;
                s_corner[5][tid] = c5;
                s_corner[6][tid] = c6;
                s_corner[7][tid] = c7;
            }
            float2 v[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) v[d] = s_corner[d][tid];
            const float ux = u[0], uy = u[1], uz = u[2];
            const float mx = 1.f - ux, my = 1.f - uy, mz = 1.f - uz;
            const float2 a00 = make_float2(mx * v[0].x + ux * v[1].x, mx * v[0].y + ux * v[1].y);
            const float2 a10 = make_float2(mx * v[2].x + ux * v[3].x, mx * v[2].y + ux * v[3].y);
            const float2 a01 = make_float2(mx * v[4].x + ux * v[5].x, mx * v[4].y + ux * v[5].y);
            const float2 a11 = make_float2(mx * v[6].x + ux * v[7].x, mx * v[6].y + ux * v[7].y);
            const float2 d00 = make_float2(v[1].x - v[0].x, v[1].y - v[0].y);
            const float2 d10 = make_float2(v[3].x - v[2].x, v[3].y - v[2].y);
            const float2 d01 = make_float2(v[5].x - v[4].x, v[5].y - v[4].y);
            const float2 d11 = make_float2(v[7].x - v[6].x, v[7].y - v[6].y);
            const float2 b0 = make_float2(my * a00.x + uy * a10.x, my * a00.y + uy * a10.y);
            const float2 b1 = make_float2(my * a01.x + uy * a11.x, my * a01.y + uy * a11.y);
            tr = mz * b0.x + uz * b1.x;
            ti = mz * b0.y + uz * b1.y;
            tgr.z = b1.x - b0.x;
            tgi.z = b1.y - b0.y;
            const float2 ey0 = make_float2(a10.x - a00.x, a10.y - a00.y);
            const float2 ey1 = make_float2(a11.x - a01.x, a11.y - a01.y);
            tgr.y = mz * ey0.x + uz * ey1.x;
            tgi.y = mz * ey0.y + uz * ey1.y;
            const float2 ex0 = make_float2(my * d00.x + uy * d10.x, my * d00.y + uy * d10.y);
            const float2 ex1 = make_float2(my * d01.x + uy * d11.x, my * d01.y + uy * d11.y);
            tgr.x = mz * ex0.x + uz * ex1.x;
            tgi.x = mz * ex0.y + uz * ex1.y;
        }

        // ---- first evaluation of a sample: plane normal to the pseudo-vorticity at x0
        if (phase == PH_INIT) {
            V3 t = crs(tgr, tgi);
            float tn = nrm(t);
            if (!(tn > 1e-6f * nrm(tgr) * nrm(tgi)) || tn == 0.f) {
                status |= VX_SAMPLE_TANGENT_FALLBACK;
                t = v3((float)(dec2(desc, 0) + dec2(desc, 1)), (float)(dec2(desc, 2) + dec2(desc, 3)),
                       (float)(dec2(desc, 4) + dec2(desc, 5)));
                if (nrm(t) == 0.f) {
                    t = v3(0.f, 0.f, 1.f);
                    for (int fc = 0; fc < 6; ++fc) {
                        const int w = dec2(desc, fc);
                        if (w != 0) {
                            const int a = fc >> 1;
                            t = v3(a == 0 ? (float)w : 0.f, a == 1 ? (float)w : 0.f, a == 2 ? (float)w : 0.f);
                            break;
                        }
                    }
                }
                tn = nrm(t);
            }
            const float itn = rcp(tn);
            t = v3(t.x * itn, t.y * itn, t.z * itn);
            int ax = 0;
            if (fabsf(t.y) < fabsf(comp(t, ax))) ax = 1;
            if (fabsf(t.z) < fabsf(comp(t, ax))) ax = 2;
            e1 = crs(t, v3(ax == 0 ? 1.f : 0.f, ax == 1 ? 1.f : 0.f, ax == 2 ? 1.f : 0.f));
            const float in1 = rsq(dot(e1, e1));
            e1 = v3(e1.x * in1, e1.y * in1, e1.z * in1);
            e2 = crs(t, e1);
            ty1 = 0.f;  // taken over as the current point below
            ty2 = 0.f;
            s_prev = 0.5f * P.step0;
            mode = MODE_DESCENT;
        }

        // ---- outcome of the evaluation, without branches: the first evaluation and accepted
        // trial points become the current point; rejected trial points halve the step
        const bool init = phase == PH_INIT;
        const bool tri = phase == PH_TRIAL;
        const bool descent = mode == MODE_DESCENT;
        const float ft = tr * tr + ti * ti;
        const bool acc = tri && (descent ? (ft <= f - P.armijo * alpha * gn) : (ft < f));
        const bool take = init || acc;
        y1 = take ? ty1 : y1;
        y2 = take ? ty2 : y2;
        vr = take ? tr : vr;
        vi = take ? ti : vi;
        gr.x = take ? tgr.x : gr.x;
        gr.y = take ? tgr.y : gr.y;
        gr.z = take ? tgr.z : gr.z;
        gim.x = take ? tgi.x : gim.x;
        gim.y = take ? tgi.y : gim.y;
        gim.z = take ? tgi.z : gim.z;
        f = take ? ft : f;
        iters += acc ? 1 : 0;
        const bool acc_d = acc && descent, acc_n = acc && !descent;
        dit += acc_d ? 1 : 0;
        nit += acc_n ? 1 : 0;
        s_prev = acc_d ? alpha : s_prev;
        const bool conv_now = acc_n && alpha * sqrtf(p1 * p1 + p2 * p2) < P.newton_tol;
        converged = converged || conv_now;
        mode = (acc_d && alpha < P.descent_tol) ? MODE_NEWTON : mode;
        const bool rej = tri && !acc;
        alpha = rej ? 0.5f * alpha : alpha;
        hv += rej ? 1 : 0;
        bool begin = init || phase == PH_BEGIN || (acc && !conv_now);
        bool trial = rej;
        bool finish = conv_now;

        // ---- start a step of the current kind; a descent that cannot start hands over to
        // Newton, which then starts at the next pass
        if (begin) {
            float n1 = 0.f, n2 = 0.f, den = 1.f;  // direction = (n1, n2) * den
            bool ok = false;
            if (mode == MODE_DESCENT) {
                if (dit < P.max_descent && f != 0.f) {
                    const V3 G = v3(2.f * (vr * gr.x + vi * gim.x), 2.f * (vr * gr.y + vi * gim.y),
                                    2.f * (vr * gr.z + vi * gim.z));
                    const float g1 = dot(e1, G), g2 = dot(e2, G);
                    const float gg = g1 * g1 + g2 * g2;
                    const float ig = rsq(gg);
                    gn = gg * ig;
                    ok = gg > 0.f && ig < INFINITY;
                    n1 = -g1;
                    n2 = -g2;
                    den = ig;  // direction = -g / |g|
                    alpha = fminf(2.f * s_prev, P.step_max);
                }
                if (!ok) {
                    mode = MODE_NEWTON;
                    phase = PH_BEGIN;
                }
            } else {
                if (nit < P.max_newton) {
                    if (f == 0.f) {
                        converged = true;
                    } else {
                        const float j00 = dot(e1, gr), j01 = dot(e2, gr);
                        const float j10 = dot(e1, gim), j11 = dot(e2, gim);
                        const float det = j00 * j11 - j01 * j10;
                        const float idet = rcp(det);
                        ok = det != 0.f && fabsf(idet) < INFINITY;
                        n1 = -(j11 * vr - j01 * vi);
                        n2 = -(-j10 * vr + j00 * vi);
                        den = idet;
                        alpha = 1.f;
                    }
                }
                if (!ok) finish = true;
            }
            if (ok) {
                p1 = n1 * den;
                p2 = n2 * den;
                hv = 0;
                trial = true;
            }
        }
        // ---- the step's next trial point inside the patch (points outside are rejected unevaluated)
        if (trial) {
            bool found = false, stuck = false;
            while (hv < P.max_halvings) {
                ty1 = y1 + alpha * p1;
                ty2 = y2 + alpha * p2;
                xt = v3(x0.x + ty1 * e1.x + ty2 * e2.x, x0.y + ty1 * e1.y + ty2 * e2.y,
                        x0.z + ty1 * e1.z + ty2 * e2.z);
                const float lx = (ext & 1u) ? -1.f : 0.f, ly = (ext & 2u) ? -1.f : 0.f;
                const float lz = (ext & 4u) ? -1.f : 0.f, hx = (ext & 8u) ? 2.f : 1.f;
                const float hy = (ext & 16u) ? 2.f : 1.f, hz = (ext & 32u) ? 2.f : 1.f;
                if (xt.x >= lx && xt.x <= hx && xt.y >= ly && xt.y <= hy && xt.z >= lz && xt.z <= hz) {
                    // a Newton trial point equal to the current point (as is then every shorter
                    // one) is rejected at this and every remaining halving: |psi|^2 cannot decrease
                    if (mode == MODE_NEWTON && ty1 == y1 && ty2 == y2) stuck = true;
                    else found = true;
                    break;
                }
                status |= VX_SAMPLE_BOUNDARY;
                alpha *= 0.5f;
                ++hv;
            }
            if (found) {
                phase = PH_TRIAL;
            } else if (mode == MODE_DESCENT && !stuck) {
                mode = MODE_NEWTON;
                phase = PH_BEGIN;
            } else {
                finish = true;
            }
        }
        if (finish) {
            if (f > P.rho_tol) status |= VX_SAMPLE_NONZERO_MIN;
            if (!converged && f > P.rho_tol) status |= VX_SAMPLE_NOT_CONVERGED;
            // the current point, computed exactly as when it was a trial point
            vx_sample o;
            o.cell = cell;
            o.off[0] = x0.x + y1 * e1.x + y2 * e2.x;
            o.off[1] = x0.y + y1 * e1.y + y2 * e2.y;
            o.off[2] = x0.z + y1 * e1.z + y2 * e2.z;
            o.rho = f;
            o.iters = (uint16_t)min(iters, 65535);
            o.status = (uint16_t)status;
            o.reserved = 0;
            if constexpr (BATCH) s_fr[fr].out[s] = o;
            else A.out[A.out_index ? A.out_index[s] : s] = o;
            phase = PH_IDLE;
        }
    }
}

__global__ void zero_u64_k(unsigned long long *p) { *p = 0ull; }

// one resident round of wavefronts (they claim chunks dynamically); fewer for short lists; -1 on error
template <typename K>
int64_t ref_blocks(vx_handle *h, K kernel, int &per_cu, int64_t cap) {
    if (per_cu <= 0) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, REF_THREADS, 0);
        if (e != hipSuccess) {
            vx_hip_check(h, e, "refine_k occupancy");
            return -1;
        }
        per_cu = nb > 0 ? nb : 1;
    }
    const int64_t resident = (int64_t)per_cu * (h->num_cu > 0 ? h->num_cu : 256);
    const int64_t need = (cap + 4 * REF_CHUNK - 1) / (4 * REF_CHUNK);  // >= one chunk per wavefront
    return std::max<int64_t>(1, std::min(need, resident));
}

}  // namespace

vx_status vx_refine_launch(vx_handle *h, const vx_dims &d, const void *psi, const uint64_t *cells,
                           const uint16_t *desc, const float *seed, const int64_t *count, int64_t cap,
                           const vx_refine_params &p, vx_sample *out, hipStream_t s, const int64_t *out_index) {
    RefArgs A;
    A.out_index = out_index;
    A.psi = (const float2 *)psi;
    A.cells = cells;
    A.desc = desc;
    A.seed = seed;
    A.count = count;
    A.cap = cap;
    A.out = out;
    A.chunks = h->d_work;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    A.px = (int)(d.periodic & 1u);
    A.py = (int)((d.periodic >> 1) & 1u);
    A.pz = (int)((d.periodic >> 2) & 1u);
    A.p = p;
    const int64_t blocks = ref_blocks(h, refine_k<false>, h->ref_blocks_per_cu, cap);
    if (blocks < 0) return VX_ERR_DEVICE;
    vx_timer tm(h, s, VX_KIND_REFINE);
    hipLaunchKernelGGL(zero_u64_k, dim3(1), dim3(1), 0, s, h->d_work);
    hipLaunchKernelGGL(refine_k<false>, dim3((unsigned)blocks), dim3(REF_THREADS), 0, s, A,
                       (const vx_ref_frame *)nullptr, 1, h->ref_refill);
    tm.stop();
    return vx_hip_check(h, hipGetLastError(), "refine_k launch");
}

vx_status vx_refine_batch_enqueue(vx_handle *h, const vx_ref_frame *d_frames, int nframes, int64_t total_cap,
                                  const vx_refine_params &p, unsigned long long *d_counter, hipStream_t s) {
    if (nframes < 1 || nframes > VX_BATCH_MAX_FRAMES)
        return vx_fail(h, VX_ERR_INVALID, "refine batch: %d frames", nframes);
    RefArgs A{};
    A.chunks = d_counter;
    A.p = p;
    const int64_t blocks = ref_blocks(h, refine_k<true>, h->refb_blocks_per_cu, total_cap);
    if (blocks < 0) return VX_ERR_DEVICE;
    hipLaunchKernelGGL(zero_u64_k, dim3(1), dim3(1), 0, s, d_counter);
    hipLaunchKernelGGL(refine_k<true>, dim3((unsigned)blocks), dim3(REF_THREADS), 0, s, A, d_frames, nframes,
                       h->ref_refill);
    return vx_hip_check(h, hipGetLastError(), "refine_k batch launch");
}
