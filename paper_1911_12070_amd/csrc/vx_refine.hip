// Core-sample refinement (Sec. 3.3.1 mean-position estimate, Sec. 3.3.3 density-guided minimisation
// in the plane normal to the pseudo-vorticity, psi linearly interpolated between nodes as in Sec. 5).
//
// Work layout. The number of listed cells is read on the device (no host synchronisation), so every
// call launches two kernels and the one whose list it is not returns at once: refine_spec_k for
// lists of at most one sample per resident 16-lane group (described with that kernel below), and
// refine_k for longer ones. refine_k cuts the list into chunks of REF_CHUNK samples that wavefronts
// claim from a device counter (zeroed by refine_spec_k, which runs first on the same stream). The
// iteration count per sample varies a lot (median about 9 accepted steps, a long tail past 30), so
// lanes do not take one sample each in lockstep: every lane runs its own sample as a state machine
// that performs one trilinear evaluation per pass of the wave's loop, and a lane whose sample is done
// writes it and takes the next unclaimed sample of the wave's chunk (ballot + mbcnt, the claim
// cursor is wave-uniform). The wave thus pays for the mean iteration count of its samples, not for
// the maximum over 64.
//
// The iterate only needs the 8 corners of the unit cell that holds it; their interpolation
// polynomial is cached per lane in LDS and rebuilt from global memory (L1/L2-resident: neighbouring
// samples share nodes) when the iterate changes cell. The state machine's bookkeeping after each
// evaluation is written as selects: loop-carried state updated under divergent branches costs
// register copies at every merge. FP32 arithmetic throughout.
#include <mutex>

#include "vx_refine_math.h"

namespace {

using namespace vxr;

constexpr int REF_THREADS = 256;  // four wavefronts per workgroup
constexpr int REF_CHUNK = 64;     // samples a wavefront claims at a time
constexpr int REF_SPEC = 2;       // trial points a lane may evaluate per pass (sequential rule)
// resident refine_k workgroups per CU at most: with two trial points per pass each wavefront has
// more independent work, and four wavefronts per SIMD beat five (0.65 against 0.67 ms on the 1024^3
// tangle's list, 0.275 against 0.30 ms on the 512^3 one); three were slower (0.70 ms)
constexpr int REF_WG_PER_CU = 4;

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
    unsigned long long *flag;    // nullable: sticky overflow flags, VX_OVERFLOW_REFINE set if count > cap
    int nx, ny, nz;
    int px, py, pz;
    vx_refine_params p;
};

// a wavefront-uniform 64-bit value, made visibly uniform to the compiler (so that loops and
// branches on it stay scalar)
__device__ __forceinline__ int64_t uni64(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
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
                                                        int refill_min, int64_t skip_upto) {
    // cell cache: interpolation coefficient d of the cell cached by thread t at [d][t]
    __shared__ float2 s_corner[8][REF_THREADS];
    constexpr int NF = BATCH ? VX_BATCH_MAX_FRAMES : 1;
    __shared__ vx_ref_frame s_fr[NF];
    __shared__ double s_rnx[NF], s_rnxy[NF];
    __shared__ int64_t s_items[NF], s_cstart[NF + 1];
    const vx_refine_params &P = A.p;
    const int tid = threadIdx.x;
    const int64_t nwaves = (int64_t)gridDim.x * (REF_THREADS / 64);
    const int64_t wave = (int64_t)blockIdx.x * (REF_THREADS / 64) + __builtin_amdgcn_readfirstlane(tid >> 6);
    int64_t n_items = 0;  // single grid: number of samples
    if constexpr (BATCH) {
        // frame table, samples per frame and the prefix of chunks per frame
        if (tid < nframes) {
            const vx_ref_frame F = frames[tid];
            s_fr[tid] = F;
            const int64_t cnt = *F.count;
            const int64_t n = min(cnt, F.cap);
            if (cnt > F.cap && blockIdx.x == 0 && A.flag) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_REFINE);
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
        if (n_items <= skip_upto) return;  // a short list, refined by refine_spec_k (uniform)
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
            // (no early return: it kept the bounds in memory)
            const bool have = ci < s_cstart[nframes];
            int lo = 0, hi = nframes;  // last frame whose first chunk is <= ci
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_cstart[mid] <= ci) lo = mid;
                else hi = mid;
            }
            cf = __builtin_amdgcn_readfirstlane(lo);
            const int64_t nx = uni64((ci - s_cstart[cf]) * REF_CHUNK);
            next = have ? nx : 0;
            end = have ? uni64(min(s_items[cf], nx + REF_CHUNK)) : 0;
            more = more && have;
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
    // a list of at most two chunks per wavefront: the second is the wavefront's by number as well, so
    // that thousands of wavefronts finishing their first chunk together do not queue on the counter
    bool second_static = !BATCH && (n_items + chunk - 1) / chunk <= 2 * nwaves;

    int phase = PH_IDLE, mode = MODE_DESCENT;
    int fr = 0;  // frame of this lane's sample
    int64_t s = 0;
    uint64_t cell = 0;
    uint32_t desc = 0;
    int gi = 0, gj = 0, gk = 0;  // grid node of the sample cell's min corner
    Box box{};                   // the sample's node patch
    int ccode = -1;              // cached cell: (cx+1) + 4 (cy+1) + 16 (cz+1)
    V3 x0 = v3(0.f, 0.f, 0.f), e1 = x0, e2 = x0, xt = x0;
    float y1 = 0.f, y2 = 0.f, ty1 = 0.f, ty2 = 0.f;
    float vr = 0.f, vi = 0.f, f = 0.f;
    V3 gr = x0, gim = x0;
    float s_prev = 0.f, gn = 0.f;           // descent: last accepted length, gradient norm
    float alpha = 0.f, p1 = 0.f, p2 = 0.f;  // current step: length factor and direction
    int dit = 0, nit = 0, hv = 0;  // accepted descent and Newton steps (their sum is reported), halvings
    uint32_t status = 0;
    bool converged = false;
    // the latest evaluation (value and gradient); an idle lane keeps stale values, which it never reads
    float tr = 0.f, ti = 0.f;
    V3 tgr = x0, tgi = x0;

    while (true) {
        // ---- idle lanes claim the next samples of the wave's range, once enough of them are idle
        const uint64_t idle = __ballot(phase == PH_IDLE);
        const int n_idle = __popcll(idle);
        if (next >= end && more && (n_idle >= refill_min || n_idle == 64)) {
            if (second_static) {
                second_static = false;
                claim(wave + nwaves);
                more = false;
            } else {
                unsigned long long c = 0;
                if ((tid & 63) == 0) c = atomicAdd(A.chunks, 1ull);
                claim((int64_t)nwaves + (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)(c >> 32)) << 32) |
                                                  __builtin_amdgcn_readfirstlane((uint32_t)c)));
            }
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
                        box = patch_box(gi, gj, gk, fnx, fny, fnz, fpx, fpy, fpz);
                        ccode = -1;  // force a corner fetch at the first evaluation
                        status = 0;
                        dit = 0;
                        nit = 0;
                        converged = false;
                        x0 = first_estimate(desc, status);
                        if (A.seed) x0 = v3(A.seed[3 * s], A.seed[3 * s + 1], A.seed[3 * s + 2]);
                        xt = x0;
                        phase = PH_INIT;
                    }
                }
            }
            next += (int64_t)n_idle;
        }
        // all lanes idle with nothing left to claim: done. All lanes idle otherwise (nothing claimed
        // yet, or every claimed id out of range) runs the pass below, which leaves idle lanes as they
        // are, and claims again; a second path back to the loop's head would cost a register copy of
        // every loop-carried variable per pass
        if (next >= end && !more && __ballot(phase != PH_IDLE) == 0) break;

        // ---- one trilinear evaluation at the pending point (value and gradient, cell units); lanes
        // waiting to begin a step evaluate too (a point of their patch) and ignore the result
        if (phase != PH_IDLE) {
            int c[3];
            float u[3];
            const int code = locate(xt, box, c, u);
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
                float2 w[8], cf[8];
                fetch_corners(psi_p, fnx, fny, fnz, fpx, fpy, fpz, gi, gj, gk, c, w);
                tri_coeffs(w, cf);
#pragma unroll
                for (int d = 0; d < 8; ++d) s_corner[d][tid] = cf[d];
            }
            float2 v[8];
#pragma unroll
            for (int d = 0; d < 8; ++d) v[d] = s_corner[d][tid];
            trilinear(v, u, tr, ti, tgr, tgi);
        }

        // ---- first evaluation of a sample: plane normal to the pseudo-vorticity at x0
        if (phase == PH_INIT) {
            plane_basis(tgr, tgi, desc, e1, e2, status);
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
        const float fa = rho2(tr, ti);
        bool acc = tri && (descent ? (fa <= f - P.armijo * alpha * gn) : (fa < f));
        // a rejected trial point is followed by the one at half its step, and so on: up to
        // REF_SPEC - 1 of these are evaluated in the same pass, from the cached polynomial, while each
        // lies in the cell just evaluated (inside the patch, within the halving limit and, for Newton,
        // not the current point; other cases are left to the sequential rule of the next pass). The
        // points, tests and halvings are those of the sequential rule, so results do not change; a step
        // that needs one or two halvings costs one pass instead of two or three.
        if (tri && !acc) {
            bool go = true;
#pragma unroll
            for (int q = 1; q < REF_SPEC; ++q) {
                const float ah = 0.5f * alpha;
                const float sy1 = y1 + ah * p1, sy2 = y2 + ah * p2;
                const V3 xs = plane_point(x0, e1, e2, sy1, sy2);
                int cs[3];
                float us[3];
                const int code = locate(xs, box, cs, us);
                go = go && hv + 1 < P.max_halvings && in_patch(xs, box) &&
                     !(mode == MODE_NEWTON && sy1 == y1 && sy2 == y2) && code == ccode;
                if (go) {
                    float2 v[8];
#pragma unroll
                    for (int d = 0; d < 8; ++d) v[d] = s_corner[d][tid];
                    float br, bi;
                    V3 bgr, bgi;
                    trilinear(v, us, br, bi, bgr, bgi);
                    const float fb = rho2(br, bi);
                    alpha = ah;  // the previous point's rejection
                    ++hv;
                    if (descent ? (fb <= f - P.armijo * alpha * gn) : (fb < f)) {
                        tr = br;
                        ti = bi;
                        tgr = bgr;
                        tgi = bgi;
                        ty1 = sy1;
                        ty2 = sy2;
                        acc = true;
                        go = false;
                    }
                }
            }
        }
        const bool take = init || acc;
        const float ft = rho2(tr, ti);  // of the point taken (the first one, or a later one of the pass)
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
        const bool acc_d = acc && descent, acc_n = acc && !descent;
        dit += acc_d ? 1 : 0;
        nit += acc_n ? 1 : 0;
        s_prev = acc_d ? alpha : s_prev;
        const bool conv_now = acc_n && newton_short(alpha, p1, p2, P.newton_tol);
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
            const PlaneJ J = plane_jac(gr, gim, e1, e2);
            if (mode == MODE_DESCENT) {
                if (dit < P.max_descent && f != 0.f) {
                    ok = descent_dir(vr, vi, J, n1, n2, den, gn);
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
                        ok = newton_dir(vr, vi, J, n1, n2, den);
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
                xt = plane_point(x0, e1, e2, ty1, ty2);
                if (in_patch(xt, box)) {
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
            const V3 xe = plane_point(x0, e1, e2, y1, y2);
            o.off[0] = xe.x;
            o.off[1] = xe.y;
            o.off[2] = xe.z;
            o.rho = f;
            o.iters = (uint16_t)min(dit + nit, 65535);
            o.status = (uint16_t)status;
            o.reserved = 0;
            if constexpr (BATCH) s_fr[fr].out[s] = o;
            else A.out[A.out_index ? A.out_index[s] : s] = o;
            phase = PH_IDLE;
        }
    }
}

// Short lists. A list that does not fill the chip (the fallback cells of the surrogate, say) takes
// as long as its slowest sample, and refine_k spends one pass per evaluation: a slowly converging
// descent pays two or three passes per accepted step (the trial at twice the last length, rejected,
// then the halved one). Here a group of SPEC_G lanes runs one sample and evaluates the trial points
// of SPEC_G consecutive halvings of the current step at once (lane h: the length halved h more
// times). The first of them at which the sequential rule stops (accepted, or a Newton step that no
// longer moves the point) decides, and its values are broadcast from its lane, so that a step costs
// one pass; the points outside the patch before it set VX_SAMPLE_BOUNDARY as they would have one at
// a time. Every lane of a group holds the sample's state. The arithmetic is refine_k's: the shared
// functions above, the same expressions for the trial point and the acceptance tests, and halvings
// equal to the same sequence of exact multiplications by 1/2, so the samples are bit-identical to
// refine_k's.
// A lane keeps the interpolation coefficients of the cell of its last evaluation in registers.
constexpr int SPEC_G = 16;

__device__ __forceinline__ float halve_n(float a, int n) {  // n multiplications by 0.5f, n in [0, SPEC_G]
    // each halving of a normal number is exact, so n of them are one exponent change, as long as the
    // result stays normal (a >= 2^-100 covers n <= SPEC_G with room); below that, one at a time
    if (fabsf(a) >= 0x1p-100f) return __builtin_ldexpf(a, -n);
#pragma unroll 1
    for (int j = 0; j < n; ++j) a = 0.5f * a;
    return a;
}

__global__ __launch_bounds__(REF_THREADS) void refine_spec_k(RefArgs A, int64_t run_limit) {
    // the 4x4x4 node patch of each group's sample, node (a, b, c) at a + 4 b + 16 c (offsets -1 .. 2)
    __shared__ float2 s_patch[REF_THREADS / SPEC_G][64];
    const int tid = threadIdx.x, lane = tid & 63, h = lane & (SPEC_G - 1), gl = lane - h;
    float2 *patch = s_patch[tid / SPEC_G];
    const int64_t cnt = *A.count;
    if (blockIdx.x == 0 && tid == 0) {
        *A.chunks = 0ull;  // chunk counter of the refine_k launch that follows
        if (cnt > A.cap && A.flag) atomicOr(A.flag, (unsigned long long)VX_OVERFLOW_REFINE);
    }
    const int64_t n = min(cnt, A.cap);
    if (n > run_limit) return;  // a long list, refined by refine_k (uniform)
    const vx_refine_params &P = A.p;
    const int64_t ngroups = (int64_t)gridDim.x * (REF_THREADS / SPEC_G);
    const uint64_t nx64 = (uint64_t)A.nx, nxy = nx64 * (uint64_t)A.ny;
    const double rnx = 1.0 / (double)A.nx, rnxy = 1.0 / ((double)A.nx * (double)A.ny);
    for (int64_t s = (int64_t)blockIdx.x * (REF_THREADS / SPEC_G) + tid / SPEC_G; s < n; s += ngroups) {
        const uint64_t cell = A.cells[s];
        const uint32_t desc = A.desc[s];
        vx_sample *dst = A.out + (A.out_index ? A.out_index[s] : s);
        if (cell >= nxy * (uint64_t)A.nz) {
            if (h == 0) {
                vx_sample o{};
                o.cell = cell;
                o.rho = -1.f;
                o.status = (uint16_t)VX_SAMPLE_BAD_CELL;
                *dst = o;
            }
            continue;
        }
        uint64_t rxy, ri;
        const int gk = (int)divmod53(cell, nxy, rnxy, rxy);
        const int gj = (int)divmod53(rxy, nx64, rnx, ri);
        const int gi = (int)ri;
        const Box box = patch_box(gi, gj, gk, A.nx, A.ny, A.nz, A.px, A.py, A.pz);
        // the whole patch at once (lane h: row h, x offsets -1 .. 2), so that a cell change costs an
        // LDS read instead of a round trip to memory; the nodes are those fetch_corners would read
        {
            const uint32_t jj = wrap(gj, (h & 3) - 1, A.ny, A.py), kk = wrap(gk, (h >> 2) - 1, A.nz, A.pz);
            const float2 *row = A.psi + nx64 * jj + nxy * kk;
#pragma unroll
            for (int a = 0; a < 4; ++a) patch[4 * h + a] = row[wrap(gi, a - 1, A.nx, A.px)];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        uint32_t status = 0;
        V3 x0 = first_estimate(desc, status);
        if (A.seed) x0 = v3(A.seed[3 * s], A.seed[3 * s + 1], A.seed[3 * s + 2]);
        int ccode = -1;
        float2 cw[8];
        auto eval = [&](const V3 &xt, float &tr, float &ti, V3 &tgr, V3 &tgi) {
            int c[3];
            float u[3];
            const int code = locate(xt, box, c, u);
            if (code != ccode) {
                ccode = code;
                const int base = (c[0] + 1) + 4 * (c[1] + 1) + 16 * (c[2] + 1);
                float2 w[8];
#pragma unroll
                for (int d = 0; d < 8; ++d) w[d] = patch[base + (d & 1) + 4 * ((d >> 1) & 1) + 16 * (d >> 2)];
                tri_coeffs(w, cw);
            }
            trilinear(cw, u, tr, ti, tgr, tgi);
        };
        // first evaluation, at x0 (every lane of the group), and the plane of the search
        float tr, ti;
        V3 tgr, tgi, e1, e2;
        eval(x0, tr, ti, tgr, tgi);
        plane_basis(tgr, tgi, desc, e1, e2, status);
        float y1 = 0.f, y2 = 0.f, vr = tr, vi = ti;
        V3 gr = tgr, gim = tgi;
        float f = rho2(tr, ti);
        float s_prev = 0.5f * P.step0, gn = 0.f;
        float alpha = 0.f, p1 = 0.f, p2 = 0.f;  // current step: length at halving hv, direction
        int mode = MODE_DESCENT, dit = 0, nit = 0, hv = 0;
        bool converged = false, done = false;
        // start a step of the current kind (a descent that cannot start hands over to Newton at
        // once), or end the sample
        auto begin = [&]() {
            float n1 = 0.f, n2 = 0.f, den = 1.f;
            bool ok = false;
            const PlaneJ J = plane_jac(gr, gim, e1, e2);
            if (mode == MODE_DESCENT) {
                if (dit < P.max_descent && f != 0.f) {
                    ok = descent_dir(vr, vi, J, n1, n2, den, gn);
                    alpha = fminf(2.f * s_prev, P.step_max);
                }
                if (!ok) mode = MODE_NEWTON;
            }
            if (mode == MODE_NEWTON) {
                if (nit < P.max_newton) {
                    if (f == 0.f) {
                        converged = true;
                    } else {
                        ok = newton_dir(vr, vi, J, n1, n2, den);
                        alpha = 1.f;
                    }
                }
                if (!ok) done = true;
            }
            if (ok) {
                p1 = n1 * den;
                p2 = n2 * den;
                hv = 0;
            }
        };
        begin();
        while (!done) {
            const float a = halve_n(alpha, h);
            const float ty1 = y1 + a * p1;
            const float ty2 = y2 + a * p2;
            const V3 xt = plane_point(x0, e1, e2, ty1, ty2);
            const bool valid = hv + h < P.max_halvings;
            const bool inside = valid && in_patch(xt, box);
            const bool stuck = inside && mode == MODE_NEWTON && ty1 == y1 && ty2 == y2;
            // a lane that does not evaluate keeps stale values, which are never taken: only an
            // accepting lane's are broadcast
            if (inside && !stuck) eval(xt, tr, ti, tgr, tgi);
            const float ft = rho2(tr, ti);
            const bool descent = mode == MODE_DESCENT;
            const bool acc = inside && !stuck && (descent ? (ft <= f - P.armijo * a * gn) : (ft < f));
            const uint32_t res = (uint32_t)(__ballot(stuck || acc) >> gl) & ((1u << SPEC_G) - 1u);
            const uint32_t outside = (uint32_t)(__ballot(valid && !inside) >> gl) & ((1u << SPEC_G) - 1u);
            if (res) {
                const int hs = __builtin_ctz(res), src = gl + hs;
                if (outside & ((1u << hs) - 1u)) status |= VX_SAMPLE_BOUNDARY;
                if (__shfl((int)stuck, src)) {
                    done = true;
                } else {
                    const float aa = __shfl(a, src);
                    y1 = __shfl(ty1, src);
                    y2 = __shfl(ty2, src);
                    vr = __shfl(tr, src);
                    vi = __shfl(ti, src);
                    gr = v3(__shfl(tgr.x, src), __shfl(tgr.y, src), __shfl(tgr.z, src));
                    gim = v3(__shfl(tgi.x, src), __shfl(tgi.y, src), __shfl(tgi.z, src));
                    f = __shfl(ft, src);
                    if (descent) {
                        ++dit;
                        s_prev = aa;
                    } else {
                        ++nit;
                    }
                    const bool conv_now = !descent && newton_short(aa, p1, p2, P.newton_tol);
                    converged = converged || conv_now;
                    if (descent && aa < P.descent_tol) mode = MODE_NEWTON;
                    if (conv_now) done = true;
                    else begin();
                }
            } else {
                if (outside) status |= VX_SAMPLE_BOUNDARY;
                hv += SPEC_G;
                alpha = halve_n(alpha, SPEC_G);
                if (hv >= P.max_halvings) {
                    if (mode == MODE_DESCENT) {
                        mode = MODE_NEWTON;
                        begin();
                    } else {
                        done = true;
                    }
                }
            }
        }
        if (h == 0) {
            if (f > P.rho_tol) status |= VX_SAMPLE_NONZERO_MIN;
            if (!converged && f > P.rho_tol) status |= VX_SAMPLE_NOT_CONVERGED;
            vx_sample o;
            o.cell = cell;
            const V3 xe = plane_point(x0, e1, e2, y1, y2);
            o.off[0] = xe.x;
            o.off[1] = xe.y;
            o.off[2] = xe.z;
            o.rho = f;
            o.iters = (uint16_t)min(dit + nit, 65535);
            o.status = (uint16_t)status;
            o.reserved = 0;
            *dst = o;
        }
    }
}

__global__ void zero_u64_k(unsigned long long *p) { *p = 0ull; }

// resident workgroups per CU of a refinement kernel (at least 1); -1 on error
template <typename K>
int occupancy(K kernel) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, REF_THREADS, 0) != hipSuccess) return -1;
    return nb > 0 ? nb : 1;
}

// resident workgroups per CU of refine_k: what fits, at most REF_WG_PER_CU; -1 on error
int long_per_cu() {
    const int r = occupancy(refine_k<false>);
    return r < 0 ? -1 : std::min(r, REF_WG_PER_CU);
}

// one resident round of wavefronts (they claim chunks dynamically, at most REF_WG_PER_CU workgroups
// per CU); fewer for short lists; -1 on error
template <typename K>
int64_t ref_blocks(vx_handle *h, K kernel, int &per_cu, int64_t cap) {
    if (per_cu <= 0) {
        per_cu = occupancy(kernel);
        if (per_cu > REF_WG_PER_CU) per_cu = REF_WG_PER_CU;
        if (per_cu < 0) {
            vx_fail(h, VX_ERR_DEVICE, "refinement kernel occupancy query failed");
            return -1;
        }
    }
    const int64_t resident = (int64_t)per_cu * (h->num_cu > 0 ? h->num_cu : 256);
    const int64_t need = (cap + 4 * REF_CHUNK - 1) / (4 * REF_CHUNK);  // >= one chunk per wavefront
    return std::max<int64_t>(1, std::min(need, resident));
}

// What a launch of the two kernels of one list needs to know about the device.
struct RefCfg {
    int num_cu;       // compute units
    int ref_per_cu;   // resident refine_k workgroups per CU
    int spec_per_cu;  // resident refine_spec_k workgroups per CU
    int refill;       // idle lanes a refine_k wavefront waits for before claiming samples
};

// The number of samples is known on the device only: refine_spec_k takes lists of at most one
// sample per resident group and zeroes the chunk counter A.chunks, refine_k (if the capacity allows a
// longer list) the others; each returns at once when the list is not its own.
hipError_t refine_enqueue(const RefCfg &c, const RefArgs &A, int64_t cap, hipStream_t s) {
    const int64_t resident = (int64_t)c.ref_per_cu * c.num_cu;
    const int64_t need = (cap + 4 * REF_CHUNK - 1) / (4 * REF_CHUNK);  // >= one chunk per wavefront
    const int64_t blocks = std::max<int64_t>(1, std::min(need, resident));
    const int64_t sblocks = (int64_t)c.spec_per_cu * c.num_cu;
    constexpr int64_t GPB = REF_THREADS / SPEC_G;  // groups per workgroup
    const int64_t limit = sblocks * GPB;
    const bool short_only = cap <= limit;
    const int64_t sgrid = std::max<int64_t>(1, std::min(sblocks, (cap + GPB - 1) / GPB));
    hipLaunchKernelGGL(refine_spec_k, dim3((unsigned)sgrid), dim3(REF_THREADS), 0, s, A,
                       short_only ? INT64_MAX : limit);
    if (!short_only)
        hipLaunchKernelGGL(refine_k<false>, dim3((unsigned)blocks), dim3(REF_THREADS), 0, s, A,
                           (const vx_ref_frame *)nullptr, 1, c.refill, limit);
    return hipGetLastError();
}

RefArgs make_args(const vx_dims &d, const void *psi, const uint64_t *cells, const uint16_t *desc, const float *seed,
                  const int64_t *count, int64_t cap, const vx_refine_params &p, vx_sample *out,
                  const int64_t *out_index, unsigned long long *chunks, unsigned long long *flag) {
    RefArgs A;
    A.out_index = out_index;
    A.psi = (const float2 *)psi;
    A.cells = cells;
    A.desc = desc;
    A.seed = seed;
    A.count = count;
    A.cap = cap;
    A.out = out;
    A.chunks = chunks;
    A.flag = flag;
    A.nx = d.nx;
    A.ny = d.ny;
    A.nz = d.nz;
    A.px = (int)(d.periodic & 1u);
    A.py = (int)((d.periodic >> 1) & 1u);
    A.pz = (int)((d.periodic >> 2) & 1u);
    A.p = p;
    return A;
}

}  // namespace

vx_status vx_refine_launch(vx_handle *h, const vx_dims &d, const void *psi, const uint64_t *cells,
                           const uint16_t *desc, const float *seed, const int64_t *count, int64_t cap,
                           const vx_refine_params &p, vx_sample *out, hipStream_t s, const int64_t *out_index) {
    if (h->ref_blocks_per_cu <= 0) h->ref_blocks_per_cu = long_per_cu();
    if (h->refs_blocks_per_cu <= 0) h->refs_blocks_per_cu = occupancy(refine_spec_k);
    if (h->ref_blocks_per_cu < 0 || h->refs_blocks_per_cu < 0)
        return vx_fail(h, VX_ERR_DEVICE, "refinement kernel occupancy query failed");
    const RefCfg c{h->num_cu > 0 ? h->num_cu : 256, h->ref_blocks_per_cu, h->refs_blocks_per_cu, h->ref_refill};
    const RefArgs A = make_args(d, psi, cells, desc, seed, count, cap, p, out, out_index, h->d_work, vx_overflow_flag(h));
    vx_timer tm(h, s, VX_KIND_REFINE);
    const hipError_t e = refine_enqueue(c, A, cap, s);
    tm.stop();
    return vx_hip_check(h, e, "refine launch");
}

int vx_refine_batch_max_wg(vx_handle *h) {
    (void)h;
    return occupancy(refine_k<true>);
}

vx_status vx_refine_batch_enqueue(vx_handle *h, const vx_ref_frame *d_frames, int nframes, int64_t total_cap,
                                  const vx_refine_params &p, unsigned long long *d_counter, int wg_per_cu,
                                  hipStream_t s) {
    if (nframes < 1 || nframes > VX_BATCH_MAX_FRAMES)
        return vx_fail(h, VX_ERR_INVALID, "refine batch: %d frames", nframes);
    RefArgs A{};
    A.chunks = d_counter;
    A.flag = vx_overflow_flag(h);
    A.p = p;
    int64_t blocks = ref_blocks(h, refine_k<true>, h->refb_blocks_per_cu, total_cap);
    if (blocks < 0) return VX_ERR_DEVICE;
    if (wg_per_cu > 0) {  // the batch's own choice, within what fits
        const int64_t resident = (int64_t)std::min(wg_per_cu, occupancy(refine_k<true>)) * (h->num_cu > 0 ? h->num_cu : 256);
        const int64_t need = (total_cap + 4 * REF_CHUNK - 1) / (4 * REF_CHUNK);
        blocks = std::max<int64_t>(1, std::min(need, resident));
    }
    hipLaunchKernelGGL(zero_u64_k, dim3(1), dim3(1), 0, s, d_counter);
    hipLaunchKernelGGL(refine_k<true>, dim3((unsigned)blocks), dim3(REF_THREADS), 0, s, A, d_frames, nframes,
                       h->ref_refill, (int64_t)-1);
    return vx_hip_check(h, hipGetLastError(), "refine_k batch launch");
}

// ---------------------------------------------------------------------------------------------
// Refinement without any allocation (vx_refine_noalloc): the scratch that vx_refine keeps in the
// handle's workspace -- the chunk counter that refine_spec_k zeroes and refine_k's wavefronts claim
// work from -- lives here in a fixed device array instead, one copy per device. Its device address
// is looked up once per device (the array's name is a host-side stand-in in host code and must never
// be passed to a kernel), together with the occupancy figures the launch needs, so that a call
// makes no allocation and no handle is needed.
namespace {

constexpr int NOALLOC_SCRATCH_WORDS = 32;  // 256 bytes; word 0 = chunk counter
static __device__ __align__(256) unsigned long long scratch[NOALLOC_SCRATCH_WORDS];

constexpr int NOALLOC_MAX_DEVICES = 64;
struct NoallocDev {
    bool ready = false;
    unsigned long long *scratch = nullptr;  // device address of this device's copy of `scratch`
    RefCfg cfg{};
};
std::mutex g_noalloc_mu;
NoallocDev g_noalloc[NOALLOC_MAX_DEVICES];

// Set-up of the current device (its first call): the scratch array's device address and the launch
// figures. Returns VX_OK or an error status.
vx_status noalloc_setup(int dev, NoallocDev &nd) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || ptr == nullptr) return VX_ERR_DEVICE;
    int num_cu = 0;
    if (hipDeviceGetAttribute(&num_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || num_cu <= 0)
        return VX_ERR_DEVICE;
    const int r = long_per_cu(), sp = occupancy(refine_spec_k);
    if (r < 0 || sp < 0) return VX_ERR_DEVICE;
    nd.scratch = (unsigned long long *)ptr;
    nd.cfg = RefCfg{num_cu, r, sp, 8};
    nd.ready = true;
    return VX_OK;
}

}  // namespace

extern "C" vx_status vx_refine_noalloc(vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                                       const uint16_t *d_cell_desc, const float *d_seed_off, const int64_t *d_count,
                                       int64_t cap, const vx_refine_params *p, vx_sample *d_out, vx_stream s) {
    if (vx_check_dims(nullptr, dims) != VX_OK) return VX_ERR_INVALID;
    if (cap < 0) return VX_ERR_INVALID;
    if (cap == 0) return VX_OK;
    if (!d_psi || !d_cells || !d_cell_desc || !d_count || !d_out) return VX_ERR_INVALID;
    const vx_refine_params prm = p ? *p : vx_refine_defaults();
    if (vx_check_refine_params(nullptr, prm) != VX_OK) return VX_ERR_INVALID;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return VX_ERR_DEVICE;
    if (dev >= NOALLOC_MAX_DEVICES) return VX_ERR_UNSUPPORTED;
    RefCfg cfg;
    unsigned long long *scr;
    {
        std::lock_guard<std::mutex> lock(g_noalloc_mu);
        NoallocDev &nd = g_noalloc[dev];
        if (!nd.ready)
            if (vx_status st = noalloc_setup(dev, nd)) return st;
        cfg = nd.cfg;
        scr = nd.scratch;
    }
    const RefArgs A = make_args(dims, d_psi, d_cells, d_cell_desc, d_seed_off, d_count, cap, prm, d_out, nullptr, scr,
                                nullptr);
    return refine_enqueue(cfg, A, cap, (hipStream_t)s) == hipSuccess ? VX_OK : VX_ERR_DEVICE;
}
