// Batching of many grids (a time series of frames of uneven size) and the z-chunk autotuner.
//
// A batch owns three small device tables built once at creation: the winding arguments of every
// frame, the prefix of their tile counts, and the refinement description of every frame that has a
// sample buffer. Its work is two kernel launches (plus two one-thread counter resets): the winding
// of all tiles of all frames, then the refinement of all listed cells of all frames. They are
// captured into a HIP graph on a private stream and replayed with one hipGraphLaunch. Counters are
// reset by small kernels, never by memset nodes.
//
// The autotuner picks the planes marched per wavefront (z-chunk depth) of the winding kernel. Deeper
// chunks re-read fewer halo planes; shallower ones make more tiles, which a lone small grid needs to
// fill the GPU but a batch does not. For a batch it then picks the refinement's resident workgroups
// per CU (more hide latency; fewer leave each wavefront's lanes more cache and issue slots), timing
// the refinement of the batch's own lists. Candidates are timed with HIP events; z-chunk results can
// be kept in a JSON-lines cache file.
#include <algorithm>
#include <cstring>
#include <fstream>
#include <new>
#include <set>
#include <sstream>

#include "vx_internal.h"

struct vx_batch {
    vx_handle *h = nullptr;
    std::vector<vx_frame> frames;
    vx_refine_params p{};
    std::vector<int> zc;  // planes per z-chunk of each frame
    int ref_wg = 0;       // resident refinement workgroups per CU (0: the library's default)
    int wind_wg = 0;      // resident winding workgroups per CU (0: as many as fit)
    int wind_pad = 0;     // the dynamic LDS per winding workgroup that caps them there
    vx_wind_args *d_wargs = nullptr;
    int *d_tile_start = nullptr;
    vx_ref_frame *d_rframes = nullptr;
    int n_ref = 0;
    int64_t total_tiles = 0;
    int64_t total_cap = 0;
    unsigned long long *d_counter = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

constexpr int TUNE_CANDIDATES[] = {8, 16, 32, 64, 128};
constexpr int BATCH_DEFAULT_ZC = 32;

using Key = std::array<int, 4>;  // nx, ny, nz, periodic
Key key_of(const vx_dims &d) { return {d.nx, d.ny, d.nz, (int)d.periodic}; }

std::vector<int> candidates(int nz) {
    std::vector<int> c;
    for (int z : TUNE_CANDIDATES)
        if (z <= std::max(nz, 8)) c.push_back(z);
    if (c.empty()) c.push_back(nz);
    return c;
}

// ---- JSON-lines cache: {"kind": "...", "dims": [nx, ny, nz], "periodic": p, "zchunk": z, ...}
bool parse_line(const std::string &line, std::string &kind, Key &k, int &zc) {
    auto field = [&](const char *name) -> const char * {
        const size_t at = line.find(name);
        return at == std::string::npos ? nullptr : line.c_str() + at + std::strlen(name);
    };
    const char *pk = field("\"kind\": \"");
    const char *pd = field("\"dims\": [");
    const char *pp = field("\"periodic\": ");
    const char *pz = field("\"zchunk\": ");
    if (!pk || !pd || !pp || !pz) return false;
    const char *q = std::strchr(pk, '"');
    if (!q) return false;
    kind.assign(pk, q);
    if (std::sscanf(pd, "%d , %d , %d", &k[0], &k[1], &k[2]) != 3) return false;
    if (std::sscanf(pp, "%d", &k[3]) != 1 || std::sscanf(pz, "%d", &zc) != 1) return false;
    return zc > 0;
}

std::map<Key, int> read_cache(const char *path, const char *kind) {
    std::map<Key, int> m;
    if (!path) return m;
    std::ifstream in(path);
    std::string line, k;
    Key key;
    int zc;
    while (std::getline(in, line))
        if (parse_line(line, k, key, zc) && k == kind) m[key] = zc;
    return m;
}

void append_cache(const char *path, const char *kind, const Key &k, int zc, double ms) {
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    out << "{\"kind\": \"" << kind << "\", \"dims\": [" << k[0] << ", " << k[1] << ", " << k[2]
        << "], \"periodic\": " << k[3] << ", \"zchunk\": " << zc << ", \"ms\": " << ms << "}\n";
}

// median duration (ms) of `reps` runs of fn on stream s after one warm-up
template <typename F>
vx_status time_median(vx_handle *h, hipStream_t s, int reps, F fn, double *ms_out) {
    hipEvent_t a, b;
    if (vx_status st = vx_hip_check(h, hipEventCreate(&a), "hipEventCreate")) return st;
    if (vx_status st = vx_hip_check(h, hipEventCreate(&b), "hipEventCreate")) {
        (void)hipEventDestroy(a);
        return st;
    }
    std::vector<double> t;
    vx_status st = fn();
    for (int i = 0; i < reps && st == VX_OK; ++i) {
        st = vx_hip_check(h, hipEventRecord(a, s), "hipEventRecord");
        if (st == VX_OK) st = fn();
        if (st == VX_OK) st = vx_hip_check(h, hipEventRecord(b, s), "hipEventRecord");
        if (st == VX_OK) st = vx_hip_check(h, hipEventSynchronize(b), "hipEventSynchronize");
        float ms = 0.f;
        if (st == VX_OK) st = vx_hip_check(h, hipEventElapsedTime(&ms, a, b), "hipEventElapsedTime");
        t.push_back(ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st) return st;
    std::sort(t.begin(), t.end());
    *ms_out = t[t.size() / 2];
    return VX_OK;
}

// build the tables for the current z-chunk depths and copy them to the device (synchronous)
vx_status upload(vx_batch *b) {
    vx_handle *h = b->h;
    const int n = (int)b->frames.size();
    std::vector<vx_wind_args> wa(n);
    std::vector<int> start(n + 1, 0);
    int64_t total = 0;
    for (int f = 0; f < n; ++f) {
        const vx_frame &F = b->frames[f];
        int64_t nt = 0;
        if (vx_status st = vx_wind_make_args(h, F.dims, F.d_psi, F.out, b->zc[f], &wa[f], &nt)) return st;
        start[f] = (int)total;
        total += nt;
        if (total > 2147483647LL) return vx_fail(h, VX_ERR_UNSUPPORTED, "vx_batch: too many tiles");
    }
    start[n] = (int)total;
    b->total_tiles = total;
    std::vector<vx_ref_frame> rf;
    int64_t cap = 0;
    for (const vx_frame &F : b->frames) {
        if (!F.d_samples || F.sample_cap <= 0 || F.out.cell_cap <= 0) continue;
        vx_ref_frame r;
        r.psi = (const float2 *)F.d_psi;
        r.cells = F.out.d_cells;
        r.desc = F.out.d_cell_desc;
        r.count = F.out.d_counts + 1;
        r.cap = std::min(F.sample_cap, F.out.cell_cap);
        r.out = F.d_samples;
        r.nx = F.dims.nx;
        r.ny = F.dims.ny;
        r.nz = F.dims.nz;
        r.periodic = F.dims.periodic;
        cap += r.cap;
        rf.push_back(r);
    }
    b->n_ref = (int)rf.size();
    b->total_cap = cap;
    if (vx_status st = vx_hip_check(h, hipMemcpy(b->d_wargs, wa.data(), n * sizeof(vx_wind_args), hipMemcpyHostToDevice),
                                    "vx_batch: table copy"))
        return st;
    if (vx_status st = vx_hip_check(h, hipMemcpy(b->d_tile_start, start.data(), (n + 1) * sizeof(int),
                                                 hipMemcpyHostToDevice),
                                    "vx_batch: table copy"))
        return st;
    if (!rf.empty())
        return vx_hip_check(h, hipMemcpy(b->d_rframes, rf.data(), rf.size() * sizeof(vx_ref_frame), hipMemcpyHostToDevice),
                            "vx_batch: table copy");
    return VX_OK;
}

vx_status enqueue_wind(vx_batch *b, hipStream_t s) {
    return vx_wind_batch_enqueue(b->h, b->d_wargs, b->d_tile_start, (int)b->frames.size(), b->total_tiles,
                                 b->wind_pad, s);
}

// timed: record the winding and refinement launches separately (eager launches only, never inside
// a capture)
vx_status enqueue(vx_batch *b, hipStream_t s, bool timed = false) {
    {
        vx_timer tm(b->h, s, timed ? VX_KIND_WIND : -1);
        const vx_status st = enqueue_wind(b, s);
        tm.stop();
        if (st) return st;
    }
    if (b->n_ref == 0) return VX_OK;
    vx_timer tm(b->h, s, timed ? VX_KIND_REFINE : -1);
    const vx_status st =
        vx_refine_batch_enqueue(b->h, b->d_rframes, b->n_ref, b->total_cap, b->p, b->d_counter, b->ref_wg, s);
    tm.stop();
    return st;
}

vx_status capture(vx_batch *b) {
    vx_handle *h = b->h;
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    hipStream_t cs;
    if (vx_status st = vx_hip_check(h, hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate"))
        return st;
    vx_status st = vx_hip_check(h, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    if (st == VX_OK) {
        const vx_status est = enqueue(b, cs);
        hipGraph_t g = nullptr;
        st = vx_hip_check(h, hipStreamEndCapture(cs, &g), "hipStreamEndCapture");
        if (st == VX_OK) st = est;
        if (st == VX_OK) {
            b->graph = g;
            st = vx_hip_check(h, hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0), "hipGraphInstantiate");
        } else if (g) {
            (void)hipGraphDestroy(g);
        }
    }
    (void)hipStreamDestroy(cs);
    return st;
}

void release(vx_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->d_wargs) (void)hipFree(b->d_wargs);
    if (b->d_tile_start) (void)hipFree(b->d_tile_start);
    if (b->d_rframes) (void)hipFree(b->d_rframes);
    if (b->d_counter) (void)hipFree(b->d_counter);
    delete b;
}

}  // namespace

extern "C" vx_status vx_batch_create(vx_handle *h, const vx_frame *frames, int nframes, const vx_refine_params *p,
                                     vx_batch **out) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (!out) return vx_fail(h, VX_ERR_INVALID, "vx_batch_create: null out");
    *out = nullptr;
    if (!frames || nframes < 1 || nframes > VX_BATCH_MAX_FRAMES)
        return vx_fail(h, VX_ERR_INVALID, "vx_batch_create: nframes = %d (1..%d)", nframes, VX_BATCH_MAX_FRAMES);
    const vx_refine_params prm = p ? *p : vx_refine_defaults();
    if (vx_status st = vx_check_refine_params(h, prm)) return st;
    for (int f = 0; f < nframes; ++f) {
        if (vx_status st = vx_check_winding(h, frames[f].dims, frames[f].d_psi, &frames[f].out, "vx_batch_create"))
            return vx_fail(h, st, "vx_batch_create: frame %d: %s", f, h->err.c_str());
        if (frames[f].sample_cap < 0)
            return vx_fail(h, VX_ERR_INVALID, "vx_batch_create: frame %d: negative sample_cap", f);
    }
    if (vx_status st = vx_bind(h)) return st;
    vx_batch *b = new (std::nothrow) vx_batch();
    if (!b) return VX_ERR_NOMEM;
    b->h = h;
    b->frames.assign(frames, frames + nframes);
    b->p = prm;
    b->zc.resize(nframes);
    for (int f = 0; f < nframes; ++f) {
        const auto it = h->tuned_zc.find(key_of(frames[f].dims));
        b->zc[f] = it != h->tuned_zc.end() ? it->second : std::min(BATCH_DEFAULT_ZC, frames[f].dims.nz);
    }
    vx_status st = vx_hip_check(h, hipMalloc((void **)&b->d_wargs, nframes * sizeof(vx_wind_args)), "hipMalloc");
    if (st == VX_OK) st = vx_hip_check(h, hipMalloc((void **)&b->d_tile_start, (nframes + 1) * sizeof(int)), "hipMalloc");
    if (st == VX_OK) st = vx_hip_check(h, hipMalloc((void **)&b->d_rframes, nframes * sizeof(vx_ref_frame)), "hipMalloc");
    if (st == VX_OK) st = vx_hip_check(h, hipMalloc((void **)&b->d_counter, 256), "hipMalloc");
    if (st == VX_OK) st = upload(b);
    if (st == VX_OK) st = capture(b);
    if (st) {
        release(b);
        return st;
    }
    *out = b;
    return VX_OK;
}

extern "C" vx_status vx_batch_launch(vx_batch *b, vx_stream s) {
    if (!b) return VX_ERR_INVALID;
    vx_handle *h = b->h;
    h->err.clear();
    if (vx_status st = vx_bind(h)) return st;
    vx_timer tm(h, (hipStream_t)s, VX_KIND_BATCH);
    const vx_status st = vx_hip_check(h, hipGraphLaunch(b->exec, (hipStream_t)s), "hipGraphLaunch");
    tm.stop();
    return st;
}

extern "C" vx_status vx_batch_launch_eager(vx_batch *b, vx_stream s) {
    if (!b) return VX_ERR_INVALID;
    vx_handle *h = b->h;
    h->err.clear();
    if (vx_status st = vx_bind(h)) return st;
    vx_timer tm(h, (hipStream_t)s, VX_KIND_BATCH);
    const vx_status st = enqueue(b, (hipStream_t)s, true);
    tm.stop();
    return st;
}

extern "C" vx_status vx_batch_zchunk(const vx_batch *b, int frame, int *zchunk) {
    if (!b || !zchunk || frame < 0 || frame >= (int)b->frames.size()) return VX_ERR_INVALID;
    *zchunk = b->zc[frame];
    return VX_OK;
}

extern "C" vx_status vx_batch_refine_wg(const vx_batch *b, int *wg_per_cu) {
    if (!b || !wg_per_cu) return VX_ERR_INVALID;
    *wg_per_cu = b->ref_wg;
    return VX_OK;
}

extern "C" vx_status vx_batch_wind_wg(const vx_batch *b, int *wg_per_cu) {
    if (!b || !wg_per_cu) return VX_ERR_INVALID;
    *wg_per_cu = b->wind_wg;
    return VX_OK;
}

extern "C" vx_status vx_batch_autotune(vx_batch *b, const char *cache_path, vx_stream s) {
    if (!b) return VX_ERR_INVALID;
    vx_handle *h = b->h;
    h->err.clear();
    if (vx_status st = vx_bind(h)) return st;
    hipStream_t hs = (hipStream_t)s;
    const std::map<Key, int> cached = read_cache(cache_path, "batch");
    std::vector<Key> todo;
    std::set<Key> seen;
    for (size_t f = 0; f < b->frames.size(); ++f) {
        const Key k = key_of(b->frames[f].dims);
        const auto it = cached.find(k);
        if (it != cached.end()) b->zc[f] = it->second;
        else if (seen.insert(k).second) todo.push_back(k);
    }
    const bool prof = h->profile;
    h->profile = false;  // tuning launches are not part of the caller's timing
    vx_status st = VX_OK;
    // coordinate descent over the frame sizes, timing the whole batch's winding: each size takes the
    // depth that is fastest with the others at their current depths; a second sweep revisits every
    // size once the others have settled (the gain of one size's depth is a small part of the batch)
    std::map<Key, double> best_ms;
    for (int sweep = 0; sweep < 2 && st == VX_OK; ++sweep) {
        for (const Key &k : todo) {
            int best_zc = 0;
            double best = 1e30;
            for (int cand : candidates(k[2])) {
                for (size_t f = 0; f < b->frames.size(); ++f)
                    if (key_of(b->frames[f].dims) == k) b->zc[f] = cand;
                st = upload(b);
                double ms = 0.0;
                if (st == VX_OK) st = time_median(h, hs, 7, [&] { return enqueue_wind(b, hs); }, &ms);
                if (st) break;
                if (ms < best) {
                    best = ms;
                    best_zc = cand;
                }
            }
            if (st) break;
            for (size_t f = 0; f < b->frames.size(); ++f)
                if (key_of(b->frames[f].dims) == k) b->zc[f] = best_zc;
            best_ms[k] = best;
        }
    }
    if (st == VX_OK)
        for (const Key &k : todo) {
            int zc = 0;
            for (size_t f = 0; f < b->frames.size(); ++f)
                if (key_of(b->frames[f].dims) == k) zc = b->zc[f];
            append_cache(cache_path, "batch", k, zc, best_ms[k]);
        }
    if (st == VX_OK) st = upload(b);
    // resident winding workgroups per CU with the chosen depths: as many as fit and one or two fewer
    // (fewer keep more of the halo lines that neighbouring tiles share in L2, more hide more latency)
    if (st == VX_OK) {
        const int top = vx_wind_batch_max_wg(h);
        int best_wg = 0, best_pad = 0;
        double best = 1e30;
        for (int wg = top; st == VX_OK && wg >= std::max(1, top - 2); --wg) {
            b->wind_pad = wg == top ? 0 : vx_wind_batch_pad(h, wg);
            double ms = 0.0;
            st = time_median(h, hs, 7, [&] { return enqueue_wind(b, hs); }, &ms);
            if (st == VX_OK && ms < best) {
                best = ms;
                best_wg = wg;
                best_pad = b->wind_pad;
            }
        }
        if (top < 1 && st == VX_OK) st = vx_fail(h, VX_ERR_DEVICE, "vx_batch_autotune: winding occupancy query failed");
        b->wind_wg = best_wg;
        b->wind_pad = best_pad;
    }
    // resident refinement workgroups per CU, on the lists of one winding with the chosen depths
    if (st == VX_OK && b->n_ref > 0) {
        st = enqueue_wind(b, hs);
        const int top = vx_refine_batch_max_wg(h);
        int best_wg = 0;
        double best = 1e30;
        for (int wg = 2; st == VX_OK && wg <= top; ++wg) {
            double ms = 0.0;
            st = time_median(h, hs, 7, [&] {
                return vx_refine_batch_enqueue(h, b->d_rframes, b->n_ref, b->total_cap, b->p, b->d_counter, wg, hs);
            }, &ms);
            if (st == VX_OK && ms < best) {
                best = ms;
                best_wg = wg;
            }
        }
        if (st == VX_OK) b->ref_wg = best_wg;
    }
    h->profile = prof;
    if (st == VX_OK) st = capture(b);
    return st;
}

extern "C" vx_status vx_batch_destroy(vx_batch *b) {
    if (!b) return VX_OK;
    (void)vx_bind(b->h);
    release(b);
    return VX_OK;
}

extern "C" vx_status vx_autotune(vx_handle *h, vx_dims dims, const void *d_psi, const char *cache_path, int *zchunk,
                                 vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (!d_psi) return vx_fail(h, VX_ERR_INVALID, "vx_autotune: null psi");
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (((uintptr_t)d_psi & 7u) != 0) return vx_fail(h, VX_ERR_INVALID, "vx_autotune: psi must be 8-byte aligned");
    if (vx_status st = vx_bind(h)) return st;
    const Key k = key_of(dims);
    const std::map<Key, int> cached = read_cache(cache_path, "grid");
    const auto it = cached.find(k);
    if (it != cached.end()) {
        h->tuned_zc[k] = it->second;
        if (zchunk) *zchunk = it->second;
        return VX_OK;
    }
    // scratch outputs shaped like a real call (packed field and lists)
    const int64_t N = (int64_t)dims.nx * dims.ny * dims.nz;
    const int64_t cap = std::max<int64_t>(4096, N / 16);
    uint8_t *wind = nullptr, *lists = nullptr;
    int64_t *counts = nullptr;
    vx_status st = vx_hip_check(h, hipMalloc((void **)&wind, (size_t)N), "hipMalloc");
    if (st == VX_OK) st = vx_hip_check(h, hipMalloc((void **)&lists, (size_t)cap * 19), "hipMalloc");
    if (st == VX_OK) st = vx_hip_check(h, hipMalloc((void **)&counts, 64), "hipMalloc");
    int best_zc = 0;
    double best = 1e30;
    if (st == VX_OK) {
        vx_winding_out o;
        o.d_wind = wind;
        o.d_faces = (uint64_t *)lists;
        o.d_cells = (uint64_t *)(lists + 8 * cap);
        o.d_cell_desc = (uint16_t *)(lists + 16 * cap);
        o.d_face_sign = (int8_t *)(lists + 18 * cap);
        o.face_cap = o.cell_cap = cap;
        o.d_counts = counts;
        const bool prof = h->profile;
        h->profile = false;
        for (int cand : candidates(dims.nz)) {
            vx_wind_args A;
            int64_t nt = 0;
            st = vx_wind_make_args(h, dims, d_psi, o, cand, &A, &nt);
            double ms = 0.0;
            if (st == VX_OK)
                st = time_median(h, (hipStream_t)s, 3, [&] { return vx_wind_enqueue(h, A, nt, (hipStream_t)s); }, &ms);
            if (st) break;
            if (ms < best) {
                best = ms;
                best_zc = cand;
            }
        }
        h->profile = prof;
    }
    (void)hipStreamSynchronize((hipStream_t)s);
    if (wind) (void)hipFree(wind);
    if (lists) (void)hipFree(lists);
    if (counts) (void)hipFree(counts);
    if (st) return st;
    h->tuned_zc[k] = best_zc;
    append_cache(cache_path, "grid", k, best_zc, best);
    if (zchunk) *zchunk = best_zc;
    return VX_OK;
}
