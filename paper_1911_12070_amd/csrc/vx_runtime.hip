// Handle, error state, validation, event timing and the C-ABI entry points of libvx.so.
#include <cstdarg>
#include <cstring>
#include <new>

#include "vx_internal.h"

extern "C" int vx_version(void) { return 10000; }

extern "C" const char *vx_status_str(int st) {
    switch (st) {
        case VX_OK: return "VX_OK";
        case VX_ERR_INVALID: return "VX_ERR_INVALID";
        case VX_ERR_CAPACITY: return "VX_ERR_CAPACITY";
        case VX_ERR_DEVICE: return "VX_ERR_DEVICE";
        case VX_ERR_NOMEM: return "VX_ERR_NOMEM";
        case VX_ERR_UNSUPPORTED: return "VX_ERR_UNSUPPORTED";
        default: return "VX_ERR_UNKNOWN";
    }
}

vx_status vx_fail(vx_handle *h, vx_status st, const char *fmt, ...) {
    if (h) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        h->err = buf;
    }
    return st;
}

vx_status vx_hip_check(vx_handle *h, hipError_t e, const char *what) {
    if (e == hipSuccess) return VX_OK;
    return vx_fail(h, e == hipErrorOutOfMemory ? VX_ERR_NOMEM : VX_ERR_DEVICE, "%s: %s", what,
                   hipGetErrorString(e));
}

vx_status vx_bind(vx_handle *h) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device)
        return vx_hip_check(h, hipSetDevice(h->device), "hipSetDevice");
    return VX_OK;
}

extern "C" vx_status vx_create(int device, vx_handle **out) {
    if (!out) return VX_ERR_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return VX_ERR_INVALID;
    vx_handle *h = new (std::nothrow) vx_handle();
    if (!h) return VX_ERR_NOMEM;
    h->device = device;
    if (hipSetDevice(device) != hipSuccess) {
        delete h;
        return VX_ERR_DEVICE;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) {
        delete h;
        return VX_ERR_DEVICE;
    }
    h->num_cu = prop.multiProcessorCount;
    h->lds_per_cu = (int)prop.maxSharedMemoryPerMultiProcessor;
    if (hipMalloc((void **)&h->d_work, 256) != hipSuccess) {
        delete h;
        return VX_ERR_NOMEM;
    }
    if (hipMemset(h->d_work, 0, 256) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipFree(h->d_work);
        delete h;
        return VX_ERR_DEVICE;
    }
    *out = h;
    return VX_OK;
}

extern "C" vx_status vx_destroy(vx_handle *h) {
    if (!h) return VX_OK;
    (void)hipSetDevice(h->device);
    for (auto &p : h->events) {
        (void)hipEventDestroy(p.start);
        (void)hipEventDestroy(p.stop);
    }
    if (h->d_work) (void)hipFree(h->d_work);
    delete h;
    return VX_OK;
}

extern "C" const char *vx_last_error(const vx_handle *h) { return h ? h->err.c_str() : ""; }

// ------------------------------------------------------------------------------- timing
vx_timer::vx_timer(vx_handle *h_, hipStream_t s_, int kind_) : h(h_), s(s_), kind(kind_) {
    if (!h->profile || kind < 0) return;
    if (h->events_used == h->events.size()) {
        vx_event_pair p{};
        if (hipEventCreate(&p.start) != hipSuccess) return;
        if (hipEventCreate(&p.stop) != hipSuccess) {
            (void)hipEventDestroy(p.start);
            return;
        }
        h->events.push_back(p);
    }
    slot = (int64_t)h->events_used++;
    h->events[slot].kind = kind;
    (void)hipEventRecord(h->events[slot].start, s);
}

void vx_timer::stop() {
    if (slot >= 0) (void)hipEventRecord(h->events[slot].stop, s);
    slot = -1;
}

extern "C" vx_status vx_profile_enable(vx_handle *h, int enable) {
    if (!h) return VX_ERR_INVALID;
    h->profile = enable != 0;
    h->events_used = 0;
    return VX_OK;
}

extern "C" vx_status vx_profile_read(vx_handle *h, int kind, double *total_ms, int64_t *launches) {
    if (!h || !total_ms || !launches || kind < 0 || kind >= VX_KIND_COUNT)
        return vx_fail(h, VX_ERR_INVALID, "vx_profile_read: bad arguments");
    vx_status st = vx_bind(h);
    if (st) return st;
    double sum = 0.0;
    int64_t n = 0;
    for (size_t i = 0; i < h->events_used; ++i) {
        auto &p = h->events[i];
        if (p.kind != kind) continue;
        st = vx_hip_check(h, hipEventSynchronize(p.stop), "hipEventSynchronize");
        if (st) return st;
        float ms = 0.f;
        st = vx_hip_check(h, hipEventElapsedTime(&ms, p.start, p.stop), "hipEventElapsedTime");
        if (st) return st;
        sum += ms;
        ++n;
    }
    *total_ms = sum;
    *launches = n;
    return VX_OK;
}

extern "C" vx_status vx_wind_config(vx_handle *h, int zchunk) {
    if (!h) return VX_ERR_INVALID;
    if (zchunk < 0) return vx_fail(h, VX_ERR_INVALID, "vx_wind_config: negative zchunk");
    h->wind_zc = zchunk;
    return VX_OK;
}

extern "C" vx_status vx_sync_status(vx_handle *h, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_bind(h)) return st;
    hipStream_t hs = (hipStream_t)s;
    unsigned long long flags = 0;
    static const unsigned long long zero = 0;
    vx_status st = vx_hip_check(h, hipMemcpyAsync(&flags, vx_overflow_flag(h), sizeof flags, hipMemcpyDeviceToHost, hs),
                                "vx_sync_status: read");
    if (st == VX_OK) st = vx_hip_check(h, hipStreamSynchronize(hs), "vx_sync_status: synchronise");
    if (st == VX_OK && flags != 0) {
        st = vx_hip_check(h, hipMemcpyAsync(vx_overflow_flag(h), &zero, sizeof zero, hipMemcpyHostToDevice, hs),
                          "vx_sync_status: clear");
        if (st == VX_OK) st = vx_hip_check(h, hipStreamSynchronize(hs), "vx_sync_status: synchronise");
        if (st == VX_OK)
            return vx_fail(h, VX_ERR_CAPACITY, "a list was longer than its capacity:%s%s%s",
                           (flags & VX_OVERFLOW_WIND) ? " pierced faces or cells (winding)" : "",
                           (flags & VX_OVERFLOW_REFINE) ? " listed cells beyond the sample capacity" : "",
                           (flags & VX_OVERFLOW_DATASET) ? " training rows beyond n_cap" : "");
    }
    return st;
}

// ------------------------------------------------------------------------------- validation
vx_status vx_check_dims(vx_handle *h, const vx_dims &d) {
    const int32_t n[3] = {d.nx, d.ny, d.nz};
    if (d.periodic > 7u) return vx_fail(h, VX_ERR_INVALID, "periodic mask 0x%x has bits above 2", d.periodic);
    for (int a = 0; a < 3; ++a) {
        bool per = (d.periodic >> a) & 1u;
        if (n[a] < (per ? 2 : 1))
            return vx_fail(h, VX_ERR_INVALID, "dims[%d] = %d must be >= %d", a, n[a], per ? 2 : 1);
    }
    const double nodes = (double)d.nx * d.ny * d.nz;
    if (nodes * 3.0 >= 18446744073709551615.0)
        return vx_fail(h, VX_ERR_UNSUPPORTED, "grid too large for 64-bit face ids");
    return VX_OK;
}

// ------------------------------------------------------------------------------- entry points
vx_status vx_check_winding(vx_handle *h, const vx_dims &dims, const void *d_psi, const vx_winding_out *out,
                           const char *who) {
    if (!d_psi || !out) return vx_fail(h, VX_ERR_INVALID, "%s: null psi or out", who);
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (((uintptr_t)d_psi & 7u) != 0) return vx_fail(h, VX_ERR_INVALID, "%s: psi must be 8-byte aligned", who);
    if (!out->d_counts) return vx_fail(h, VX_ERR_INVALID, "%s: d_counts is required", who);
    if (((uintptr_t)out->d_counts & 7u) != 0)
        return vx_fail(h, VX_ERR_INVALID, "%s: d_counts must be 8-byte aligned", who);
    if (out->face_cap < 0 || out->cell_cap < 0) return vx_fail(h, VX_ERR_INVALID, "%s: negative capacity", who);
    if (out->face_cap > 0 && (!out->d_faces || !out->d_face_sign))
        return vx_fail(h, VX_ERR_INVALID, "%s: face_cap > 0 needs d_faces and d_face_sign", who);
    if (out->cell_cap > 0 && (!out->d_cells || !out->d_cell_desc))
        return vx_fail(h, VX_ERR_INVALID, "%s: cell_cap > 0 needs d_cells and d_cell_desc", who);
    return VX_OK;
}

vx_status vx_check_refine_params(vx_handle *h, const vx_refine_params &prm) {
    if (prm.max_descent < 0 || prm.max_newton < 0 || prm.max_halvings < 0 || prm.max_descent > 100000 ||
        prm.max_newton > 100000 || prm.max_halvings > 200 || !(prm.step0 > 0.f) || !(prm.step_max > 0.f))
        return vx_fail(h, VX_ERR_INVALID, "refine: bad parameters");
    return VX_OK;
}

extern "C" vx_status vx_winding(vx_handle *h, vx_dims dims, const void *d_psi, const vx_winding_out *out,
                                vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_winding(h, dims, d_psi, out, "vx_winding")) return st;
    if (vx_status st = vx_bind(h)) return st;
    return vx_wind_launch(h, dims, d_psi, *out, (hipStream_t)s);
}

extern "C" vx_refine_params vx_refine_defaults(void) {
    vx_refine_params p;
    p.max_descent = 32;
    p.max_newton = 20;
    p.max_halvings = 30;
    p.step0 = 0.25f;
    p.step_max = 1.0f;
    p.armijo = 1e-4f;
    p.descent_tol = 1e-2f;
    p.newton_tol = 1e-6f;
    p.rho_tol = 1e-10f;
    return p;
}

extern "C" vx_status vx_refine(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                               const uint16_t *d_cell_desc, const float *d_seed_off,
                               const int64_t *d_count, int64_t cap, const vx_refine_params *p,
                               vx_sample *d_out, vx_stream s) {
    if (!h) return VX_ERR_INVALID;
    h->err.clear();
    if (vx_status st = vx_check_dims(h, dims)) return st;
    if (cap < 0) return vx_fail(h, VX_ERR_INVALID, "vx_refine: negative capacity");
    if (cap == 0) return VX_OK;
    if (!d_psi || !d_cells || !d_cell_desc || !d_count || !d_out)
        return vx_fail(h, VX_ERR_INVALID, "vx_refine: null pointer argument");
    vx_refine_params prm = p ? *p : vx_refine_defaults();
    if (vx_status st = vx_check_refine_params(h, prm)) return st;
    if (vx_status st = vx_bind(h)) return st;
    return vx_refine_launch(h, dims, d_psi, d_cells, d_cell_desc, d_seed_off, d_count, cap, prm, d_out,
                            (hipStream_t)s);
}
