// Internal declarations shared by the translation units of libvx.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/vx.h"

enum { VX_KIND_WIND = 0, VX_KIND_REFINE = 1, VX_KIND_MLP = 2, VX_KIND_BATCH = 3, VX_KIND_COUNT = 4 };

struct vx_event_pair {
    hipEvent_t start, stop;
    int kind;
};

struct vx_handle {
    int device = 0;
    int num_cu = 0;
    std::string err;
    bool profile = false;
    std::vector<vx_event_pair> events;  // recorded pairs (pool grows as needed)
    size_t events_used = 0;
    int wind_ty = 0;  // rows per wavefront of the winding kernel (0 = default)
    int wind_zc = 0;  // planes per z-chunk (0 = chosen from the grid)
    int ref_blocks_per_cu = 0;  // resident refinement workgroups per CU (0 = not yet queried)
    int ref_refill = 8;         // idle lanes a refinement wavefront waits for before claiming samples
    unsigned long long *d_work = nullptr;  // device workspace: [0] refinement chunk counter
};

// error helpers -----------------------------------------------------------------------------
vx_status vx_fail(vx_handle *h, vx_status st, const char *fmt, ...);
vx_status vx_hip_check(vx_handle *h, hipError_t e, const char *what);
vx_status vx_bind(vx_handle *h);  // make the handle's device current

// timing helpers: record a start/stop pair around a launch when profiling is on
struct vx_timer {
    vx_handle *h;
    hipStream_t s;
    int kind;
    vx_event_pair *pair = nullptr;
    vx_timer(vx_handle *h_, hipStream_t s_, int kind_);
    void stop();
};

// validation
vx_status vx_check_dims(vx_handle *h, const vx_dims &d);

// kernels (one translation unit each)
vx_status vx_wind_launch(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o,
                         hipStream_t s);
vx_status vx_refine_launch(vx_handle *h, const vx_dims &d, const void *psi, const uint64_t *cells,
                           const uint16_t *desc, const float *seed, const int64_t *count, int64_t cap,
                           const vx_refine_params &p, vx_sample *out, hipStream_t s);
