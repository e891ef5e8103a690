// Internal declarations shared by the translation units of libvx.so.
#pragma once

#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <cstdio>
#include <map>
#include <string>
#include <vector>

#include "../../include/vx.h"

enum {
    VX_KIND_WIND = 0,
    VX_KIND_REFINE = 1,
    VX_KIND_MLP = 2,
    VX_KIND_BATCH = 3,
    VX_KIND_POLISH = 4,
    VX_KIND_NODE = 5,
    VX_KIND_COUNT = 6
};

struct vx_event_pair {
    hipEvent_t start, stop;
    int kind;
};

struct vx_handle {
    int device = 0;
    int num_cu = 0;
    int lds_per_cu = 0;  // bytes of LDS per CU
    std::string err;
    bool profile = false;
    std::vector<vx_event_pair> events;  // recorded pairs (pool grows as needed)
    size_t events_used = 0;
    int wind_zc = 0;  // planes per z-chunk (0 = chosen from the grid)
    int ref_blocks_per_cu = 0;   // resident refinement workgroups per CU (0 = not yet queried)
    int refb_blocks_per_cu = 0;  // the same for the batched refinement kernel
    int refs_blocks_per_cu = 0;  // the same for the short-list refinement kernel
    int wind_lds_pad = -1;       // dynamic LDS bytes per winding workgroup (-1 = not yet computed)
    int ref_refill = 8;          // idle lanes a refinement wavefront waits for before claiming samples
    unsigned long long *d_work = nullptr;  // device workspace: [0] refinement chunk counter, [1] overflow flags
    std::map<std::array<int, 4>, int> tuned_zc;  // (nx, ny, nz, periodic) -> planes per z-chunk
};

// Sticky overflow flags in the handle's workspace (device word d_work[1]): set by kernels that find
// a list longer than its capacity, read and cleared by vx_sync_status.
enum : unsigned { VX_OVERFLOW_WIND = 1u, VX_OVERFLOW_REFINE = 2u, VX_OVERFLOW_DATASET = 4u };
inline unsigned long long *vx_overflow_flag(vx_handle *h) { return h->d_work + 1; }

// Arguments of the winding kernel for one grid (one frame of a batch).
struct vx_wind_args {
    const float2 *psi;
    uint8_t *wind;
    uint64_t *faces;
    int8_t *fsign;
    int64_t fcap;
    uint64_t *cells;
    uint16_t *cdesc;
    int64_t ccap;
    int64_t *counts;
    unsigned long long *flag;  // sticky overflow flags (VX_OVERFLOW_WIND set when a list overflows)
    int nx, ny, nz;
    int px, py, pz;
    int ntx, nty, ntz, zc;
    int psi_a16;   // psi is 16-byte aligned (16-byte loads allowed)
    int wind_a16;  // packed field 16-byte aligned
    int wind_a4;   // packed field 4-byte aligned
};

// One frame of a batched refinement (64 bytes; the kernel keeps the table in LDS).
struct vx_ref_frame {
    const float2 *psi;
    const uint64_t *cells;
    const uint16_t *desc;
    const int64_t *count;  // number of listed cells (device)
    int64_t cap;           // at most this many are refined
    vx_sample *out;
    int nx, ny, nz;
    uint32_t periodic;
};

// error helpers -----------------------------------------------------------------------------
vx_status vx_fail(vx_handle *h, vx_status st, const char *fmt, ...);
vx_status vx_hip_check(vx_handle *h, hipError_t e, const char *what);
vx_status vx_bind(vx_handle *h);  // make the handle's device current

// timing helpers: record a start/stop pair around a launch when profiling is on (kind < 0: off).
// Timers may nest; each keeps the index of its pair (the pool may grow meanwhile).
struct vx_timer {
    vx_handle *h;
    hipStream_t s;
    int kind;
    int64_t slot = -1;
    vx_timer(vx_handle *h_, hipStream_t s_, int kind_);
    void stop();
};

// validation
vx_status vx_check_dims(vx_handle *h, const vx_dims &d);
vx_status vx_check_winding(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out *out,
                           const char *who);
vx_status vx_check_refine_params(vx_handle *h, const vx_refine_params &p);

// kernels (one translation unit each)
vx_status vx_wind_launch(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o,
                         hipStream_t s);
// out_index (nullable): sample s of the list goes to out[out_index[s]]
vx_status vx_refine_launch(vx_handle *h, const vx_dims &d, const void *psi, const uint64_t *cells,
                           const uint16_t *desc, const float *seed, const int64_t *count, int64_t cap,
                           const vx_refine_params &p, vx_sample *out, hipStream_t s,
                           const int64_t *out_index = nullptr);

// winding arguments of one grid with a given z-chunk depth (0 = the handle's choice); *ntiles
// receives the number of tiles (workgroups)
vx_status vx_wind_make_args(vx_handle *h, const vx_dims &d, const void *psi, const vx_winding_out &o, int zc,
                            vx_wind_args *A, int64_t *ntiles);
// zero the grid's counts and launch its winding kernel
vx_status vx_wind_enqueue(vx_handle *h, const vx_wind_args &A, int64_t ntiles, hipStream_t s);
// planes per z-chunk the handle uses for a single grid of these dims
int vx_wind_zc_for(vx_handle *h, const vx_dims &d);
// one launch over the tiles of several grids (tables in device memory; tile_start[nframes] = total)
// (lds_pad: dynamic LDS per workgroup, which caps the resident workgroups per CU; 0 = as many as fit)
vx_status vx_wind_batch_enqueue(vx_handle *h, const vx_wind_args *d_frames, const int *d_tile_start, int nframes,
                                int64_t total_tiles, int lds_pad, hipStream_t s);
// resident batch-winding workgroups per CU without a pad (-1 on error), and the pad that leaves N
int vx_wind_batch_max_wg(vx_handle *h);
int vx_wind_batch_pad(vx_handle *h, int wg_per_cu);
// one launch refining the listed cells of several grids (table in device memory)
// wg_per_cu > 0: resident refinement workgroups per CU to launch (capped by what fits); 0: the default
vx_status vx_refine_batch_enqueue(vx_handle *h, const vx_ref_frame *d_frames, int nframes, int64_t total_cap,
                                  const vx_refine_params &p, unsigned long long *d_counter, int wg_per_cu,
                                  hipStream_t s);
// resident workgroups per CU that the batch refinement kernel can have at most (-1 on error)
int vx_refine_batch_max_wg(vx_handle *h);
