/*
 * vx.h -- C ABI of libvx.so, the MI355X (gfx950) vortex-core extraction library.
 *
 * Method: Liu, Xiong & Liu, "Vectorizing Quantum Turbulence Vortex-Core Lines for Real-Time
 * Visualization" (arXiv 1911.12070). Given a complex wavefunction psi sampled on a 3D grid, the
 * library computes
 *   - the circulation of the phase around every unit face of the grid (Sec. 2.2, circulation
 *     equation; |C| = 2 pi where a core pierces the face, sign by the right-hand rule of
 *     Sec. 3.4), as an exact winding number w in {-1, 0, +1};
 *   - the lists of pierced faces and pierced cells (the vortex nodes and their links of
 *     Sec. 3.1, in dual form);
 *   - one sub-grid core sample per listed cell: the mean-position estimate (Sec. 3.3.1) refined
 *     by minimising |psi|^2 in the plane normal to the pseudo-vorticity (Sec. 3.3.3), with psi
 *     linearly interpolated between nodes (Sec. 5).
 *
 * Conventions
 *   Grid       node (i,j,k), 0 <= i < nx etc., linear id n = i + nx*(j + ny*k) (x fastest).
 *   psi        complex64, interleaved (re, im), nx*ny*nz values in node order, device memory,
 *              8-byte aligned. Values must be finite.
 *   Periodic   bit a of vx_dims.periodic makes axis a periodic (index nx wraps to 0). On a
 *              non-periodic axis the faces and cells that would need index n_a do not exist:
 *              their windings are 0 and they are never listed.
 *   Faces      face (n, a) is the unit square at node n with normal +e_a (a=0 yz-face, a=1
 *              zx-face, a=2 xy-face); id = 3*n + a; winding counted about +e_a.
 *   Cells      cell n is the unit cube with min corner n; id = n. A cell is pierced if any of
 *              its six faces has w != 0. Descriptor (12 bits): 2-bit two's complement windings
 *              (01 = +1, 11 = -1) of the faces -x,+x,-y,+y,-z,+z = w_x(n), w_x(n+ex), w_y(n),
 *              w_y(n+ey), w_z(n), w_z(n+ez), lowest bits first, each about +e_axis.
 *   Packed     one byte per node: bits 1:0 w_x(n), 3:2 w_y(n), 5:4 w_z(n) (2-bit two's
 *              complement), bit 6 = cell n pierced, bit 7 = 0.
 *
 * Memory and streams
 *   Every buffer argument named d_* is device memory owned by the caller. The library owns only
 *   its handle and the handle's small internal state; vx_destroy frees them. All compute calls
 *   are asynchronous on the given stream (NULL = the device's null stream) and allocate nothing;
 *   the set-up calls (vx_create, vx_batch_create, vx_mlp_create, vx_mlp_reserve, the autotuners)
 *   allocate and synchronise. Argument errors are detected on the host before anything is
 *   launched. A handle belongs to one device and must not be used by two threads at once.
 *
 * Errors
 *   Every call returns vx_status. Nothing throws, exits or prints. vx_last_error() gives the
 *   detail of the handle's last failure.
 */
#ifndef VX_H
#define VX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VX_OK = 0,
    VX_ERR_INVALID = -1,     /* bad argument: null pointer, bad dims, bad sizes */
    VX_ERR_CAPACITY = -2,    /* an output list was too small (true counts were still written) */
    VX_ERR_DEVICE = -3,      /* a HIP call failed */
    VX_ERR_NOMEM = -4,       /* host or device allocation failed */
    VX_ERR_UNSUPPORTED = -5  /* valid request outside what the library supports */
} vx_status;

typedef struct vx_handle vx_handle;
typedef void *vx_stream; /* a hipStream_t */

typedef struct {
    int32_t nx, ny, nz;
    uint32_t periodic; /* bit 0: x, bit 1: y, bit 2: z */
} vx_dims;

/* Capacity status of the work enqueued so far on this handle. Synchronises stream s (the caller
 * synchronises any other stream it used), then returns VX_ERR_CAPACITY if any call since the last
 * vx_sync_status found a list longer than its capacity -- pierced faces or cells beyond face_cap /
 * cell_cap (vx_winding, batches), listed cells beyond the sample capacity (vx_refine, vx_mlp_infer,
 * vx_mlp_predict, batches), training rows beyond n_cap (vx_mlp_dataset) -- with the detail in vx_last_error, and
 * clears the flag; VX_OK otherwise. The flag is a device word of the handle that those kernels set
 * (sticky: it is never cleared by the compute calls themselves); it travels with captured graphs. */
vx_status vx_sync_status(vx_handle *h, vx_stream s);

/* Library version (major*10000 + minor*100 + patch). */
int vx_version(void);

/* Create a handle bound to HIP device `device`. *out receives the handle. */
vx_status vx_create(int device, vx_handle **out);
/* Destroy a handle. NULL is accepted. Waits for nothing: the caller synchronises its streams. */
vx_status vx_destroy(vx_handle *h);
/* Static text of a status code. */
const char *vx_status_str(int status);
/* Detail of the handle's last failure ("" if none). Valid until the next call on the handle. */
const char *vx_last_error(const vx_handle *h);

/* ------------------------------------------------------------------------------------------
 * Synthetic inputs (support: the paper's simulation data is replaced by seeded fields).
 * ---------------------------------------------------------------------------------------- */

/* Random-wave tangle psi(x) = sum_k c_k T[(ax_k x + ay_k y + az_k z) mod M], T[m] = exp(2 pi i m/M),
 * evaluated in FP64 in wave order with one rounding per operation and rounded to complex64.
 * Arrays are device memory: d_ax, d_ay, d_az uint32[nwaves] (each < table_size), d_coef
 * double[2*nwaves] (re, im), d_table double[2*table_size]. table_size <= 46340. */
typedef struct {
    int32_t nwaves;
    uint32_t table_size;
    const uint32_t *d_ax, *d_ay, *d_az;
    const double *d_coef;
    const double *d_table;
} vx_tangle;
vx_status vx_gen_tangle(vx_handle *h, vx_dims dims, const vx_tangle *t, void *d_psi, vx_stream s);

/* Straight z-line (winding +1) times a ring in the plane z = ring_cz (winding -1 about its
 * azimuthal direction), core profile d / sqrt(d^2 + 2 xi^2), minimum-image displacements, plus
 * optional noise d_noise (float[2*N], nullable). FP64 arithmetic rounded to complex64. */
typedef struct {
    double line_x, line_y, ring_cx, ring_cy, ring_cz, radius, xi;
} vx_line_ring;
vx_status vx_gen_line_ring(vx_handle *h, vx_dims dims, const vx_line_ring *p, const float *d_noise,
                           void *d_psi, vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Winding + compaction (Sec. 2.2 circulation, Sec. 3.1 vortex-node graph in dual form).
 *
 * The winding of a face is the exact winding number, about the point q = (-delta, +eps)
 * (0 < eps << delta << 1), of the image of the face's boundary under psi with straight edges:
 * an edge a->b counts +1 if Im a <= 0 < Im b and Re a Im b - Im a Re b >= 0, -1 if
 * Im a > 0 >= Im b and Re a Im b - Im a Re b <= 0. The determinant sign is exact (FP32 products
 * formed in FP64). Results are bit-identical to any exact implementation of this definition.
 *
 * Outputs (all device memory, caller-owned):
 *   d_wind       uint8[N] packed field, or NULL to skip it.
 *   d_faces      uint64[face_cap] pierced face ids;  d_face_sign int8[face_cap] their w (+1/-1).
 *   d_cells      uint64[cell_cap] pierced cell ids;  d_cell_desc uint16[cell_cap] descriptors.
 *   d_counts     int64[2]: true number of pierced faces, cells. Written even on overflow; only
 *                the first *_cap entries are stored. The call zeroes d_counts first.
 * Lists are sets: their order is unspecified and may differ between runs. Sort to compare.
 * Overflow (a true count above its capacity) sets the handle's sticky capacity flag on the device;
 * vx_sync_status reports it as VX_ERR_CAPACITY. The counts themselves also show it.
 * d_faces/d_face_sign may be NULL when face_cap == 0 (likewise cells).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    uint8_t *d_wind;
    uint64_t *d_faces;
    int8_t *d_face_sign;
    int64_t face_cap;
    uint64_t *d_cells;
    uint16_t *d_cell_desc;
    int64_t cell_cap;
    int64_t *d_counts;
} vx_winding_out;
vx_status vx_winding(vx_handle *h, vx_dims dims, const void *d_psi, const vx_winding_out *out,
                     vx_stream s);

/* Depth of the winding kernel's z-chunks on this handle: planes marched per wavefront (0 = chosen
 * from the grid size, or by vx_autotune for that shape). Results do not depend on it. */
vx_status vx_wind_config(vx_handle *h, int zchunk);

/* ------------------------------------------------------------------------------------------
 * Node-centred circulation (Sec. 2.2: three rings per grid node in the coordinate planes, the
 * largest |C| kept, vortex node where it exceeds pi), derived from the packed face windings.
 *
 * The ring of node n in the plane normal to axis a is the boundary of the 2 x 2 faces around n in
 * that plane (corners n +- e_u +- e_v); its circulation / 2 pi is the sum of those four faces'
 * windings, e.g. C_z(n) / 2 pi = w_z(n) + w_z(n-ex) + w_z(n-ey) + w_z(n-ex-ey) (faces outside a
 * non-periodic axis count 0). Exact integers, |C| / 2 pi <= 3.
 *   d_wind   uint8[N] packed field of vx_winding (device, input).
 *   d_node   uint8[N] (nullable): bits 1:0 |C| / 2 pi of the plane with the largest |C| (ties: lowest
 *            axis), bit 2 its sign (1 = negative), bits 4:3 that plane's normal axis (0 x, 1 y, 2 z),
 *            bit 6 = vortex node (|C| > pi), bits 5 and 7 zero; 0 where every ring has C = 0.
 *   d_nodes  uint64[node_cap] vortex node ids (unspecified order; nullable when node_cap == 0).
 *   d_count  int64[1]: true number of vortex nodes (zeroed by the call; overflow sets the handle's
 *            capacity flag, see vx_sync_status).
 * ---------------------------------------------------------------------------------------- */
vx_status vx_node_circulation(vx_handle *h, vx_dims dims, const uint8_t *d_wind, uint8_t *d_node, uint64_t *d_nodes,
                              int64_t node_cap, int64_t *d_count, vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Core-sample refinement (Sec. 3.3.1 mean estimate, Sec. 3.3.3 density-guided minimisation).
 *
 * For listed cell i (i < min(*d_count, cap)): x0 = mean of the centres of its pierced faces;
 * t = grad Re psi x grad Im psi at x0 (fallback: the cell's face flux); in the plane through x0
 * normal to t, gradient descent of |psi|^2 (trilinear psi) from x0 with a halving step rule,
 * then a Newton polish on (Re psi, Im psi); trial points must stay inside the cell's 4x4x4
 * node patch. FP32 arithmetic. d_count is read on the device (no host synchronisation).
 * d_seed_off (float[3*cap], nullable) replaces x0 by caller seeds (cell-local coordinates).
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int32_t max_descent;   /* accepted descent steps (32) */
    int32_t max_newton;    /* Newton steps (20) */
    int32_t max_halvings;  /* step halvings per trial (30) */
    float step0;           /* first descent step length, cells (0.25) */
    float step_max;        /* largest descent step length, cells (1.0) */
    float armijo;          /* sufficient-decrease constant (1e-4) */
    float descent_tol;     /* descent stops after an accepted step shorter than this (1e-2) */
    float newton_tol;      /* Newton stops after a step shorter than this (1e-6) */
    float rho_tol;         /* |psi|^2 above this at the end sets NONZERO_MIN (1e-10) */
} vx_refine_params;

/* status bits of a sample */
#define VX_SAMPLE_MULTI 1u            /* 4 or 6 pierced faces (branch / reconnection cell) */
#define VX_SAMPLE_TANGENT_FALLBACK 2u /* pseudo-vorticity degenerate; face flux used */
#define VX_SAMPLE_BOUNDARY 4u         /* a trial point left the patch and was rejected */
#define VX_SAMPLE_NONZERO_MIN 8u      /* |psi|^2 > rho_tol at the end */
#define VX_SAMPLE_NOT_CONVERGED 16u   /* Newton ended without a short step, rho > rho_tol */
#define VX_SAMPLE_NO_FACES 32u        /* the listed cell has no pierced face */
#define VX_SAMPLE_BAD_CELL 64u        /* the listed cell id is >= nx*ny*nz: nothing was read */

typedef struct {
    uint64_t cell;    /* cell id */
    float off[3];     /* sample position relative to the cell's min corner, cells */
    float rho;        /* |psi|^2 at the sample */
    uint16_t iters;   /* descent + Newton steps taken */
    uint16_t status;  /* VX_SAMPLE_* bits */
    uint32_t reserved;
} vx_sample; /* 32 bytes */

/* Defaults of vx_refine_params. */
vx_refine_params vx_refine_defaults(void);

vx_status vx_refine(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                    const uint16_t *d_cell_desc, const float *d_seed_off, const int64_t *d_count,
                    int64_t cap, const vx_refine_params *p, vx_sample *d_out, vx_stream s);

/* The refinement of vx_refine for callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid device allocation): no handle, and no allocation at any
 * point -- not even at its first call. Same kernels, same results bit for bit as vx_refine with the
 * same arguments, on the current HIP device and stream s. The scratch that vx_refine keeps in its
 * handle (the work counter of the refinement kernels) is a fixed 256-byte device array of the
 * library, one copy per device, held until the process ends; it does not grow with the list, so
 * any cap is accepted. The first call on a device looks up that array's address and the launch
 * figures (host-side queries only) and keeps them. Every call on one device shares the array: calls
 * that overlap in time on one device (two streams, two threads) race and give wrong samples.
 * Overflow (*d_count > cap) refines the first cap cells and sets no flag (there is no handle).
 * Errors: VX_ERR_INVALID (arguments, checked on the host), VX_ERR_DEVICE (a HIP call failed),
 * VX_ERR_UNSUPPORTED (device index >= 64); no error detail is kept. */
vx_status vx_refine_noalloc(vx_dims dims, const void *d_psi, const uint64_t *d_cells, const uint16_t *d_cell_desc,
                            const float *d_seed_off, const int64_t *d_count, int64_t cap,
                            const vx_refine_params *p, vx_sample *d_out, vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Learned surrogate of the refinement (an extension of the method; the plain refinement above
 * labels its training data, is the reference for its error and takes over below a confidence
 * threshold).
 *
 * Network: inputs f (128) from the 4x4x4 patch of nodes around a cell (offsets -1..2 on each
 * axis from the min corner; patch node q = a + 4b + 16c, x fastest): f[2q] = Re psi_q / s,
 * f[2q+1] = Im psi_q / s, s = sqrt(mean_q |psi_q|^2) (s = 1 if zero). Z1 = f W1 + b1,
 * H1 = gelu(Z1), Z2 = H1 W2 + b2, H2 = gelu(Z2), Z3 = H2 W3 + b3 with W1 128xH, W2 HxH, W3 Hx4
 * (row index = input; hidden width H = VX_MLP_NHID = 128), gelu(x) = x (1 + erf(x / sqrt 2)) / 2.
 * Outputs: Z3[0..2] = the
 * core sample minus the cell's first estimate x0 (mean of its pierced-face centres, cell units);
 * conf = 1 / (1 + exp(-Z3[3])).
 * Arithmetic: BF16 matrix operands (features, weights, activations) on the matrix cores with FP32
 * accumulation; biases, master weights, Adam moments and the loss in FP32; in training, gelu and
 * its derivative read from FP32 tables of the exact function (erff/expf at creation, 1/64 spacing
 * on [-8, 8], linear interpolation, error below 3e-5; identity / zero outside); in inference, gelu
 * from a fitted closed form x sigmoid(x (a + b x^2 + c x^4)) (x clamped to [-8, 8] inside the
 * sigmoid), error below 3e-5 as well.
 * Parameters (host layout, VX_MLP_NPARAMS floats): W1 row-major, b1, W2, b2, W3, b3.
 * Training loss per sample: |Z3[0..2] - t|^2 + lambda * (log(1 + exp(Z3[3])) - y Z3[3]), y = 1 if
 * the current prediction is within conf_tol of t on every axis (no gradient through y); the mean
 * over the minibatch is minimised with Adam.
 * ---------------------------------------------------------------------------------------- */
#define VX_MLP_NIN 128
#define VX_MLP_NHID 128
#define VX_MLP_NOUT 4
#define VX_MLP_NPARAMS 33540
#define VX_SAMPLE_SURROGATE 128u  /* position from the surrogate network + one Newton step */

typedef struct vx_mlp vx_mlp;
typedef struct {
    float lr, beta1, beta2, eps; /* Adam */
    float conf_lambda;           /* weight of the confidence loss */
    float conf_tol;              /* prediction counted as good within this many cells per axis */
} vx_adam_params;

/* h_params: VX_MLP_NPARAMS initial values (host memory, copied). max_batch: largest minibatch of
 * the training calls (their scratch, about 1.5 KiB per row, is allocated here). */
vx_status vx_mlp_create(vx_handle *h, const float *h_params, int64_t max_batch, vx_mlp **out);
vx_status vx_mlp_destroy(vx_mlp *m);
/* Reserve the inference buffers of vx_mlp_infer for lists of up to max_cells cells (98 bytes per
 * cell: network outputs, the cells' corners for the polish, the fallback queue). Allocating and
 * synchronous (it waits for the device first, since earlier work may still read the old buffers);
 * a smaller max_cells than already reserved keeps the buffers. vx_mlp_infer itself never allocates. */
vx_status vx_mlp_reserve(vx_mlp *m, int64_t max_cells);
/* Copy the FP32 parameters to / from host memory (synchronous). */
vx_status vx_mlp_get_params(vx_mlp *m, float *h_params);
vx_status vx_mlp_set_params(vx_mlp *m, const float *h_params);
/* Save / load the parameters as a little-endian file ("VXMLP1", count, floats). */
vx_status vx_mlp_save(vx_mlp *m, const char *path);
vx_status vx_mlp_load(vx_mlp *m, const char *path);

/* Training data from refined samples: for listed cell i < min(*d_count, cap) whose sample
 * d_samples[i] has none of the status bits MULTI, NO_FACES, NONZERO_MIN, NOT_CONVERGED, BOUNDARY,
 * BAD_CELL and whose patch lies inside the grid, append its features (BF16, 128 per row) to
 * d_feat and its target (sample offset minus x0, 3 floats) to d_target. *d_n (device int64,
 * zeroed by the caller) counts appended rows; rows beyond n_cap are counted but not stored. */
vx_status vx_mlp_dataset(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                         const uint16_t *d_cell_desc, const vx_sample *d_samples, const int64_t *d_count,
                         int64_t cap, uint16_t *d_feat, float *d_target, int64_t *d_n, int64_t n_cap,
                         vx_stream s);
/* Features of the listed cells (BF16 [n][128], n = min(*d_count, cap)); cells whose patch leaves
 * a non-periodic grid get the clamped patch. */
vx_status vx_mlp_features(vx_handle *h, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                          const int64_t *d_count, int64_t cap, uint16_t *d_feat, vx_stream s);

/* One Adam step on the minibatch rows d_idx[0..n-1] of (d_feat, d_target) (d_idx NULL: rows
 * 0..n-1), n <= max_batch. d_loss (nullable, 2 floats) receives the batch's mean squared error
 * and mean confidence loss. */
vx_status vx_mlp_train_step(vx_mlp *m, const uint16_t *d_feat, const float *d_target, const int32_t *d_idx,
                            int64_t n, const vx_adam_params *p, float *d_loss, vx_stream s);
/* Gradient of the mean loss on rows 0..n-1 into d_grad (VX_MLP_NPARAMS floats, host layout),
 * without updating the parameters. */
vx_status vx_mlp_grad(vx_mlp *m, const uint16_t *d_feat, const float *d_target, int64_t n, float conf_lambda,
                      float conf_tol, float *d_grad, float *d_loss, vx_stream s);
/* Network outputs for rows 0..n-1: d_out[n][4] = (Z3[0], Z3[1], Z3[2], conf). */
vx_status vx_mlp_forward(vx_mlp *m, const uint16_t *d_feat, int64_t n, float *d_out, vx_stream s);

/* The network alone on listed cells (for measuring it before the Newton step): d_out[i][0..3] =
 * (Z3[0], Z3[1], Z3[2], conf) of cell d_cells[i] for i < min(*d_count, cap), from the 4x4x4 patch of
 * nodes at offsets -1..2 around the cell (the features of vx_mlp_features; on an open axis a patch
 * that leaves the grid takes the nearest nodes; an id outside the grid takes cell 0's patch),
 * computed by the inference kernel of vx_mlp_infer. d_out: device, 16-byte aligned. cap must not
 * exceed the cells reserved with vx_mlp_reserve (VX_ERR_INVALID otherwise); a count above cap is
 * reported by vx_sync_status. Allocates nothing, does not synchronise, uses the surrogate's
 * inference buffers (calls on one surrogate must not overlap in time). */
vx_status vx_mlp_predict(vx_mlp *m, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                         const int64_t *d_count, int64_t cap, float *d_out, vx_stream s);

/* Core samples of the listed cells (as vx_refine) through the surrogate. A cell whose first
 * estimate has two pierced faces, whose patch lies inside the grid and whose conf >= conf_threshold
 * gets the network's point x0 + Z3[0..2], projected onto the refinement's plane (through x0, normal
 * to grad Re psi x grad Im psi at x0) and polished by one Newton step on (Re psi, Im psi) in that
 * plane, FP32, with the refinement's own arithmetic (status VX_SAMPLE_SURROGATE, iters 1,
 * rho = |trilinear psi|^2 there). The polished point is kept only if the Newton step that would
 * follow it is at most max_step cells long (an estimate of its distance from the zero of psi in
 * the plane; max_step = 0 skips this test). Every other cell, and every cell whose polish fails
 * (degenerate tangent, singular Jacobian, point outside the patch, longer step), is refined by the
 * plain method with p (NULL = defaults), exactly as vx_refine would.
 * cap must not exceed the cells reserved with vx_mlp_reserve (VX_ERR_INVALID otherwise). The call
 * allocates nothing and does not synchronise; it uses the surrogate's inference buffers, so calls
 * on one surrogate must not overlap in time. */
vx_status vx_mlp_infer(vx_mlp *m, vx_dims dims, const void *d_psi, const uint64_t *d_cells,
                       const uint16_t *d_cell_desc, const int64_t *d_count, int64_t cap, float conf_threshold,
                       float max_step, const vx_refine_params *p, vx_sample *d_out, vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Batching: winding + compaction and refinement of many grids of uneven size (a time series of
 * frames, Sec. 5 timing over time steps) in one captured HIP graph.
 *
 * vx_batch_create validates the frames, builds the per-frame argument tables in device memory
 * (copied synchronously, once) and captures the work into a graph: the winding of every tile of
 * every frame is ONE kernel launch over the combined tile range, the refinement of every listed
 * cell of every frame is ONE launch whose work chunks never straddle frames. Each frame's results
 * are exactly those of vx_winding + vx_refine on that frame alone (same kernels, same arithmetic).
 *
 *   frames[f].d_psi, .dims, .out   as for vx_winding (out.d_counts receives the frame's counts)
 *   frames[f].d_samples            nullable; vx_sample[sample_cap]: refine the frame's listed cells
 *                                  (the first min(count, cell_cap, sample_cap) of them)
 * The buffers named in `frames` must stay allocated while the batch exists; their contents may
 * change between launches (new psi values, same shapes): that is the point of the replay.
 * nframes <= VX_BATCH_MAX_FRAMES. Launches of one batch must not overlap in time (they share the
 * batch's work counter); different batches are independent.
 * ---------------------------------------------------------------------------------------- */
#define VX_BATCH_MAX_FRAMES 128
typedef struct {
    vx_dims dims;
    const void *d_psi;
    vx_winding_out out;
    vx_sample *d_samples;
    int64_t sample_cap;
} vx_frame;
typedef struct vx_batch vx_batch;

/* p: refinement parameters (NULL = vx_refine_defaults()). The frame table is copied. */
vx_status vx_batch_create(vx_handle *h, const vx_frame *frames, int nframes, const vx_refine_params *p,
                          vx_batch **out);
/* Replay the captured graph on stream s. */
vx_status vx_batch_launch(vx_batch *b, vx_stream s);
/* The same kernels launched directly on s, without the graph (for checking the replay). */
vx_status vx_batch_launch_eager(vx_batch *b, vx_stream s);
/* Planes per z-chunk used for frame f (after autotuning, the tuned value). */
vx_status vx_batch_zchunk(const vx_batch *b, int frame, int *zchunk);
/* Resident refinement workgroups per CU the batch launches: 0 until vx_batch_autotune has chosen
 * one (the library's default is used), then the tuned value. */
vx_status vx_batch_refine_wg(const vx_batch *b, int *wg_per_cu);
/* Resident winding workgroups per CU the batch launches: 0 until vx_batch_autotune has chosen (as
 * many as fit), then the tuned value. */
vx_status vx_batch_wind_wg(const vx_batch *b, int *wg_per_cu);
/* Autotune the z-chunk depth of every distinct frame shape for this batch, by coordinate descent
 * over {8, 16, 32, 64, 128} (values above nz dropped) in two sweeps over the shapes, timing the
 * batched winding launch with HIP events on s (median of 7 after one warm-up); synchronises s.
 * cache_path (nullable) is a JSON
 * file of earlier results, one object per line: {"kind": "batch", "dims": [nx, ny, nz],
 * "periodic": p, "zchunk": z}; entries found there are used without timing, new results are
 * appended. Then, with those depths, the winding's resident workgroups per CU (as many as fit and
 * one or two fewer, set by the workgroup's LDS) and, on the lists of one winding, the refinement's
 * resident workgroups per CU (2 .. what fits), timed the same way, not cached. The graph is captured
 * again with the choices. */
vx_status vx_batch_autotune(vx_batch *b, const char *cache_path, vx_stream s);
vx_status vx_batch_destroy(vx_batch *b);

/* Autotune the z-chunk depth of vx_winding for one grid shape on the caller's field d_psi
 * (same candidates as above, one pass, timing the winding launch with HIP events on s, median of
 * 3 after one warm-up, with internal scratch outputs allocated for the duration of the call;
 * synchronises s); the handle then uses it for that shape.
 * cache_path as above with "kind": "grid". *zchunk (nullable) receives the choice. */
vx_status vx_autotune(vx_handle *h, vx_dims dims, const void *d_psi, const char *cache_path, int *zchunk,
                      vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Density for the error metric of the vectorised lines (Sec. 5: e = sum_i rho(x_i) / (mean rho * N)
 * over N points x_i of the lines; rho = 0 on a true core).
 *   vx_density       d_rho float[n] = |psi|^2 at d_points double[n][3] (grid coordinates; wrapped on
 *                    periodic axes, extrapolated from the last cell on open ones), psi linearly
 *                    interpolated between nodes (Sec. 5) in the refinement's FP32 arithmetic. Every
 *                    axis needs >= 2 nodes.
 *   vx_mean_density  *d_out (device double) = mean over all nodes of |psi|^2, accumulated in FP64.
 * ---------------------------------------------------------------------------------------- */
vx_status vx_density(vx_handle *h, vx_dims dims, const void *d_psi, const double *d_points, int64_t n, float *d_rho,
                     vx_stream s);
vx_status vx_mean_density(vx_handle *h, vx_dims dims, const void *d_psi, double *d_out, vx_stream s);

/* ------------------------------------------------------------------------------------------
 * Host consumers of the lists (host memory in and out; synchronous; no device work).
 *
 * Dual graph of the vortex lines (Sec. 3.1 graph of vortex nodes, in dual form): the vertices are
 * the listed pierced cells, and every pierced face joins the two cells that share it (the face's
 * winding orients the edge by the right-hand rule, Sec. 3.4). Connected components by depth-first
 * traversal (Sec. 3.2) started from the unvisited cell of lowest id, so component c is the one whose
 * lowest cell id is the c-th smallest of all components' lowest ids. Class of a component from the
 * connectivity (number of neighbour cells) of its vertices (Sec. 3.4): Type I simple open line
 * (all <= 2, some < 2: it ends on a non-periodic boundary), Type II simple closed line (all 2),
 * Type III complex line (some > 2). Vertices of connectivity > 2 are branch points, the
 * reconnection candidates of Sec. 4.2 (cells with four or six pierced faces). A pierced face on a
 * non-periodic boundary has no second cell: it is a boundary face of its cell.
 *   h_cells, h_cell_desc  the pierced cells and their descriptors (as vx_winding lists them, any
 *                         order, n entries; every pierced face's other cell must be listed)
 *   h_comp    int64[n]  component of each input cell
 *   h_degree  int32[n]  (nullable) its connectivity
 *   h_comp_type int32[n] (nullable) type (1, 2, 3) of component c at index c (at most n components)
 * VX_ERR_INVALID for a duplicate cell, a cell id outside the grid, or a pierced face whose other cell
 * is not listed (stats->bad_input then gives the input position). */
typedef struct {
    int64_t nvert;      /* vertices (listed cells) */
    int64_t nedge;      /* edges: pierced faces shared by two listed cells */
    int64_t nboundary;  /* pierced faces on a non-periodic boundary */
    int64_t ncomp;      /* connected components */
    int64_t ntype[3];   /* components of Type I, II, III */
    int64_t nbranch;    /* vertices of connectivity > 2 */
    int64_t bad_input;  /* input position of an invalid entry (-1 if none) */
} vx_graph_stats;
vx_status vx_graph_lines(vx_dims dims, const uint64_t *h_cells, const uint16_t *h_cell_desc, int64_t n,
                         int64_t *h_comp, int32_t *h_degree, int32_t *h_comp_type, vx_graph_stats *stats);

/* Sample points by box means and iterative graph reduction (Sec. 3.3.1 candidate sample points,
 * Sec. 3.3.2 graph reduction), on the dual graph above. Each vertex (pierced cell) stands at its
 * first estimate: min corner + mean of its pierced-face centres. One pass: take the unprocessed
 * vertex of lowest id (or the seed chosen below); collect, by depth-first traversal from it, the
 * connected unprocessed vertices whose position lies in the box of side box_k cells centred on it
 * (|dx|, |dy|, |dz| <= box_k / 2, minimum image on periodic axes); they collapse into one new node at
 * their mean position (sums in ascending vertex order, relative to the first vertex, wrapped into
 * the grid); the next vertex is the lowest-id unprocessed neighbour of the collapsed ones, else the
 * lowest unprocessed vertex. The new nodes, numbered in creation order, are joined where any of their
 * members were. Passes repeat on the reduced graph until one merges nothing (the positions have
 * converged) or max_passes is reached. Host memory; synchronous.
 *   vx_reduce         builds the reduced graph (*out, freed by vx_reduced_destroy); VX_ERR_INVALID
 *                     for lists vx_graph_lines rejects, box_k outside 1..64, max_passes outside 1..64
 *   vx_reduced_info   number of nodes, of edges, passes run
 *   vx_reduced_get    (each nullable) h_pos double[nnode][3] node positions; h_edges int64[nedge][2]
 *                     (u < v, ascending); h_members int64[nnode] pierced cells merged into each node;
 *                     h_comp int64[nnode] component of the dual graph it came from
 *   vx_reduced_seeds  the refinement inputs of the nodes (for vx_refine's caller seeds): the cell that
 *                     holds each node (clamped to the cells of an open axis), that cell's descriptor
 *                     if it is in the given pierced list (else 0), and the node's offset from the
 *                     cell's min corner (FP32, cell-local as vx_refine takes it) */
typedef struct vx_reduced vx_reduced;
vx_status vx_reduce(vx_dims dims, const uint64_t *h_cells, const uint16_t *h_cell_desc, int64_t n, int box_k,
                    int max_passes, vx_reduced **out);
vx_status vx_reduced_info(const vx_reduced *r, int64_t *nnode, int64_t *nedge, int32_t *passes);
vx_status vx_reduced_get(const vx_reduced *r, double *h_pos, int64_t *h_edges, int64_t *h_members, int64_t *h_comp);
vx_status vx_reduced_seeds(const vx_reduced *r, const uint64_t *h_cells, const uint16_t *h_cell_desc, int64_t n,
                           uint64_t *h_seed_cell, uint16_t *h_seed_desc, float *h_seed_off);
vx_status vx_reduced_destroy(vx_reduced *r);

/* Vectorisation (Sec. 3.4) of a sample graph (positions h_pos double[n][3] in grid coordinates,
 * undirected edges h_edges int64[nedge][2]; e.g. vx_reduced_get's output after refinement): the graph
 * is split at its ends and branch points (connectivity other than 2) into chains -- from each such
 * node in ascending order, along its edges in ascending neighbour order, through connectivity-2
 * nodes to the next such node; what remains are loops, each started at its lowest node towards its
 * lower neighbour (Type II lines, closed curves); an isolated node is a chain of one point. Each
 * chain's samples are unwrapped along it (minimum image on periodic axes) and interpolated by a
 * uniform Catmull-Rom spline: seg_points points per segment plus the last point (a loop closes on
 * its first node, shifted by the loop's lattice displacement if it winds round the periodic grid);
 * open chains repeat their end points as outer control points. Curve length = length of that
 * polyline. Host memory; synchronous.
 *   vx_curves_info  number of curves, points, chain nodes, and the total length
 *   vx_curves_get   (each nullable) h_pt_start int64[ncurve+1] (curve c: points [start[c],
 *                   start[c+1])), h_points double[npoint][3], h_length double[ncurve], h_closed
 *                   int32[ncurve], h_node_start int64[ncurve+1], h_nodes int64[nnode] (the ordered
 *                   sample nodes of each chain) */
typedef struct vx_curves vx_curves;
vx_status vx_curves_build(vx_dims dims, const double *h_pos, int64_t n, const int64_t *h_edges, int64_t nedge,
                          int seg_points, vx_curves **out);
vx_status vx_curves_info(const vx_curves *c, int64_t *ncurve, int64_t *npoint, int64_t *nnode, double *total_length);
vx_status vx_curves_get(const vx_curves *c, int64_t *h_pt_start, double *h_points, double *h_length, int32_t *h_closed,
                        int64_t *h_node_start, int64_t *h_nodes);
vx_status vx_curves_destroy(vx_curves *c);

/* ------------------------------------------------------------------------------------------
 * Kernel timing with HIP events on the launch stream (measurement support).
 * kind: 0 = winding kernel, 1 = refinement kernel, 2 = surrogate network (inference: the network
 * kernel; training: a whole step), 3 = batch, 4 = surrogate polish, 5 = node circulation.
 * ---------------------------------------------------------------------------------------- */
vx_status vx_profile_enable(vx_handle *h, int enable); /* enabling clears the accumulators */
/* Sum of the recorded kernel durations (ms) and their number; synchronises the recorded events. */
vx_status vx_profile_read(vx_handle *h, int kind, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* VX_H */
