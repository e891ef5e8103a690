"""Python binding of libvx.so: argument marshalling only.

Every compute step runs in the library's HIP kernels. PyTorch provides device memory and the
stream; tensors are passed by data pointer. The functions carry the C-ABI names and raise
``VxError`` when a call returns a non-zero status. There is no CPU fallback: without a built
``libvx.so`` (and a GPU) the calls fail.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvx.so")

_lib = None

VX_OK, VX_ERR_INVALID, VX_ERR_CAPACITY, VX_ERR_DEVICE, VX_ERR_NOMEM, VX_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5

SAMPLE_MULTI = 1
SAMPLE_TANGENT_FALLBACK = 2
SAMPLE_BOUNDARY = 4
SAMPLE_NONZERO_MIN = 8
SAMPLE_NOT_CONVERGED = 16
SAMPLE_NO_FACES = 32
SAMPLE_BAD_CELL = 64

KIND_WIND, KIND_REFINE, KIND_MLP, KIND_BATCH, KIND_POLISH, KIND_NODE = 0, 1, 2, 3, 4, 5

# every symbol include/vx.h declares
EXPORTS = ["vx_sync_status", "vx_version", "vx_create", "vx_destroy", "vx_status_str", "vx_last_error", "vx_gen_tangle",
           "vx_gen_line_ring", "vx_winding", "vx_wind_config", "vx_refine_defaults", "vx_refine",
           "vx_refine_noalloc", "vx_node_circulation", "vx_graph_lines",
           "vx_reduce", "vx_reduced_info", "vx_reduced_get", "vx_reduced_seeds", "vx_reduced_destroy",
           "vx_curves_build", "vx_curves_info", "vx_curves_get", "vx_curves_destroy",
           "vx_density", "vx_mean_density",
           "vx_batch_create", "vx_batch_launch", "vx_batch_launch_eager", "vx_batch_zchunk", "vx_batch_refine_wg",
           "vx_batch_wind_wg",
           "vx_batch_autotune", "vx_batch_destroy", "vx_autotune", "vx_mlp_create", "vx_mlp_destroy",
           "vx_mlp_reserve", "vx_mlp_get_params", "vx_mlp_set_params", "vx_mlp_save", "vx_mlp_load", "vx_mlp_dataset",
           "vx_mlp_features", "vx_mlp_train_step", "vx_mlp_grad", "vx_mlp_forward", "vx_mlp_predict", "vx_mlp_infer",
           "vx_profile_enable", "vx_profile_read"]

MLP_NHID = 128
MLP_NPARAMS = 128 * MLP_NHID + MLP_NHID + MLP_NHID * MLP_NHID + MLP_NHID + MLP_NHID * 4 + 4  # 33540
SAMPLE_SURROGATE = 128

BATCH_MAX_FRAMES = 128


class VxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{status}: {msg}")
        self.status = status


class Dims(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("periodic", ctypes.c_uint32)]


class Tangle(ctypes.Structure):
    _fields_ = [("nwaves", ctypes.c_int32), ("table_size", ctypes.c_uint32), ("d_ax", ctypes.c_void_p),
                ("d_ay", ctypes.c_void_p), ("d_az", ctypes.c_void_p), ("d_coef", ctypes.c_void_p),
                ("d_table", ctypes.c_void_p)]


class LineRing(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("line_x", "line_y", "ring_cx", "ring_cy", "ring_cz", "radius", "xi")]


class WindingOut(ctypes.Structure):
    _fields_ = [("d_wind", ctypes.c_void_p), ("d_faces", ctypes.c_void_p), ("d_face_sign", ctypes.c_void_p),
                ("face_cap", ctypes.c_int64), ("d_cells", ctypes.c_void_p), ("d_cell_desc", ctypes.c_void_p),
                ("cell_cap", ctypes.c_int64), ("d_counts", ctypes.c_void_p)]


class RefineParams(ctypes.Structure):
    _fields_ = [("max_descent", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("step0", ctypes.c_float), ("step_max", ctypes.c_float),
                ("armijo", ctypes.c_float), ("descent_tol", ctypes.c_float), ("newton_tol", ctypes.c_float),
                ("rho_tol", ctypes.c_float)]


class Sample(ctypes.Structure):
    _fields_ = [("cell", ctypes.c_uint64), ("off", ctypes.c_float * 3), ("rho", ctypes.c_float),
                ("iters", ctypes.c_uint16), ("status", ctypes.c_uint16), ("reserved", ctypes.c_uint32)]


assert ctypes.sizeof(Sample) == 32


class AdamParams(ctypes.Structure):
    _fields_ = [(n, ctypes.c_float) for n in ("lr", "beta1", "beta2", "eps", "conf_lambda", "conf_tol")]


class GraphStats(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int64), ("nedge", ctypes.c_int64), ("nboundary", ctypes.c_int64),
                ("ncomp", ctypes.c_int64), ("ntype", ctypes.c_int64 * 3), ("nbranch", ctypes.c_int64),
                ("bad_input", ctypes.c_int64)]


class Frame(ctypes.Structure):
    _fields_ = [("dims", Dims), ("d_psi", ctypes.c_void_p), ("out", WindingOut), ("d_samples", ctypes.c_void_p),
                ("sample_cap", ctypes.c_int64)]


def build():
    from . import _build
    return _build.build()


def lib() -> ctypes.CDLL:
    """Load libvx.so (building it first if it has never been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P, i, st = ctypes.c_void_p, ctypes.c_int, ctypes.c_int
        L.vx_version.restype = i
        L.vx_create.argtypes = [i, ctypes.POINTER(P)]
        L.vx_create.restype = st
        L.vx_destroy.argtypes = [P]
        L.vx_destroy.restype = st
        L.vx_sync_status.argtypes = [P, P]
        L.vx_sync_status.restype = st
        L.vx_status_str.argtypes = [i]
        L.vx_status_str.restype = ctypes.c_char_p
        L.vx_last_error.argtypes = [P]
        L.vx_last_error.restype = ctypes.c_char_p
        L.vx_gen_tangle.argtypes = [P, Dims, ctypes.POINTER(Tangle), P, P]
        L.vx_gen_tangle.restype = st
        L.vx_gen_line_ring.argtypes = [P, Dims, ctypes.POINTER(LineRing), P, P, P]
        L.vx_gen_line_ring.restype = st
        L.vx_winding.argtypes = [P, Dims, P, ctypes.POINTER(WindingOut), P]
        L.vx_winding.restype = st
        L.vx_wind_config.argtypes = [P, i]
        L.vx_wind_config.restype = st
        L.vx_refine_defaults.argtypes = []
        L.vx_refine_defaults.restype = RefineParams
        L.vx_refine.argtypes = [P, Dims, P, P, P, P, P, ctypes.c_int64, ctypes.POINTER(RefineParams), P, P]
        L.vx_refine.restype = st
        L.vx_graph_lines.argtypes = [Dims, P, P, ctypes.c_int64, P, P, P, ctypes.POINTER(GraphStats)]
        L.vx_graph_lines.restype = st
        L.vx_reduce.argtypes = [Dims, P, P, ctypes.c_int64, i, i, ctypes.POINTER(P)]
        L.vx_reduced_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int32)]
        L.vx_reduced_get.argtypes = [P, P, P, P, P]
        L.vx_reduced_seeds.argtypes = [P, P, P, ctypes.c_int64, P, P, P]
        L.vx_reduced_destroy.argtypes = [P]
        for name in ("vx_reduce", "vx_reduced_info", "vx_reduced_get", "vx_reduced_seeds", "vx_reduced_destroy"):
            getattr(L, name).restype = st
        L.vx_curves_build.argtypes = [Dims, P, ctypes.c_int64, P, ctypes.c_int64, i, ctypes.POINTER(P)]
        L.vx_curves_info.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                     ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double)]
        L.vx_curves_get.argtypes = [P, P, P, P, P, P, P]
        L.vx_curves_destroy.argtypes = [P]
        for name in ("vx_curves_build", "vx_curves_info", "vx_curves_get", "vx_curves_destroy"):
            getattr(L, name).restype = st
        L.vx_density.argtypes = [P, Dims, P, P, ctypes.c_int64, P, P]
        L.vx_density.restype = st
        L.vx_mean_density.argtypes = [P, Dims, P, P, P]
        L.vx_mean_density.restype = st
        L.vx_node_circulation.argtypes = [P, Dims, P, P, P, ctypes.c_int64, P, P]
        L.vx_node_circulation.restype = st
        L.vx_refine_noalloc.argtypes = [Dims, P, P, P, P, P, ctypes.c_int64, ctypes.POINTER(RefineParams), P, P]
        L.vx_refine_noalloc.restype = st
        L.vx_batch_create.argtypes = [P, ctypes.POINTER(Frame), i, ctypes.POINTER(RefineParams), ctypes.POINTER(P)]
        L.vx_batch_create.restype = st
        L.vx_batch_launch.argtypes = [P, P]
        L.vx_batch_launch.restype = st
        L.vx_batch_launch_eager.argtypes = [P, P]
        L.vx_batch_launch_eager.restype = st
        L.vx_batch_zchunk.argtypes = [P, i, ctypes.POINTER(i)]
        L.vx_batch_zchunk.restype = st
        L.vx_batch_refine_wg.argtypes = [P, ctypes.POINTER(i)]
        L.vx_batch_refine_wg.restype = st
        L.vx_batch_wind_wg.argtypes = [P, ctypes.POINTER(i)]
        L.vx_batch_wind_wg.restype = st
        L.vx_batch_autotune.argtypes = [P, ctypes.c_char_p, P]
        L.vx_batch_autotune.restype = st
        L.vx_batch_destroy.argtypes = [P]
        L.vx_batch_destroy.restype = st
        L.vx_autotune.argtypes = [P, Dims, P, ctypes.c_char_p, ctypes.POINTER(i), P]
        L.vx_autotune.restype = st
        i64, f = ctypes.c_int64, ctypes.c_float
        L.vx_mlp_create.argtypes = [P, P, i64, ctypes.POINTER(P)]
        L.vx_mlp_destroy.argtypes = [P]
        L.vx_mlp_reserve.argtypes = [P, i64]
        L.vx_mlp_get_params.argtypes = [P, P]
        L.vx_mlp_set_params.argtypes = [P, P]
        L.vx_mlp_save.argtypes = [P, ctypes.c_char_p]
        L.vx_mlp_load.argtypes = [P, ctypes.c_char_p]
        L.vx_mlp_dataset.argtypes = [P, Dims, P, P, P, P, P, i64, P, P, P, i64, P]
        L.vx_mlp_features.argtypes = [P, Dims, P, P, P, i64, P, P]
        L.vx_mlp_train_step.argtypes = [P, P, P, P, i64, ctypes.POINTER(AdamParams), P, P]
        L.vx_mlp_grad.argtypes = [P, P, P, i64, f, f, P, P, P]
        L.vx_mlp_forward.argtypes = [P, P, i64, P, P]
        L.vx_mlp_predict.argtypes = [P, Dims, P, P, P, i64, P, P]
        L.vx_mlp_infer.argtypes = [P, Dims, P, P, P, P, i64, f, f, ctypes.POINTER(RefineParams), P, P]
        for name in ("vx_mlp_create", "vx_mlp_destroy", "vx_mlp_reserve", "vx_mlp_get_params", "vx_mlp_set_params", "vx_mlp_save",
                     "vx_mlp_load", "vx_mlp_dataset", "vx_mlp_features", "vx_mlp_train_step", "vx_mlp_grad",
                     "vx_mlp_forward", "vx_mlp_predict", "vx_mlp_infer"):
            getattr(L, name).restype = st
        L.vx_profile_enable.argtypes = [P, i]
        L.vx_profile_enable.restype = st
        L.vx_profile_read.argtypes = [P, i, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.vx_profile_read.restype = st
        _lib = L
    return _lib


# ---------------------------------------------------------------------------------------------- helpers
def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _check(h, status: int, what: str):
    if status != VX_OK:
        L = lib()
        detail = L.vx_last_error(h).decode() if h else ""
        raise VxError(status, f"{what}: {L.vx_status_str(status).decode()} {detail}")


def dims(nx: int, ny: int, nz: int, periodic: int = 7) -> Dims:
    return Dims(int(nx), int(ny), int(nz), int(periodic))


# ---------------------------------------------------------------------------------------------- C-ABI
def vx_version() -> int:
    return lib().vx_version()


def vx_create(device: int = 0):
    h = ctypes.c_void_p()
    _check(None, lib().vx_create(int(device), ctypes.byref(h)), "vx_create")
    return h


def vx_destroy(h) -> None:
    _check(None, lib().vx_destroy(h), "vx_destroy")


def vx_last_error(h) -> str:
    return lib().vx_last_error(h).decode()


def vx_gen_tangle(h, d: Dims, ax, ay, az, coef, table, psi, stream=None):
    t = Tangle(int(ax.numel()), int(table.shape[0]), _ptr(ax), _ptr(ay), _ptr(az), _ptr(coef), _ptr(table))
    _check(h, lib().vx_gen_tangle(h, d, ctypes.byref(t), _ptr(psi), _stream(stream)), "vx_gen_tangle")


def vx_gen_line_ring(h, d: Dims, params, noise, psi, stream=None):
    p = LineRing(*[float(v) for v in params])
    _check(h, lib().vx_gen_line_ring(h, d, ctypes.byref(p), _ptr(noise), _ptr(psi), _stream(stream)),
           "vx_gen_line_ring")


def vx_winding(h, d: Dims, psi, counts, wind=None, faces=None, fsign=None, cells=None, cdesc=None,
               stream=None):
    out = WindingOut(_ptr(wind), _ptr(faces), _ptr(fsign), int(faces.numel()) if faces is not None else 0,
                     _ptr(cells), _ptr(cdesc), int(cells.numel()) if cells is not None else 0, _ptr(counts))
    _check(h, lib().vx_winding(h, d, _ptr(psi), ctypes.byref(out), _stream(stream)), "vx_winding")


def vx_wind_config(h, zchunk: int = 0):
    _check(h, lib().vx_wind_config(h, int(zchunk)), "vx_wind_config")


def vx_sync_status(h, stream=None):
    """Raises VxError(VX_ERR_CAPACITY) if a list overflowed since the last call (clears the flag)."""
    _check(h, lib().vx_sync_status(h, _stream(stream)), "vx_sync_status")


def vx_refine_defaults() -> RefineParams:
    return lib().vx_refine_defaults()


def vx_refine(h, d: Dims, psi, cells, cdesc, count, out, params: RefineParams | None = None, seed=None,
              stream=None, cap: int | None = None):
    cap = int(out.numel() * out.element_size() // 32) if cap is None else int(cap)
    prm = params if params is not None else vx_refine_defaults()
    _check(h, lib().vx_refine(h, d, _ptr(psi), _ptr(cells), _ptr(cdesc), _ptr(seed), _ptr(count), cap,
                              ctypes.byref(prm), _ptr(out), _stream(stream)), "vx_refine")


def vx_graph_lines(d: Dims, cells, cdesc):
    """Dual graph of host lists (numpy uint64 cells, uint16 descriptors): (comp int64[n], degree
    int32[n], comp_type int32[ncomp], stats dict)."""
    import numpy as np
    cells = np.ascontiguousarray(cells, np.uint64)
    cdesc = np.ascontiguousarray(cdesc, np.uint16)
    n = len(cells)
    comp = np.empty(n, np.int64)
    deg = np.empty(n, np.int32)
    ctype = np.empty(max(n, 1), np.int32)
    st = GraphStats()
    status = lib().vx_graph_lines(d, cells.ctypes.data, cdesc.ctypes.data, n, comp.ctypes.data, deg.ctypes.data,
                                  ctype.ctypes.data, ctypes.byref(st))
    if status != VX_OK:
        raise VxError(status, f"vx_graph_lines: {lib().vx_status_str(status).decode()} (input {st.bad_input})")
    stats = {"nvert": st.nvert, "nedge": st.nedge, "nboundary": st.nboundary, "ncomp": st.ncomp,
             "ntype": list(st.ntype), "nbranch": st.nbranch}
    return comp, deg, ctype[:st.ncomp].copy(), stats


def vx_reduce(d: Dims, cells, cdesc, box_k: int, max_passes: int = 5):
    """Reduced sample graph of host lists: dict with pos (m, 3), edges (e, 2), members, comp, passes,
    and the refinement seeds (seed_cell, seed_desc, seed_off) of the nodes."""
    import numpy as np
    cells = np.ascontiguousarray(cells, np.uint64)
    cdesc = np.ascontiguousarray(cdesc, np.uint16)
    r = ctypes.c_void_p()
    L = lib()
    st = L.vx_reduce(d, cells.ctypes.data, cdesc.ctypes.data, len(cells), int(box_k), int(max_passes), ctypes.byref(r))
    if st != VX_OK:
        raise VxError(st, f"vx_reduce: {L.vx_status_str(st).decode()}")
    try:
        nn, ne, npass = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
        L.vx_reduced_info(r, ctypes.byref(nn), ctypes.byref(ne), ctypes.byref(npass))
        m, e = nn.value, ne.value
        pos = np.empty((m, 3), np.float64)
        edges = np.empty((e, 2), np.int64)
        members = np.empty(m, np.int64)
        comp = np.empty(m, np.int64)
        L.vx_reduced_get(r, pos.ctypes.data, edges.ctypes.data, members.ctypes.data, comp.ctypes.data)
        seed_cell = np.empty(m, np.uint64)
        seed_desc = np.empty(m, np.uint16)
        seed_off = np.empty((m, 3), np.float32)
        st = L.vx_reduced_seeds(r, cells.ctypes.data, cdesc.ctypes.data, len(cells), seed_cell.ctypes.data,
                                seed_desc.ctypes.data, seed_off.ctypes.data)
        if st != VX_OK:
            raise VxError(st, "vx_reduced_seeds")
    finally:
        L.vx_reduced_destroy(r)
    return {"pos": pos, "edges": edges, "members": members, "comp": comp, "passes": npass.value,
            "seed_cell": seed_cell, "seed_desc": seed_desc, "seed_off": seed_off}


def vx_curves(d: Dims, pos, edges, seg_points: int = 8):
    """Catmull-Rom curves of a sample graph (host arrays): dict with pt_start, points, length, closed,
    node_start, nodes, total_length."""
    import numpy as np
    pos = np.ascontiguousarray(pos, np.float64).reshape(-1, 3)
    edges = np.ascontiguousarray(edges, np.int64).reshape(-1, 2)
    L = lib()
    c = ctypes.c_void_p()
    st = L.vx_curves_build(d, pos.ctypes.data, len(pos), edges.ctypes.data, len(edges), int(seg_points),
                           ctypes.byref(c))
    if st != VX_OK:
        raise VxError(st, f"vx_curves_build: {L.vx_status_str(st).decode()}")
    try:
        nc, npt, nn, tot = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64(), ctypes.c_double()
        L.vx_curves_info(c, ctypes.byref(nc), ctypes.byref(npt), ctypes.byref(nn), ctypes.byref(tot))
        r = {"pt_start": np.empty(nc.value + 1, np.int64), "points": np.empty((npt.value, 3), np.float64),
             "length": np.empty(nc.value, np.float64), "closed": np.empty(nc.value, np.int32),
             "node_start": np.empty(nc.value + 1, np.int64), "nodes": np.empty(nn.value, np.int64)}
        L.vx_curves_get(c, *(r[k].ctypes.data for k in ("pt_start", "points", "length", "closed", "node_start",
                                                         "nodes")))
        r["total_length"] = tot.value
    finally:
        L.vx_curves_destroy(c)
    return r


def vx_density(h, d: Dims, psi, points, rho, stream=None):
    """rho (float32 [n]) = |trilinear psi|^2 at points (float64 [n, 3] device tensor)."""
    _check(h, lib().vx_density(h, d, _ptr(psi), _ptr(points), int(points.shape[0]), _ptr(rho), _stream(stream)),
           "vx_density")


def vx_mean_density(h, d: Dims, psi, out, stream=None):
    _check(h, lib().vx_mean_density(h, d, _ptr(psi), _ptr(out), _stream(stream)), "vx_mean_density")


def vx_node_circulation(h, d: Dims, wind, count, node=None, nodes=None, stream=None):
    cap = int(nodes.numel()) if nodes is not None else 0
    _check(h, lib().vx_node_circulation(h, d, _ptr(wind), _ptr(node), _ptr(nodes), cap, _ptr(count),
                                        _stream(stream)), "vx_node_circulation")


def vx_refine_noalloc(d: Dims, psi, cells, cdesc, count, out, params: RefineParams | None = None, seed=None,
                      stream=None, cap: int | None = None):
    """vx_refine without a handle or any allocation (on the current device; see include/vx.h)."""
    cap = int(out.numel() * out.element_size() // 32) if cap is None else int(cap)
    prm = params if params is not None else vx_refine_defaults()
    st = lib().vx_refine_noalloc(d, _ptr(psi), _ptr(cells), _ptr(cdesc), _ptr(seed), _ptr(count), cap,
                                 ctypes.byref(prm), _ptr(out), _stream(stream))
    if st != VX_OK:
        raise VxError(st, f"vx_refine_noalloc: {lib().vx_status_str(st).decode()}")


def winding_out(counts, wind=None, faces=None, fsign=None, cells=None, cdesc=None) -> WindingOut:
    return WindingOut(_ptr(wind), _ptr(faces), _ptr(fsign), int(faces.numel()) if faces is not None else 0,
                      _ptr(cells), _ptr(cdesc), int(cells.numel()) if cells is not None else 0, _ptr(counts))


def vx_batch_create(h, frames, params: RefineParams | None = None):
    """frames: sequence of Frame structures. Returns the batch handle."""
    arr = (Frame * len(frames))(*frames)
    b = ctypes.c_void_p()
    prm = ctypes.byref(params) if params is not None else None
    _check(h, lib().vx_batch_create(h, arr, len(frames), prm, ctypes.byref(b)), "vx_batch_create")
    return b


def vx_batch_launch(h, b, stream=None):
    _check(h, lib().vx_batch_launch(b, _stream(stream)), "vx_batch_launch")


def vx_batch_launch_eager(h, b, stream=None):
    _check(h, lib().vx_batch_launch_eager(b, _stream(stream)), "vx_batch_launch_eager")


def vx_batch_zchunk(h, b, frame: int) -> int:
    z = ctypes.c_int()
    _check(h, lib().vx_batch_zchunk(b, int(frame), ctypes.byref(z)), "vx_batch_zchunk")
    return z.value


def vx_batch_refine_wg(h, b) -> int:
    w = ctypes.c_int()
    _check(h, lib().vx_batch_refine_wg(b, ctypes.byref(w)), "vx_batch_refine_wg")
    return w.value


def vx_batch_wind_wg(h, b) -> int:
    w = ctypes.c_int()
    _check(h, lib().vx_batch_wind_wg(b, ctypes.byref(w)), "vx_batch_wind_wg")
    return w.value


def vx_batch_autotune(h, b, cache_path: str | None = None, stream=None):
    path = cache_path.encode() if cache_path else None
    _check(h, lib().vx_batch_autotune(b, path, _stream(stream)), "vx_batch_autotune")


def vx_batch_destroy(h, b):
    _check(h, lib().vx_batch_destroy(b), "vx_batch_destroy")


def vx_autotune(h, d: Dims, psi, cache_path: str | None = None, stream=None) -> int:
    z = ctypes.c_int()
    path = cache_path.encode() if cache_path else None
    _check(h, lib().vx_autotune(h, d, _ptr(psi), path, ctypes.byref(z), _stream(stream)), "vx_autotune")
    return z.value


# ---------------------------------------------------------------------------------------------- surrogate
def _host_f32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    if a.size != MLP_NPARAMS:
        raise ValueError(f"expected {MLP_NPARAMS} parameters, got {a.size}")
    return a


def vx_mlp_create(h, params, max_batch: int):
    a = _host_f32(params)
    m = ctypes.c_void_p()
    _check(h, lib().vx_mlp_create(h, a.ctypes.data, int(max_batch), ctypes.byref(m)), "vx_mlp_create")
    return m


def vx_mlp_destroy(h, m):
    _check(h, lib().vx_mlp_destroy(m), "vx_mlp_destroy")


def vx_mlp_reserve(h, m, max_cells: int):
    _check(h, lib().vx_mlp_reserve(m, int(max_cells)), "vx_mlp_reserve")


def vx_mlp_get_params(h, m):
    import numpy as np
    a = np.empty(MLP_NPARAMS, np.float32)
    _check(h, lib().vx_mlp_get_params(m, a.ctypes.data), "vx_mlp_get_params")
    return a


def vx_mlp_set_params(h, m, params):
    a = _host_f32(params)
    _check(h, lib().vx_mlp_set_params(m, a.ctypes.data), "vx_mlp_set_params")


def vx_mlp_save(h, m, path: str):
    _check(h, lib().vx_mlp_save(m, path.encode()), "vx_mlp_save")


def vx_mlp_load(h, m, path: str):
    _check(h, lib().vx_mlp_load(m, path.encode()), "vx_mlp_load")


def vx_mlp_dataset(h, d: Dims, psi, cells, cdesc, samples, count, cap, feat, target, n_out, n_cap, stream=None):
    _check(h, lib().vx_mlp_dataset(h, d, _ptr(psi), _ptr(cells), _ptr(cdesc), _ptr(samples), _ptr(count), int(cap),
                                   _ptr(feat), _ptr(target), _ptr(n_out), int(n_cap), _stream(stream)),
           "vx_mlp_dataset")


def vx_mlp_features(h, d: Dims, psi, cells, count, cap, feat, stream=None):
    _check(h, lib().vx_mlp_features(h, d, _ptr(psi), _ptr(cells), _ptr(count), int(cap), _ptr(feat),
                                    _stream(stream)), "vx_mlp_features")


def vx_mlp_train_step(h, m, feat, target, idx, n: int, adam: AdamParams, loss=None, stream=None):
    _check(h, lib().vx_mlp_train_step(m, _ptr(feat), _ptr(target), _ptr(idx), int(n), ctypes.byref(adam), _ptr(loss),
                                      _stream(stream)), "vx_mlp_train_step")


def vx_mlp_grad(h, m, feat, target, n: int, conf_lambda: float, conf_tol: float, grad, loss=None, stream=None):
    _check(h, lib().vx_mlp_grad(m, _ptr(feat), _ptr(target), int(n), float(conf_lambda), float(conf_tol), _ptr(grad),
                                _ptr(loss), _stream(stream)), "vx_mlp_grad")


def vx_mlp_forward(h, m, feat, n: int, out, stream=None):
    _check(h, lib().vx_mlp_forward(m, _ptr(feat), int(n), _ptr(out), _stream(stream)), "vx_mlp_forward")


def vx_mlp_predict(h, m, d: Dims, psi, cells, count, cap, out, stream=None):
    _check(h, lib().vx_mlp_predict(m, d, _ptr(psi), _ptr(cells), _ptr(count), int(cap), _ptr(out), _stream(stream)),
           "vx_mlp_predict")


# default acceptance bound of the surrogate's polished point: the Newton step that would follow it (an
# estimate of its distance from the core) must be at most this many cells
MLP_MAX_STEP = 0.02


def vx_mlp_infer(h, m, d: Dims, psi, cells, cdesc, count, cap, conf_threshold: float, out,
                 params: RefineParams | None = None, stream=None, max_step: float = MLP_MAX_STEP):
    prm = params if params is not None else vx_refine_defaults()
    _check(h, lib().vx_mlp_infer(m, d, _ptr(psi), _ptr(cells), _ptr(cdesc), _ptr(count), int(cap),
                                 float(conf_threshold), float(max_step), ctypes.byref(prm), _ptr(out),
                                 _stream(stream)), "vx_mlp_infer")


def vx_profile_enable(h, enable: bool = True):
    _check(h, lib().vx_profile_enable(h, int(bool(enable))), "vx_profile_enable")


def vx_profile_read(h, kind: int):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(h, lib().vx_profile_read(h, int(kind), ctypes.byref(ms), ctypes.byref(n)), "vx_profile_read")
    return ms.value, n.value


from .pipeline import (Batch, Extractor, FramePipeline, length_histogram, lines_by_length,  # noqa: E402,F401
                       samples_to_numpy, upload_tangle)
