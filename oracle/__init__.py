"""CPU ORACLE -- test infrastructure only.

Plain, slow reference implementation of the vortex-core hot path of Liu, Xiong & Liu,
"Vectorizing Quantum Turbulence Vortex-Core Lines for Real-Time Visualization"
(arXiv 1911.12070). Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import it. It shares no code with the GPU library (``paper_1911_12070_amd``)
and never imports it.

Parts:
  * ``vxo.c`` (plain C, built here with gcc): face windings, pierced sets, packed field,
    core-sample refinement -- see the comments there for the paper passages each follows.
  * this module: ctypes wrappers, the plain-definition evaluation of the synthetic fields
    (generator check) and the FP64 surrogate network (``oracle.mlp``).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libvxo.so")
_SRC = os.path.join(_HERE, "vxo.c")
_lib = None

# status bits of a refined sample
MULTI = 1
TANGENT_FALLBACK = 2
BOUNDARY = 4
NONZERO_MIN = 8
NOT_CONVERGED = 16
NO_FACES = 32


def build(force: bool = True) -> str:
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


class _RefineParams(ctypes.Structure):
    _fields_ = [("max_descent", ctypes.c_int32), ("max_newton", ctypes.c_int32),
                ("max_halvings", ctypes.c_int32), ("step0", ctypes.c_double),
                ("step_max", ctypes.c_double), ("armijo", ctypes.c_double),
                ("descent_tol", ctypes.c_double), ("newton_tol", ctypes.c_double),
                ("rho_tol", ctypes.c_double)]


@dataclass
class RefineParams:
    """Step rule of the in-plane minimisation (the paper fixes none; see vxo.c)."""
    max_descent: int = 32
    max_newton: int = 20
    max_halvings: int = 30
    step0: float = 0.25
    step_max: float = 1.0
    armijo: float = 1e-4
    descent_tol: float = 1e-2
    newton_tol: float = 1e-12
    rho_tol: float = 1e-10

    def c(self) -> _RefineParams:
        return _RefineParams(self.max_descent, self.max_newton, self.max_halvings, self.step0,
                             self.step_max, self.armijo, self.descent_tol, self.newton_tol,
                             self.rho_tol)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P, i = ctypes.c_void_p, ctypes.c_int
        lib.vxo_edge.argtypes = [P, P]
        lib.vxo_edge.restype = i
        lib.vxo_polygon.argtypes = [P, P, P, P]
        lib.vxo_polygon.restype = i
        lib.vxo_winding.argtypes = [i, i, i, ctypes.c_uint, P, P, P, P, P, ctypes.c_int64, P, P,
                                    ctypes.c_int64, P]
        lib.vxo_winding.restype = None
        lib.vxo_winding_box.argtypes = [i, i, i, ctypes.c_uint, i, i, i, i, i, i, P, P, P, P]
        lib.vxo_winding_box.restype = None
        lib.vxo_refine.argtypes = [i, i, i, ctypes.c_uint, P, ctypes.c_int64, P, P, P,
                                   ctypes.POINTER(_RefineParams), P, P, P, P, P]
        lib.vxo_refine.restype = None
        lib.vxo_refine_one.argtypes = [P, P, P, P, ctypes.c_uint, ctypes.POINTER(_RefineParams),
                                       P, P, P, P]
        lib.vxo_refine_one.restype = None
        lib.vxo_trilerp.argtypes = [P, P, P, P, P, P]
        lib.vxo_trilerp.restype = None
        _lib = lib
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f32pairs(psi: np.ndarray) -> np.ndarray:
    psi = np.ascontiguousarray(psi, dtype=np.complex64)
    return psi.view(np.float32)


# ----------------------------------------------------------------------------------------------
# winding (Sec. 2.2 circulation, Sec. 3.1 graph of vortex nodes in dual form)
# ----------------------------------------------------------------------------------------------

def edge(a: complex, b: complex) -> int:
    """Crossing-number contribution of the directed edge a->b about q = (-delta, +eps)."""
    va = np.array([a.real, a.imag], np.float32)
    vb = np.array([b.real, b.imag], np.float32)
    return _load().vxo_edge(_p(va), _p(vb))


def polygon(v) -> int:
    arr = [np.array([complex(z).real, complex(z).imag], np.float32) for z in v]
    return _load().vxo_polygon(*[_p(a) for a in arr])


@dataclass
class Winding:
    w: np.ndarray          # int8 (nz, ny, nx, 3) face windings
    packed: np.ndarray     # uint8 (nz, ny, nx)
    faces: np.ndarray      # uint64 ascending face ids 3n+a
    fsign: np.ndarray      # int8
    cells: np.ndarray      # uint64 ascending cell ids n
    cdesc: np.ndarray      # uint16 descriptors


def winding(psi: np.ndarray, periodic: int = 7) -> Winding:
    """Whole-grid winding pass. psi: complex64 array of shape (nz, ny, nx)."""
    nz, ny, nx = psi.shape
    f = _f32pairs(psi)
    N = nx * ny * nz
    w = np.zeros((nz, ny, nx, 3), np.int8)
    packed = np.zeros((nz, ny, nx), np.uint8)
    counts = np.zeros(2, np.int64)
    lib = _load()
    lib.vxo_winding(nx, ny, nz, periodic, _p(f), _p(w), _p(packed), None, None, 0, None, None, 0,
                    _p(counts))
    nf, nc = int(counts[0]), int(counts[1])
    faces = np.zeros(max(nf, 1), np.uint64)
    fsign = np.zeros(max(nf, 1), np.int8)
    cells = np.zeros(max(nc, 1), np.uint64)
    cdesc = np.zeros(max(nc, 1), np.uint16)
    lib.vxo_winding(nx, ny, nz, periodic, _p(f), None, None, _p(faces), _p(fsign), nf, _p(cells),
                    _p(cdesc), nc, _p(counts))
    return Winding(w, packed, faces[:nf], fsign[:nf], cells[:nc], cdesc[:nc])


def winding_box(sub: np.ndarray, dims, origin, periodic: int = 7, want_w: bool = True):
    """Windings of the nodes of a box from the box values plus one node in each positive
    direction. sub: complex64 (bz+1, by+1, bx+1), already wrapped. Returns (w, packed, cdesc)
    (w is None unless want_w)."""
    nx, ny, nz = dims
    bz, by, bx = (s - 1 for s in sub.shape)
    f = _f32pairs(sub)
    w = np.zeros((bz, by, bx, 3), np.int8) if want_w else None
    packed = np.zeros((bz, by, bx), np.uint8)
    cdesc = np.zeros((bz, by, bx), np.uint16)
    x0, y0, z0 = origin
    _load().vxo_winding_box(nx, ny, nz, periodic, x0, y0, z0, bx, by, bz, _p(f),
                            _p(w) if w is not None else None, _p(packed), _p(cdesc))
    return w, packed, cdesc


def _slab_sub(psi: np.ndarray, k0: int, k1: int, periodic: int) -> np.ndarray:
    """Planes k0 .. k1 of a grid plus one node in each positive direction, wrapped where the axis is
    periodic (an open axis repeats its last node: those values are never read)."""
    nz, ny, nx = psi.shape
    kk = np.arange(k0, k1 + 1)
    kk = kk % nz if periodic & 4 else np.minimum(kk, nz - 1)
    jj = np.arange(ny + 1) % ny if periodic & 2 else np.minimum(np.arange(ny + 1), ny - 1)
    ii = np.arange(nx + 1) % nx if periodic & 1 else np.minimum(np.arange(nx + 1), nx - 1)
    return psi[kk][:, jj][:, :, ii]


def lists_from_packed(packed: np.ndarray, cdesc: np.ndarray, base: int = 0):
    """Pierced faces (ids 3n+a ascending, signs) and pierced cells (ids ascending, descriptors) of a
    run of nodes starting at node id `base`, from its packed bytes and cell descriptors."""
    pk = packed.reshape(-1)
    cd = cdesc.reshape(-1)
    ids, signs = [], []
    for a in range(3):
        v = (pk >> (2 * a)) & 3
        n = np.flatnonzero(v)
        ids.append(3 * (n.astype(np.uint64) + np.uint64(base)) + np.uint64(a))
        signs.append(np.where(v[n] == 1, 1, -1).astype(np.int8))
    fid = np.concatenate(ids)
    fs = np.concatenate(signs)
    o = np.argsort(fid, kind="stable")
    cn = np.flatnonzero(pk & 0x40)
    return fid[o], fs[o], cn.astype(np.uint64) + np.uint64(base), cd[cn]


def winding_slabs(psi: np.ndarray, periodic: int = 7, threads: int = 1, slab: int = 16):
    """The whole-grid winding pass computed slab by slab (z-slabs of `slab` planes, in `threads`
    host threads) with the box evaluation, which gives node for node what vxo_winding gives.
    Yields (k0, k1, packed, cdesc) per slab in plane order."""
    from concurrent.futures import ThreadPoolExecutor
    nz, ny, nx = psi.shape

    def one(k0):
        k1 = min(nz, k0 + slab)
        sub = _slab_sub(psi, k0, k1, periodic)
        _, packed, cdesc = winding_box(sub, (nx, ny, nz), (0, 0, k0), periodic, want_w=False)
        return k0, k1, packed, cdesc

    starts = list(range(0, nz, slab))
    if threads <= 1:
        for k0 in starts:
            yield one(k0)
        return
    with ThreadPoolExecutor(max_workers=threads) as ex:
        # bounded look-ahead: at most 2 * threads slabs in flight
        pending = []
        it = iter(starts)
        for k0 in it:
            pending.append(ex.submit(one, k0))
            if len(pending) >= 2 * threads:
                break
        for k0 in it:
            yield pending.pop(0).result()
            pending.append(ex.submit(one, k0))
        for f in pending:
            yield f.result()


# ----------------------------------------------------------------------------------------------
# node-centred circulation (Sec. 2.2: rings in the three coordinate planes through a node)
# ----------------------------------------------------------------------------------------------

def node_circulation(w: np.ndarray, periodic: int = 7):
    """Circulation / 2 pi around the ring of every node in each coordinate plane, from the face
    windings w (nz, ny, nx, 3) of the whole-grid pass. The ring of node n in the plane normal to
    axis a is the boundary of the four faces of orientation a that have n as a corner: the faces at
    n, n - e_u, n - e_v and n - e_u - e_v (u, v the other two axes); the windings of faces add, so the
    ring's circulation / 2 pi is their sum. A face that would sit at index -1 of a non-periodic axis
    does not exist (0). Returns C (nz, ny, nx, 3) int and the node bytes: bits 1:0 |C| of the plane
    with the largest |C| (ties: lowest axis), bit 2 its sign, bits 4:3 that axis, bit 6 = vortex node
    (|C| / 2 pi >= 1, i.e. |C| > pi)."""
    nz, ny, nx = w.shape[:3]
    W = w.astype(np.int64)
    axis_of = {0: 2, 1: 1, 2: 0}  # grid axis a -> array axis of (z, y, x)

    def back(f, a):
        """f at n - e_a (zero where n - e_a is outside a non-periodic axis)."""
        g = np.roll(f, 1, axis=axis_of[a])
        if not (periodic >> a) & 1:
            sl = [slice(None)] * 3
            sl[axis_of[a]] = 0
            g[tuple(sl)] = 0
        return g

    C = np.zeros((nz, ny, nx, 3), np.int64)
    for a in range(3):
        u, v = [b for b in range(3) if b != a]
        f = W[..., a]
        C[..., a] = f + back(f, u) + back(f, v) + back(back(f, u), v)
    mag = np.abs(C)
    best = np.argmax(mag, axis=-1)  # the first maximum: ties go to the lowest axis
    val = np.take_along_axis(C, best[..., None], axis=-1)[..., 0]
    m = np.minimum(np.abs(val), 3)
    node = np.where(m > 0, m | np.where(val < 0, 4, 0) | (best << 3) | 0x40, 0).astype(np.uint8)
    return C, node


# ----------------------------------------------------------------------------------------------
# refinement (Sec. 3.3.1 mean estimate, Sec. 3.3.3 density-guided minimisation)
# ----------------------------------------------------------------------------------------------

@dataclass
class Samples:
    x: np.ndarray       # float64 (n, 3) cell-local position
    rho: np.ndarray     # float64 |psi|^2 at x
    iters: np.ndarray   # int32
    status: np.ndarray  # int32 status bits
    cond: np.ndarray    # float64 condition number of the in-plane Jacobian at x (diagnostic)


def refine(psi: np.ndarray, cells: np.ndarray, cdesc: np.ndarray, params: RefineParams | None = None,
           periodic: int = 7, threads: int = 1, seeds: np.ndarray | None = None) -> Samples:
    """Refine the listed cells; with threads > 1 the list is cut into contiguous chunks refined in
    host threads (each sample is independent, so the results are the same). seeds (n, 3), cell-local,
    replace the face-centre first estimates as starting points."""
    params = params or RefineParams()
    nz, ny, nx = psi.shape
    f = _f32pairs(psi)
    cells = np.ascontiguousarray(cells, np.uint64)
    cdesc = np.ascontiguousarray(cdesc, np.uint16)
    n = len(cells)
    x = np.zeros((n, 3), np.float64)
    rho = np.zeros(n, np.float64)
    iters = np.zeros(n, np.int32)
    status = np.zeros(n, np.int32)
    cond = np.zeros(n, np.float64)
    sd = np.ascontiguousarray(seeds, np.float64).reshape(n, 3) if seeds is not None else None
    pr = params.c()
    lib = _load()

    def run(a, b):
        if b > a:
            lib.vxo_refine(nx, ny, nz, periodic, _p(f), b - a, _p(cells[a:]), _p(cdesc[a:]),
                           _p(sd[a:]) if sd is not None else None, ctypes.byref(pr),
                           _p(x[a:]), _p(rho[a:]), _p(iters[a:]), _p(status[a:]), _p(cond[a:]))

    if threads <= 1 or n < 2 * threads:
        run(0, n)
    else:
        from concurrent.futures import ThreadPoolExecutor
        step = (n + 4 * threads - 1) // (4 * threads)
        with ThreadPoolExecutor(max_workers=threads) as ex:
            list(ex.map(lambda a: run(a, min(n, a + step)), range(0, n, step)))
    return Samples(x, rho, iters, status, cond)


def refine_patch(re: np.ndarray, im: np.ndarray, desc: int, params: RefineParams | None = None,
                 lo=(-1, -1, -1), hi=(2, 2, 2)):
    """Refine one sample from a 4x4x4 patch given as arrays indexed [c][b][a] (z, y, x)."""
    params = params or RefineParams()
    re = np.ascontiguousarray(re, np.float64).reshape(64)
    im = np.ascontiguousarray(im, np.float64).reshape(64)
    lo_ = np.array(lo, np.int32)
    hi_ = np.array(hi, np.int32)
    x = np.zeros(3, np.float64)
    rho = np.zeros(1, np.float64)
    it = np.zeros(1, np.int32)
    st = np.zeros(1, np.int32)
    pr = params.c()
    _load().vxo_refine_one(_p(re), _p(im), _p(lo_), _p(hi_), desc, ctypes.byref(pr), _p(x), _p(rho),
                           _p(it), _p(st))
    return x, float(rho[0]), int(it[0]), int(st[0])


def trilerp(re, im, x, lo=(-1, -1, -1), hi=(2, 2, 2)):
    re = np.ascontiguousarray(re, np.float64).reshape(64)
    im = np.ascontiguousarray(im, np.float64).reshape(64)
    lo_ = np.array(lo, np.int32)
    hi_ = np.array(hi, np.int32)
    xx = np.ascontiguousarray(x, np.float64)
    out = np.zeros(8, np.float64)
    _load().vxo_trilerp(_p(re), _p(im), _p(lo_), _p(hi_), _p(xx), _p(out))
    return out[0] + 1j * out[1], out[2:5] + 1j * out[5:8]


def density_at(psi: np.ndarray, points: np.ndarray, periodic: int = 7) -> np.ndarray:
    """|psi|^2 at points (grid coordinates, rows (x, y, z)) with psi linearly interpolated between
    nodes (Sec. 5), FP64: each point wrapped on periodic axes, in the cell that holds it (on an open
    axis the cell of min corner 0 .. n - 2 nearest to it, extrapolating)."""
    nz, ny, nx = psi.shape
    dims = (nx, ny, nz)
    out = np.empty(len(points), np.float64)
    for k, p in enumerate(np.asarray(points, np.float64)):
        c, u = [], []
        for q in range(3):
            x = p[q]
            if (periodic >> q) & 1:
                x = x - dims[q] * np.floor(x / dims[q])
                f = int(np.floor(x))
                u.append(x - f)
                c.append(f % dims[q])
            else:
                f = min(max(int(np.floor(x)), 0), dims[q] - 2)
                u.append(x - f)
                c.append(f)
        v = 0j
        for dz in (0, 1):
            for dy in (0, 1):
                for dx in (0, 1):
                    w = (u[0] if dx else 1 - u[0]) * (u[1] if dy else 1 - u[1]) * (u[2] if dz else 1 - u[2])
                    node = psi[(c[2] + dz) % nz, (c[1] + dy) % ny, (c[0] + dx) % nx]
                    v += w * complex(node)
        out[k] = abs(v) ** 2
    return out


def gather_patch(psi: np.ndarray, cell: int):
    """4x4x4 patch around a cell of a periodic grid, as (re, im) arrays indexed [c][b][a]."""
    nz, ny, nx = psi.shape
    i, j, k = cell % nx, (cell // nx) % ny, cell // (nx * ny)
    zi = (np.arange(k - 1, k + 3) % nz)[:, None, None]
    yi = (np.arange(j - 1, j + 3) % ny)[None, :, None]
    xi = (np.arange(i - 1, i + 3) % nx)[None, None, :]
    p = psi[zi, yi, xi].astype(np.complex128)
    return p.real.copy(), p.imag.copy()


# ----------------------------------------------------------------------------------------------
# synthetic-field definitions (for checking the GPU generator)
# ----------------------------------------------------------------------------------------------

def tangle_at(n: np.ndarray, c: np.ndarray, dims, nodes: np.ndarray) -> np.ndarray:
    """psi(x) = sum_k c_k exp(2 pi i sum_a n_ka x_a / N_a), evaluated in FP64 at integer nodes
    (rows of (x, y, z)). Plain definition with exp; no phase table."""
    nodes = np.asarray(nodes, np.float64)
    N = np.asarray(dims, np.float64)
    out = np.zeros(len(nodes), np.complex128)
    for s in range(0, len(nodes), 4096):
        ph = 2.0 * np.pi * (nodes[s:s + 4096] / N) @ n.T.astype(np.float64)
        out[s:s + 4096] = np.exp(1j * ph) @ c
    return out


def line_ring_at(dims, line, center, radius, xi, nodes: np.ndarray) -> np.ndarray:
    """Noise-free line x ring field in FP64 at integer nodes, minimum-image displacements."""
    nodes = np.asarray(nodes, np.float64)
    N = np.asarray(dims, np.float64)

    def mi(d, n):
        return d - n * np.round(d / n)

    dx = mi(nodes[:, 0] - line[0], N[0])
    dy = mi(nodes[:, 1] - line[1], N[1])
    fl = (dx + 1j * dy) / np.sqrt(dx * dx + dy * dy + 2 * xi * xi)
    rx = mi(nodes[:, 0] - center[0], N[0])
    ry = mi(nodes[:, 1] - center[1], N[1])
    rz = mi(nodes[:, 2] - center[2], N[2])
    u = np.sqrt(rx * rx + ry * ry) - radius
    fr = (u + 1j * rz) / np.sqrt(u * u + rz * rz + 2 * xi * xi)
    return fl * fr
