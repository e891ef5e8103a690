"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This package holds only input construction: wave-vector and coefficient sampling, the phase
table, noise, and a host evaluation of the synthetic fields. It contains none of the vortex
identification or refinement arithmetic. The GPU library has its own generator kernels that
perform the same FP64 operations; the tests check that both produce identical bytes.

Workloads (the paper's 2048^3 NLKG turbulence data is not available, so random-wave tangles of
the same kind -- a periodic complex64 grid threaded by vortex lines -- stand in for it):

* ``line_ring``  32^3: one straight z-line (winding +1) times one ring of radius 8 (winding -1
  about its azimuthal direction), core profile d/sqrt(d^2 + 2 xi^2), xi = 1, plus Gaussian noise.
* ``tangle_256``  256^3, 512 waves with |n| in [4, 8].
* ``tangle_1024`` 1024^3, 4096 waves with |n| in [8, 24].
* ``series``      64 frames of sizes drawn from {128, 192, 256, 384}^3, 1024 waves, |n| in [4, 12],
  advanced by exp(-i |n|^2/2 t) with t = 0.05 per frame.
* ``tangle_512``  512^3, 2048 waves with |n| in [6, 16] (surrogate evaluation field).

Wave coefficients: c_k = a_k exp(i phi_k) / sqrt(sum |a|^2), a_k complex Gaussian with unit
variance, phi_k uniform in [0, 2 pi); wave vectors are distinct lattice points n of the shell, so
the grid mean of |psi|^2 is exactly 1 by discrete Parseval (|n_i| < N/2 keeps the modes distinct).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libvxsynth.so")
_SRC = os.path.join(_HERE, "synth.c")
_lib = None

# FP64 table sizes above this would overflow the 32-bit phase products of the GPU generator.
MAX_TABLE = 46340


def build(force: bool = True) -> str:
    """Compile the host evaluator (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                               "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        i = ctypes.c_int
        lib.vxs_tangle.argtypes = [i, i, i, i, i, i, i, i, i, i, P, P, P, P, ctypes.c_uint32, P, P]
        lib.vxs_tangle.restype = None
        lib.vxs_line_ring.argtypes = [i, i, i, P, P, P]
        lib.vxs_line_ring.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ----------------------------------------------------------------------------------------------
# Tangle parameters
# ----------------------------------------------------------------------------------------------

def shell_points(a: float, b: float) -> np.ndarray:
    """All integer vectors n with a <= |n| <= b, in lexicographic order."""
    r = int(math.floor(b))
    g = np.arange(-r, r + 1)
    n = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    s = (n * n).sum(1)
    keep = (s >= a * a - 1e-9) & (s <= b * b + 1e-9)
    return n[keep].astype(np.int64)


@dataclass
class Tangle:
    """A random-wave field: psi(x) = sum_k c[k] exp(2 pi i n[k] . (x / N))."""
    n: np.ndarray            # (W, 3) int64 wave vectors (lattice units)
    c: np.ndarray            # (W,) complex128 coefficients
    dims: tuple              # (nx, ny, nz)

    def at_time(self, t: float) -> "Tangle":
        """Advance each wave by exp(-i omega t), omega = |n|^2 / 2 (box of side 2 pi)."""
        w = 0.5 * (self.n * self.n).sum(1).astype(np.float64)
        return Tangle(self.n, self.c * np.exp(-1j * w * t), self.dims)

    def on_grid(self, dims) -> "Tangle":
        return Tangle(self.n, self.c, tuple(int(d) for d in dims))

    # integer phase-index form shared by the host evaluator and the GPU generator
    def table_size(self) -> int:
        nx, ny, nz = self.dims
        M = math.lcm(nx, ny, nz)
        if M > MAX_TABLE:
            raise ValueError(f"lcm of dims {self.dims} = {M} exceeds {MAX_TABLE}")
        return M

    def phase_steps(self):
        """Per-wave phase-index increments (ax, ay, az) modulo M, as uint32."""
        nx, ny, nz = self.dims
        M = self.table_size()
        ax = np.mod(self.n[:, 0] * (M // nx), M).astype(np.uint32)
        ay = np.mod(self.n[:, 1] * (M // ny), M).astype(np.uint32)
        az = np.mod(self.n[:, 2] * (M // nz), M).astype(np.uint32)
        return ax, ay, az

    def table(self) -> np.ndarray:
        M = self.table_size()
        m = np.arange(M, dtype=np.float64)
        th = 2.0 * np.pi * m / M
        return np.stack([np.cos(th), np.sin(th)], 1).astype(np.float64).copy()

    def coef_pairs(self) -> np.ndarray:
        return np.stack([self.c.real, self.c.imag], 1).astype(np.float64).copy()


def make_tangle(dims, nwaves: int, shell, seed: int) -> Tangle:
    rng = np.random.default_rng(seed)
    pts = shell_points(*shell)
    if nwaves > len(pts):
        raise ValueError("shell has fewer lattice points than waves")
    idx = rng.choice(len(pts), size=nwaves, replace=False)
    n = pts[np.sort(idx)]
    g = rng.standard_normal((nwaves, 2))
    a = (g[:, 0] + 1j * g[:, 1]) / math.sqrt(2.0)
    phi = rng.uniform(0.0, 2.0 * np.pi, nwaves)
    c = a * np.exp(1j * phi)
    c = c / math.sqrt(float((np.abs(c) ** 2).sum()))
    return Tangle(n=n, c=c, dims=tuple(int(d) for d in dims))


def eval_tangle(t: Tangle, box=None) -> np.ndarray:
    """Host evaluation of a tangle on the grid, or on a box (x0, y0, z0, bx, by, bz) that wraps
    periodically. Returns complex64 with shape (bz, by, bx) (x fastest in memory)."""
    nx, ny, nz = t.dims
    if box is None:
        box = (0, 0, 0, nx, ny, nz)
    x0, y0, z0, bx, by, bz = (int(v) for v in box)
    ax, ay, az = t.phase_steps()
    coef = t.coef_pairs()
    tab = t.table()
    out = np.empty((bz, by, bx, 2), np.float32)
    _load().vxs_tangle(nx, ny, nz, x0, y0, z0, bx, by, bz, len(ax), _ptr(ax), _ptr(ay), _ptr(az),
                       _ptr(coef), t.table_size(), _ptr(tab), _ptr(out))
    return out.view(np.complex64)[..., 0]


# ----------------------------------------------------------------------------------------------
# Line + ring field
# ----------------------------------------------------------------------------------------------

@dataclass
class LineRing:
    dims: tuple = (32, 32, 32)
    line: tuple = (16.31, 15.77)
    ring_center: tuple = (16.23, 15.81, 16.47)
    radius: float = 8.0
    xi: float = 1.0
    noise_sigma: float = 1e-3
    seed: int = 1

    def params(self) -> np.ndarray:
        return np.array([*self.line, *self.ring_center, self.radius, self.xi], np.float64)

    def noise(self) -> np.ndarray | None:
        if self.noise_sigma == 0:
            return None
        nx, ny, nz = self.dims
        rng = np.random.default_rng(self.seed)
        return (rng.standard_normal((nz, ny, nx, 2)) * self.noise_sigma).astype(np.float32)


def eval_line_ring(lr: LineRing) -> np.ndarray:
    nx, ny, nz = lr.dims
    prm = lr.params()
    nz_ = lr.noise()
    out = np.empty((nz, ny, nx, 2), np.float32)
    _load().vxs_line_ring(nx, ny, nz, _ptr(prm), _ptr(nz_) if nz_ is not None else None, _ptr(out))
    return out.view(np.complex64)[..., 0]


# ----------------------------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------------------------

def line_ring_32() -> LineRing:
    return LineRing()


def tangle_256(seed: int = 2) -> Tangle:
    return make_tangle((256, 256, 256), 512, (4, 8), seed)


def tangle_1024(seed: int = 3) -> Tangle:
    return make_tangle((1024, 1024, 1024), 4096, (8, 24), seed)


def tangle_512(seed: int = 5) -> Tangle:
    return make_tangle((512, 512, 512), 2048, (6, 16), seed)


@dataclass
class Series:
    """Time series of frames with uneven sizes sharing one wave set."""
    sizes: list
    base: Tangle
    dt: float = 0.05

    def frame(self, f: int) -> Tangle:
        n = self.sizes[f]
        return self.base.at_time(self.dt * f).on_grid((n, n, n))


def series_64(seed: int = 4, nframes: int = 64) -> Series:
    rng = np.random.default_rng(seed)
    sizes = [int(v) for v in rng.choice([128, 192, 256, 384], size=nframes)]
    base = make_tangle((128, 128, 128), 1024, (4, 12), seed + 10_000)
    return Series(sizes=sizes, base=base)


def random_small_int_field(dims, seed: int, lo: int = -2, hi: int = 2) -> np.ndarray:
    """Small-integer complex field (zeros and collinear values included) for brute-force checks."""
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    v = rng.integers(lo, hi + 1, size=(nz, ny, nx, 2)).astype(np.float32)
    return v.view(np.complex64)[..., 0].copy()


# ----------------------------------------------------------------------------------------------
# Surrogate network: initial weights and the flat parameter layout
# ----------------------------------------------------------------------------------------------

MLP_NHID = 128  # hidden width
MLP_SHAPES = (("W1", (128, MLP_NHID)), ("b1", (MLP_NHID,)), ("W2", (MLP_NHID, MLP_NHID)), ("b2", (MLP_NHID,)),
              ("W3", (MLP_NHID, 4)), ("b3", (4,)))
MLP_NPARAMS = sum(int(np.prod(s)) for _, s in MLP_SHAPES)


def mlp_init(seed: int) -> dict:
    """Random initial weights (float64): W ~ N(0, 1/fan_in) (last layer scaled by 0.1), biases 0."""
    rng = np.random.default_rng(seed)
    P = {}
    for name, shape in MLP_SHAPES:
        if name.startswith("W"):
            scale = 1.0 / np.sqrt(shape[0]) * (0.1 if name == "W3" else 1.0)
            P[name] = rng.normal(0.0, scale, size=shape)
        else:
            P[name] = np.zeros(shape)
    return P


def mlp_pack(P: dict) -> np.ndarray:
    """Flat float32 vector in the library's layout: W1 (row-major, rows = inputs), b1, W2, b2, W3, b3."""
    return np.concatenate([np.asarray(P[n], np.float64).reshape(-1) for n, _ in MLP_SHAPES]).astype(np.float32)


def mlp_unpack(v: np.ndarray) -> dict:
    P, o = {}, 0
    for n, s in MLP_SHAPES:
        k = int(np.prod(s))
        P[n] = np.asarray(v[o:o + k], np.float64).reshape(s)
        o += k
    return P


def surrogate_train_tangles(first: int = 1000, count: int = 150):
    """Training fields: 256^3 random-wave tangles like the 256^3 case (512 waves, |n| in [4, 8])."""
    return [make_tangle((256, 256, 256), 512, (4, 8), s) for s in range(first, first + count)]
