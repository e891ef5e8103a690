"""Convenience layer over the C-ABI: allocates caller-owned buffers with torch and chains the calls.

Nothing here computes on the data: it only sizes buffers, moves pointers and copies results to
the host for inspection.
"""
from __future__ import annotations

import numpy as np

from . import (VX_ERR_CAPACITY, VxError, dims as make_dims, vx_create, vx_destroy, vx_gen_line_ring, vx_gen_tangle,
               vx_refine, vx_refine_defaults, vx_winding, vx_wind_config)

SAMPLE_DTYPE = np.dtype([("cell", "<u8"), ("off", "<f4", (3,)), ("rho", "<f4"), ("iters", "<u2"),
                         ("status", "<u2"), ("reserved", "<u4")])


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("libvx needs a ROCm GPU; none is visible")
    return torch


def upload_tangle(tangle, device="cuda"):
    """Device copies of a tangle's integer phase steps, coefficients and phase table."""
    torch = _torch()
    ax, ay, az = tangle.phase_steps()
    to = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
    return dict(ax=to(ax.astype(np.int32), torch.int32), ay=to(ay.astype(np.int32), torch.int32),
                az=to(az.astype(np.int32), torch.int32), coef=to(tangle.coef_pairs(), torch.float64),
                table=to(tangle.table(), torch.float64))


def samples_to_numpy(t, n: int | None = None) -> np.ndarray:
    a = t.detach().cpu().numpy().view(np.uint8).reshape(-1)
    s = a.view(SAMPLE_DTYPE)
    return s if n is None else s[:n]


class Extractor:
    """One handle plus torch-allocated output buffers."""

    def __init__(self, device: int = 0):
        self.torch = _torch()
        self.device = device
        self.h = vx_create(device)

    def close(self):
        if self.h is not None:
            vx_destroy(self.h)
            self.h = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def config(self, zchunk: int = 0):
        vx_wind_config(self.h, zchunk)

    # ------------------------------------------------------------------ inputs
    def gen_tangle(self, tangle, stream=None):
        torch = self.torch
        nx, ny, nz = tangle.dims
        prm = upload_tangle(tangle, f"cuda:{self.device}")
        psi = torch.empty((nz, ny, nx), dtype=torch.complex64, device=f"cuda:{self.device}")
        vx_gen_tangle(self.h, make_dims(nx, ny, nz), prm["ax"], prm["ay"], prm["az"], prm["coef"],
                      prm["table"], psi, stream)
        return psi

    def gen_line_ring(self, lr, stream=None):
        torch = self.torch
        nx, ny, nz = lr.dims
        noise = lr.noise()
        d_noise = torch.from_numpy(noise).to(f"cuda:{self.device}") if noise is not None else None
        psi = torch.empty((nz, ny, nx), dtype=torch.complex64, device=f"cuda:{self.device}")
        prm = [*lr.line, *lr.ring_center, lr.radius, lr.xi]
        vx_gen_line_ring(self.h, make_dims(nx, ny, nz), prm, d_noise, psi, stream)
        return psi

    # ------------------------------------------------------------------ outputs
    def alloc_winding(self, shape, face_cap: int | None = None, cell_cap: int | None = None,
                      wind: bool = True):
        torch = self.torch
        nz, ny, nx = shape
        n = nx * ny * nz
        # a tangle pierces a few per cent of faces at most; dense small test fields need more room
        face_cap = max(4096, n // 4) if face_cap is None else face_cap
        cell_cap = max(4096, n // 4) if cell_cap is None else cell_cap
        dev = f"cuda:{self.device}"
        return dict(
            wind=torch.empty((nz, ny, nx), dtype=torch.uint8, device=dev) if wind else None,
            faces=torch.empty(face_cap, dtype=torch.int64, device=dev),
            fsign=torch.empty(face_cap, dtype=torch.int8, device=dev),
            cells=torch.empty(cell_cap, dtype=torch.int64, device=dev),
            cdesc=torch.empty(cell_cap, dtype=torch.int16, device=dev),
            counts=torch.zeros(2, dtype=torch.int64, device=dev),
        )

    def winding(self, psi, periodic: int = 7, out=None, stream=None):
        nz, ny, nx = psi.shape
        out = out or self.alloc_winding(psi.shape)
        vx_winding(self.h, make_dims(nx, ny, nz, periodic), psi, out["counts"], out["wind"], out["faces"],
                   out["fsign"], out["cells"], out["cdesc"], stream)
        return out

    def alloc_samples(self, cap: int):
        return self.torch.empty((cap, 8), dtype=self.torch.int32, device=f"cuda:{self.device}")

    def refine(self, psi, wout, periodic: int = 7, samples=None, params=None, seed=None, stream=None):
        nz, ny, nx = psi.shape
        cap = wout["cells"].numel()
        samples = samples if samples is not None else self.alloc_samples(cap)
        vx_refine(self.h, make_dims(nx, ny, nz, periodic), psi, wout["cells"], wout["cdesc"],
                  wout["counts"][1:], samples, params or vx_refine_defaults(), seed, stream,
                  cap=min(cap, samples.shape[0]))
        return samples

    def vectorize(self, psi, periodic: int = 7, box_k: int = 4, max_passes: int = 5, seg_points: int = 8,
                  wout=None, params=None):
        """The paper's pipeline from a field to vector lines, in one call (synchronous): winding and
        compaction on the GPU; the dual graph of the pierced cells and its line classes, box-mean
        samples with graph reduction (host, in the library); refinement of the reduced samples from
        their box means on the GPU; Catmull-Rom curves through the refined samples (host). Returns a
        dict: graph (per-cell component and connectivity, class per component, counts), samples
        (absolute positions [m, 3], the refinement records, the sample graph's edges, members and
        components) and curves (as vx_curves returns them)."""
        from . import vx_curves, vx_graph_lines, vx_reduce
        torch = self.torch
        nz, ny, nx = psi.shape
        d = make_dims(nx, ny, nz, periodic)
        wout = self.winding(psi, periodic, wout)
        nf, nc = (int(v) for v in wout["counts"].cpu())
        if nf > wout["faces"].numel() or nc > wout["cells"].numel():
            raise VxError(VX_ERR_CAPACITY, f"vectorize: {nf} faces / {nc} cells exceed the list capacity")
        cells = wout["cells"][:nc].cpu().numpy().view(np.uint64)
        cdesc = wout["cdesc"][:nc].cpu().numpy().view(np.uint16)
        comp, degree, ctype, stats = vx_graph_lines(d, cells, cdesc)
        R = vx_reduce(d, cells, cdesc, box_k, max_passes)
        m = len(R["seed_cell"])
        dev = psi.device
        smp = self.alloc_samples(max(m, 1))
        if m:
            vx_refine(self.h, d, psi, torch.from_numpy(R["seed_cell"].view(np.int64)).to(dev),
                      torch.from_numpy(R["seed_desc"].view(np.int16)).to(dev),
                      torch.tensor([m], dtype=torch.int64, device=dev), smp, params or vx_refine_defaults(),
                      torch.from_numpy(R["seed_off"]).to(dev), None, cap=m)
        s = samples_to_numpy(smp, m)
        c = R["seed_cell"].astype(np.int64)
        pos = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], 1).astype(np.float64) + s["off"].astype(np.float64)
        curves = vx_curves(d, pos, R["edges"], seg_points)
        return {"graph": {"comp": comp, "degree": degree, "comp_type": ctype, "stats": stats},
                "samples": {"pos": pos, "records": s, "edges": R["edges"], "members": R["members"],
                            "comp": R["comp"], "passes": R["passes"]},
                "curves": curves}


def lines_by_length(curves, lo: float, hi: float, scale: float = 1.0) -> np.ndarray:
    """Indices of the curves whose length, times scale (e.g. domain size / cells per axis, for lengths
    in units of the domain), lies in [lo, hi): the selection of the paper's multi-scale view
    (Sec. 4.1.2), on the lengths vx_curves measures."""
    L = np.asarray(curves["length"], np.float64) * scale
    return np.nonzero((L >= lo) & (L < hi))[0]


def length_histogram(curves, edges, scale: float = 1.0):
    """Number of curves and their total length, times scale, per length bin [edges[i], edges[i+1])."""
    L = np.asarray(curves["length"], np.float64) * scale
    e = np.asarray(edges, np.float64)
    which = np.searchsorted(e, L, side="right") - 1
    inside = (which >= 0) & (which < len(e) - 1)
    count = np.bincount(which[inside], minlength=len(e) - 1)
    total = np.bincount(which[inside], weights=L[inside], minlength=len(e) - 1)
    return count, total


class Batch:
    """A vx_batch over frames (psi tensors of uneven shapes) with torch-allocated outputs.

    frames: list of (psi, periodic). Outputs per frame: dict as from Extractor.alloc_winding plus
    "samples" (sample_cap rows) when refine is set.
    """

    def __init__(self, ex: Extractor, frames, face_cap=None, cell_cap=None, wind: bool = True,
                 refine: bool = True, params=None):
        from . import Frame, dims as make_dims_, winding_out, vx_batch_create
        self.ex = ex
        self.psi = [p for p, _ in frames]
        self.outs = []
        structs = []
        for psi, periodic in frames:
            nz, ny, nx = psi.shape
            n = nx * ny * nz
            fc = face_cap(n) if callable(face_cap) else (face_cap or max(4096, n // 16))
            cc = cell_cap(n) if callable(cell_cap) else (cell_cap or max(4096, n // 16))
            o = ex.alloc_winding(psi.shape, face_cap=fc, cell_cap=cc, wind=wind)
            if refine:
                o["samples"] = ex.alloc_samples(cc)
            self.outs.append(o)
            wo = winding_out(o["counts"], o["wind"], o["faces"], o["fsign"], o["cells"], o["cdesc"])
            structs.append(Frame(make_dims_(nx, ny, nz, periodic), psi.data_ptr(), wo,
                                 o["samples"].data_ptr() if refine else None, cc if refine else 0))
        self.b = vx_batch_create(ex.h, structs, params)

    def launch(self, stream=None, graph: bool = True):
        from . import vx_batch_launch, vx_batch_launch_eager
        (vx_batch_launch if graph else vx_batch_launch_eager)(self.ex.h, self.b, stream)

    def autotune(self, cache_path=None, stream=None):
        from . import vx_batch_autotune
        vx_batch_autotune(self.ex.h, self.b, cache_path, stream)

    def refine_wg(self) -> int:
        """Resident refinement workgroups per CU of the batch (0 until autotuned: the default)."""
        from . import vx_batch_refine_wg
        return vx_batch_refine_wg(self.ex.h, self.b)

    def wind_wg(self) -> int:
        """Resident winding workgroups per CU of the batch (0 until autotuned: as many as fit)."""
        from . import vx_batch_wind_wg
        return vx_batch_wind_wg(self.ex.h, self.b)

    def zchunk(self, frame: int) -> int:
        from . import vx_batch_zchunk
        return vx_batch_zchunk(self.ex.h, self.b, frame)

    def close(self):
        from . import vx_batch_destroy
        if self.b is not None:
            vx_batch_destroy(self.ex.h, self.b)
            self.b = None

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass


class FramePipeline:
    """Winding and refinement of a stream of same-shape frames on two streams, so that the winding
    of frame k runs while frame k-1 is refined: the winding is bound by HBM, the refinement by
    vector issue, and the two kernels fit side by side on every CU. Two sets of output buffers
    alternate; frame k's results are in slot push(k) returned, valid once `done(slot)` has been
    waited for (or after `sync()`), and until frame k+2 is pushed. Every psi tensor must stay alive
    until its frame is done. All calls go to one handle, which must not be used by other work
    while frames are in flight (the refinements share its chunk counter, on one stream)."""

    def __init__(self, ex: Extractor, shape, face_cap: int, cell_cap: int, wind: bool = True,
                 periodic: int = 7, params=None):
        torch = ex.torch
        self.ex = ex
        self.periodic = periodic
        self.params = params
        self.outs = [ex.alloc_winding(shape, face_cap=face_cap, cell_cap=cell_cap, wind=wind) for _ in range(2)]
        self.samples = [ex.alloc_samples(cell_cap) for _ in range(2)]
        dev = torch.device("cuda", ex.device)
        self.s_wind = torch.cuda.Stream(device=dev)
        self.s_refine = torch.cuda.Stream(device=dev)
        self._refined = [None, None]
        self.k = 0

    def push(self, psi) -> int:
        """Enqueue the next frame; returns its output slot (0 or 1)."""
        torch = self.ex.torch
        b = self.k % 2
        if self._refined[b] is not None:  # frame k-2 has finished with this slot
            self.s_wind.wait_event(self._refined[b])
        self.ex.winding(psi, self.periodic, self.outs[b], self.s_wind)
        wound = torch.cuda.Event()
        wound.record(self.s_wind)
        self.s_refine.wait_event(wound)
        self.ex.refine(psi, self.outs[b], self.periodic, self.samples[b], self.params, None, self.s_refine)
        refined = torch.cuda.Event()
        refined.record(self.s_refine)
        self._refined[b] = refined
        self.k += 1
        return b

    def done(self, slot: int):
        """Event recorded after the last refinement written to `slot` (None before any)."""
        return self._refined[slot]

    def sync(self):
        self.s_wind.synchronize()
        self.s_refine.synchronize()
