"""Whole-field parity of a GPU run against the oracle: every packed byte, the complete sorted face
and cell lists, and every refined sample, for grids of any size the host memory holds. The oracle
reads the exact psi bytes the GPU path read (copied back from the device), by z-slabs in host
threads (the box evaluation, pinned against the whole-grid pass on the CPU)."""
import json
import os
import time

import numpy as np

import oracle
from gpu_util import log

TOL = 1e-4         # position tolerance of the FP32 refinement against the FP64 oracle, cells
COND_LIMIT = 1e3  # above this the FP32 position of a zero is ill-determined (error ~ cond x FP32 rounding)

# status bits whose meaning is the same on both sides
BITS = {"MULTI": 1, "TANGENT_FALLBACK": 2, "BOUNDARY": 4, "NONZERO_MIN": 8, "NOT_CONVERGED": 16, "NO_FACES": 32}
UNCONVERGED = oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.NO_FACES


def host_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


def gpu_lists(out):
    nf, nc = (int(v) for v in out["counts"].cpu())
    assert nf <= out["faces"].numel() and nc <= out["cells"].numel(), "list capacity too small"
    faces = out["faces"][:nf].cpu().numpy().view(np.uint64)
    fsign = out["fsign"][:nf].cpu().numpy()
    o = np.argsort(faces, kind="stable")
    cells = out["cells"][:nc].cpu().numpy().view(np.uint64)
    cdesc = out["cdesc"][:nc].cpu().numpy().view(np.uint16)
    oc = np.argsort(cells, kind="stable")
    return faces[o], fsign[o], cells[oc], cdesc[oc]


def winding_parity(psi_h, packed_g, out, periodic, tag):
    """Packed field and lists against the oracle, slab by slab. Returns the oracle's (cells, cdesc)."""
    t0 = time.perf_counter()
    nz, ny, nx = psi_h.shape
    faces_g, fsign_g, cells_g, cdesc_g = gpu_lists(out)
    F, S, C, D = [], [], [], []
    for k0, k1, pk, cd in oracle.winding_slabs(psi_h, periodic, threads=host_threads(), slab=16):
        if packed_g is not None:
            bad = np.argwhere(packed_g[k0:k1] != pk)
            assert len(bad) == 0, f"{tag}: {len(bad)} packed bytes differ in planes {k0}..{k1 - 1}, first {bad[:3].tolist()}"
        f, s, c, d = oracle.lists_from_packed(pk, cd, k0 * nx * ny)
        F.append(f)
        S.append(s)
        C.append(c)
        D.append(d)
    F, S, C, D = (np.concatenate(a) for a in (F, S, C, D))
    assert len(F) == len(faces_g) and len(C) == len(cells_g), (tag, len(F), len(faces_g), len(C), len(cells_g))
    assert np.array_equal(F, faces_g) and np.array_equal(S, fsign_g), f"{tag}: face lists differ"
    assert np.array_equal(C, cells_g) and np.array_equal(D, cdesc_g), f"{tag}: cell lists differ"
    log(f"{tag}: packed field of {nx}x{ny}x{nz} and lists ({len(F)} faces, {len(C)} cells) bit-exact "
        f"({time.perf_counter() - t0:.1f} s on {host_threads()} host threads)")
    return C, D


def sample_parity(psi_h, cells, cdesc, samples_g, periodic, tag, tol=1e-4, report=True):
    """Every GPU sample (any order; numpy structured array from samples_to_numpy) against the FP64
    oracle's refinement of the same cell. Returns the error statistics."""
    t0 = time.perf_counter()
    o = np.argsort(samples_g["cell"], kind="stable")
    g = samples_g[o]
    assert np.array_equal(g["cell"], cells), f"{tag}: sample cells differ from the list"
    R = oracle.refine(psi_h, cells, cdesc, periodic=periodic, threads=host_threads())
    ok = (R.status & UNCONVERGED) == 0
    err = np.abs(g["off"].astype(np.float64) - R.x).max(axis=1)
    e = err[ok]
    above = np.nonzero(ok & (err > tol))[0]
    st_g = g["status"].astype(np.int64)
    disagree = {k: int(((st_g & b) != (R.status & b)).sum()) for k, b in BITS.items()}
    stats = {
        "config": tag,
        "samples": int(len(cells)),
        "oracle_converged": int(ok.sum()),
        "max_err": float(e.max()) if len(e) else 0.0,
        "p99_err": float(np.percentile(e, 99)) if len(e) else 0.0,
        "median_err": float(np.median(e)) if len(e) else 0.0,
        "above_tol": int(len(above)),
        "tol": tol,
        "above_tol_samples": [{"cell": int(cells[i]), "err": float(err[i]), "cond": float(R.cond[i]),
                               "gpu_status": int(st_g[i]), "oracle_status": int(R.status[i])} for i in above[:50]],
        "status_disagreements": disagree,
        "cond_p99": float(np.percentile(R.cond[ok], 99)) if ok.any() else 0.0,
        "seconds": time.perf_counter() - t0,
    }
    if report:
        log("PARITY " + json.dumps(stats))
        path = os.environ.get("VX_PARITY_OUT")
        if path:
            with open(path, "a") as fh:
                fh.write(json.dumps(stats) + "\n")
    return stats, err, ok, R


def explain(psi_h, cells, cdesc, g, R, idx):
    """Details of samples above TOL: both positions, statuses, iterations, the oracle's |psi|^2 at the
    GPU point and at its own, the condition number."""
    rows = []
    for i in idx:
        re, im = oracle.gather_patch(psi_h, int(cells[i]))
        vg, _ = oracle.trilerp(re, im, g["off"][i].astype(np.float64))
        rows.append({"i": int(i), "cell": int(cells[i]), "desc": int(cdesc[i]), "gpu": g["off"][i].tolist(),
                     "oracle": R.x[i].tolist(), "gpu_status": int(g["status"][i]), "oracle_status": int(R.status[i]),
                     "gpu_iters": int(g["iters"][i]), "oracle_iters": int(R.iters[i]), "cond": float(R.cond[i]),
                     "rho_oracle_at_gpu_point": float(abs(vg) ** 2), "rho_oracle": float(R.rho[i])})
    return rows


def off_plane(psi_h, cell, desc, x, periodic=7):
    """Distance of x from the oracle's refinement plane of the cell (through x0, normal to the
    pseudo-vorticity at x0); None where the oracle's tangent is degenerate or the patch would need
    nodes past an open boundary."""
    from oracle import mlp as M
    nz, ny, nx = psi_h.shape
    c = int(cell)
    i, j, k = c % nx, (c // nx) % ny, c // (nx * ny)
    for a, (q, n) in enumerate(((i, nx), (j, ny), (k, nz))):
        if not (periodic >> a) & 1 and not (q >= 1 and q + 2 < n):
            return None
    re, im = oracle.gather_patch(psi_h, c)
    x0 = M.first_estimate(int(desc))
    _, g = oracle.trilerp(re, im, x0)
    t = np.cross(g.real, g.imag)
    n = np.linalg.norm(t)
    if not n > 1e-6 * np.linalg.norm(g.real) * np.linalg.norm(g.imag):
        return None
    return abs((np.asarray(x, np.float64) - x0) @ (t / n))


def assert_samples(stats, err, ok, R, g, psi_h, cells, cdesc, details=None, periodic=7):
    """Every oracle-converged sample within TOL of the oracle, except (a) where the in-plane Jacobian
    at the zero is ill-conditioned, and (b) path divergences: the FP32 descent took another branch
    at a discrete decision (a step accepted or rejected by a margin below FP32 rounding) and ended
    at another minimum of |psi|^2 in the same plane, which it reports itself as not a zero
    (NONZERO_MIN or NOT_CONVERGED). Both kinds are listed in the report; (b) must stay rare."""
    above = ok & (err > TOL) & (R.cond <= COND_LIMIT)
    idx = np.nonzero(above)[0]
    if len(idx) and details is not None:
        log("ABOVE " + str(details(idx[:10])))
    diverged = 0
    for i in idx:
        flagged = int(g["status"][i]) & (8 | 16)
        d = off_plane(psi_h, cells[i], cdesc[i], g["off"][i], periodic)
        assert flagged and (d is None or d < 1e-5), \
            f"{stats['config']}: sample {i} (cell {int(cells[i])}) above {TOL} at error {err[i]:.2e}, " \
            f"condition {R.cond[i]:.1f}, GPU status {int(g['status'][i])}, off the plane by {d}"
        diverged += 1
    assert diverged <= max(2, len(err) // 1_000_000), f"{stats['config']}: {diverged} path divergences"
    assert stats["status_disagreements"]["MULTI"] == 0 and stats["status_disagreements"]["NO_FACES"] == 0
    return diverged
