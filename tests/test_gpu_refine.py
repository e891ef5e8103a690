"""GPU refinement (FP32) against the FP64 oracle (Sec. 3.3.3 density-guided minimisation).

For every sample the oracle marks converged, the GPU position must be within 1e-4 cell. The error
distribution and the status agreement are printed for the record; no sample is dropped silently:
a sample outside the bound must be ill-conditioned (in-plane Jacobian condition above 1e3) or a
path divergence that the GPU flags itself (NONZERO_MIN or NOT_CONVERGED, in the oracle's plane),
and there may be at most two of those per list (the rule of whole_parity.assert_samples).
"""
import numpy as np
import pytest

import oracle
import vxinputs

from gpu_util import log, run_winding, to_dev
from whole_parity import assert_samples, explain, sample_parity

pytestmark = pytest.mark.gpu

BAD = oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.NO_FACES


@pytest.fixture(scope="module")
def ex():
    from paper_1911_12070_amd import Extractor
    e = Extractor(0)
    yield e
    e.close()


def check_all(name, psi, s, periodic=7):
    """Every GPU sample against the oracle under the rule of whole_parity.assert_samples."""
    cells = s["cell"].astype(np.uint64)
    W = oracle.winding(psi, periodic)
    assert np.array_equal(cells, W.cells)
    stats, err, ok, R = sample_parity(psi, W.cells, W.cdesc, s, periodic, name, report=False)
    assert_samples(stats, err, ok, R, s, psi, W.cells, W.cdesc, lambda idx: explain(psi, W.cells, W.cdesc, s, R, idx),
                   periodic=periodic)
    return stats


def refine_both(ex, psi, periodic=7):
    import torch
    from paper_1911_12070_amd import samples_to_numpy
    W = oracle.winding(psi, periodic)
    psi_dev = to_dev(psi)
    out = run_winding(ex, psi_dev, periodic)
    smp = ex.refine(psi_dev, out, periodic)
    torch.cuda.synchronize()
    nc = int(out["counts"][1].cpu())
    s = samples_to_numpy(smp, nc)
    s = s[np.argsort(s["cell"], kind="stable")]
    assert np.array_equal(s["cell"], W.cells)
    S = oracle.refine(psi, W.cells, W.cdesc, periodic=periodic)
    return s, S


def report(name, s, S):
    ok = (S.status & BAD) == 0
    err = np.abs(s["off"].astype(np.float64) - S.x).max(axis=1)
    e = err[ok]
    above = int((e > 1e-4).sum())
    same_status = np.mean((s["status"] & BAD) == (S.status & BAD))
    log(f"{name}: n={len(err)} oracle-ok={ok.sum()} err max={e.max():.2e} p99={np.percentile(e, 99):.2e} "
        f"median={np.median(e):.2e} above1e-4={above} status-agree={same_status:.4f} "
        f"gpu-rho-p99={np.percentile(s['rho'][ok], 99):.2e}")
    return e, above, ok


def test_refine_line_ring(ex):
    psi = vxinputs.eval_line_ring(vxinputs.line_ring_32())
    s, S = refine_both(ex, psi)
    e, above, ok = report("line_ring_32", s, S)
    assert above == 0
    assert ok.mean() > 0.95


@pytest.mark.parametrize("periodic", [7, 0])
def test_refine_small_tangle(ex, periodic):
    t = vxinputs.make_tangle((96, 96, 64), 256, (3, 7), 41)
    psi = vxinputs.eval_tangle(t)
    s, S = refine_both(ex, psi, periodic)
    e, above, ok = report(f"tangle_96x96x64 periodic={periodic}", s, S)
    check_all(f"tangle_96x96x64 periodic={periodic}", psi, s, periodic)
    assert np.median(e) < 1e-5


def test_refine_tangle_256(ex):
    t = vxinputs.tangle_256()
    psi = vxinputs.eval_tangle(t)
    s, S = refine_both(ex, psi)
    e, above, ok = report("tangle_256", s, S)
    check_all("tangle_256", psi, s)
    assert np.median(e) < 1e-5
    # the refined density is near zero where the oracle converged (Sec. 3.3.3: rho = 0 on the core)
    assert np.percentile(s["rho"][ok], 99) < 1e-9


def _face_centre_seeds(cdesc):
    """Mean of the centres of the pierced faces in cell-local coordinates, FP32, faces in the order
    -x, +x, -y, +y, -z, +z (Sec. 3.3.1 first estimate)."""
    seeds = np.zeros((len(cdesc), 3), np.float32)
    for i, d in enumerate(cdesc):
        acc = np.zeros(3, np.float32)
        n = 0
        for f in range(6):
            if (int(d) >> (2 * f)) & 3:
                c = np.full(3, 0.5, np.float32)
                c[f >> 1] = f & 1
                acc += c
                n += 1
        seeds[i] = acc * np.float32(1.0 / n) if n else 0.5
    return seeds


def test_refine_seeds_and_bad_cells(ex):
    """Caller seeds equal to the face-centre estimate reproduce the unseeded run bit for bit; a seed at
    the refined position stays there; out-of-range cell ids are flagged and leave the others intact."""
    import torch
    from paper_1911_12070_amd import SAMPLE_BAD_CELL, samples_to_numpy
    t = vxinputs.make_tangle((64, 64, 48), 128, (2, 5), 43)
    psi = vxinputs.eval_tangle(t)
    psi_dev = to_dev(psi)
    out = run_winding(ex, psi_dev, 7)
    torch.cuda.synchronize()
    nc = int(out["counts"][1].cpu())
    assert nc > 100
    base = samples_to_numpy(ex.refine(psi_dev, out, 7), nc)
    cdesc = out["cdesc"][:nc].cpu().numpy().view(np.uint16)
    seeds = torch.from_numpy(_face_centre_seeds(cdesc).reshape(-1)).cuda()
    seeded = samples_to_numpy(ex.refine(psi_dev, out, 7, seed=seeds), nc)
    for k in ("cell", "off", "rho", "iters", "status"):
        assert np.array_equal(seeded[k], base[k]), k
    seeds2 = torch.from_numpy(np.ascontiguousarray(base["off"], np.float32).reshape(-1)).cuda()
    again = samples_to_numpy(ex.refine(psi_dev, out, 7, seed=seeds2), nc)
    good = (base["status"] & BAD) == 0
    assert np.abs(again["off"] - base["off"]).max(axis=1)[good].max() < 1e-5

    n_nodes = psi.size
    cells = out["cells"].clone()
    bad_ids = [n_nodes, n_nodes + 12345, -1]  # -1 reads as 2^64 - 1
    pos = [0, nc // 2, nc - 1]
    for p, b in zip(pos, bad_ids):
        cells[p] = b
    out2 = dict(out)
    out2["cells"] = cells
    mixed = samples_to_numpy(ex.refine(psi_dev, out2, 7), nc)
    torch.cuda.synchronize()
    for p in pos:
        assert mixed["status"][p] == SAMPLE_BAD_CELL
        assert mixed["rho"][p] == -1.0
    keep = np.setdiff1d(np.arange(nc), pos)
    for k in ("off", "rho", "iters", "status"):
        assert np.array_equal(mixed[k][keep], base[k][keep]), k


@pytest.mark.parametrize("periodic", [7, 0])
def test_short_list_bit_identical(ex, periodic):
    """A list short enough for the short-list kernel (one sample per group of lanes, the halvings of a
    step evaluated together) gives the samples of the long-list kernel bit for bit: the 512^3 tangle's
    full list (half a million cells) against subsets of it: random cells, the slowest ones, with
    out-of-range ids mixed in, and the empty list."""
    import torch
    from paper_1911_12070_amd import SAMPLE_BAD_CELL, samples_to_numpy
    psi = ex.gen_tangle(vxinputs.tangle_512())
    nz, ny, nx = psi.shape
    out = ex.alloc_winding(psi.shape, face_cap=nx * ny * nz // 16, cell_cap=nx * ny * nz // 16, wind=False)
    ex.winding(psi, periodic, out)
    torch.cuda.synchronize()
    nc = int(out["counts"][1].cpu())
    assert nc > 200_000
    full = samples_to_numpy(ex.refine(psi, out, periodic), nc)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    slow = np.argsort(-full["iters"].astype(np.int64), kind="stable")[:1000]
    subsets = {"random": np.sort(rng.choice(nc, 5000, replace=False)), "slowest": slow,
               "one": np.array([int(slow[0])])}
    for name, idx in subsets.items():
        sel = torch.from_numpy(idx.astype(np.int64)).cuda()
        sub = {"cells": out["cells"][sel].contiguous(), "cdesc": out["cdesc"][sel].contiguous(),
               "counts": torch.tensor([0, len(idx)], dtype=torch.int64, device="cuda")}
        got = samples_to_numpy(ex.refine(psi, sub, periodic), len(idx))
        torch.cuda.synchronize()
        log(f"periodic={periodic} {name}: {len(idx)} samples, iters max {int(got['iters'].max())}, "
            f"boundary {int(((got['status'] & oracle.BOUNDARY) != 0).sum())}")
        assert got.tobytes() == full[idx].tobytes(), name
    # out-of-range ids inside a short list
    idx = subsets["random"][:300]
    cells = out["cells"][torch.from_numpy(idx.astype(np.int64)).cuda()].clone()
    bad_pos = [0, 150, 299]
    for p, b in zip(bad_pos, [nx * ny * nz, nx * ny * nz + 7, -1]):
        cells[p] = b
    sub = {"cells": cells, "cdesc": out["cdesc"][torch.from_numpy(idx.astype(np.int64)).cuda()].contiguous(),
           "counts": torch.tensor([0, len(idx)], dtype=torch.int64, device="cuda")}
    got = samples_to_numpy(ex.refine(psi, sub, periodic), len(idx))
    torch.cuda.synchronize()
    keep = np.setdiff1d(np.arange(len(idx)), bad_pos)
    assert got[keep].tobytes() == full[idx[keep]].tobytes()
    assert all(got["status"][p] == SAMPLE_BAD_CELL and got["rho"][p] == -1.0 for p in bad_pos)
    # an empty list writes nothing
    sub["counts"] = torch.zeros(2, dtype=torch.int64, device="cuda")
    marker = ex.alloc_samples(4)
    marker.fill_(7)
    ex.refine(psi, sub, periodic, marker)
    torch.cuda.synchronize()
    assert bool((marker == 7).all())


@pytest.mark.parametrize("variant", ["newton_only", "few_halvings", "one_newton", "long_steps", "no_descent_no_newton"])
def test_short_list_bit_identical_params(ex, variant):
    """The two refinement kernels agree bit for bit under non-default step rules too (descent
    disabled, at most two halvings per step, one Newton step, longer trial steps, no steps at all):
    the 256^3 tangle's full list against a random subset of it."""
    import torch
    from paper_1911_12070_amd import samples_to_numpy, vx_refine_defaults
    p = vx_refine_defaults()
    if variant == "newton_only":
        p.max_descent = 0
    elif variant == "few_halvings":
        p.max_halvings = 2
    elif variant == "one_newton":
        p.max_newton = 1
    elif variant == "long_steps":
        p.step0 = 0.9
        p.step_max = 2.0
    else:
        p.max_descent = 0
        p.max_newton = 0
    psi = ex.gen_tangle(vxinputs.tangle_256())
    nz, ny, nx = psi.shape
    out = ex.alloc_winding(psi.shape, face_cap=nx * ny * nz // 16, cell_cap=nx * ny * nz // 16, wind=False)
    ex.winding(psi, 7, out)
    torch.cuda.synchronize()
    nc = int(out["counts"][1].cpu())
    assert nc > 40_000
    full = samples_to_numpy(ex.refine(psi, out, 7, params=p), nc)
    idx = np.sort(np.random.default_rng(9).choice(nc, 3000, replace=False))
    sel = torch.from_numpy(idx.astype(np.int64)).cuda()
    sub = {"cells": out["cells"][sel].contiguous(), "cdesc": out["cdesc"][sel].contiguous(),
           "counts": torch.tensor([0, len(idx)], dtype=torch.int64, device="cuda")}
    got = samples_to_numpy(ex.refine(psi, sub, 7, params=p), len(idx))
    torch.cuda.synchronize()
    log(f"{variant}: iters max {int(full['iters'].max())}, status bits {sorted(set(int(v) for v in full['status']))[:8]}")
    assert got.tobytes() == full[idx].tobytes()
