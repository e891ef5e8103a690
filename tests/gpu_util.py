"""Helpers for the GPU parity tests: run the library through its C-ABI binding and bring results
back to the host in the oracle's canonical (sorted) form."""
import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(psi_np):
    import torch
    return torch.from_numpy(np.ascontiguousarray(psi_np)).to("cuda:0")


def run_winding(ex, psi_dev, periodic=7, face_cap=None, cell_cap=None, wind=True):
    import torch
    n = int(np.prod(psi_dev.shape))
    if n <= (1 << 22):  # small grids: room for every face and cell (upper bounds 3N and N)
        face_cap = 3 * n if face_cap is None else face_cap
        cell_cap = n if cell_cap is None else cell_cap
    out = ex.alloc_winding(psi_dev.shape, face_cap, cell_cap, wind)
    ex.winding(psi_dev, periodic, out)
    torch.cuda.synchronize()
    return out


def canonical(out):
    """(packed, faces, fsign, cells, cdesc, counts) with the lists sorted by id."""
    nf, nc = (int(v) for v in out["counts"].cpu())
    kf = min(nf, out["faces"].numel())
    kc = min(nc, out["cells"].numel())
    faces = out["faces"][:kf].cpu().numpy().astype(np.uint64)
    fsign = out["fsign"][:kf].cpu().numpy()
    o = np.argsort(faces, kind="stable")
    cells = out["cells"][:kc].cpu().numpy().astype(np.uint64)
    cdesc = out["cdesc"][:kc].cpu().numpy().view(np.uint16)
    oc = np.argsort(cells, kind="stable")
    packed = out["wind"].cpu().numpy() if out["wind"] is not None else None
    return packed, faces[o], fsign[o], cells[oc], cdesc[oc], (nf, nc)


def assert_winding_equal(out, W):
    packed, faces, fsign, cells, cdesc, (nf, nc) = canonical(out)
    assert nf <= out["faces"].numel() and nc <= out["cells"].numel(), "list capacity too small for the test"
    assert nf == len(W.faces), (nf, len(W.faces))
    assert nc == len(W.cells), (nc, len(W.cells))
    if packed is not None:
        bad = np.argwhere(packed != W.packed)
        assert len(bad) == 0, f"{len(bad)} packed bytes differ, first at {bad[:5].tolist()}"
    assert np.array_equal(faces, W.faces)
    assert np.array_equal(fsign, W.fsign)
    assert np.array_equal(cells, W.cells)
    assert np.array_equal(cdesc, W.cdesc)


def window_packed(t, packed_dev, origin, size, periodic=7):
    """The packed field of a box of a GPU-generated tangle field, next to the oracle's windings of
    the same box computed from host-evaluated values (the generator is bit-exact with the host
    evaluator). Returns (gpu, oracle_packed, oracle_cdesc), all of shape (bz, by, bx)."""
    import torch
    import oracle
    import vxinputs
    nx, ny, nz = t.dims
    x0, y0, z0 = origin
    bx, by, bz = size
    sub = vxinputs.eval_tangle(t, (x0, y0, z0, bx + 1, by + 1, bz + 1))
    _, packed, cdesc = oracle.winding_box(sub, t.dims, origin, periodic)
    dev = packed_dev.device
    zi = torch.as_tensor((z0 + np.arange(bz)) % nz, device=dev)
    yi = torch.as_tensor((y0 + np.arange(by)) % ny, device=dev)
    xi = torch.as_tensor((x0 + np.arange(bx)) % nx, device=dev)
    g = packed_dev.index_select(0, zi).index_select(1, yi).index_select(2, xi).cpu().numpy()
    return g, packed, cdesc


def window_samples(t, samples_np, origin, size, cdesc_box, max_cells=200, seed=0):
    """GPU samples of (up to max_cells) pierced cells of a box against the oracle refinement of the
    same cells from host-evaluated 4x4x4 patches. samples_np: the GPU samples of the whole field
    (any order). Returns (errors of oracle-converged cells, number of oracle-converged cells,
    number checked)."""
    import oracle
    import vxinputs
    nx, ny, nz = t.dims
    x0, y0, z0 = origin
    bad = oracle.NONZERO_MIN | oracle.NOT_CONVERGED | oracle.NO_FACES
    kz, ky, kx = np.nonzero(cdesc_box)
    rng = np.random.default_rng(seed)
    pick = rng.permutation(len(kx))[:max_cells]
    order = np.argsort(samples_np["cell"], kind="stable")
    sc = samples_np["cell"][order]
    errs, ok = [], 0
    for p in pick:
        i, j, k = (x0 + kx[p]) % nx, (y0 + ky[p]) % ny, (z0 + kz[p]) % nz
        cell = i + nx * (j + ny * k)
        at = np.searchsorted(sc, cell)
        assert at < len(sc) and sc[at] == cell, f"cell {cell} missing from the GPU samples"
        s = samples_np[order[at]]
        patch = vxinputs.eval_tangle(t, (i - 1, j - 1, k - 1, 4, 4, 4)).astype(np.complex128)
        x, rho, it, st = oracle.refine_patch(patch.real, patch.imag, int(cdesc_box[kz[p], ky[p], kx[p]]))
        if st & bad:
            continue
        ok += 1
        errs.append(np.abs(s["off"].astype(np.float64) - x).max())
    return np.array(errs), ok, len(pick)
