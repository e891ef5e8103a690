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
