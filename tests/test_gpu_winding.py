"""GPU parity of the generator and of winding + compaction against the CPU oracle.

Winding numbers, the packed field and the pierced face/cell sets must match bit for bit: both
sides evaluate the same exact predicate (Sec. 2.2 circulation as a winding number). Lists are
sets on the GPU, so they are compared after sorting.
"""
import numpy as np
import pytest

import oracle
import vxinputs

from gpu_util import assert_winding_equal, canonical, log, run_winding, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    from paper_1911_12070_amd import Extractor
    e = Extractor(0)
    yield e
    e.close()


# ------------------------------------------------------------------ generator
@pytest.mark.parametrize("dims,nw,shell,seed", [((64, 48, 40), 128, (3, 6), 1), ((36, 20, 12), 40, (2, 4), 2),
                                                ((128, 128, 128), 1024, (4, 12), 3)])
def test_gen_tangle_bit_exact(ex, dims, nw, shell, seed):
    log(f"gen_tangle {dims} nw={nw}")
    t = vxinputs.make_tangle(dims, nw, shell, seed)
    psi = ex.gen_tangle(t).cpu().numpy()
    host = vxinputs.eval_tangle(t)
    assert np.array_equal(psi.view(np.uint64), host.view(np.uint64))
    nx, ny, nz = dims
    rng = np.random.default_rng(seed)
    nodes = np.stack([rng.integers(0, n, 2000) for n in dims], 1)
    ref = oracle.tangle_at(t.n, t.c, dims, nodes)
    got = psi[nodes[:, 2], nodes[:, 1], nodes[:, 0]]
    assert np.abs(got - ref).max() < 2e-5


def test_gen_line_ring_close_to_definition(ex):
    log("gen_line_ring 32^3")
    lr = vxinputs.line_ring_32()
    psi = ex.gen_line_ring(lr).cpu().numpy()
    host = vxinputs.eval_line_ring(lr)
    assert np.abs(psi - host).max() < 1e-6
    clean = vxinputs.LineRing(noise_sigma=0.0)
    psi0 = ex.gen_line_ring(clean).cpu().numpy()
    z, y, x = np.meshgrid(*(np.arange(32),) * 3, indexing="ij")
    nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    ref = oracle.line_ring_at((32, 32, 32), lr.line, lr.ring_center, lr.radius, lr.xi, nodes)
    assert np.abs(psi0.ravel() - ref).max() < 2e-6


# ------------------------------------------------------------------ winding parity, small grids
CASES = [
    # (dims, periodic, kind, seed)
    ((32, 32, 32), 7, "line_ring", 1),
    ((64, 48, 40), 7, "tangle", 2),
    ((260, 37, 19), 7, "tangle", 3),     # two x-tiles + ragged tail, ragged y and z
    ((516, 9, 5), 7, "tangle", 4),
    ((4, 2, 2), 7, "int", 5),            # smallest grids
    ((8, 3, 2), 7, "int", 6),
    ((12, 7, 6), 7, "int", 7),           # zeros, collinear values: degenerate predicate cases
    ((40, 33, 17), 0, "tangle", 8),      # non-periodic everywhere
    ((40, 33, 17), 1, "tangle", 9),
    ((40, 33, 17), 2, "tangle", 10),
    ((40, 33, 17), 4, "tangle", 11),
    ((40, 33, 17), 6, "int", 12),
    ((8, 8, 1), 3, "tangle", 13),        # single plane, z not periodic (a 2D field)
    ((37, 29, 13), 7, "tangle", 14),     # odd sizes, one tile with wrapped halo column and row
    ((127, 63, 5), 7, "tangle", 15),     # 63/31 tile boundaries: 3 x-tiles, 3 y-tiles
    ((126, 62, 4), 5, "tangle", 16),     # exact multiples of the tile outputs, y not periodic
    ((1, 5, 3), 6, "int", 17),           # one column, x not periodic
    ((2, 2, 2), 7, "int", 18),
    ((64, 32, 8), 3, "int", 19),
]


def _field(dims, kind, seed):
    if kind == "line_ring":
        return vxinputs.eval_line_ring(vxinputs.line_ring_32())
    if kind == "int":
        return vxinputs.random_small_int_field(dims, seed)
    # a box cropped from a periodic parent grid whose phase table is small (any dims work)
    parent = 1 << max(int(np.ceil(np.log2(max(dims)))), 4)
    t = vxinputs.make_tangle((parent,) * 3, 96, (2, 5), seed)
    return vxinputs.eval_tangle(t, (0, 0, 0, *dims))


@pytest.mark.parametrize("dims,periodic,kind,seed", CASES)
@pytest.mark.parametrize("zc", [0, 3, 1])
def test_winding_parity(ex, dims, periodic, kind, seed, zc):
    log(f"winding {dims} periodic={periodic} {kind} zc={zc}")
    psi = _field(dims, kind, seed)
    W = oracle.winding(psi, periodic)
    ex.config(zc)
    try:
        out = run_winding(ex, to_dev(psi), periodic)
    finally:
        ex.config(0)
    assert_winding_equal(out, W)


def test_winding_deterministic_sets(ex):
    t = vxinputs.make_tangle((128, 64, 64), 256, (3, 8), 31)
    psi = to_dev(vxinputs.eval_tangle(t))
    a = canonical(run_winding(ex, psi))
    b = canonical(run_winding(ex, psi))
    for x, y in zip(a[:5], b[:5]):
        assert np.array_equal(x, y)


def test_winding_without_packed_field(ex):
    t = vxinputs.make_tangle((64, 64, 32), 128, (3, 6), 32)
    psi = vxinputs.eval_tangle(t)
    W = oracle.winding(psi)
    out = run_winding(ex, to_dev(psi), wind=False)
    _, faces, fsign, cells, cdesc, (nf, nc) = canonical(out)
    assert np.array_equal(faces, W.faces) and np.array_equal(cells, W.cells)


def test_capacity_overflow_keeps_true_counts(ex):
    t = vxinputs.make_tangle((64, 64, 64), 256, (3, 8), 33)
    psi = vxinputs.eval_tangle(t)
    W = oracle.winding(psi)
    out = run_winding(ex, to_dev(psi), face_cap=7, cell_cap=5)
    nf, nc = (int(v) for v in out["counts"].cpu())
    assert (nf, nc) == (len(W.faces), len(W.cells))
    f = out["faces"].cpu().numpy().astype(np.uint64)
    c = out["cells"].cpu().numpy().astype(np.uint64)
    assert np.isin(f, W.faces).all() and len(np.unique(f)) == 7
    assert np.isin(c, W.cells).all() and len(np.unique(c)) == 5


def test_capacity_status_is_sticky_until_read(ex):
    """A list longer than its capacity sets the handle's capacity flag on the device; vx_sync_status
    reports it once (VX_ERR_CAPACITY) and clears it. Zero capacities, the refinement's sample
    capacity below the listed count, and the surrogate dataset's row capacity all count."""
    import torch
    from paper_1911_12070_amd import VX_ERR_CAPACITY, VxError, dims, vx_refine, vx_sync_status, vx_winding
    t = vxinputs.make_tangle((64, 64, 64), 256, (3, 8), 33)
    psi = to_dev(vxinputs.eval_tangle(t))
    try:
        vx_sync_status(ex.h)  # clears what earlier tests on this handle left (their overflow tests)
    except VxError:
        pass
    full = run_winding(ex, psi)
    vx_sync_status(ex.h)  # room for every face and cell: no overflow
    nf, nc = (int(v) for v in full["counts"].cpu())
    assert nf > 0 and nc > 0
    # capacity 0 on both lists (no list buffers at all)
    counts = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    vx_winding(ex.h, dims(64, 64, 64), psi, counts)
    torch.cuda.synchronize()
    assert tuple(int(v) for v in counts.cpu()) == (nf, nc)  # true counts still written
    with pytest.raises(VxError) as e:
        vx_sync_status(ex.h)
    assert e.value.status == VX_ERR_CAPACITY and "winding" in str(e.value)
    vx_sync_status(ex.h)  # read once, then cleared
    # the cell list fits, the face list does not
    run_winding(ex, psi, face_cap=nf - 1, cell_cap=nc)
    with pytest.raises(VxError):
        vx_sync_status(ex.h)
    run_winding(ex, psi, face_cap=nf, cell_cap=nc)
    vx_sync_status(ex.h)
    # refinement: sample capacity below the listed count
    smp = ex.alloc_samples(nc)
    vx_refine(ex.h, dims(64, 64, 64), psi, full["cells"], full["cdesc"], full["counts"][1:], smp, cap=nc - 1)
    with pytest.raises(VxError) as e:
        vx_sync_status(ex.h)
    assert e.value.status == VX_ERR_CAPACITY and "sample capacity" in str(e.value)
    vx_refine(ex.h, dims(64, 64, 64), psi, full["cells"], full["cdesc"], full["counts"][1:], smp, cap=nc)
    vx_sync_status(ex.h)


def test_invalid_arguments_are_rejected(ex):
    import torch
    from paper_1911_12070_amd import VxError, dims, vx_winding
    psi = torch.zeros((4, 4, 6), dtype=torch.complex64, device="cuda:0")
    counts = torch.zeros(2, dtype=torch.int64, device="cuda:0")
    with pytest.raises(VxError):   # bits above the three axes in the periodic mask
        vx_winding(ex.h, dims(6, 4, 4, 8), psi, counts)
    with pytest.raises(VxError):   # misaligned psi
        vx_winding(ex.h, dims(6, 4, 4), psi.data_ptr() + 4, counts)
    with pytest.raises(VxError):   # periodic axis of size 1
        vx_winding(ex.h, dims(4, 4, 1, 7), psi, counts)
    with pytest.raises(VxError):   # no counts buffer
        vx_winding(ex.h, dims(4, 4, 4), psi, None)


# ------------------------------------------------------------------ 256^3 tangle, whole grid
def test_tangle_256_full_grid(ex):
    t = vxinputs.tangle_256()
    log("tangle_256: generate on GPU")
    psi_dev = ex.gen_tangle(t)
    log("tangle_256: host evaluation")
    host = vxinputs.eval_tangle(t)
    assert np.array_equal(psi_dev.cpu().numpy().view(np.uint64), host.view(np.uint64))
    log("tangle_256: oracle winding")
    W = oracle.winding(host)
    log("tangle_256: GPU winding")
    out = run_winding(ex, psi_dev)
    assert_winding_equal(out, W)
    log(f"tangle_256: {len(W.faces)} faces, {len(W.cells)} cells")
