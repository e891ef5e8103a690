"""Node-centred circulation on the GPU (vx_node_circulation) against the oracle: every node byte and
the sorted vortex-node list bit for bit, on the GPU's own packed field (itself bit-exact with the
oracle's), for ragged and tile-boundary shapes, every periodic mask, degenerate small-integer
fields (dense in vortex nodes), tangles and the 1024^3 benchmark field (in z-slabs). Rows whose
length is a multiple of 16 take the wide kernel, the others the general one."""
import numpy as np
import pytest

import oracle
import vxinputs
from gpu_util import log, run_winding, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ex():
    from paper_1911_12070_amd import Extractor
    e = Extractor(0)
    yield e
    e.close()


def gpu_nodes(ex, wind, periodic, cap=None):
    import torch
    from paper_1911_12070_amd import dims, vx_node_circulation
    nz, ny, nx = wind.shape
    cap = nx * ny * nz if cap is None else cap
    node = torch.empty_like(wind)
    lst = torch.empty(max(cap, 1), dtype=torch.int64, device=wind.device)
    count = torch.zeros(1, dtype=torch.int64, device=wind.device)
    vx_node_circulation(ex.h, dims(nx, ny, nz, periodic), wind, count, node, lst[:cap] if cap else None)
    torch.cuda.synchronize()
    n = int(count.cpu())
    ids = np.sort(lst[:min(n, cap)].cpu().numpy().view(np.uint64))
    return node.cpu().numpy(), ids, n


def w_from_packed(packed):
    w = np.zeros(packed.shape + (3,), np.int8)
    for a in range(3):
        v = (packed >> (2 * a)) & 3
        w[..., a] = np.where(v == 3, -1, v).astype(np.int8)
    return w


CASES = [((7, 5, 4), 7, "int"), ((13, 9, 6), 0, "int"), ((256, 3, 3), 5, "int"), ((260, 6, 5), 7, "int"),
         ((31, 17, 70), 3, "int"), ((96, 80, 64), 7, "tangle"), ((100, 66, 70), 6, "tangle"),
         ((257, 40, 33), 1, "tangle"), ((64, 64, 130), 4, "tangle"), ((2, 2, 2), 7, "int"),
         # whole 16-node words per lane (the wide kernel): two row segments, open and periodic axes,
         # rows not a multiple of the rows per wavefront
         ((1040, 6, 5), 5, "int"), ((112, 9, 70), 0, "tangle"), ((16, 3, 2), 7, "int"), ((2048, 5, 3), 2, "int")]


@pytest.mark.parametrize("shape,periodic,kind", CASES)
def test_node_circulation_parity(ex, shape, periodic, kind):
    nx, ny, nz = shape
    log(f"node circulation {shape} periodic={periodic} {kind}")
    if kind == "int":
        psi = vxinputs.random_small_int_field((nx, ny, nz), seed=nx * 7 + nz)
    else:
        psi = vxinputs.eval_tangle(vxinputs.make_tangle((128, 128, 128), 256, (3, 7), nx), (0, 0, 0, nx, ny, nz))
    W = oracle.winding(psi, periodic)
    out = run_winding(ex, to_dev(psi), periodic)
    assert np.array_equal(out["wind"].cpu().numpy(), W.packed)
    node, ids, n = gpu_nodes(ex, out["wind"], periodic)
    _, onode = oracle.node_circulation(W.w, periodic)
    bad = np.argwhere(node != onode)
    assert len(bad) == 0, f"{len(bad)} node bytes differ, first {bad[:4].tolist()}"
    oid = np.flatnonzero(onode.reshape(-1) & 0x40).astype(np.uint64)
    assert n == len(oid) and np.array_equal(ids, oid)


def test_node_circulation_capacity_and_status(ex):
    from paper_1911_12070_amd import VX_ERR_CAPACITY, VxError, vx_sync_status
    psi = vxinputs.eval_tangle(vxinputs.make_tangle((64, 64, 64), 256, (3, 8), 33))
    out = run_winding(ex, to_dev(psi), 7)
    try:
        vx_sync_status(ex.h)
    except VxError:
        pass
    node, ids, n = gpu_nodes(ex, out["wind"], 7)
    vx_sync_status(ex.h)
    node2, ids2, n2 = gpu_nodes(ex, out["wind"], 7, cap=n // 3)
    assert n2 == n and np.array_equal(node2, node) and np.isin(ids2, ids).all() and len(ids2) == n // 3
    with pytest.raises(VxError) as e:
        vx_sync_status(ex.h)
    assert e.value.status == VX_ERR_CAPACITY


def test_node_circulation_tangle_1024(ex):
    """The benchmark field: node bytes of every plane against the oracle from the GPU's packed field,
    by z-slabs of 64 planes (plus the plane below each slab)."""
    import torch
    t = vxinputs.tangle_1024()
    psi = ex.gen_tangle(t)
    out = ex.alloc_winding(psi.shape, face_cap=1 << 24, cell_cap=1 << 24, wind=True)
    ex.winding(psi, 7, out)
    torch.cuda.synchronize()
    del psi
    torch.cuda.empty_cache()
    node, ids, n = gpu_nodes(ex, out["wind"], 7, cap=1 << 26)
    packed = out["wind"].cpu().numpy()
    nf = int(out["counts"][0])
    total = 0
    for k0 in range(0, 1024, 64):
        # planes k0-1 .. k0+63 as an open-z grid: planes k0 .. k0+63 see their whole rings
        kk = np.arange(k0 - 1, k0 + 64) % 1024
        _, onode = oracle.node_circulation(w_from_packed(packed[kk]), 3)
        assert np.array_equal(node[k0:k0 + 64], onode[1:]), f"planes {k0}..{k0 + 63}"
        total += int((onode[1:] & 0x40 != 0).sum())
    assert n == total == len(ids)
    log(f"1024^3: {n} vortex nodes for {nf} pierced faces ({n / nf:.2f} per face)")
