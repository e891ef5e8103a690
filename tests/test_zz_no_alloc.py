"""The refinement entry point that allocates nothing (vx_refine_noalloc) against vx_refine: the same
kernels with their work counter in the library's fixed per-device scratch array instead of the
handle's workspace, so every sample must be the same bit for bit. Two calls in a row, the second
on a smaller input (a long list that runs the long-list kernel, then a short one that runs the
short-list kernel), plus seeds, a capacity below the count and an empty list."""
import numpy as np
import pytest

import vxinputs
from gpu_util import log, run_winding, to_dev

pytestmark = pytest.mark.gpu


def _ref_and_noalloc(ex, psi, out, periodic, cap=None, seed=None, count=None):
    import torch
    from paper_1911_12070_amd import dims, vx_refine, vx_refine_noalloc
    nz, ny, nx = psi.shape
    d = dims(nx, ny, nz, periodic)
    n = out["cells"].numel()
    cap = n if cap is None else cap
    count = out["counts"][1:] if count is None else count
    a = torch.full((n, 8), -3, dtype=torch.int32, device="cuda:0")
    b = torch.full((n, 8), -5, dtype=torch.int32, device="cuda:0")
    vx_refine(ex.h, d, psi, out["cells"], out["cdesc"], count, a, seed=seed, cap=cap)
    vx_refine_noalloc(d, psi, out["cells"], out["cdesc"], count, b, seed=seed, cap=cap)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy()


def test_noalloc_refine_equals_refine():
    import torch
    from paper_1911_12070_amd import Extractor
    ex = Extractor(0)
    try:
        # first call: every pierced cell of a 256^3 tangle (a long list: the long-list kernel)
        t = vxinputs.make_tangle((256, 256, 256), 512, (4, 8), 2)
        psi = ex.gen_tangle(t)
        out = run_winding(ex, psi, 7, face_cap=1 << 20, cell_cap=1 << 20)
        nc = int(out["counts"][1])
        log(f"no-alloc refinement: long list of {nc} cells")
        assert nc > 20000
        a, b = _ref_and_noalloc(ex, psi, out, 7)
        assert np.array_equal(a[:nc], b[:nc])
        assert (b[nc:] == -5).all()
        # second call, smaller input: an open 40x36x32 grid (a short list: the short-list kernel)
        psi2_np = vxinputs.eval_tangle(vxinputs.make_tangle((64, 64, 64), 256, (3, 7), 41), (0, 0, 0, 40, 36, 32))
        psi2 = to_dev(psi2_np)
        out2 = run_winding(ex, psi2, 0)
        nc2 = int(out2["counts"][1])
        log(f"no-alloc refinement: short list of {nc2} cells")
        assert 0 < nc2 < nc
        a, b = _ref_and_noalloc(ex, psi2, out2, 0)
        assert np.array_equal(a[:nc2], b[:nc2])
        # caller seeds, and a capacity below the count (the first cap samples only)
        seed = torch.rand((out2["cells"].numel(), 3), dtype=torch.float32, device="cuda:0")
        a, b = _ref_and_noalloc(ex, psi2, out2, 0, cap=nc2 // 2, seed=seed)
        assert np.array_equal(a[:nc2 // 2], b[:nc2 // 2])
        assert (a[nc2 // 2:] == -3).all() and (b[nc2 // 2:] == -5).all()
        # an empty list writes nothing
        zero = torch.zeros(1, dtype=torch.int64, device="cuda:0")
        a, b = _ref_and_noalloc(ex, psi2, out2, 0, count=zero)
        assert (b == -5).all()
        # the long list again after the short one (the shared counter starts from zero each call)
        a, b = _ref_and_noalloc(ex, psi, out, 7)
        assert np.array_equal(a[:nc], b[:nc])
    finally:
        ex.close()


def test_noalloc_rejects_bad_arguments():
    import torch
    from paper_1911_12070_amd import VX_ERR_INVALID, dims, lib
    from paper_1911_12070_amd import vx_refine_defaults
    import ctypes
    L = lib()
    psi = torch.zeros((4, 4, 4), dtype=torch.complex64, device="cuda:0")
    p = vx_refine_defaults()
    assert L.vx_refine_noalloc(dims(4, 4, 4, 8), psi.data_ptr(), None, None, None, None, 4, ctypes.byref(p), None,
                               None) == VX_ERR_INVALID
    assert L.vx_refine_noalloc(dims(4, 4, 4, 7), psi.data_ptr(), None, None, None, None, 4, ctypes.byref(p), None,
                               None) == VX_ERR_INVALID
    assert L.vx_refine_noalloc(dims(4, 4, 4, 7), psi.data_ptr(), None, None, None, None, -1, ctypes.byref(p), None,
                               None) == VX_ERR_INVALID
