"""Training of the surrogate by the library's own kernels, end to end on the GPU.

Rows are built by vx_mlp_dataset from the plain refinement of a few small tangles; a network
initialised from the seeded initial weights is trained with vx_mlp_train_step (BF16 matrix-core
forward/backward, FP32 Adam) for a few hundred steps. Checks: the training loss falls; on a held-out
field, one Newton step from the trained network's point lands closer to the plain refinement than
one Newton step from the first estimate (the zero network), which is what the network adds to the
method."""
import numpy as np
import pytest

import vxinputs
from gpu_util import log

pytestmark = pytest.mark.gpu


def test_training_from_scratch_beats_the_zero_network():
    import torch
    from paper_1911_12070_amd import (MLP_NPARAMS, SAMPLE_SURROGATE, Extractor, dims, samples_to_numpy, vx_mlp_create,
                                      vx_mlp_destroy, vx_mlp_infer, vx_mlp_reserve)
    from paper_1911_12070_amd.surrogate import build_dataset, train
    ex = Extractor(0)
    try:
        tangles = [vxinputs.make_tangle((128, 128, 128), 512, (4, 8), 3000 + s) for s in range(8)]
        feat, target, n = build_dataset(ex, tangles, n_cap=120_000)
        log(f"training rows: {n}")
        assert n > 40_000
        m, hist, secs, steps = train(ex, feat, target, n, vxinputs.mlp_pack(vxinputs.mlp_init(7)), epochs=6,
                                     batch=1024, lr=2e-3, seed=1, log_every=20)
        first, last = hist[0], hist[-1]
        log(f"{steps} steps in {secs:.2f} s: mse {first[1]:.3e} -> {last[1]:.3e}, conf loss {first[2]:.3e} -> "
            f"{last[2]:.3e}")
        assert steps >= 300
        assert last[1] < 0.5 * first[1], "the position loss must fall"
        # held-out field: one Newton step from the trained network's point vs from x0 (zero network)
        psi = ex.gen_tangle(vxinputs.make_tangle((128, 128, 128), 512, (4, 8), 4000))
        out = ex.alloc_winding(psi.shape, face_cap=1 << 17, cell_cap=1 << 17, wind=False)
        ex.winding(psi, 7, out)
        plain = ex.refine(psi, out, 7)
        torch.cuda.synchronize()
        nc = int(out["counts"][1])
        cap = out["cells"].numel()
        P = samples_to_numpy(plain, nc)
        zero = vx_mlp_create(ex.h, np.zeros(MLP_NPARAMS, np.float32), 64)
        errs = {}
        for name, net in (("zero", zero), ("trained", m)):
            vx_mlp_reserve(ex.h, net, cap)
            res = ex.alloc_samples(cap)
            vx_mlp_infer(ex.h, net, dims(128, 128, 128, 7), psi, out["cells"], out["cdesc"], out["counts"][1:], cap,
                         0.0, res, max_step=0.0)
            torch.cuda.synchronize()
            S = samples_to_numpy(res, nc)
            used = (S["status"] & SAMPLE_SURROGATE) != 0
            good = used & ((P["status"] & (8 | 16 | 32 | 64)) == 0)
            errs[name] = np.abs(S["off"][good].astype(np.float64) - P["off"][good]).max(axis=1)
        vx_mlp_destroy(ex.h, zero)
        vx_mlp_destroy(ex.h, m)
        for name, e in errs.items():
            log(f"held-out, one Newton step from the {name} network: median {np.median(e):.2e}, "
                f"within 0.02: {np.mean(e < 0.02):.4f} ({len(e)} cells)")
        assert np.median(errs["trained"]) < 0.5 * np.median(errs["zero"])
        assert np.mean(errs["trained"] < 0.02) > np.mean(errs["zero"] < 0.02)
    finally:
        ex.close()
