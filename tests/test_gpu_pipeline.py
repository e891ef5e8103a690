"""Two-stream frame pipeline: the winding of frame k overlaps the refinement of frame k-1. Results
must equal the serial calls frame by frame (pierced sets exactly; samples bit for bit, matched by
cell, since list order follows the winding kernel's atomics)."""
import numpy as np
import pytest

import vxinputs

from gpu_util import log

pytestmark = pytest.mark.gpu


def _by_cell(s):
    return s[np.argsort(s["cell"], kind="stable")]


def test_pipeline_matches_serial():
    import torch
    from paper_1911_12070_amd import Extractor, FramePipeline, samples_to_numpy
    ex = Extractor(0)
    shape = (96, 128, 160)
    frames = [ex.gen_tangle(vxinputs.make_tangle(shape, 256, (3, 7), 70 + f)) for f in range(5)]
    torch.cuda.synchronize()
    n = shape[0] * shape[1] * shape[2]
    cap = n // 8
    serial = []
    for psi in frames:
        out = ex.alloc_winding(psi.shape, face_cap=cap, cell_cap=cap, wind=True)
        ex.winding(psi, 7, out)
        smp = ex.refine(psi, out, 7)
        torch.cuda.synchronize()
        nf, nc = (int(v) for v in out["counts"].cpu())
        serial.append((nf, nc, out["wind"].cpu().numpy().copy(), np.sort(out["faces"][:nf].cpu().numpy()),
                       _by_cell(samples_to_numpy(smp, nc))))
    pipe = FramePipeline(ex, frames[0].shape, cap, cap)
    pending = []
    for f, psi in enumerate(frames):
        pending.append((f, pipe.push(psi)))
        if len(pending) == 2:  # the older frame's slot is reused two pushes later: read it now
            f0, b0 = pending.pop(0)
            pipe.done(b0).synchronize()
            _check(pipe, f0, b0, serial)
    pipe.sync()
    for f0, b0 in pending:
        _check(pipe, f0, b0, serial)
    ex.close()


def _check(pipe, f, b, serial):
    from paper_1911_12070_amd import samples_to_numpy
    nf, nc, wind, faces, smp = serial[f]
    out = pipe.outs[b]
    got_nf, got_nc = (int(v) for v in out["counts"].cpu())
    assert (got_nf, got_nc) == (nf, nc), f
    assert np.array_equal(out["wind"].cpu().numpy(), wind), f
    assert np.array_equal(np.sort(out["faces"][:nf].cpu().numpy()), faces), f
    got = _by_cell(samples_to_numpy(pipe.samples[b], nc))
    assert got.tobytes() == smp.tobytes(), f
    log(f"frame {f}: {nf} faces, {nc} cells identical to the serial calls")
