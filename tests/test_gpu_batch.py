"""Batching (frames of uneven size in one graph launch) against the oracle and the single-frame path.

Each frame's winding output must equal the oracle's exactly (as sets), and each refined sample
must equal, bit for bit, the sample the single-frame vx_refine produces for the same cell (same
kernel arithmetic; the single-frame path is itself checked against the oracle). Graph replays are
checked against the eager launch, with eager torch work in between, and after the frames' psi
values change in place. The autotuner must pick a listed depth, keep results unchanged and reuse
its cache.
"""
import os

import numpy as np
import pytest

import oracle
import vxinputs

from gpu_util import assert_winding_equal, canonical, log, to_dev

pytestmark = pytest.mark.gpu

# (nx, ny, nz, periodic): aligned, ragged/odd, non-periodic, ragged x tile + thin z, 2D, mixed mask
SHAPES = [(64, 48, 40, 7), (33, 17, 29, 7), (128, 30, 20, 0), (130, 16, 3, 5), (40, 40, 1, 3), (256, 45, 18, 6)]
CANDIDATES = {8, 16, 32, 64, 128}


@pytest.fixture(scope="module")
def ex():
    from paper_1911_12070_amd import Extractor
    e = Extractor(0)
    yield e
    e.close()


def frames_np(seed):
    parent = vxinputs.make_tangle((256, 64, 64), 192, (2, 6), seed)
    return [vxinputs.eval_tangle(parent, (0, 0, 0, nx, ny, nz)) for nx, ny, nz, _ in SHAPES]


def make_batch(ex, psis):
    from paper_1911_12070_amd import Batch
    frames = [(p, per) for p, (_, _, _, per) in zip(psis, SHAPES)]
    n_all = lambda n: 3 * n
    return Batch(ex, frames, face_cap=n_all, cell_cap=lambda n: n)


def samples_by_cell(out):
    from paper_1911_12070_amd import samples_to_numpy
    nc = min(int(out["counts"][1]), out["cells"].numel())
    s = samples_to_numpy(out["samples"], nc)
    return s[np.argsort(s["cell"], kind="stable")]


def results(batch):
    import torch
    torch.cuda.synchronize()
    return [(canonical(o), samples_by_cell(o)) for o in batch.outs]


def assert_same(ra, rb):
    for (ca, sa), (cb, sb) in zip(ra, rb):
        for x, y in zip(ca, cb):
            assert np.array_equal(np.asarray(x), np.asarray(y))
        assert sa.tobytes() == sb.tobytes()


def check_against_oracle(ex, batch, psis_np):
    import torch
    from paper_1911_12070_amd import samples_to_numpy
    torch.cuda.synchronize()
    for f, (psi, (nx, ny, nz, per)) in enumerate(zip(psis_np, SHAPES)):
        log(f"frame {f}: {nx}x{ny}x{nz} periodic={per} zchunk={batch.zchunk(f)}")
        o = batch.outs[f]
        assert_winding_equal(o, oracle.winding(psi, per))
        # the single-frame refinement of the same list, sample by sample
        single = ex.refine(batch.psi[f], o, per)
        torch.cuda.synchronize()
        nc = min(int(o["counts"][1]), o["cells"].numel())
        a = samples_to_numpy(o["samples"], nc)
        b = samples_to_numpy(single, nc)
        assert a.tobytes() == b.tobytes(), f"frame {f}: batched samples differ from vx_refine"


def test_batch_matches_oracle_eager_and_graph(ex):
    psis_np = frames_np(51)
    psis = [to_dev(p) for p in psis_np]
    batch = make_batch(ex, psis)
    batch.launch(graph=False)
    check_against_oracle(ex, batch, psis_np)
    r_eager = results(batch)
    for rep in range(3):
        for o in batch.outs:  # eager work between replays: scribble over every output
            for k in ("faces", "cells", "counts", "samples"):
                o[k].fill_(-1)
            o["wind"].fill_(255)
        batch.launch(graph=True)
        assert_same(results(batch), r_eager)
        log(f"graph replay {rep} matches the eager launch")
    batch.close()


def test_batch_replay_with_new_data(ex):
    psis = [to_dev(p) for p in frames_np(52)]
    batch = make_batch(ex, psis)
    batch.launch()
    new_np = frames_np(53)
    for dst, src in zip(psis, new_np):
        dst.copy_(to_dev(src))
    batch.launch()
    check_against_oracle(ex, batch, new_np)
    batch.close()


def test_batch_autotune_and_cache(ex, tmp_path):
    psis = [to_dev(p) for p in frames_np(54)]
    batch = make_batch(ex, psis)
    batch.launch(graph=False)
    ref = results(batch)
    cache = str(tmp_path / "tune.jsonl")
    assert batch.refine_wg() == 0 and batch.wind_wg() == 0  # the defaults until tuned
    batch.autotune(cache)
    chosen = [batch.zchunk(f) for f in range(len(SHAPES))]
    log(f"tuned z-chunks {chosen}, winding workgroups per CU {batch.wind_wg()}, refinement workgroups per CU "
        f"{batch.refine_wg()}")
    assert 2 <= batch.refine_wg() <= 8 and 1 <= batch.wind_wg() <= 16
    for z, (_, _, nz, _) in zip(chosen, SHAPES):
        assert z in CANDIDATES
    lines = open(cache).read().strip().splitlines()
    assert len(lines) == len({s for s in SHAPES})
    batch.launch()
    assert_same(results(batch), ref)
    batch.close()
    again = make_batch(ex, psis)
    again.autotune(cache)  # every shape is in the cache: no depth is timed, nothing is appended
    assert [again.zchunk(f) for f in range(len(SHAPES))] == chosen
    assert open(cache).read().strip().splitlines() == lines
    again.launch()
    assert_same(results(again), ref)
    again.close()


def test_autotune_single_grid(ex, tmp_path):
    import torch
    from paper_1911_12070_amd import dims, vx_autotune
    t = vxinputs.make_tangle((96, 80, 72), 128, (2, 6), 55)
    psi_np = vxinputs.eval_tangle(t)
    psi = to_dev(psi_np)
    z = vx_autotune(ex.h, dims(96, 80, 72, 7), psi, str(tmp_path / "g.jsonl"))
    log(f"tuned z-chunk {z}")
    assert z in CANDIDATES
    out = ex.alloc_winding(psi.shape, 3 * psi.numel(), psi.numel())
    ex.winding(psi, 7, out)
    torch.cuda.synchronize()
    assert_winding_equal(out, oracle.winding(psi_np, 7))


def test_batch_invalid_arguments(ex):
    from paper_1911_12070_amd import BATCH_MAX_FRAMES, Frame, VxError, dims, vx_batch_create, winding_out
    import torch
    psi = to_dev(frames_np(56)[0])
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    good = Frame(dims(64, 48, 40, 7), psi.data_ptr(), winding_out(counts), None, 0)
    with pytest.raises(VxError):
        vx_batch_create(ex.h, [])
    with pytest.raises(VxError):
        vx_batch_create(ex.h, [good] * (BATCH_MAX_FRAMES + 1))
    bad = Frame(dims(64, 48, 40, 7), None, winding_out(counts), None, 0)
    with pytest.raises(VxError):
        vx_batch_create(ex.h, [good, bad])
    b = vx_batch_create(ex.h, [good] * BATCH_MAX_FRAMES)  # the maximum is accepted
    from paper_1911_12070_amd import vx_batch_destroy
    vx_batch_destroy(ex.h, b)
