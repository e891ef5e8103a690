"""The consumers of the GPU lists, end to end: the dual graph (Sec. 3.1-3.2, 3.4 classes), sample
points by box means and graph reduction (Sec. 3.3.1-3.3.2) refined on the GPU from their seeds
(Sec. 3.3.3), Catmull-Rom curves (Sec. 3.4) and the density error metric e (Sec. 5), against the
oracle: the host steps bit for bit on the GPU's own lists, the seeded refinement to 1e-4 cell, the
density at points to FP32 rounding. At 1024^3 (the benchmark field) through invariants and the
oracle's refinement of sampled seeds."""
import numpy as np
import pytest

import oracle
import vxinputs
from gpu_util import log
from oracle import graph as G
from whole_parity import COND_LIMIT, TOL, gpu_lists

pytestmark = pytest.mark.gpu


def refine_seeds(ex, psi, periodic, R):
    """GPU refinement of the reduced nodes from their seeds; absolute positions and the samples."""
    import torch
    from paper_1911_12070_amd import dims, samples_to_numpy, vx_refine
    nz, ny, nx = psi.shape
    dev = psi.device
    m = len(R["seed_cell"])
    cells = torch.from_numpy(R["seed_cell"].view(np.int64)).to(dev)
    desc = torch.from_numpy(R["seed_desc"].view(np.int16)).to(dev)
    seed = torch.from_numpy(R["seed_off"]).to(dev)
    count = torch.tensor([m], dtype=torch.int64, device=dev)
    out = torch.empty((m, 8), dtype=torch.int32, device=dev)
    vx_refine(ex.h, dims(nx, ny, nz, periodic), psi, cells, desc, count, out, seed=seed, cap=m)
    torch.cuda.synchronize()
    s = samples_to_numpy(out, m)
    c = R["seed_cell"].astype(np.int64)
    corner = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], 1).astype(np.float64)
    return s, corner + s["off"].astype(np.float64)


def gpu_density(ex, psi, periodic, pts):
    import torch
    from paper_1911_12070_amd import dims, vx_density
    nz, ny, nx = psi.shape
    p = torch.from_numpy(np.ascontiguousarray(pts, np.float64)).to(psi.device)
    rho = torch.empty(len(pts), dtype=torch.float32, device=psi.device)
    vx_density(ex.h, dims(nx, ny, nz, periodic), psi, p, rho)
    torch.cuda.synchronize()
    return rho.cpu().numpy().astype(np.float64)


def mean_density(ex, psi, periodic):
    import torch
    from paper_1911_12070_amd import dims, vx_mean_density
    nz, ny, nx = psi.shape
    out = torch.zeros(1, dtype=torch.float64, device=psi.device)
    vx_mean_density(ex.h, dims(nx, ny, nz, periodic), psi, out)
    torch.cuda.synchronize()
    return float(out.cpu())


@pytest.mark.parametrize("name,k", [("line_ring_32", 3), ("tangle_256", 4), ("tangle_96_open", 5)])
def test_vectorize_against_oracle(name, k):
    import torch
    from paper_1911_12070_amd import Extractor, dims, vx_curves, vx_graph_lines, vx_reduce
    ex = Extractor(0)
    try:
        if name == "line_ring_32":
            psi, per = ex.gen_line_ring(vxinputs.line_ring_32()), 7
        elif name == "tangle_256":
            psi, per = ex.gen_tangle(vxinputs.tangle_256()), 7
        else:
            t = vxinputs.make_tangle((128, 128, 128), 256, (3, 7), 77)
            psi = torch.from_numpy(vxinputs.eval_tangle(t, (0, 0, 0, 96, 80, 72))).cuda()
            per = 0
        nz, ny, nx = psi.shape
        d = dims(nx, ny, nz, per)
        out = ex.alloc_winding(psi.shape, face_cap=1 << 20, cell_cap=1 << 20, wind=False)
        ex.winding(psi, per, out)
        torch.cuda.synchronize()
        faces, fsign, cells, cdesc = gpu_lists(out)
        psi_h = psi.cpu().numpy()
        # graph
        comp, deg, types, st = vx_graph_lines(d, cells, cdesc)
        ocomp, odeg, otypes, ost = G.graph_lines((nx, ny, nz), per, cells, cdesc)
        assert np.array_equal(comp, ocomp) and np.array_equal(deg, odeg) and np.array_equal(types, otypes) and st == ost
        assert st["nedge"] + st["nboundary"] == len(faces)
        # sample points
        R = vx_reduce(d, cells, cdesc, k, 5)
        pos, edges, mem, rcomp, passes = G.reduce_graph((nx, ny, nz), per, cells, cdesc, k, 5)
        assert np.array_equal(R["pos"], pos) and np.array_equal(R["edges"], np.array(edges, np.int64).reshape(-1, 2))
        # refinement of the samples from their seeds, GPU against the FP64 oracle
        s, xstar = refine_seeds(ex, psi, per, R)
        O = oracle.refine(psi_h, R["seed_cell"], R["seed_desc"], periodic=per,
                          seeds=R["seed_off"].astype(np.float64))
        ok = (O.status & (oracle.NONZERO_MIN | oracle.NOT_CONVERGED)) == 0
        err = np.abs(s["off"].astype(np.float64) - O.x).max(axis=1)
        bad = ok & (err > TOL) & (O.cond <= COND_LIMIT) & ((s["status"] & (8 | 16)) == 0)
        log(f"{name} k={k}: {len(cells)} cells -> {len(pos)} samples in {passes} passes; refined: "
            f"{ok.sum()} converged, max err {err[ok].max():.2e}, above {TOL}: {(ok & (err > TOL)).sum()}")
        assert not bad.any()
        # curves of the refined samples
        C = vx_curves(d, xstar, R["edges"], 8)
        ch = G.chains(len(xstar), [tuple(e) for e in R["edges"].tolist()])
        assert len(ch) == len(C["length"])
        for c, (nodes, closed) in enumerate(ch):
            pts, L = G.curve((nx, ny, nz), per, xstar.tolist(), nodes, closed, 8)
            assert np.array_equal(C["points"][C["pt_start"][c]:C["pt_start"][c + 1]], np.array(pts))
            assert C["length"][c] == L and bool(C["closed"][c]) == closed
        # density at points and the error metric e = sum rho / (mean rho N)
        rbar = mean_density(ex, psi, per)
        assert abs(rbar - float(np.mean(np.abs(psi_h.astype(np.complex128)) ** 2))) < 1e-9 * rbar
        e = {}
        for tag, pts in (("x0", R["pos"]), ("x_refined", xstar), ("curve", C["points"])):
            g = gpu_density(ex, psi, per, pts)
            sel = np.arange(0, len(pts), max(1, len(pts) // 3000))
            o = oracle.density_at(psi_h, pts[sel], per)
            assert np.abs(g[sel] - o).max() <= 1e-5 * rbar + 1e-5 * o.max(), tag
            e[tag] = float(g.sum() / (rbar * len(pts)))
        log(f"{name}: {len(C['length'])} curves ({int(C['closed'].sum())} closed), total length "
            f"{C['total_length']:.1f}; e(x0) {e['x0']:.3e}, e(refined) {e['x_refined']:.3e}, e(curve) {e['curve']:.3e}")
        assert e["x_refined"] < 0.1 * e["x0"]  # the refinement moves the samples onto the cores
    finally:
        ex.close()


def test_vectorize_tangle_1024():
    """The benchmark field's lists through every consumer; exact invariants, sampled oracle refinement."""
    import time

    import torch
    from paper_1911_12070_amd import Extractor, dims, vx_curves, vx_graph_lines, vx_reduce
    ex = Extractor(0)
    try:
        psi = ex.gen_tangle(vxinputs.tangle_1024())
        out = ex.alloc_winding(psi.shape, face_cap=1 << 24, cell_cap=1 << 24, wind=False)
        ex.winding(psi, 7, out)
        torch.cuda.synchronize()
        faces, fsign, cells, cdesc = gpu_lists(out)
        d = dims(1024, 1024, 1024, 7)
        t0 = time.perf_counter()
        comp, deg, types, st = vx_graph_lines(d, cells, cdesc)
        t1 = time.perf_counter()
        R = vx_reduce(d, cells, cdesc, 4, 5)
        t2 = time.perf_counter()
        assert st["nedge"] == len(faces) and st["nboundary"] == 0 and (deg % 2 == 0).all()
        assert st["ntype"][0] == 0  # no open line on a periodic grid
        assert R["members"].sum() == len(cells) and len(np.unique(R["comp"])) == st["ncomp"]
        s, xstar = refine_seeds(ex, psi, 7, R)
        t3 = time.perf_counter()
        C = vx_curves(d, xstar, R["edges"], 8)
        t4 = time.perf_counter()
        # sampled seeds against the oracle (patches of the GPU field's own bytes)
        rng = np.random.default_rng(0)
        pick = rng.choice(len(xstar), 300, replace=False)
        worst, nchk = 0.0, 0
        for i in pick:
            c = int(R["seed_cell"][i])
            x, y, z = c % 1024, (c // 1024) % 1024, c // (1024 * 1024)
            zi = torch.tensor([(z + q) % 1024 for q in (-1, 0, 1, 2)], device=psi.device)
            yi = torch.tensor([(y + q) % 1024 for q in (-1, 0, 1, 2)], device=psi.device)
            xi = torch.tensor([(x + q) % 1024 for q in (-1, 0, 1, 2)], device=psi.device)
            patch = psi.index_select(0, zi).index_select(1, yi).index_select(2, xi).cpu().numpy()
            grid = np.zeros((4, 4, 4), np.complex64)
            grid[:] = patch
            O = oracle.refine(grid, np.array([21], np.uint64), R["seed_desc"][i:i + 1], periodic=0,
                              seeds=R["seed_off"][i:i + 1].astype(np.float64))
            if O.status[0] & (8 | 16 | 4) or O.cond[0] > COND_LIMIT or s["status"][i] & (8 | 16):
                continue
            worst = max(worst, float(np.abs(s["off"][i] - O.x[0]).max()))
            nchk += 1
        log(f"1024^3: graph {t1 - t0:.2f} s ({st['ncomp']} lines, {st['ntype']} by type, {st['nbranch']} branch "
            f"cells), reduction {t2 - t1:.2f} s ({len(cells)} cells -> {len(xstar)} samples, {R['passes']} passes), "
            f"seeded refinement {t3 - t2:.2f} s, curves {t4 - t3:.2f} s ({len(C['length'])} curves, total length "
            f"{C['total_length']:.0f}); sampled seeds vs oracle: {nchk} checked, worst {worst:.2e}")
        assert nchk > 200 and worst <= TOL
    finally:
        ex.close()


@pytest.mark.parametrize("name", ["line_ring_32", "tangle_96_open"])
def test_extractor_vectorize_equals_the_steps(name):
    """Extractor.vectorize (one call from the field to curves) gives exactly what its steps give when
    called one by one: graph, reduced samples, their refinement and the curves."""
    import torch
    from paper_1911_12070_amd import Extractor, dims, vx_curves, vx_graph_lines, vx_reduce
    ex = Extractor(0)
    try:
        if name == "line_ring_32":
            psi, per = ex.gen_line_ring(vxinputs.line_ring_32()), 7
        else:
            t = vxinputs.make_tangle((128, 128, 128), 256, (3, 7), 77)
            psi = torch.from_numpy(vxinputs.eval_tangle(t, (0, 0, 0, 96, 80, 72))).cuda()
            per = 0
        nz, ny, nx = psi.shape
        d = dims(nx, ny, nz, per)
        V = ex.vectorize(psi, per, box_k=4, max_passes=5, seg_points=8)
        out = ex.alloc_winding(psi.shape, face_cap=1 << 20, cell_cap=1 << 20, wind=False)
        ex.winding(psi, per, out)
        torch.cuda.synchronize()
        _, _, cells, cdesc = gpu_lists(out)
        comp, deg, types, st = vx_graph_lines(d, cells, cdesc)
        # the list order differs between two windings (compaction order): compare what does not
        # depend on it
        assert V["graph"]["stats"] == st
        assert np.array_equal(np.bincount(V["graph"]["comp_type"], minlength=4), np.bincount(types, minlength=4))
        assert np.array_equal(np.sort(V["graph"]["degree"]), np.sort(deg))
        # the reduction sorts the cells itself: same samples whatever the list order
        R = vx_reduce(d, cells, cdesc, 4, 5)
        assert np.array_equal(V["samples"]["edges"], R["edges"]) and V["samples"]["passes"] == R["passes"]
        s, xstar = refine_seeds(ex, psi, per, R)
        assert np.array_equal(V["samples"]["pos"], xstar)
        assert V["samples"]["records"].tobytes() == s.tobytes()
        C = vx_curves(d, xstar, R["edges"], 8)
        for k in ("pt_start", "points", "length", "closed", "node_start", "nodes"):
            assert np.array_equal(V["curves"][k], C[k]), k
        log(f"{name}: vectorize = steps ({len(cells)} cells, {len(xstar)} samples, {len(C['length'])} curves)")
    finally:
        ex.close()
