"""Checks of the seeded input construction against the plain definitions of the fields.

The host evaluator uses an integer phase index and an FP64 table; the oracle evaluates the
defining sums with complex exponentials. Both must agree to FP32 rounding; the grid mean of
|psi|^2 is 1 by discrete Parseval; the noise has the requested statistics.
"""
import numpy as np

import oracle
import vxinputs


def test_shell_sizes():
    # distinct lattice points available for each workload's shell
    assert len(vxinputs.shell_points(4, 8)) == 1858
    assert len(vxinputs.shell_points(8, 24)) == 55674
    assert len(vxinputs.shell_points(4, 12)) == 6902
    assert len(vxinputs.shell_points(6, 16)) == 16182


def test_tangle_matches_definition_and_parseval():
    for dims, nw, shell, seed in [((32, 32, 32), 128, (3, 6), 1), ((24, 20, 36), 64, (2, 5), 2)]:
        t = vxinputs.make_tangle(dims, nw, shell, seed)
        psi = vxinputs.eval_tangle(t)
        nx, ny, nz = dims
        z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
        ref = oracle.tangle_at(t.n, t.c, dims, nodes).reshape(psi.shape)
        assert np.abs(psi - ref).max() < 2e-6
        assert abs(np.mean(np.abs(ref) ** 2) - 1.0) < 1e-12
        assert abs(np.mean(np.abs(psi.astype(np.complex128)) ** 2) - 1.0) < 1e-5


def test_tangle_box_wraps_periodically():
    t = vxinputs.make_tangle((16, 16, 16), 32, (2, 4), 3)
    full = vxinputs.eval_tangle(t)
    box = vxinputs.eval_tangle(t, (-3, 14, 30, 8, 8, 8))
    zi = (np.arange(30, 38) % 16)[:, None, None]
    yi = (np.arange(14, 22) % 16)[None, :, None]
    xi = (np.arange(-3, 5) % 16)[None, None, :]
    assert np.array_equal(box.view(np.uint64), full[zi, yi, xi].view(np.uint64))


def test_time_advance_is_the_wave_dispersion():
    t = vxinputs.make_tangle((16, 16, 16), 16, (2, 4), 4)
    t1 = t.at_time(0.05)
    w = 0.5 * (t.n ** 2).sum(1)
    assert np.allclose(t1.c, t.c * np.exp(-0.05j * w), rtol=0, atol=1e-15)


def test_line_ring_matches_definition_and_noise_statistics():
    lr = vxinputs.line_ring_32()
    clean = vxinputs.LineRing(noise_sigma=0.0)
    psi = vxinputs.eval_line_ring(clean)
    z, y, x = np.meshgrid(*(np.arange(32),) * 3, indexing="ij")
    nodes = np.stack([x.ravel(), y.ravel(), z.ravel()], 1)
    ref = oracle.line_ring_at((32, 32, 32), lr.line, lr.ring_center, lr.radius, lr.xi, nodes)
    assert np.abs(psi.ravel() - ref).max() < 1e-6
    noisy = vxinputs.eval_line_ring(lr)
    d = (noisy.astype(np.complex128) - psi).ravel()
    for comp in (d.real, d.imag):
        n = comp.size
        assert abs(comp.mean()) < 3 * lr.noise_sigma / np.sqrt(n)
        assert abs(comp.std() - lr.noise_sigma) < 3 * lr.noise_sigma / np.sqrt(2 * n)


def test_series_sizes_and_shared_waves():
    s = vxinputs.series_64()
    assert len(s.sizes) == 64 and set(s.sizes) <= {128, 192, 256, 384}
    f3 = s.frame(3)
    assert f3.dims == (s.sizes[3],) * 3 and np.array_equal(f3.n, s.base.n)
    assert np.abs(np.abs(s.base.n).max()) < 128 // 2
