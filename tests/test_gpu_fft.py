"""GPU parity of the fused wave-space transform kernels (power-of-two grids,
64 <= M <= 2048) against the rocFFT path of the same library (real-to-complex
transform, multiplier kernel, complex-to-real transform; FBIM_FLAG_LIBRARY_FFT).

Both compute M^(w) mu (Section 3.2) and the random field (Section 3.3) by the
same algorithm and differ only in the order of rounding: FP64 results agree to
1e-12 relative (the transforms' own error is ~1e-15 log M), FP32 results of a
mixed context to 2e-5 relative (FP32 transforms of length 2048 reach ~1e-6;
the spreading and interpolation are shared).  The oracle parity of the fused
path is covered by the matvec and solver tests, whose power-of-two workloads
now run it (tiny2, M = 48, keeps the rocFFT path covered)."""
import numpy as np
import pytest

import workloads as W
from gpu_util import dev, host, log, make_ctx, relerr, zeros

pytestmark = pytest.mark.gpu


def _pair(M, **over):
    import paper_1709_01480_amd as fb
    wl = W.make("starfish4", grid_M=M)
    a = make_ctx(wl, **over)
    flags = over.pop("flags", 0)
    b = make_ctx(wl, flags=flags | fb.FLAG_LIBRARY_FFT, **over)
    return wl, a, b


@pytest.mark.parametrize("M", [64, 128, 256, 512, 1024, 2048])
def test_fused_wave_part_matches_library_fft(M):
    import paper_1709_01480_amd as fb
    log("fused vs rocFFT M^(w), M = %d" % M)
    wl, a, b = _pair(M)
    mu = np.random.default_rng(M).standard_normal(2 * wl.n_nodes)
    oa, ob = zeros(2 * wl.n_nodes), zeros(2 * wl.n_nodes)
    a.apply_M(dev(mu), oa, fb.PART_WAVE)
    b.apply_M(dev(mu), ob, fb.PART_WAVE)
    assert relerr(host(oa), host(ob)) < 1e-12


@pytest.mark.parametrize("M", [64, 256, 2048])
def test_fused_random_field_matches_library_fft(M):
    log("fused vs rocFFT random field, M = %d" % M)
    wl, a, b = _pair(M)
    Wg = np.random.default_rng(M + 1).standard_normal(2 * M * M)
    oa, ob = zeros(2 * wl.n_nodes), zeros(2 * wl.n_nodes)
    a.random_field(dev(Wg), oa)
    b.random_field(dev(Wg), ob)
    assert relerr(host(oa), host(ob)) < 1e-12


@pytest.mark.parametrize("M", [64, 512, 2048])
def test_fused_fp32_wave_part_matches_library_fft(M):
    import paper_1709_01480_amd as fb
    log("fused vs rocFFT FP32 M^(w), M = %d" % M)
    wl, a, b = _pair(M, precision=fb.PREC_MIXED)
    mu = np.random.default_rng(M + 2).standard_normal(2 * wl.n_nodes)
    oa, ob = zeros(2 * wl.n_nodes), zeros(2 * wl.n_nodes)
    a.apply_M(dev(mu), oa, fb.PART_WAVE)  # a mixed context applies the FP32 operator
    b.apply_M(dev(mu), ob, fb.PART_WAVE)
    assert relerr(host(oa), host(ob)) < 2e-5


def test_batched_fused_matches_single_library_fft():
    """Two systems of grids 64 and 128 in one batch (fused kernels, one size
    class each) against single contexts on the rocFFT path."""
    import paper_1709_01480_amd as fb
    wls = [W.make("starfish4", grid_M=64), W.make("starfish4", grid_M=128, seed=3)]
    b = fb.Batch([w.params() for w in wls])
    for m, wl in zip(b.members, wls):
        sid = m.add_shape(fb.starfish(wl.r_s, wl.b, wl.n_arm, wl.n_p))
        m.set_bodies(np.full(wl.n_bodies, sid), wl.q, wl.theta)
    rng = np.random.default_rng(5)
    mus = [rng.standard_normal(2 * wl.n_nodes) for wl in wls]
    outs = [zeros(2 * wl.n_nodes) for wl in wls]
    b.apply_M([dev(m) for m in mus], outs)
    for wl, mu, out in zip(wls, mus, outs):
        ref = zeros(2 * wl.n_nodes)
        make_ctx(wl, flags=fb.FLAG_LIBRARY_FFT).apply_M(dev(mu), ref)
        assert relerr(host(out), host(ref)) < 1e-12
