"""GPU: the delay-filtered likelihood (eq. rime_filter, eq. gpr, eq. filtered_noise)
against the FP64 oracle, and its gradient against central differences of the
GPU chi^2_F at full 61-dish size."""
import math

import numpy as np
import pytest

from oracle import filter as fl
from oracle import model
from paper_2504_07090_amd import workload as w
from tests.gpu_common import GRAD_ELEM_FP32, max_rel, rel_norm, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_07090_amd import vis as v
    return v


def _params(d, cfg, scale=1.0):
    alm = torch.tensor(d.alm * scale, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    return alm, g, fw


@pytest.mark.parametrize("synthesis,side,nf", [(0, 4, 32), (1, 4, 32), (1, 3, 13), (0, 3, 70)],
                         ids=["dense", "separable", "ragged13", "two_row_blocks70"])
def test_filtered_chi2_and_gradient_match_oracle(vis, synthesis, side, nf):
    """13 channels leave a ragged contraction and row block, 70 channels need
    two 64-row blocks; 19 dishes (342 real columns) a ragged column block."""
    cfg = w.scaled(w.C0, array="hex", array_size=side, n_freq=nf, n_time=3, lmax=12,
                   freq_lo_hz=120e6, freq_hi_hz=130e6)
    basis = vis.Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, 1 | vis.STORAGE_SEPARABLE)
    fld = vis.Field.from_config(basis, cfg, vis.VIS_FP32, synthesis)
    filt = vis.Filter(w.frequencies(cfg))
    d = w.draw(cfg)
    of = model.Field(cfg)
    _, sig, data = model.make_data(of, d)
    f = fl.delay_filter(w.frequencies(cfg))
    rx2, rga, rgg, rgf = fl.chi2_filtered_and_grad(of, data, sig, f, d.alm * 1.2, d.gains,
                                                   w.fwhm_ref_rad(cfg))
    alm, g, fw = _params(d, cfg, 1.2)
    ddev = torch.tensor(np.ascontiguousarray(data), dtype=torch.complex64, device="cuda")
    x2, ga, gg, gf = vis.chi2_filtered_and_grad(fld, filt, ddev, sig, alm, g, fw)
    e = [abs(float(x2) - rx2) / rx2, rel_norm(ga.cpu().numpy(), rga), rel_norm(gg.cpu().numpy(), rgg),
         abs(float(gf) - rgf) / abs(rgf)]
    em = [max_rel(ga.cpu().numpy(), rga), max_rel(gg.cpu().numpy(), rgg)]
    say("filtered chi2 errs (chi2, a, g, F)", synthesis, e, "element-wise (a, g)", em)
    assert max(e) <= 2e-4
    assert max(em) <= GRAD_ELEM_FP32
    x2b, *_ = vis.chi2_filtered_and_grad(fld, filt, ddev, sig, alm, g, fw, grads=False)
    assert float(x2b) == float(x2)


def test_filter_channel_mismatch_rejected(vis):
    cfg = w.scaled(w.C0, n_freq=4, n_time=2)
    basis = vis.Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, 1)
    fld = vis.Field.from_config(basis, cfg)
    filt = vis.Filter(w.frequencies(w.scaled(cfg, n_freq=5)))
    d = w.draw(cfg)
    alm, g, fw = _params(d, cfg)
    data = torch.zeros((cfg.n_time, cfg.n_freq, fld.n_bl), dtype=torch.complex64, device="cuda")
    with pytest.raises(vis.VisError):
        vis.chi2_filtered_and_grad(fld, filt, data, 1.0, alm, g, fw)


def test_filtered_gradient_central_differences_c1(vis):
    """Full 61-dish size: chi^2_F is quadratic along every sky coefficient and every
    single real gain component, so central differences of the GPU chi^2_F are exact
    up to rounding for any step; 24 random coordinates.  The step moves chi^2_F by
    about 1e-3 of itself, so the FP32 rounding of the two chi^2_F values (a few
    1e-7 of chi^2_F) stays below 1e-3 of the difference.  The filter removes most
    of the smooth residual, so a sky-coefficient gradient is a sum with
    cancellation whose FP32 error is about uniform across coordinates (~1e-4 of a
    typical one, the same as against the oracle): the bar is 1e-3 of
    max(|g_k|, 0.1 rms of the sampled g)."""
    cfg = w.C1
    basis = vis.Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, vis.STORAGE_SEPARABLE)
    fld = vis.Field.from_config(basis, cfg, vis.VIS_FP32, vis.VIS_SYNTH_SEPARABLE)
    filt = vis.Filter(w.frequencies(cfg))
    d = w.draw(cfg)
    alm0, g0, fw0 = _params(d, cfg)
    m = vis.forward(fld, alm0, g0, fw0)
    rms = float(torch.sqrt(torch.mean(torch.abs(m) ** 2)))
    sig = 0.01 * rms / math.sqrt(2.0)
    data = (m + sig * math.sqrt(2.0) * torch.tensor(d.noise_unit, dtype=torch.complex64,
                                                    device="cuda")).contiguous()
    alm, g, fw = _params(d, cfg, 1.2)
    x2, ga, gg, gf = vis.chi2_filtered_and_grad(fld, filt, data, sig, alm, g, fw)
    chi0 = float(x2)

    def chi(a_, g_):
        return float(vis.chi2_filtered_and_grad(fld, filt, data, sig, a_, g_, fw, grads=False)[0])

    rng = np.random.default_rng(20)
    worst = 0.0
    rows = []
    for n in range(24):
        if n < 20:
            f, c = int(rng.integers(cfg.n_freq)), int(rng.integers(fld.n_modes))
            gk = float(ga[f, c])
            h = min(1e-3 * chi0 / max(abs(gk), 1e-30), 1e3 * float(alm[f].abs().max()))
            xp, xm = np.float32(float(alm[f, c]) + h), np.float32(float(alm[f, c]) - h)
            ap, am = alm.clone(), alm.clone()
            ap[f, c], am[f, c] = float(xp), float(xm)
            fd = (chi(ap, g) - chi(am, g)) / (float(xp) - float(xm))
        else:
            f, a, part = int(rng.integers(cfg.n_freq)), int(rng.integers(fld.n_ant)), n % 2
            z = complex(gg[f, a])
            gk = z.real if part == 0 else z.imag
            h = min(1e-3 * chi0 / max(abs(gk), 1e-30), 1.0)
            x = float(torch.view_as_real(g)[f, a, part])
            xp, xm = np.float32(x + h), np.float32(x - h)
            gp, gm = g.clone(), g.clone()
            torch.view_as_real(gp)[f, a, part] = float(xp)
            torch.view_as_real(gm)[f, a, part] = float(xm)
            fd = (chi(alm, gp) - chi(alm, gm)) / (float(xp) - float(xm))
        rows.append((gk, fd))
    scale = 0.1 * math.sqrt(np.mean([gk * gk for gk, _ in rows]))
    for n, (gk, fd) in enumerate(rows):
        rel = abs(fd - gk) / max(abs(gk), scale)
        worst = max(worst, rel)
        say("fd", n, "grad", gk, "fd", fd, "rel", rel)
    say("filtered fd c1 worst relative error", worst)
    assert worst <= 1e-3
