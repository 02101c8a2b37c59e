"""The chi^2 autograd.Function: its backward against the FP64 oracle gradient
(16-dish field) and against central finite differences of the GPU chi^2 on 200
random coordinates of the 61-dish field (~6.6e5 parameters).

Finite differences.  The model is linear in the sky coefficients and, because
every visibility pairs two different antennas, linear in each single real gain
component; chi^2 is therefore exactly quadratic along every such coordinate
and the central difference equals the derivative for any step.  The step is
chosen so that the first-order change of chi^2 is 1e-4 of chi^2 itself, far
above the rounding noise of the FP64 total of FP32 terms (~1e-9 relative).
Only the beam width enters non-polynomially: its step is 1e-3 of F, where the
truncation error is ~(h/F)^2 ~ 1e-6 relative.  Steps are the differences of
the FP32 values actually evaluated.  Bar: relative error <= 1e-3 on every
sampled coordinate.
"""
import math

import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from oracle import model
from tests.gpu_common import rel_norm, say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_07090_amd import vis as v
    return v


def _params(d, cfg, alm_scale, fw_scale=1.0, grad=False):
    alm = torch.tensor(d.alm * alm_scale, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg) * fw_scale], dtype=torch.float32, device="cuda")
    if grad:
        for x in (alm, g, fw):
            x.requires_grad_(True)
    return alm, g, fw


def test_autograd_function_c0_matches_oracle(vis):
    """backward of 3 * chi^2 through VisChi2Function equals 3 x the oracle gradient."""
    cfg = w.C0
    basis = vis.basis_for(cfg, storage=1)
    fld = vis.Field.from_config(basis, cfg)
    d = w.draw(cfg)
    of = model.Field(cfg)
    _, sig, data = model.make_data(of, d)
    alm, g, fw = _params(d, cfg, 1.2, grad=True)
    ddev = torch.tensor(data, dtype=torch.complex64, device="cuda")
    x2 = vis.VisChi2Function.apply(alm, g, fw, fld, ddev, sig)
    (3.0 * x2).backward()
    rx2, rga, rgg, rgf = model.chi2_and_grad(of, data, sig, d.alm * 1.2, d.gains, w.fwhm_ref_rad(cfg))
    e = [rel_norm(alm.grad.cpu().numpy(), 3 * rga), rel_norm(g.grad.cpu().numpy(), 3 * rgg),
         abs(float(fw.grad) - 3 * rgf) / abs(3 * rgf), abs(float(x2) - rx2) / rx2]
    say("autograd c0 errs (a, g, F, chi2)", e)
    assert max(e) <= 2e-4


def _coordinates(nf, nm, nant, rng):
    """200 coordinates uniform over the flat parameter vector [a | gains (Re, Im) | F],
    plus 16 gain components and F so that every parameter kind is exercised."""
    na, ng = nf * nm, nf * nant * 2
    flat = rng.choice(na + ng + 1, size=200, replace=False)
    extra = na + rng.choice(ng, size=16, replace=False)
    out = []
    for k in np.concatenate([flat, extra, [na + ng]]):
        k = int(k)
        if k < na:
            out.append(("a", divmod(k, nm)))
        elif k < na + ng:
            f, r = divmod(k - na, nant * 2)
            out.append(("g", (f, r // 2, r % 2)))
        else:
            out.append(("F", None))
    return out


def test_finite_differences_200_coordinates_c1(vis):
    cfg = w.C1
    basis = vis.basis_for(cfg, storage=1)
    fld = vis.Field.from_config(basis, cfg)
    d = w.draw(cfg)
    alm0, g0, fw0 = _params(d, cfg, 1.0)
    m = vis.forward(fld, alm0, g0, fw0)
    rms = float(torch.sqrt(torch.mean(torch.abs(m) ** 2)))
    sig = 0.01 * rms / math.sqrt(2.0)
    data = (m + sig * math.sqrt(2.0) * torch.tensor(d.noise_unit, dtype=torch.complex64,
                                                    device="cuda")).contiguous()
    del m
    alm, g, fw = _params(d, cfg, 1.2, fw_scale=1.03, grad=True)
    x2 = vis.VisChi2Function.apply(alm, g, fw, fld, data, sig)
    x2.backward()
    chi0 = float(x2)
    ga, gg, gf = alm.grad.detach(), g.grad.detach(), fw.grad.detach()
    alm, g, fw = alm.detach().clone(), g.detach().clone(), fw.detach().clone()

    def chi(a_, g_, f_):
        return float(vis.chi2_and_grad(fld, data, sig, a_, g_, f_, grads=False)[0])

    coords = _coordinates(cfg.n_freq, fld.n_modes, fld.n_ant, np.random.default_rng(20250409))
    say("fd c1: chi2", chi0, "coordinates", len(coords))
    worst = 0.0
    for kind, ix in coords:
        if kind == "a":
            f, c = ix
            gk = float(ga[f, c])
            h = min(1e-4 * chi0 / max(abs(gk), 1e-30), 1e3 * float(alm[f].abs().max()))
            x = float(alm[f, c])
            xp, xm = np.float32(x + h), np.float32(x - h)
            a_p, a_m = alm.clone(), alm.clone()
            a_p[f, c], a_m[f, c] = float(xp), float(xm)
            fd = (chi(a_p, g, fw) - chi(a_m, g, fw)) / (float(xp) - float(xm))
        elif kind == "g":
            f, i, part = ix
            z = complex(gg[f, i])
            gk = z.real if part == 0 else z.imag
            h = min(1e-4 * chi0 / max(abs(gk), 1e-30), 1.0)
            gr = torch.view_as_real(g)
            x = float(gr[f, i, part])
            xp, xm = np.float32(x + h), np.float32(x - h)
            g_p, g_m = g.clone(), g.clone()
            torch.view_as_real(g_p)[f, i, part] = float(xp)
            torch.view_as_real(g_m)[f, i, part] = float(xm)
            fd = (chi(alm, g_p, fw) - chi(alm, g_m, fw)) / (float(xp) - float(xm))
        else:
            gk = float(gf[0])
            x = float(fw[0])
            xp, xm = np.float32(x * 1.001), np.float32(x * 0.999)
            f_p = torch.tensor([float(xp)], dtype=torch.float32, device="cuda")
            f_m = torch.tensor([float(xm)], dtype=torch.float32, device="cuda")
            fd = (chi(alm, g, f_p) - chi(alm, g, f_m)) / (float(xp) - float(xm))
        rel = abs(fd - gk) / abs(gk)
        worst = max(worst, rel)
        if rel > 1e-3:
            say("fd mismatch", kind, ix, "grad", gk, "fd", fd, "rel", rel)
    say("fd c1 worst relative error", worst)
    assert worst <= 1e-3
