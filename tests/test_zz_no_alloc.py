"""GPU test of chi2_filtered_and_grad_noalloc (the entry point that allocates
nothing: its scratch is a static per-GPU device array): its outputs equal
chi2_filtered_and_grad's (which takes a caller work buffer) bit for bit, on two
calls in a row, the second on a smaller field, and a field whose scratch would
exceed the static array is refused."""
import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vis():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_07090_amd import vis as v
    return v


def _case(vis, cfg):
    basis = vis.Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, 1)
    fld = vis.Field.from_config(basis, cfg)
    filt = vis.Filter(w.frequencies(cfg))
    d = w.draw(cfg)
    alm = torch.tensor(d.alm * 1.2, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    m = vis.forward(fld, torch.tensor(d.alm, dtype=torch.float32, device="cuda"), g, fw)
    sig = 0.05 * float(torch.sqrt(torch.mean(m.abs().double() ** 2)))
    data = (m + sig * torch.tensor(d.noise_unit, dtype=torch.complex64, device="cuda")).contiguous()
    return basis, fld, filt, data, sig, alm, g, fw


def test_noalloc_equals_work_buffer_entry_point(vis):
    big = w.scaled(w.C0, n_freq=8, n_time=4)
    small = w.scaled(w.C0, array="hex", array_size=3, n_freq=3, n_time=2, lmax=10,
                     freq_lo_hz=120e6, freq_hi_hz=130e6)
    for name, cfg in (("16 dishes, 8 ch, 4 t", big), ("19 dishes, 3 ch, 2 t (smaller)", small)):
        basis, fld, filt, data, sig, alm, g, fw = _case(vis, cfg)
        say("no-alloc filtered chi2:", name)
        ref = vis.chi2_filtered_and_grad(fld, filt, data, sig, alm, g, fw)
        got = vis.chi2_filtered_and_grad_noalloc(fld, filt, data, sig, alm, g, fw)
        torch.cuda.synchronize()
        say("chi2", float(ref[0]), float(got[0]))
        assert float(got[0]) == float(ref[0])
        for a, b, what in zip(got[1:], ref[1:], ("grad a", "grad g", "grad F")):
            assert torch.equal(a, b), what
        # chi^2 only (no gradient outputs) through the same array
        x2 = vis.chi2_filtered_and_grad_noalloc(fld, filt, data, sig, alm, g, fw, grads=False)[0]
        assert float(x2) == float(ref[0])


def test_noalloc_refuses_fields_beyond_the_static_array(vis):
    """127 dishes x 64 channels x 20 times need 2 x 82 MB of model and residual
    scratch, more than the 128 MiB array: VIS_ENOMEM before any launch."""
    cfg = w.scaled(w.C0, array="hex", array_size=7, n_freq=64, n_time=20, lmax=4,
                   freq_lo_hz=120e6, freq_hi_hz=130e6)
    basis, fld, filt, data, sig, alm, g, fw = _case(vis, cfg)
    with pytest.raises(vis.VisError, match="status -2"):
        vis.chi2_filtered_and_grad_noalloc(fld, filt, data, sig, alm, g, fw)
