"""GPU map-making (eq. vis_to_map with a diagonal normalisation) against the
FP64 oracle's explicit response matrix."""
import numpy as np
import pytest

from oracle import mapmaking as mm
from oracle import model
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


CASES = [
    ("c0", w.scaled(w.C0, n_freq=3, n_time=4), 0),
    ("c0-separable", w.scaled(w.C0, n_freq=3, n_time=4), 1),
    ("hex61", w.scaled(w.C0, array="hex", array_size=5, n_freq=2, n_time=3, lmax=12,
                       freq_lo_hz=120e6, freq_hi_hz=130e6), 0),
]


@pytest.mark.parametrize("name,cfg,synthesis", CASES, ids=[c[0] for c in CASES])
def test_make_map_matches_oracle(vis, name, cfg, synthesis):
    basis = vis.Basis(cfg.grid_nz, cfg.grid_nphi, cfg.lmax, 1 | vis.STORAGE_SEPARABLE)
    fld = vis.Field.from_config(basis, cfg, vis.VIS_FP32, synthesis)
    d = w.draw(cfg)
    of = model.Field(cfg)
    rng = np.random.default_rng(21)
    y = rng.normal(size=(cfg.n_time, cfg.n_freq, fld.n_bl)) + 1j * rng.normal(size=(cfg.n_time, cfg.n_freq, fld.n_bl))
    ref_map, ref_w = mm.dirty_map(of, y, d.gains, w.fwhm_ref_rad(cfg))
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    m, wt = vis.make_map(fld, torch.tensor(y, dtype=torch.complex64, device="cuda"), g, fw)
    m, wt = m.cpu().numpy(), wt.cpu().numpy()
    e_m = np.linalg.norm(m - ref_map, axis=1) / np.linalg.norm(ref_map, axis=1)
    e_w = np.max(np.abs(wt - ref_w)) / np.max(ref_w)
    # element-wise: max over pixels |error| / rms of the channel's map
    e_x = np.max(np.abs(m - ref_map), axis=1) / np.sqrt(np.mean(ref_map ** 2, axis=1))
    say("map", name, "per-channel rel err", e_m, "element-wise", e_x, "weight", e_w)
    assert np.all(e_m <= 1e-5) and e_w <= 1e-5
    assert np.all(e_x <= 1e-4)
    assert np.all(m[ref_w == 0] == 0.0)
