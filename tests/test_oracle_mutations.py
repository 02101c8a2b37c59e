"""Planted mistakes in the oracle (on the CPU) must each fail one of its pins.

Each case replaces one oracle function by a copy with a plausible error (a
flipped sign, a dropped factor, a conjugated operand) and re-runs the pin
that should catch it.
"""
import math

import numpy as np
import pytest

from oracle import model, rime, sky
from tests import test_oracle_geometry as tg
from tests import test_oracle_harmonics as th
from tests import test_oracle_model as tm


def _vis_wrong_sign(bvec, enu, weight, freqs):
    return np.conj(_orig_vis(bvec, enu, weight, freqs))


_orig_vis = rime.vis_direct


def test_flipped_fringe_sign_is_caught(monkeypatch):
    monkeypatch.setattr(rime, "vis_direct", _vis_wrong_sign)
    with pytest.raises(AssertionError):
        tm.test_fringe_sign_worked_example()


def test_missing_sqrt2_in_ylm_is_caught(monkeypatch):
    orig = sky.real_ylm

    def bad(lmax, z, phi):
        y = orig(lmax, z, phi)
        for l in range(1, lmax + 1):
            y[:, l * l + l + 1:(l + 1) ** 2] /= math.sqrt(2)
        return y

    monkeypatch.setattr(sky, "real_ylm", bad)
    with pytest.raises(AssertionError):
        th.test_orthonormal_gauss_legendre(20, 1e-13)


def test_wrong_north_component_is_caught(monkeypatch):
    orig = rime.enu_directions

    def bad(dec, ra, lst, lat):
        s = orig(dec, ra, lst, lat)
        s[..., 1] *= -1
        return s

    monkeypatch.setattr(rime, "enu_directions", bad)
    with pytest.raises(AssertionError):
        tg.test_directions_unit_and_landmarks()


def test_swapped_gain_conjugation_is_caught(monkeypatch):
    monkeypatch.setattr(model.Field, "gain_products",
                        lambda self, g: np.conj(g[:, self.pairs[:, 0]]) * g[:, self.pairs[:, 1]])
    f = model.Field(tm.w.C0)
    d = tm.w.draw(tm.w.C0)
    with pytest.raises(AssertionError):
        tm.test_point_source_at_zenith_check_a((f, d))


def test_unconjugated_adjoint_is_caught(monkeypatch):
    orig = rime.fringe_adjoint
    monkeypatch.setattr(rime, "fringe_adjoint",
                        lambda b, e, om, fr, mk: orig(b, e, np.conj(om), fr, mk))
    f = model.Field(tm.w.C0)
    d = tm.w.draw(tm.w.C0)
    with pytest.raises(AssertionError):
        tm.test_adjoint_dot_check_e((f, d))


def test_fwhm_used_as_sigma_is_caught(monkeypatch):
    monkeypatch.setattr(rime, "FWHM_TO_SIGMA", 1.0)
    with pytest.raises(AssertionError):
        tg.test_beam_landmarks()


def test_transposed_lattice_basis_is_caught(monkeypatch):
    """Unique baselines built with the two lattice axes swapped break the dedup pin."""
    from oracle import array
    orig = array.unique_lattice

    def bad(ij, pairs):
        ubl, u, s = orig(ij, pairs)
        return ubl[:, ::-1].copy(), u, s

    monkeypatch.setattr(array, "unique_lattice", bad)
    with pytest.raises(AssertionError):
        tg.test_hex_unique_count_closed_form(5)
