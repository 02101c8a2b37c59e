"""Pins of the oracle's array, baseline, grid and direction code."""
import json
import math
import os

import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from oracle import array, rime, sky


def test_hera91_baseline_counts(golden_dir):
    """Sec. 3.1: HERA-91 with 0 < |b| < 60 m gives 1785 physical / 30 unique baselines."""
    g = json.load(open(os.path.join(golden_dir, "hera91_counts.json")))
    ij = w.hex_lattice(g["hex_side"])
    assert len(ij) == g["n_ant"]
    cfg = w.scaled(w.C1, array="hex", array_size=g["hex_side"], spacing_m=g["spacing_m"])
    enu = w.antenna_enu(cfg)
    pairs = array.baseline_pairs(len(ij))
    b = array.baseline_vectors(enu, pairs)
    keep = np.linalg.norm(b, axis=1) < g["bl_max_m"]
    assert int(keep.sum()) == g["physical"]
    ubl, u_of_bl, sign = array.unique_lattice(ij, pairs[keep])
    assert len(ubl) == g["unique"]


@pytest.mark.parametrize("side", [3, 4, 5, 7])
def test_hex_unique_count_closed_form(side):
    """Differences of a side-n hexagon fill a hexagon of radius R = 2(n-1):
    3R(R+1)+1 points; without the origin and modulo sign, 3R(R+1)/2 unique."""
    ij = w.hex_lattice(side)
    pairs = array.baseline_pairs(len(ij))
    ubl, u_of_bl, sign = array.unique_lattice(ij, pairs)
    r = 2 * (side - 1)
    assert len(ubl) == 3 * r * (r + 1) // 2
    # every unique baseline is canonical and the broadcast reproduces each difference
    d = ij[pairs[:, 0]] - ij[pairs[:, 1]]
    np.testing.assert_array_equal(sign[:, None] * ubl[u_of_bl], d)
    assert np.all((ubl[:, 0] > 0) | ((ubl[:, 0] == 0) & (ubl[:, 1] > 0)))


@pytest.mark.parametrize("cfg", [w.C0, w.C1, w.scaled(w.C1, array_size=7)])
def test_unique_lattice_matches_vector_grouping(cfg):
    """Lattice-coordinate dedup agrees with dedup by rounded metre vectors."""
    ij = w.antenna_lattice(cfg)
    enu = w.antenna_enu(cfg)
    pairs = array.baseline_pairs(len(ij))
    ubl, u_of_bl, sign = array.unique_lattice(ij, pairs)
    n, groups = array.unique_by_vector(array.baseline_vectors(enu, pairs))
    assert n == len(ubl)
    for members in groups.values():
        us = {int(u_of_bl[k]) for k, _ in members}
        assert len(us) == 1
        rel = {int(sign[k]) * s for k, s in members}
        assert len(rel) == 1


def test_rhombus16_counts():
    """16-dish 4x4 rhombus: 120 baselines, 24 unique (7x7 differences, 49-1 halved)."""
    ij = w.rhombus_lattice(4)
    pairs = array.baseline_pairs(16)
    ubl, _, _ = array.unique_lattice(ij, pairs)
    assert len(pairs) == 120 and len(ubl) == 24


def test_grid_equal_area():
    """Rings uniform in z have equal area (Archimedes): sum dOmega = 4 pi."""
    for nz, nphi in [(32, 96), (128, 384)]:
        z, alpha, dom = sky.grid(nz, nphi)
        edges = np.linspace(-1.0, 1.0, nz + 1)
        ring_area = 2.0 * math.pi * np.diff(edges)
        np.testing.assert_allclose(ring_area / nphi, dom, rtol=1e-15)
        np.testing.assert_allclose(dom * nz * nphi, 4 * math.pi, rtol=1e-15)
        np.testing.assert_allclose(z, 0.5 * (edges[1:] + edges[:-1]), atol=1e-15)


def test_paper_grid_pixel_count(golden_dir):
    """Sec. 3.2: the 0.5 deg equal-area grid of the observable sky has 153,360 pixels."""
    g = json.load(open(os.path.join(golden_dir, "sky_grid_count.json")))
    cell = math.radians(g["cell_deg"])
    nphi = int(round(2 * math.pi / cell))
    zmax = math.sin(math.radians(90.0 - abs(g["latitude_deg"])))
    nrings = int(math.floor((1.0 + zmax) / cell))
    assert nphi * nrings == g["n_pix"]


def test_directions_unit_and_landmarks():
    lat = math.radians(-30.7)
    rng = np.random.default_rng(1)
    dec = np.arcsin(rng.uniform(-1, 1, 200))
    ra = rng.uniform(0, 2 * math.pi, 200)
    s = rime.enu_directions(dec, ra, np.array([0.0, 1.0, 3.0]), lat)
    np.testing.assert_allclose(np.linalg.norm(s, axis=-1), 1.0, atol=1e-15)
    # a source at dec = latitude transits through the zenith
    z = rime.enu_directions(np.array([lat]), np.array([0.7]), np.array([0.7]), lat)[0, 0]
    np.testing.assert_allclose(z, [0.0, 0.0, 1.0], atol=1e-15)
    # south celestial pole: due south at altitude |lat|
    p = rime.enu_directions(np.array([-math.pi / 2]), np.array([0.0]), np.array([1.3]), lat)[0, 0]
    np.testing.assert_allclose(p, [0.0, -math.cos(lat), math.sin(-lat)], atol=1e-15)
    # a source on the celestial equator rises due east 6 h before transit (H = -pi/2)
    e = rime.enu_directions(np.array([0.0]), np.array([math.pi / 2]), np.array([0.0]), lat)[0, 0]
    np.testing.assert_allclose(e, [1.0, 0.0, 0.0], atol=1e-15)
    # after transit (H > 0) a source is in the west (E < 0)
    west = rime.enu_directions(np.array([lat]), np.array([0.0]), np.array([0.2]), lat)[0, 0]
    assert west[0] < 0


def test_beam_landmarks():
    """Power beam: 1 at zenith, 1/2 at theta = FWHM(nu)/2, 0 at/below the horizon."""
    f = np.array([120e6, 150e6, 180e6])
    fw = math.radians(10.0)
    th = fw * (150e6 / f) / 2.0
    enu = np.zeros((1, 5, 3))
    enu[0, 0] = [0, 0, 1]
    enu[0, 1] = [0, -1.0, 0]
    enu[0, 2] = [0.3, 0, -math.sqrt(1 - 0.09)]
    enu[0, 3] = [math.sin(th[0]), 0, math.cos(th[0])]
    enu[0, 4] = [0, math.sin(th[2]), math.cos(th[2])]
    b = rime.beam(enu, f, fw, 150e6)
    np.testing.assert_allclose(b[0, :, 0], 1.0, rtol=1e-15)
    assert np.all(b[0, :, 1] == 0.0) and np.all(b[0, :, 2] == 0.0)
    assert abs(b[0, 0, 3] - 0.5) < 1e-14 and abs(b[0, 2, 4] - 0.5) < 1e-14


def test_dbeam_dfwhm_finite_difference():
    rng = np.random.default_rng(3)
    v = rng.normal(size=(2, 50, 3))
    v[..., 2] = np.abs(v[..., 2])
    v /= np.linalg.norm(v, axis=-1, keepdims=True)
    f = np.array([121e6, 177e6])
    fw, h = math.radians(10.0), 1e-6
    num = (rime.beam(v, f, fw + h, 150e6) - rime.beam(v, f, fw - h, 150e6)) / (2 * h)
    np.testing.assert_allclose(rime.dbeam_dfwhm(v, f, fw, 150e6), num, rtol=1e-7, atol=1e-12)
