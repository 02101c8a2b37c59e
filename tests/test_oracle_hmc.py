"""Pins of the oracle's Philox stream and HMC integrator."""
import json
import math
import os

import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from oracle import hmc, model, philox


def test_philox_known_answers(golden_dir):
    g = json.load(open(os.path.join(golden_dir, "philox_kat.json")))
    for v in g["vectors"]:
        out = philox.philox4x32_10([int(x, 16) for x in v["ctr"]], [int(x, 16) for x in v["key"]])
        assert list(out) == [int(x, 16) for x in v["out"]]


def test_box_muller_moments():
    z = philox.normals(20000, seed=7, stream=3, traj=0)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 5 * math.sqrt(2 / z.size)
    z2 = philox.normals(20000, seed=7, stream=3, traj=1)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 / math.sqrt(z.size)


def test_leapfrog_harmonic_oscillator_closed_form():
    """U = k q^2/2, unit mass: one leapfrog step is the matrix
    [[1 - e^2 k/2, e], [-e k (1 - e^2 k/4), 1 - e^2 k/2]]."""
    k, eps = 1.7, 0.3
    pg = lambda q: (0.5 * k * float(q @ q), k * q)
    q0, p0 = np.array([0.4]), np.array([-1.1])
    q1, p1, _, _ = hmc.leapfrog(q0, p0, k * q0, eps, 1, np.ones(1), pg)
    a = 1 - eps * eps * k / 2
    assert abs(q1[0] - (a * q0[0] + eps * p0[0])) < 1e-15
    assert abs(p1[0] - (-eps * k * (1 - eps * eps * k / 4) * q0[0] + a * p0[0])) < 1e-15


def _tiny():
    cfg = w.scaled(w.C0, lmax=2, n_freq=2, n_time=2, grid_nz=16, grid_nphi=48)
    f = model.Field(cfg)
    d = w.draw(cfg)
    _, sig, data = model.make_data(f, d)
    post = hmc.Posterior(f, data, sig, d.alm_var, cfg.gain_scatter)
    q0 = hmc.pack(d.alm, d.gains, w.fwhm_ref_rad(cfg))
    # inverse mass = 1 / diagonal Hessian, by differences of the gradient
    _, g0 = post.potential_and_grad(q0)
    hdiag = np.empty(q0.size)
    for i in range(q0.size):
        h = 1e-6 * max(1.0, abs(q0[i]))
        qp = q0.copy()
        qp[i] += h
        hdiag[i] = (post.potential_and_grad(qp)[1][i] - g0[i]) / h
    return post, q0, 1.0 / hdiag


@pytest.fixture(scope="module")
def tiny_posterior():
    return _tiny()


def test_posterior_gradient_fd(tiny_posterior):
    post, q0, _ = tiny_posterior
    u0, g0 = post.potential_and_grad(q0)
    rng = np.random.default_rng(4)
    for i in rng.choice(q0.size, 6, replace=False):
        h = 1e-6 * max(1.0, abs(q0[i]))
        qp, qm = q0.copy(), q0.copy()
        qp[i] += h
        qm[i] -= h
        fd = (post.potential_and_grad(qp)[0] - post.potential_and_grad(qm)[0]) / (2 * h)
        assert abs(fd - g0[i]) < 1e-5 * max(1.0, abs(g0[i]))


def test_leapfrog_reversible_and_second_order(tiny_posterior):
    post, q0, minv = tiny_posterior
    assert np.all(minv > 0)
    u0, g0 = post.potential_and_grad(q0)
    p0 = hmc.draw_momentum(minv, seed=5, stream=0, traj=0)
    q1, p1, u1, g1 = hmc.leapfrog(q0, p0, g0, 0.1, 10, minv, post.potential_and_grad)
    q2, p2, _, _ = hmc.leapfrog(q1, -p1, g1, 0.1, 10, minv, post.potential_and_grad)
    assert np.max(np.abs(q2 - q0)) < 1e-10 * np.max(np.abs(q0))
    assert np.max(np.abs(-p2 - p0)) < 1e-8 * np.max(np.abs(p0))
    # energy error shrinks as eps^2 at fixed trajectory length
    errs = []
    for eps, n in ((0.1, 5), (0.05, 10)):
        qe, pe, ue, _ = hmc.leapfrog(q0, p0, g0, eps, n, minv, post.potential_and_grad)
        errs.append(abs((ue + hmc.kinetic(pe, minv)) - (u0 + hmc.kinetic(p0, minv))))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_hmc_samples_gaussian():
    """HMC on a 2-D Gaussian reproduces its mean and variances (statistical)."""
    mu = np.array([1.0, -2.0])
    var = np.array([0.5, 2.0])
    pg = lambda q: (0.5 * float(np.sum((q - mu) ** 2 / var)), (q - mu) / var)
    q = np.zeros(2)
    u, g = pg(q)
    xs = []
    for t in range(3000):
        q, u, g, acc, h0, h1 = hmc.trajectory(q, u, g, 0.4, 8, np.ones(2), pg, 9, 0, t)
        if t >= 200:
            xs.append(q.copy())
    xs = np.array(xs)
    assert np.all(np.abs(xs.mean(0) - mu) < 6 * np.sqrt(var / 300))
    assert np.all(np.abs(xs.var(0) / var - 1) < 0.25)


# ---- dense mass matrices via Cholesky factors (App. B) ----

def _spd(n, rng, cond=30.0):
    q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    return (q * np.geomspace(1.0, cond, n)) @ q.T


def _block_mass(rng, n=12, nb=2, off=3):
    total = off + nb * n + 2
    minv = rng.uniform(0.5, 2.0, total)
    ms = [_spd(n, rng) for _ in range(nb)]
    mass = hmc.BlockMass(minv, [(off + b * n, np.linalg.cholesky(m)) for b, m in enumerate(ms)])
    full = np.diag(1.0 / minv)
    for b, m in enumerate(ms):
        s = slice(off + b * n, off + (b + 1) * n)
        full[s, s] = m
    return mass, full


def test_block_mass_kinetic_and_velocity_match_full_solve():
    """K = p^T M^-1 p / 2 and dq/dt = M^-1 p through the triangular solves equal a
    general (LU) solve with the assembled mass matrix."""
    rng = np.random.default_rng(21)
    mass, full = _block_mass(rng)
    for _ in range(3):
        p = rng.normal(size=len(full))
        v = np.linalg.solve(full, p)
        assert np.max(np.abs(mass.velocity(p) - v)) <= 1e-12 * np.max(np.abs(v))
        assert abs(mass.kinetic(p) - 0.5 * p @ v) <= 1e-12 * abs(p @ v)


def test_block_mass_momentum_covariance():
    """Momenta p = L z0 have covariance M (Monte Carlo over trajectories)."""
    rng = np.random.default_rng(22)
    mass, full = _block_mass(rng, n=4, nb=1, off=1)
    ps = np.array([hmc.draw_momentum(mass, seed=3, stream=1, traj=t) for t in range(6000)])
    cov = ps.T @ ps / len(ps)
    scale = np.sqrt(np.outer(np.diag(full), np.diag(full)))
    assert np.max(np.abs(cov - full) / scale) < 0.08


def test_block_mass_with_diagonal_factor_is_diagonal_mass():
    """A diagonal Cholesky factor reproduces the diagonal-mass trajectory."""
    rng = np.random.default_rng(23)
    n = 6
    minv = rng.uniform(0.5, 2.0, n)
    lvals = rng.uniform(0.7, 1.5, 4)
    bm = hmc.BlockMass(minv, [(1, np.diag(lvals))])
    dm = minv.copy()
    dm[1:5] = 1.0 / lvals ** 2
    mu = rng.normal(size=n)
    pg = lambda q: (0.5 * float(np.sum((q - mu) ** 2)), q - mu)
    q0 = np.zeros(n)
    u0, g0 = pg(q0)
    a = hmc.trajectory(q0, u0, g0, 0.3, 6, bm, pg, 5, 2, 1)
    b = hmc.trajectory(q0, u0, g0, 0.3, 6, dm, pg, 5, 2, 1)
    assert a[3] == b[3]
    assert np.max(np.abs(a[0] - b[0])) <= 1e-12
    assert abs(a[4] - b[4]) <= 1e-12 * abs(b[4]) and abs(a[5] - b[5]) <= 1e-12 * abs(b[5])


def _gain_mass(post, q0, minv):
    nf, nm, na = post.shape
    alm, gains, fw = hmc.unpack(q0, nf, nm, na)
    h = hmc.gain_gauss_newton_blocks(post.field, alm, gains, fw, post.sigma_n)
    h += np.eye(2 * na)[None] / post.gvar
    return hmc.gain_block_mass(minv, np.linalg.cholesky(h), nf * nm), h


def test_gain_gauss_newton_blocks_match_gradient_differences(tiny_posterior):
    """The Gauss-Newton gain block equals the gain-gain Hessian of chi^2 / 2 at a
    noise-free point (residual zero), where the two coincide; the Hessian is taken
    by central differences of the oracle gradient."""
    post, q0, _ = tiny_posterior
    nf, nm, na = post.shape
    alm, gains, fw = hmc.unpack(q0, nf, nm, na)
    exact = hmc.Posterior(post.field, model.forward(post.field, alm, gains, fw), post.sigma_n,
                          post.alm_var, 1e6)
    h = hmc.gain_gauss_newton_blocks(post.field, alm, gains, fw, post.sigma_n)
    f = 1
    off = nf * nm + f * 2 * na
    for k in (0, 3, 2 * na - 1):
        hh = 1e-4
        qp, qm = q0.copy(), q0.copy()
        qp[off + k] += hh
        qm[off + k] -= hh
        col = (exact.potential_and_grad(qp)[1] - exact.potential_and_grad(qm)[1]) / (2 * hh)
        ref = col[off:off + 2 * na] - np.eye(2 * na)[k] / exact.gvar
        assert np.max(np.abs(h[f, :, k] - ref)) <= 1e-6 * np.max(np.abs(h[f]))
        # no coupling into the other channel's gains
        other = nf * nm
        assert np.max(np.abs(col[other:other + 2 * na])) <= 1e-6 * np.max(np.abs(h[f]))


def test_dense_mass_leapfrog_reversible_and_second_order(tiny_posterior):
    post, q0, minv = tiny_posterior
    mass, _ = _gain_mass(post, q0, minv)
    u0, g0 = post.potential_and_grad(q0)
    p0 = hmc.draw_momentum(mass, seed=5, stream=0, traj=0)
    q1, p1, u1, g1 = hmc.leapfrog(q0, p0, g0, 0.1, 10, mass, post.potential_and_grad)
    q2, p2, _, _ = hmc.leapfrog(q1, -p1, g1, 0.1, 10, mass, post.potential_and_grad)
    assert np.max(np.abs(q2 - q0)) < 1e-10 * np.max(np.abs(q0))
    assert np.max(np.abs(-p2 - p0)) < 1e-8 * np.max(np.abs(p0))
    errs = []
    for eps, n in ((0.05, 10), (0.025, 20)):
        qe, pe, ue, _ = hmc.leapfrog(q0, p0, g0, eps, n, mass, post.potential_and_grad)
        errs.append(abs((ue + mass.kinetic(pe)) - (u0 + mass.kinetic(p0))))
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_dense_mass_samples_correlated_gaussian():
    """With M equal to the precision of a strongly correlated 2-D Gaussian, HMC
    reproduces its mean and covariance (statistical)."""
    mu = np.array([0.5, -1.0])
    cov = np.array([[1.0, 0.95], [0.95, 1.0]])
    prec = np.linalg.inv(cov)
    pg = lambda q: (0.5 * float((q - mu) @ prec @ (q - mu)), prec @ (q - mu))
    mass = hmc.BlockMass(np.ones(2), [(0, np.linalg.cholesky(prec))])
    q = np.zeros(2)
    u, g = pg(q)
    xs = []
    for t in range(3000):
        q, u, g, acc, h0, h1 = hmc.trajectory(q, u, g, 0.5, 4, mass, pg, 13, 0, t)
        if t >= 100:
            xs.append(q.copy())
    xs = np.array(xs)
    c = np.cov(xs.T)
    assert np.all(np.abs(xs.mean(0) - mu) < 0.1)
    assert np.max(np.abs(c - cov)) < 0.12


def test_planted_forward_only_velocity_is_caught(monkeypatch):
    """Dropping the backward substitution (velocity L^-1 p) breaks the solve pin."""
    def vel(self, p):
        v = hmc.DiagonalMass.velocity(self, p)
        for o, l in self.blocks:
            v[o:o + len(l)] = np.linalg.solve(l, p[o:o + len(l)])
        return v
    monkeypatch.setattr(hmc.BlockMass, "velocity", vel)
    with pytest.raises(AssertionError):
        test_block_mass_kinetic_and_velocity_match_full_solve()


def test_planted_transposed_draw_is_caught(monkeypatch):
    """Drawing p = L^T z0 instead of L z0 breaks the covariance pin."""
    def draw(self, z):
        p = hmc.DiagonalMass.draw(self, z)
        for o, l in self.blocks:
            p[o:o + len(l)] = l.T @ z[o:o + len(l)]
        return p
    monkeypatch.setattr(hmc.BlockMass, "draw", draw)
    with pytest.raises(AssertionError):
        test_block_mass_momentum_covariance()


# ---- step-size adaptation (App. B) ----

def test_adapt_step_scripted_sequence():
    """App. B: below 0.2 acceptance the step shrinks to eps / 1.2; otherwise it
    grows to 1.2 eps but never past the originally tuned eps0.  A scripted
    sequence of acceptance probabilities gives these steps, written out by hand
    from the rule with eps0 = 1."""
    probs = [0.05, 0.1, 0.5, 0.7, 0.9, 0.19, 0.2, 0.0]
    expect = [1 / 1.2, 1 / 1.44, 1 / 1.2, 1.0, 1.0, 1 / 1.2, 1.0, 1 / 1.2]
    eps, got = 1.0, []
    for a in probs:
        eps = hmc.adapt_step(eps, 1.0, a)
        got.append(eps)
    assert np.max(np.abs(np.array(got) - np.array(expect))) <= 1e-15


def test_run_chain_matches_oscillator_closed_form():
    """Adapted HMC on a 40-dimensional unit oscillator U = |q|^2 / 2 with unit
    mass: every trajectory of n leapfrog steps is the n-th power of the 2 x 2
    leapfrog matrix [[1 - e^2/2, e], [-e (1 - e^2/4), 1 - e^2/2]] applied to
    each (q_i, p_i); the acceptance probability, Metropolis decision and next
    step follow from the closed form.  The run shrinks the step twice, grows it
    and reaches the eps0 cap, so both branches of the rule are exercised."""
    d, eps0, n, seed, stream = 40, 1.4, 3, 3, 1
    pg = lambda q: (0.5 * float(q @ q), q.copy())
    q0 = np.linspace(-1.0, 1.0, d)
    _, _, _, recs = hmc.run_chain(q0, eps0, n, np.ones(d), pg, seed, stream, 8)
    q, eps = q0.copy(), eps0
    shrunk = grown = 0
    for t, r in enumerate(recs):
        p = philox.normals(d, seed, stream, t)
        m = np.array([[1 - eps ** 2 / 2, eps], [-eps * (1 - eps ** 2 / 4), 1 - eps ** 2 / 2]])
        mn = np.linalg.matrix_power(m, n)
        q1 = mn[0, 0] * q + mn[0, 1] * p
        p1 = mn[1, 0] * q + mn[1, 1] * p
        h0 = 0.5 * (q @ q + p @ p)
        h1 = 0.5 * (q1 @ q1 + p1 @ p1)
        prob = min(1.0, math.exp(h0 - h1))
        acc = philox.accept_uniform(seed, stream, t) < prob
        assert r["eps"] == pytest.approx(eps, rel=1e-14)
        assert r["h0"] == pytest.approx(h0, rel=1e-12) and r["h1"] == pytest.approx(h1, rel=1e-12)
        assert r["accept_prob"] == pytest.approx(prob, rel=1e-10, abs=1e-300)
        assert r["accepted"] == acc
        if acc:
            q = q1
        if prob < 0.2:
            eps, shrunk = eps / 1.2, shrunk + 1
        else:
            eps, grown = min(eps0, 1.2 * eps), grown + 1
    assert shrunk >= 2 and grown >= 2
    assert any(r["eps"] < eps0 / 1.3 for r in recs)


def test_nuts_run_chain_chains_states_and_adapts():
    """NUTS with adaptation: each trajectory starts where the previous one ended,
    and its step is the App. B update of the previous step with the previous
    trajectory's mean leaf acceptance as the acceptance probability."""
    from oracle import nuts
    d = 10
    pg = lambda q: (0.5 * float(q @ q), q.copy())
    q0 = np.linspace(-1.0, 1.0, d)
    eps0 = 1.6
    _, _, _, recs = nuts.run_chain(q0, eps0, 4, np.ones(d), pg, 7, 2, 6)
    q, eps = q0, eps0
    branches = set()
    for t, rec in enumerate(recs):
        u, g = pg(q)
        ref = nuts.trajectory(q, u, g, eps, 4, np.ones(d), pg, 7, 2, t)
        assert rec["eps"] == eps
        assert rec["result"].accept_stat == ref.accept_stat and np.array_equal(rec["result"].q, ref.q)
        branches.add(ref.accept_stat < 0.2)
        eps = eps / 1.2 if ref.accept_stat < 0.2 else min(eps0, 1.2 * eps)
        q = ref.q
    assert branches == {True, False}


def test_planted_grow_on_reject_is_caught(monkeypatch):
    """Multiplying by 1.2 after a poor trajectory (and dividing after a good one)
    breaks the scripted-sequence pin; so does dropping the eps0 cap."""
    monkeypatch.setattr(hmc, "adapt_step",
                        lambda eps, eps0, a, threshold=0.2, factor=1.2:
                        min(eps0, eps * factor) if a < threshold else eps / factor)
    with pytest.raises(AssertionError):
        test_adapt_step_scripted_sequence()
    monkeypatch.setattr(hmc, "adapt_step",
                        lambda eps, eps0, a, threshold=0.2, factor=1.2:
                        eps / factor if a < threshold else factor * eps)
    with pytest.raises(AssertionError):
        test_adapt_step_scripted_sequence()


# ---- diagonal mass matrix: Gauss-Newton diagonal (Sec. 4.2, App. B) ----

def _exact_jtj_diag(post, q0):
    """diag(J^T J) from the explicit Jacobian: the model is linear in every sky
    coefficient (column = model of a unit coefficient, gains and F fixed) and F
    takes a central difference (O(h^2) error)."""
    f = post.field
    nf, nm, na = post.shape
    alm, gains, fw = hmc.unpack(q0, nf, nm, na)
    out = np.empty(nf * nm + 1)
    for k in range(nf * nm):
        e = np.zeros(nf * nm)
        e[k] = 1.0
        col = model.forward(f, e.reshape(nf, nm), gains, fw)
        out[k] = np.sum(np.abs(col) ** 2)
    h = 1e-5 * fw
    col = (model.forward(f, alm, gains, fw + h) - model.forward(f, alm, gains, fw - h)) / (2 * h)
    out[-1] = np.sum(np.abs(col) ** 2)
    return out


def test_gauss_newton_diag_gains_equal_dense_block_diagonal(tiny_posterior):
    """The closed-form gain entries equal the diagonals of the Gauss-Newton gain
    blocks, whose Jacobian comes from central differences of the forward model."""
    post, q0, _ = tiny_posterior
    nf, nm, na = post.shape
    alm, gains, fw = hmc.unpack(q0, nf, nm, na)
    h = hmc.gauss_newton_diag(post.field, alm, gains, fw, post.sigma_n, 1, seed=3)
    blocks = hmc.gain_gauss_newton_blocks(post.field, alm, gains, fw, post.sigma_n)
    ref = np.concatenate([np.diag(b) for b in blocks])
    got = h[nf * nm:nf * nm + 2 * nf * na]
    assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(ref)


def test_gauss_newton_diag_hutchinson_converges(tiny_posterior):
    """With K Gaussian probes each sky / F entry is the mean of K draws of
    (J^T z)^2 ~ (J^T J)_kk chi^2_1, so it lies within a few sqrt(2 / K) of the
    exact diagonal; the mean ratio over the 19 entries is tighter."""
    post, q0, _ = tiny_posterior
    nf, nm, na = post.shape
    alm, gains, fw = hmc.unpack(q0, nf, nm, na)
    k = 400
    h = hmc.gauss_newton_diag(post.field, alm, gains, fw, post.sigma_n, k, seed=11)
    est = np.concatenate([h[:nf * nm], h[-1:]]) * post.sigma_n ** 2
    ratio = est / _exact_jtj_diag(post, q0)
    sd = math.sqrt(2.0 / k)
    assert np.max(np.abs(ratio - 1)) < 5 * sd
    assert abs(np.mean(ratio) - 1) < 2.5 * sd


def test_planted_real_only_probe_is_caught(monkeypatch):
    """Probes without an imaginary part see only half of J^T J: the Hutchinson pin fails."""
    orig = hmc.hutchinson_probe
    monkeypatch.setattr(hmc, "hutchinson_probe",
                        lambda shape, seed, probe: orig(shape, seed, probe).real + 0j)
    with pytest.raises(AssertionError):
        test_gauss_newton_diag_hutchinson_converges(_tiny())


def test_prior_precision_diag():
    var = np.array([[2.0, 4.0], [0.5, 1.0]])
    p = hmc.prior_precision_diag(var, 3, 0.05)
    assert np.allclose(p[:4], [0.5, 0.25, 2.0, 1.0])
    assert np.allclose(p[4:16], 2.0 / 0.05 ** 2) and p[-1] == 0.0 and p.size == 17
