"""Hamiltonian Monte Carlo with a diagonal or block-dense mass matrix (oracle).

Sec. 4.2 and App. B: HMC simulates Hamiltonian dynamics of position q
(the parameters) and momentum p in the potential U = -log posterior, with
mass matrix M; the kinetic energy is K = p^T M^-1 p / 2, the position moves
as dq/dt = M^-1 p, and momenta are drawn as p = L_M p0 with p0 ~ N(0, 1).
For a diagonal M these reduce to element-wise operations:
    K = sum p^2 minv / 2,   dq/dt = minv p,   p = p0 / sqrt(minv).
App. B (dense mass matrices): with a Cholesky factor M = L L^T the three
quantities become triangular solves, K = z^T z / 2 with L z = p, the velocity
M^-1 p = L^-T z, and momenta p = L z0 (``BlockMass``: dense blocks on chosen
index ranges, diagonal elsewhere).
One trajectory is L leapfrog steps of size eps,
    p <- p - eps/2 grad U(q);  q <- q + eps minv p;  p <- p - eps/2 grad U(q),
followed by a Metropolis test accepting with probability min(1, exp(H0 - H1)),
H = U + K.

App. B, step-size adaptation: after each trajectory the step size eps is
divided by 1.2 when the trajectory's acceptance probability falls below 0.2,
and otherwise multiplied by 1.2 but never beyond the originally tuned eps0;
it carries over from one trajectory to the next (``adapt_step``,
``run_chain``).

The potential (Sec. 2.3, eq. posterior) is
    U = chi^2 / 2 + sum a^2 / (2 C) + sum |g - 1|^2 / (2 s_g^2 / 2),
a Gaussian prior of variance C(l, nu) on every sky coefficient, a Gaussian
prior of variance s_g^2 / 2 on each real component of every gain, and a flat
prior on the beam width F.

Parameter vector layout (float64 here): [a (n_freq * n_modes, channel-major),
gains (n_freq * n_ant * 2, (Re, Im) interleaved), F].
"""
from __future__ import annotations

import math
from typing import Callable, Tuple

import numpy as np
import scipy.linalg

from . import model, philox


class DiagonalMass:
    """M = diag(1 / minv): velocity minv p, K = sum minv p^2 / 2, p = z / sqrt(minv)."""

    def __init__(self, minv: np.ndarray):
        self.minv = np.asarray(minv, dtype=np.float64)

    def velocity(self, p):
        return self.minv * p

    def kinetic(self, p) -> float:
        return 0.5 * float(np.sum(self.minv * p * p))

    def draw(self, z):
        return z / np.sqrt(self.minv)


class BlockMass(DiagonalMass):
    """Diagonal mass matrix except for dense blocks M_b = L_b L_b^T on index
    ranges [off_b, off_b + n_b) (App. B): with L z = p (forward substitution)
    the kinetic energy is z^T z / 2 and the velocity M^-1 p = L^-T z (backward
    substitution); momenta are drawn as p = L z0, z0 ~ N(0, 1)."""

    def __init__(self, minv: np.ndarray, blocks):
        super().__init__(minv)
        self.blocks = [(int(o), np.asarray(l, dtype=np.float64)) for o, l in blocks]

    def velocity(self, p):
        v = super().velocity(p)
        for o, l in self.blocks:
            n = len(l)
            z = scipy.linalg.solve_triangular(l, p[o:o + n], lower=True)
            v[o:o + n] = scipy.linalg.solve_triangular(l.T, z, lower=False)
        return v

    def kinetic(self, p) -> float:
        mask = np.ones(len(p), dtype=bool)
        k = 0.0
        for o, l in self.blocks:
            n = len(l)
            mask[o:o + n] = False
            z = scipy.linalg.solve_triangular(l, p[o:o + n], lower=True)
            k += 0.5 * float(z @ z)
        return k + 0.5 * float(np.sum(self.minv[mask] * p[mask] * p[mask]))

    def draw(self, z):
        p = super().draw(z)
        for o, l in self.blocks:
            n = len(l)
            p[o:o + n] = l @ z[o:o + n]
        return p


def _as_mass(m):
    return m if isinstance(m, DiagonalMass) else DiagonalMass(m)


def pack(alm: np.ndarray, gains: np.ndarray, fwhm: float) -> np.ndarray:
    g = np.stack([gains.real, gains.imag], axis=-1)
    return np.concatenate([alm.ravel(), g.ravel(), [fwhm]])


def unpack(q: np.ndarray, n_freq: int, n_modes: int, n_ant: int):
    na = n_freq * n_modes
    alm = q[:na].reshape(n_freq, n_modes)
    g = q[na:na + 2 * n_freq * n_ant].reshape(n_freq, n_ant, 2)
    return alm, g[..., 0] + 1j * g[..., 1], float(q[-1])


class Posterior:
    """U(q) and grad U(q) for one field, data and prior."""

    def __init__(self, field: model.Field, data: np.ndarray, sigma_n: float,
                 alm_var: np.ndarray, gain_scatter: float):
        self.field = field
        self.data = data
        self.sigma_n = sigma_n
        self.alm_var = alm_var
        self.gvar = gain_scatter ** 2 / 2.0
        c = field.cfg
        self.shape = (c.n_freq, c.n_modes, field.n_ant)

    def potential_and_grad(self, q: np.ndarray) -> Tuple[float, np.ndarray]:
        alm, gains, fw = unpack(q, *self.shape)
        x2, ga, gg, gf = model.chi2_and_grad(self.field, self.data, self.sigma_n,
                                             alm, gains, fw)
        dg = gains - 1.0
        u = 0.5 * x2 + 0.5 * float(np.sum(alm ** 2 / self.alm_var)) \
            + 0.5 * float(np.sum(dg.real ** 2 + dg.imag ** 2)) / self.gvar
        grad = pack(0.5 * ga + alm / self.alm_var, 0.5 * gg + dg / self.gvar, 0.5 * gf)
        return u, grad


def kinetic(p: np.ndarray, minv) -> float:
    return _as_mass(minv).kinetic(p)


def leapfrog(q: np.ndarray, p: np.ndarray, grad: np.ndarray, eps: float, n_steps: int,
             minv, potential_and_grad: Callable):
    """n_steps leapfrog steps from (q, p) with grad = grad U(q); returns (q, p, U, grad).
    ``minv`` is the inverse-mass diagonal or a mass object (DiagonalMass, BlockMass)."""
    mass = _as_mass(minv)
    q = q.copy()
    p = p.copy()
    u = None
    for _ in range(n_steps):
        p = p - 0.5 * eps * grad
        q = q + eps * mass.velocity(p)
        u, grad = potential_and_grad(q)
        p = p - 0.5 * eps * grad
    return q, p, u, grad


def draw_momentum(minv, seed: int, stream: int, traj: int,
                  normal_index: np.ndarray = None) -> np.ndarray:
    """p = M^(1/2)-factor times z; element j takes normal number normal_index[j]
    (default j) of the (seed, stream, traj) Philox sequence."""
    mass = _as_mass(minv)
    n = len(mass.minv)
    if normal_index is None:
        z = philox.normals(n, seed, stream, traj)
    else:
        z = philox.normals(int(np.max(normal_index)) + 1, seed, stream, traj)[normal_index]
    return mass.draw(z)


def trajectory(q0: np.ndarray, u0: float, grad0: np.ndarray, eps: float, n_steps: int,
               minv, potential_and_grad: Callable, seed: int, stream: int,
               traj: int, normal_index: np.ndarray = None):
    """One HMC transition.  Returns (q, U, grad, accepted, H0, H1)."""
    mass = _as_mass(minv)
    p0 = draw_momentum(mass, seed, stream, traj, normal_index)
    h0 = u0 + mass.kinetic(p0)
    q1, p1, u1, g1 = leapfrog(q0, p0, grad0, eps, n_steps, mass, potential_and_grad)
    h1 = u1 + mass.kinetic(p1)
    u = philox.accept_uniform(seed, stream, traj)
    accepted = math.isfinite(h1) and u < math.exp(min(0.0, h0 - h1))
    if accepted:
        return q1, u1, g1, True, h0, h1
    return q0, u0, grad0, False, h0, h1


def accept_probability(h0: float, h1: float) -> float:
    """min(1, exp(H0 - H1)); 0 for a non-finite energy (a divergence)."""
    if not (math.isfinite(h0) and math.isfinite(h1)):
        return 0.0
    return math.exp(min(0.0, h0 - h1))


def adapt_step(eps: float, eps0: float, accept_prob: float, threshold: float = 0.2,
               factor: float = 1.2) -> float:
    """App. B, step-size adaptation: a trajectory whose acceptance probability is
    below the threshold shrinks the step, eps / 1.2; any other grows it,
    min(eps0, 1.2 eps).  Reading: "below" is strict, so a probability equal to
    the threshold grows the step."""
    if accept_prob < threshold:
        return eps / factor
    return min(eps0, factor * eps)


def run_chain(q0: np.ndarray, eps0: float, n_steps: int, minv, potential_and_grad: Callable,
              seed: int, stream: int, n_traj: int, adapt: bool = True,
              normal_index: np.ndarray = None):
    """n_traj consecutive HMC transitions from q0 (trajectory indices 0 .. n_traj-1 of
    the Philox stream), the step adapted after each one when ``adapt`` (App. B).
    Returns (q, U, grad, records); record k holds the step size trajectory k used,
    its acceptance probability, the accept decision, H0, H1 and the position
    after the transition."""
    mass = _as_mass(minv)
    q = np.asarray(q0, dtype=np.float64)
    u, g = potential_and_grad(q)
    eps = eps0
    recs = []
    for t in range(n_traj):
        q, u, g, acc, h0, h1 = trajectory(q, u, g, eps, n_steps, mass, potential_and_grad,
                                          seed, stream, t, normal_index)
        prob = accept_probability(h0, h1)
        recs.append({"eps": eps, "accept_prob": prob, "accepted": acc, "h0": h0, "h1": h1,
                     "q": q.copy()})
        if adapt:
            eps = adapt_step(eps, eps0, prob)
    return q, u, g, recs


def gain_gauss_newton_blocks(field: model.Field, alm: np.ndarray, gains: np.ndarray,
                             fwhm: float, sigma_n: float) -> np.ndarray:
    """Per-channel Gauss-Newton Hessian of chi^2 / 2 in the real gain components,
    H_f = Re(J_f^H J_f) / sigma_n^2 with J_f the Jacobian of channel f's model
    visibilities with respect to (Re g_k, Im g_k) (App. B: the mass matrix
    approximates the Hessian).  Each visibility is linear in every single real
    gain component, so central differences give J_f exactly up to rounding.
    Returns [n_freq][2 n_ant][2 n_ant] in the (Re, Im)-interleaved order."""
    nf, na = gains.shape
    out = np.empty((nf, 2 * na, 2 * na))
    for f in range(nf):
        cols = []
        for k in range(na):
            for d in (1.0, 1j):
                gp, gm = gains.copy(), gains.copy()
                gp[f, k] += d
                gm[f, k] -= d
                jc = (model.forward(field, alm, gp, fwhm, [f]) - model.forward(field, alm, gm, fwhm, [f])) / 2
                cols.append(jc.reshape(-1))
        j = np.stack(cols, axis=1)
        out[f] = (j.conj().T @ j).real / sigma_n ** 2
    return out


def hutchinson_probe(shape, seed: int, probe: int) -> np.ndarray:
    """Complex probe z[t][nu][bl] with unit-variance real and imaginary parts:
    visibility v (row-major index) takes normals 2v (real) and 2v + 1 (imaginary)
    of the Philox stream (seed, stream 0, traj = probe, purpose 5)."""
    n = int(np.prod(shape))
    x = philox.normals(2 * n, seed, 0, probe, purpose=5)
    return (x[0::2] + 1j * x[1::2]).reshape(shape)


def gauss_newton_diag(field: model.Field, alm: np.ndarray, gains: np.ndarray, fwhm: float,
                      sigma_n: float, n_probes: int, seed: int) -> np.ndarray:
    """Diagonal of the Gauss-Newton Hessian of chi^2 / 2, diag(J^T J) / sigma_n^2,
    with J the Jacobian of the real and imaginary parts of the model visibilities
    (Sec. 4.2 and App. B: the mass matrix approximates the posterior Hessian).
    Sky coefficients and F: the Hutchinson estimate mean_k (J^T z_k)^2, z_k the
    Philox probes of ``hutchinson_probe`` (E[z z^T] = I, so the mean tends to the
    diagonal); J^T z is the adjoint of the model with cotangent z.  Gains: the
    exact diagonal, for either real component of g_i,
        sum over baselines (i, j) and times of |g_j|^2 |V_ij|^2,
    V the visibility without gains.  Returned in the oracle's parameter layout."""
    c = field.cfg
    shape = (c.n_time, c.n_freq, field.n_ant * (field.n_ant - 1) // 2)
    acc = np.zeros(c.n_freq * c.n_modes + 2 * c.n_freq * field.n_ant + 1)
    for k in range(n_probes):
        z = hutchinson_probe(shape, seed, k)
        ga, gg, gf = model.adjoint(field, alm, gains, fwhm, z)
        v = pack(ga, gg, gf)
        acc += v * v
    h = acc / n_probes / sigma_n ** 2
    _, v, _ = model.forward(field, alm, gains, fwhm, return_parts=True)
    v2 = np.sum(np.abs(v) ** 2, axis=0)                         # [nu][bl], summed over times
    g2 = np.abs(gains) ** 2
    hg = np.zeros((c.n_freq, field.n_ant))
    for b, (i, j) in enumerate(field.pairs):
        hg[:, i] += g2[:, j] * v2[:, b]
        hg[:, j] += g2[:, i] * v2[:, b]
    na = c.n_freq * c.n_modes
    h[na:na + 2 * c.n_freq * field.n_ant] = np.repeat(hg.ravel(), 2) / sigma_n ** 2
    return h


def prior_precision_diag(alm_var: np.ndarray, n_ant: int, gain_scatter: float) -> np.ndarray:
    """Diagonal of the prior's contribution to the Hessian of U: 1 / C for every
    sky coefficient, 2 / s_g^2 for every real gain component, 0 for F (flat)."""
    nf = alm_var.shape[0]
    return np.concatenate([1.0 / alm_var.ravel(),
                           np.full(2 * nf * n_ant, 2.0 / gain_scatter ** 2), [0.0]])


def gain_block_mass(minv: np.ndarray, chol: np.ndarray, goff: int) -> BlockMass:
    """BlockMass with dense per-channel gain blocks M_f = chol[f] chol[f]^T placed
    at goff + f * n (n = chol.shape[1]); every other parameter keeps minv."""
    n = chol.shape[1]
    return BlockMass(minv, [(goff + f * n, np.tril(chol[f])) for f in range(chol.shape[0])])
