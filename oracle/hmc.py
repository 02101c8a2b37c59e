"""Hamiltonian Monte Carlo with a diagonal mass matrix (oracle).

Sec. 4.2 and App. B: HMC simulates Hamiltonian dynamics of position q
(the parameters) and momentum p in the potential U = -log posterior, with
mass matrix M; the kinetic energy is K = p^T M^-1 p / 2, the position moves
as dq/dt = M^-1 p, and momenta are drawn as p = L_M p0 with p0 ~ N(0, 1).
For a diagonal M these reduce to element-wise operations:
    K = sum p^2 minv / 2,   dq/dt = minv p,   p = p0 / sqrt(minv).
One trajectory is L leapfrog steps of size eps,
    p <- p - eps/2 grad U(q);  q <- q + eps minv p;  p <- p - eps/2 grad U(q),
followed by a Metropolis test accepting with probability min(1, exp(H0 - H1)),
H = U + K.

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

from . import model, philox


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


def kinetic(p: np.ndarray, minv: np.ndarray) -> float:
    return 0.5 * float(np.sum(minv * p * p))


def leapfrog(q: np.ndarray, p: np.ndarray, grad: np.ndarray, eps: float, n_steps: int,
             minv: np.ndarray, potential_and_grad: Callable):
    """n_steps leapfrog steps from (q, p) with grad = grad U(q); returns (q, p, U, grad)."""
    q = q.copy()
    p = p.copy()
    u = None
    for _ in range(n_steps):
        p = p - 0.5 * eps * grad
        q = q + eps * minv * p
        u, grad = potential_and_grad(q)
        p = p - 0.5 * eps * grad
    return q, p, u, grad


def draw_momentum(minv: np.ndarray, seed: int, stream: int, traj: int,
                  normal_index: np.ndarray = None) -> np.ndarray:
    """p = z / sqrt(minv); element j takes normal number normal_index[j] (default j)
    of the (seed, stream, traj) Philox sequence."""
    if normal_index is None:
        z = philox.normals(minv.size, seed, stream, traj)
    else:
        z = philox.normals(int(np.max(normal_index)) + 1, seed, stream, traj)[normal_index]
    return z / np.sqrt(minv)


def trajectory(q0: np.ndarray, u0: float, grad0: np.ndarray, eps: float, n_steps: int,
               minv: np.ndarray, potential_and_grad: Callable, seed: int, stream: int,
               traj: int, normal_index: np.ndarray = None):
    """One HMC transition.  Returns (q, U, grad, accepted, H0, H1)."""
    p0 = draw_momentum(minv, seed, stream, traj, normal_index)
    h0 = u0 + kinetic(p0, minv)
    q1, p1, u1, g1 = leapfrog(q0, p0, grad0, eps, n_steps, minv, potential_and_grad)
    h1 = u1 + kinetic(p1, minv)
    u = philox.accept_uniform(seed, stream, traj)
    accepted = math.isfinite(h1) and u < math.exp(min(0.0, h0 - h1))
    if accepted:
        return q1, u1, g1, True, h0, h1
    return q0, u0, grad0, False, h0, h1
