"""No-U-Turn sampler with multinomial and biased progressive sampling (oracle).

Test infrastructure: only tests, the smoke check and the benchmark's CPU
baseline use this module; the product path never imports it.

Sec. 4.2: the paper samples with HMC-NUTS (Hoffman & Gelman 2014): the
trajectory length follows from the no-U-turn termination criterion, and the
end point of a trajectory is drawn by biased progressive sampling (Betancourt
2017, "A conceptual introduction to Hamiltonian Monte Carlo", App. A).  The
paper prints no algorithm, so this is the published method written out
plainly over a stored trajectory (every state kept; no checkpoint tricks):

* Momentum p0 and H0 = U(q0) + K(p0) as in ``hmc.trajectory``.  Every state
  carries the weight exp(H0 - H).
* Doubling j = 0 .. max_depth-1 picks a direction v = +1 if bit 0 of word 0
  of Philox counter (j, traj, stream, 2) is set, else -1, and grows a new
  subtree of 2^j leapfrog steps of size v eps from the trajectory's end on
  that side.
* A leaf is divergent if its H is not finite or H - H0 > 1000; a divergent
  leaf discards its subtree and ends the trajectory.
* Within a subtree the candidate is drawn multinomially in progressive form:
  leaf n replaces the candidate with probability w_n / (w_0 + ... + w_n),
  using the uniform from Philox counter (s, traj, stream, 3), s = the leaf's
  0-based leapfrog step count within the trajectory.
* No-U-turn criterion (Betancourt's generalised form, with the half-end
  correction): a span of states with end momenta p_a, p_b and momentum sum
  rho turns if (M^-1 p_a).(rho - (p_a + p_b)/2) <= 0 or
  (M^-1 p_b).(rho - (p_a + p_b)/2) <= 0.  After leaf n of a subtree every
  aligned span of m = 2, 4, ... leaves ending at n ((n + 1) divisible by m) is
  checked; a turn discards the subtree and ends the trajectory.
* A completed subtree's candidate becomes the proposal with probability
  min(1, W_subtree / W_trajectory) (biased progressive sampling; uniform from
  Philox counter (j, traj, stream, 4)); the subtree joins the trajectory, and
  the whole trajectory is checked with the criterion; a turn, or reaching
  max_depth doublings, ends it.
* The chain moves to the proposal (there is no separate Metropolis test).
  The adaptation statistic is the mean over all leaves of min(1, exp(H0 - H)).
* App. B's step-size adaptation (``hmc.adapt_step``) takes that mean as the
  trajectory's acceptance probability (``run_chain``).
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Callable, List

import numpy as np

from . import hmc, philox

DIVERGENCE = 1000.0


def _uniform(seed: int, ctr) -> float:
    key = (seed & philox.MASK, (seed >> 32) & philox.MASK)
    return philox.unit_open(philox.philox4x32_10(ctr, key)[0])


def direction(seed: int, stream: int, traj: int, j: int) -> int:
    key = (seed & philox.MASK, (seed >> 32) & philox.MASK)
    return 1 if philox.philox4x32_10((j, traj, stream, 2), key)[0] & 1 else -1


def leaf_uniform(seed: int, stream: int, traj: int, s: int) -> float:
    return _uniform(seed, (s, traj, stream, 3))


def merge_uniform(seed: int, stream: int, traj: int, j: int) -> float:
    return _uniform(seed, (j, traj, stream, 4))


@dataclass
class State:
    q: np.ndarray
    p: np.ndarray
    g: np.ndarray
    u: float
    h: float


def turns(mass, p_a: np.ndarray, p_b: np.ndarray, rho: np.ndarray, margins=None) -> bool:
    adj = rho - 0.5 * (p_a + p_b)
    va, vb = mass.velocity(p_a), mass.velocity(p_b)
    da, db = float(va @ adj), float(vb @ adj)
    if margins is not None:
        na = np.linalg.norm(adj)
        margins.append(abs(da) / max(np.linalg.norm(va) * na, 1e-300))
        margins.append(abs(db) / max(np.linalg.norm(vb) * na, 1e-300))
    return da <= 0.0 or db <= 0.0


@dataclass
class Result:
    q: np.ndarray
    u: float
    g: np.ndarray
    h0: float
    h_prop: float
    moved: bool
    n_steps: int
    depth: int          # doublings attempted (the last one may have been discarded)
    accept_stat: float
    reason: str         # "turn", "subtree-turn", "divergent" or "max-depth"
    # smallest distance of any random or threshold decision from its boundary
    # (leaf and merge draws: |u - p| / p; U-turn checks: |v . adj| / (|v| |adj|);
    # divergence: |H - H0 - 1000| / 1000); a diagnostic for comparisons with
    # lower-precision implementations, not part of the method
    min_margin: float = math.inf


def trajectory(q0: np.ndarray, u0: float, g0: np.ndarray, eps: float, max_depth: int,
               minv, potential_and_grad: Callable, seed: int, stream: int, traj: int,
               normal_index: np.ndarray = None) -> Result:
    mass = hmc._as_mass(minv)
    p0 = hmc.draw_momentum(mass, seed, stream, traj, normal_index)
    h0 = u0 + mass.kinetic(p0)
    traj_states: List[State] = [State(q0, p0, g0, u0, h0)]   # time order
    prop = traj_states[0]
    log_w = 0.0                                               # log sum of weights, exp(H0 - H0) = 1
    n_steps = 0
    acc = []
    reason = "max-depth"
    depth = 0
    margins = []
    for j in range(max_depth):
        depth = j + 1
        v = direction(seed, stream, traj, j)
        start = traj_states[-1] if v > 0 else traj_states[0]
        sub: List[State] = []          # build order
        cand, log_w_sub = None, -math.inf
        ok = True
        cur = start
        for n in range(2 ** j):
            q, p, u, g = hmc.leapfrog(cur.q, cur.p, cur.g, v * eps, 1, mass, potential_and_grad)
            h = u + mass.kinetic(p)
            s = n_steps
            n_steps += 1
            acc.append(min(1.0, math.exp(min(0.0, h0 - h))) if math.isfinite(h) else 0.0)
            cur = State(q, p, g, u, h)
            sub.append(cur)
            if math.isfinite(h):
                margins.append(abs(h - h0 - DIVERGENCE) / DIVERGENCE)
            if not math.isfinite(h) or h - h0 > DIVERGENCE:
                ok, reason = False, "divergent"
                break
            lw = h0 - h
            log_w_sub = np.logaddexp(log_w_sub, lw)
            pl, ul = math.exp(lw - log_w_sub), leaf_uniform(seed, stream, traj, s)
            margins.append(abs(ul - pl) / max(pl, 1e-300))
            if ul < pl:
                cand = cur
            m = 2
            while (n + 1) % m == 0:
                span = sub[n + 1 - m:n + 1]
                rho = np.sum([x.p for x in span], axis=0)
                if turns(mass, span[0].p, span[-1].p, rho, margins):
                    ok, reason = False, "subtree-turn"
                    break
                m *= 2
            if not ok:
                break
        if not ok:
            break
        pm, um = math.exp(min(0.0, log_w_sub - log_w)), merge_uniform(seed, stream, traj, j)
        margins.append(abs(um - pm) / max(pm, 1e-300))
        if um < pm:
            prop = cand
        log_w = np.logaddexp(log_w, log_w_sub)
        traj_states = (traj_states + sub) if v > 0 else (sub[::-1] + traj_states)
        rho = np.sum([x.p for x in traj_states], axis=0)
        if turns(mass, traj_states[0].p, traj_states[-1].p, rho, margins):
            reason = "turn"
            break
    moved = prop.q is not q0
    return Result(prop.q, prop.u, prop.g, h0, prop.h, moved, n_steps, depth,
                  float(np.mean(acc)) if acc else 0.0, reason,
                  min(margins) if margins else math.inf)


def run_chain(q0: np.ndarray, eps0: float, max_depth: int, minv, potential_and_grad: Callable,
              seed: int, stream: int, n_traj: int, adapt: bool = True,
              normal_index: np.ndarray = None):
    """n_traj consecutive NUTS transitions from q0 (trajectory indices 0 .. n_traj-1),
    the step adapted after each one when ``adapt`` (App. B), with the mean over the
    leaves of min(1, exp(H0 - H)) as the acceptance probability.  Returns
    (q, U, grad, records): the step size each trajectory used and its Result."""
    q = np.asarray(q0, dtype=np.float64)
    u, g = potential_and_grad(q)
    eps = eps0
    recs = []
    for t in range(n_traj):
        r = trajectory(q, u, g, eps, max_depth, minv, potential_and_grad, seed, stream, t,
                       normal_index)
        recs.append({"eps": eps, "result": r})
        q, u, g = r.q, r.u, r.g
        if adapt:
            eps = hmc.adapt_step(eps, eps0, r.accept_stat)
    return q, u, g, recs
