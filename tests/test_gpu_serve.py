"""GPU tests of the HMC leapfrog kernels and the continuous-batching server."""
import math

import numpy as np
import pytest

from paper_2504_07090_amd import workload as w
from oracle import hmc as ohmc
from oracle import model
from tests.gpu_common import say

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mods():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2504_07090_amd import serve, vis
    return vis, serve


def _chain_inputs(vis, serve, fld, cfg, d, sigma=None, data=None, scale=1.0):
    lay = serve.Layout(fld)
    alm = torch.tensor(d.alm * scale, dtype=torch.float32, device="cuda")
    g = torch.tensor(d.gains, dtype=torch.complex64, device="cuda")
    fw = torch.tensor([w.fwhm_ref_rad(cfg)], dtype=torch.float32, device="cuda")
    if data is None:
        m = vis.forward(fld, torch.tensor(d.alm, dtype=torch.float32, device="cuda"), g, fw)
        rms = float(torch.sqrt(torch.mean(m.abs().double() ** 2)))
        sigma = cfg.noise_frac * rms / math.sqrt(2)
        data = (m + sigma * math.sqrt(2) * torch.tensor(d.noise_unit, dtype=torch.complex64,
                                                        device="cuda")).contiguous()
    q0 = lay.pack(alm, g, fw)
    h = serve.diag_hessian(fld, alm, g, fw, sigma, n_probes=8)
    # prior precisions on the diagonal as well
    h[:lay.nalm] += 1.0 / torch.tensor(d.alm_var, device="cuda").reshape(-1).double()
    h[lay.goff:lay.goff + lay.ngain] += 2.0 / cfg.gain_scatter ** 2
    minv = (1.0 / h).float().contiguous()
    cvar = torch.tensor(d.alm_var, dtype=torch.float32, device="cuda")
    return lay, data, sigma, q0, minv, cvar


def test_trajectory_matches_oracle(mods):
    """One 5-step trajectory from the same q0, momentum stream and mass matrix:
    the GPU move agrees with the FP64 oracle's to 1e-3 of its length, and the
    accept decision and energies agree."""
    vis, serve = mods
    cfg = w.scaled(w.C0, lmax=4, n_freq=2, n_time=2)
    basis = vis.basis_for(cfg)
    fld = vis.Field.from_config(basis, cfg)
    d = w.draw(cfg)
    of = model.Field(cfg)
    _, sig, data = model.make_data(of, d)
    post = ohmc.Posterior(of, data, sig, d.alm_var, cfg.gain_scatter)
    q_or = ohmc.pack(d.alm, d.gains, w.fwhm_ref_rad(cfg))
    # inverse mass from the oracle's finite-difference Hessian diagonal (an input to both sides)
    _, g0 = post.potential_and_grad(q_or)
    hd = np.empty(q_or.size)
    for i in range(q_or.size):
        h = 1e-6 * max(1.0, abs(q_or[i]))
        qp = q_or.copy()
        qp[i] += h
        hd[i] = (post.potential_and_grad(qp)[1][i] - g0[i]) / h
    minv_or = 1.0 / hd
    eps, nl, seed, stream = 0.15, 5, 11, 3
    lay = serve.Layout(fld)
    nalm, ng = lay.nalm, lay.ngain
    # the server draws normal i for element i of its padded layout
    idx = np.concatenate([np.arange(nalm), lay.goff + np.arange(ng), [lay.length - 1]])
    u0, gr0 = post.potential_and_grad(q_or)
    q1, u1, g1, acc, h0, h1 = ohmc.trajectory(q_or, u0, gr0, eps, nl, minv_or,
                                              post.potential_and_grad, seed, stream, 0,
                                              normal_index=idx)

    def to_lay(v):
        out = np.zeros(lay.length)
        out[:nalm] = v[:nalm]
        out[lay.goff:lay.goff + ng] = v[nalm:nalm + ng]
        out[-1] = v[-1]
        return out

    def from_lay(v):
        return np.concatenate([v[:nalm], v[lay.goff:lay.goff + ng], v[-1:]])

    minv_l = to_lay(minv_or)
    minv_l[nalm:lay.goff] = 1.0
    srv = serve.Server(64 << 20, max_chains=4, max_batch=4)
    cid = srv.admit(fld, torch.tensor(data, dtype=torch.complex64, device="cuda"), sig,
                    torch.tensor(to_lay(q_or), dtype=torch.float32, device="cuda"),
                    torch.tensor(minv_l, dtype=torch.float32, device="cuda"),
                    torch.tensor(d.alm_var, dtype=torch.float32, device="cuda"),
                    cfg.gain_scatter, eps, nl, seed, stream)
    srv.submit(cid, 1)
    res = srv.wait(1)
    qg = from_lay(srv.position(cid, lay.length, "cuda").double().cpu().numpy())
    srv.close()
    r = res[0]
    say("oracle acc", acc, h0, h1, "gpu", r["accepted"], r["h0"], r["h1"])
    assert r["status"] == 0 and r["trajectory"] == 0
    assert abs(r["h0"] - h0) <= 1e-4 * abs(h0) and abs(r["h1"] - h1) <= 1e-4 * abs(h1)
    assert abs((r["h1"] - r["h0"]) - (h1 - h0)) <= 0.05 + 1e-2 * abs(h1 - h0)
    assert bool(r["accepted"]) == bool(acc)
    if acc:
        move = np.linalg.norm(q1 - q_or)
        assert move > 0
        assert np.linalg.norm(qg - q1) <= 1e-3 * move
    else:
        np.testing.assert_allclose(qg, q_or, rtol=1e-6)


# (hex side, channels, times, lmax, precision, synthesis): every evaluation path
# of the library appears in the mix
MIXED = [(3, 4, 3, 10, 1, 0), (4, 3, 5, 14, 1, 1), (3, 6, 2, 20, 2, 0), (5, 2, 4, 8, 3, 0),
         (4, 5, 3, 16, 1, 1)]


def _mixed_fields(vis, basis):
    cfgs = [w.scaled(w.C0, array="hex", array_size=s, n_freq=nf, n_time=nt, lmax=lm,
                     freq_lo_hz=120e6, freq_hi_hz=130e6, seed=3000 + i)
            for i, (s, nf, nt, lm, _, _) in enumerate(MIXED)]
    return cfgs, [vis.Field.from_config(basis, c, prec, syn)
                  for c, (*_, prec, syn) in zip(cfgs, MIXED)]


def _mixed_basis(vis):
    return vis.Basis(32, 96, 20, 1 | 2 | 4 | vis.STORAGE_SEPARABLE)


def test_alone_equals_mix(mods):
    """A chain's trajectories are bitwise identical alone and batched with others."""
    vis, serve = mods
    basis = _mixed_basis(vis)
    cfgs, flds = _mixed_fields(vis, basis)
    inputs = []
    for c, f in zip(cfgs, flds):
        inputs.append(_chain_inputs(vis, serve, f, c, w.draw(c)))

    def run(which):
        srv = serve.Server(256 << 20, max_chains=8, max_batch=8)
        ids = {}
        for k in which:
            lay, data, sig, q0, minv, cvar = inputs[k]
            ids[k] = srv.admit(flds[k], data, sig, q0, minv, cvar, cfgs[k].gain_scatter, 0.2, 4,
                               seed=99, stream_id=k, adapt_step=True)
            srv.submit(ids[k], 3)
        res = srv.wait(3 * len(which))
        pos = {k: srv.position(ids[k], inputs[k][0].length, "cuda") for k in which}
        srv.close()
        per = {k: sorted([r for r in res if r["chain"] == ids[k]], key=lambda r: r["trajectory"])
               for k in which}
        return per, pos

    alone, pos_a = run([0])
    mix, pos_m = run([0, 1, 2, 3, 4])
    assert all(r["status"] == 0 for rs in mix.values() for r in rs)
    for ra, rm in zip(alone[0], mix[0]):
        for key in ("trajectory", "accepted", "h0", "h1", "chi2", "eps"):
            assert ra[key] == rm[key], key
    assert torch.equal(pos_a[0], pos_m[0])


def test_admission_by_footprint_and_release(mods):
    vis, serve = mods
    basis = _mixed_basis(vis)
    cfgs, flds = _mixed_fields(vis, basis)
    fps = [serve.Server.footprint(f) for f in flds[:3]]
    # room for the tick tables, chains 0 and 1, and 256 bytes less than chain 2 needs:
    # chain 2 is refused until chain 1's block (adjacent to the tail) is released
    probe = serve.Server(1 << 20, max_chains=8, max_batch=2)
    tables = (1 << 20) - probe.stats()["arena_free_bytes"]
    probe.close()
    srv = serve.Server(tables + fps[0] + fps[1] + fps[2] - 256, max_chains=8, max_batch=2)
    ins = [_chain_inputs(vis, serve, f, c, w.draw(c)) for c, f in zip(cfgs[:3], flds[:3])]
    ids = []
    for k in range(3):
        lay, data, sig, q0, minv, cvar = ins[k]
        ids.append(srv.admit(flds[k], data, sig, q0, minv, cvar, 0.05, 0.1, 2, seed=1, stream_id=k))
    assert ids[0] is not None and ids[1] is not None and ids[2] is None
    srv.submit(ids[0], 2)
    srv.submit(ids[1], 1)
    srv.release(ids[1])          # released while its work may be in flight
    lay, data, sig, q0, minv, cvar = ins[2]
    third = None
    got = set()   # results that arrive while waiting for room count too
    for _ in range(200):
        third = srv.admit(flds[2], data, sig, q0, minv, cvar, 0.05, 0.1, 2, seed=1, stream_id=2)
        if third is not None:
            break
        got |= {(r["chain"], r["trajectory"]) for r in srv.poll(16, timeout_ms=20)}
    assert third is not None
    srv.submit(third, 1)
    need = {(ids[0], 0), (ids[0], 1), (third, 0)}
    for _ in range(600):
        got |= {(r["chain"], r["trajectory"]) for r in srv.poll(64, timeout_ms=100)}
        if need <= got:
            break
    assert need <= got
    srv.close()


def test_nonfinite_chain_is_isolated(mods):
    vis, serve = mods
    basis = _mixed_basis(vis)
    cfgs, flds = _mixed_fields(vis, basis)
    srv = serve.Server(128 << 20, max_chains=4, max_batch=4)
    good = _chain_inputs(vis, serve, flds[0], cfgs[0], w.draw(cfgs[0]))
    bad = _chain_inputs(vis, serve, flds[1], cfgs[1], w.draw(cfgs[1]))
    qb = bad[3].clone()
    qb[0] = float("nan")
    a = srv.admit(flds[0], good[1], good[2], good[3], good[4], good[5], 0.05, 0.1, 3, 5, 0)
    b = srv.admit(flds[1], bad[1], bad[2], qb, bad[4], bad[5], 0.05, 0.1, 3, 5, 1)
    srv.submit(a, 2)
    srv.submit(b, 2)
    res = srv.wait(3, timeout_s=60)
    ra = [r for r in res if r["chain"] == a]
    rb = [r for r in res if r["chain"] == b]
    assert len(ra) == 2 and all(r["status"] == 0 for r in ra)
    assert len(rb) == 1 and rb[0]["status"] == serve.VIS_ENUMERIC
    with pytest.raises(vis.VisError):
        srv.submit(b, 1)
    srv.close()


def test_latency_stats_recorded(mods):
    vis, serve = mods
    basis = _mixed_basis(vis)
    cfgs, flds = _mixed_fields(vis, basis)
    srv = serve.Server(128 << 20, max_chains=4, max_batch=4)
    ins = _chain_inputs(vis, serve, flds[0], cfgs[0], w.draw(cfgs[0]))
    c = srv.admit(flds[0], *ins[1:], 0.05, 0.1, 3, 5, 0)
    srv.submit(c, 2)
    srv.wait(2)
    st = srv.stats()
    assert st["requests"] == 1 + 2 * 3 and 0 < st["p50_ms"] <= st["p99_ms"] <= st["max_ms"]
    srv.close()
