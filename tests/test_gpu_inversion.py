"""The outer inversion driver on the library against the oracle's driver.

On the inversion test grid (24^3, 36 sources and 36 detectors, 27 RBFs with
five parameters, l = 6 simultaneous sources and detectors, 2 of each
optimized after the SAA phase, a truth whose absorption differs visibly,
here as a 20 mm slab)
both drivers start from the same parameters and samples, with five trial
steps per phase.  The oracle solves directly and uses numpy's SVD and
Alg. 1; the library solves by CG to relres 1e-12.  They must take the same
decisions (truncation counts, acceptances), produce the same misfits,
model reductions, ratios and radii, the same iterates, the same full
Jacobian, the same optimized directions (up to sign) and complementary
samples, and the same solve counts, which follow the paper's accounting."""

import numpy as np
import pytest
import torch

import synthetic
from oracle import estimators as oest
from oracle import inversion as oinv
from oracle import problem as oprob

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dl():
    import paper_1706_05586_amd as m
    return m


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)


def test_driver_matches_oracle_replay(dl, dev):
    # the inversion test grid as a 20 mm slab (coefficients scaled by 20
    # instead of 60): detector readings are then about 3e-5 of the field's
    # size, so CG solves to relres 1e-13 give them to about 1e-9 or better
    # and the two drivers' decisions can be compared closely
    L = 20.0
    wl = synthetic.make_workload(synthetic.get_config("inv_t", mu_out=0.01 * L, mu_in=0.05 * L,
                                                      mus_prime=L))
    cfg = wl.cfg
    prob = oprob.build(wl)
    data = oprob.synthetic_data(prob, wl)
    W0, V0 = oest.sample_matrix(wl.w_signs), oest.sample_matrix(wl.v_signs)
    p0 = oinv.params_of(wl.theta_ref, prob.active)
    # singular values below 1e-2 s_1 are left out of the steps: a term
    # (c_i / s_i) R_i moves by about s_1 / s_i times the relative difference
    # of the two sides' J_s and r
    radius0, max_iter, rcut = 0.5, 5, 1e-2
    ref = oinv.invert(oinv.SampledDOT(prob, wl, data, wl.theta_ref), p0, W0, V0, cfg.q_s, cfg.q_d,
                      wl.y_signs, wl.z_signs, cfg.noise,
                      oinv.TrustRegionOptions(radius0=radius0, max_iter=max_iter, rcut=rcut))

    T = lambda a: torch.tensor(np.asarray(a, dtype=np.float64), device=dev)  # noqa: E731
    grid, pals = dl.Grid.from_config(cfg), dl.Pals.from_config(cfg)
    _, D = dl.pals_field(grid, pals, T(wl.theta_ref), cfg.mus_prime)
    with dl.Operator(grid, D) as op:
        inv = dl.inversion
        sd = inv.SampledDOT(op, pals, T(wl.theta_ref), wl.src_cells, wl.det_cells, T(data),
                            rtol=1e-13)
        out = inv.invert(sd, T(p0), T(W0), T(V0), cfg.q_s, cfg.q_d, T(wl.y_signs), T(wl.z_signs),
                         cfg.noise, inv.TrustRegionOptions(radius0=radius0, max_iter=max_iter,
                                                           rcut=rcut))
        got = {k: (v.cpu().numpy() if isinstance(v, torch.Tensor) else v) for k, v in out.items()}
    for name in ("saa", "opt"):
        a, b = got[name], ref[name]
        say(f"[{name}] it/FE/JE {a.it}/{a.fe}/{a.je} (oracle {b.it}/{b.fe}/{b.je}), "
            f"f {a.f:.10e} vs {b.f:.10e}")
        assert (a.it, a.fe, a.je, a.converged) == (b.it, b.fe, b.je, b.converged)
        assert len(a.history) == len(b.history) > 0
        for k, (ha, hb) in enumerate(zip(a.history, b.history)):
            say(f"  step {k}: t {ha['t']} kappa {ha['kappa']:.6f} ratio {ha['ratio']:.6f} "
                f"accept {ha['accept']} (oracle t {hb['t']} ratio {hb['ratio']:.6f})")
            assert (ha["t"], bool(ha["accept"])) == (hb["t"], bool(hb["accept"]))
            for key in ("kappa", "step_norm", "pred", "f", "f_trial", "radius"):
                print(f"    {key}: rel diff {abs(ha[key] - hb[key]) / max(abs(hb[key]), 1e-300):.1e}",
                      flush=True)
            for key in ("kappa", "step_norm", "pred", "f", "f_trial", "radius"):
                assert ha[key] == pytest.approx(hb[key], rel=1e-6, abs=1e-300), key
            assert ha["ratio"] == pytest.approx(hb["ratio"], rel=1e-5, abs=1e-6)
        pa = a.p.cpu().numpy()
        assert np.linalg.norm(pa - b.p) <= 1e-7 * np.linalg.norm(b.p)
    # the full Jacobian, the optimized directions and the new samples
    eJ = np.linalg.norm(got["J_full"] - ref["J_full"]) / np.linalg.norm(ref["J_full"])
    say(f"[update] full J rel err {eJ:.2e}, HOOI objective {got['hooi_objective']:.6e} "
        f"vs {ref['hooi_objective']:.6e}")
    assert eJ <= 1e-8
    assert got["hooi_objective"] == pytest.approx(ref["hooi_objective"], rel=1e-8)
    for X, Y, q in ((got["W"], ref["W"], cfg.q_s), (got["V"], ref["V"], cfg.q_d)):
        Pa, Pb = X[:, :q] @ X[:, :q].T, Y[:, :q] @ Y[:, :q].T
        assert np.linalg.norm(Pa - Pb) <= 1e-8
        assert np.allclose(X[:, q:], Y[:, q:], rtol=0, atol=1e-8)
    say(f"[counts] solves {got['solves']} (oracle {ref['solves']}), counted {got['counted']}")
    assert got["solves"] == got["counted"] == ref["solves"] == ref["counted"]
