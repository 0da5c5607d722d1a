"""Pins of the TNMH chain (Algorithm 1; Eqs. mh-acc, tns-prior, reversibility)
and of the chain statistics (Eqs. cauto, c-auto-int) in the oracle."""
import numpy as np
from scipy.stats import chi2 as chi2_dist

from oracle import bmps, exact, ising, mh, sampler, stats
from workloads import random_instance, uniform


def model_of(inst):
    return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)


def test_untruncated_every_proposal_accepted():
    for (L, D, beta) in [(4, 4, 0.9), (8, 16, 0.44)]:
        Jh, Jv = uniform(L, L, 1.0)
        m = ising.Model(Jh, Jv, None, beta)
        env = bmps.build_envs(m, D)
        state = mh.init_state(m, env, 16)
        for t in range(5):
            acc, _, la = mh.mh_step(m, env, state, 77, t)
            assert np.all(np.abs(la) < 1e-10)
            assert acc.all()


def transition_matrix(m, env):
    cfg = exact.all_configs(m.Ly, m.Lx)
    lq = sampler.eval_logq(m, env, cfg)['logq']
    E = ising.energy(cfg, m.Jh, m.Jv, m.h)
    n = cfg.shape[0]
    # P_acc(w -> w') for every pair, by the rule the chain uses
    la = (lq[:, None] - lq[None, :]) - m.beta * (E[None, :] - E[:, None])
    T = np.exp(lq)[None, :] * np.exp(np.minimum(0.0, la))
    T[np.arange(n), np.arange(n)] = 0.0
    T[np.arange(n), np.arange(n)] = 1.0 - T.sum(1)
    return T, E


def test_detailed_balance_3x3():
    inst = random_instance(3, 3, 1.0, 1, seed=5, field_scale=0.4)
    m = model_of(inst)
    env = bmps.build_envs(m, 1)
    T, _ = transition_matrix(m, env)
    _, _, _, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    pi = np.exp(lp)
    F = pi[:, None] * T
    assert np.abs(F - F.T).max() < 1e-15
    assert np.abs(pi @ T - pi).max() < 1e-14
    assert np.all(T >= -1e-15)


def test_acceptance_rule_matches_transition_matrix_on_draws():
    # the chain's decision for a drawn (state, proposal, u) equals u < T-rule
    inst = random_instance(3, 3, 1.0, 1, seed=6)
    m = model_of(inst)
    env = bmps.build_envs(m, 1)
    state = mh.init_state(m, env, 256)
    before = state['spins'].copy()
    lq0, E0 = state['logq'].copy(), state['energy'].copy()
    acc, prop, la = mh.mh_step(m, env, state, 3, 0)
    u = mh.accept_uniforms(256, 3, 0)
    ratio = np.exp(lq0 - prop['logq']) * np.exp(-m.beta * (prop['energy'] - E0))
    assert np.array_equal(acc, u < np.minimum(1.0, ratio))
    assert np.array_equal(state['spins'][~acc], before[~acc])
    assert np.array_equal(state['spins'][acc], prop['spins'][acc])


def test_chain_histogram_matches_boltzmann():
    inst = random_instance(3, 3, 1.0, 1, seed=7, field_scale=0.3)
    m = model_of(inst)
    env = bmps.build_envs(m, 1)
    chains, steps = 20000, 12
    st, acc, _ = mh.run_chain(m, env, chains, steps, seed=99)
    idx = (((1 - st['spins'].reshape(chains, 9).astype(np.int64)) // 2) << np.arange(9)).sum(1)
    cnt = np.bincount(idx, minlength=512)
    _, _, _, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    p = np.exp(lp)
    keep = p * chains > 5
    stat = ((cnt[keep] - chains * p[keep]) ** 2 / (chains * p[keep])).sum()
    assert 0.2 < acc.mean() < 1.0
    assert chi2_dist.sf(stat, keep.sum() - 1) > 1e-3


def test_tau_int_ar1():
    rng = np.random.default_rng(0)
    rho, steps, chains = 0.6, 4000, 64
    x = np.zeros((steps, chains))
    x[0] = rng.normal(size=chains)
    for t in range(1, steps):
        x[t] = rho * x[t - 1] + np.sqrt(1 - rho ** 2) * rng.normal(size=chains)
    tau, W = stats.tau_int(x)
    assert abs(tau - (1 + rho) / (1 - rho)) < 0.15
    C = stats.autocorr(x)
    assert abs(C[1] - rho) < 0.02 and abs(C[2] - rho ** 2) < 0.02


def test_tau_int_of_exact_sampler_is_one():
    Jh, Jv = uniform(4, 4, 1.0)
    m = ising.Model(Jh, Jv, None, 0.6)
    env = bmps.build_envs(m, 4)
    _, acc, E = mh.run_chain(m, env, 64, 300, seed=5)
    assert acc.all()
    tau, _ = stats.tau_int(E)
    assert abs(tau - 1.0) < 0.15
