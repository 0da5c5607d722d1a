"""Pins of the sequential sampler (Sec. 2, Eqs. bayes / pi-approx; App. A
Eq. proba-ratio-apx) in the oracle."""
import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

from oracle import bmps, exact, ising, sampler
from workloads import random_instance, uniform, fully_frustrated
from test_oracle_bmps import random_orthogonal


def model_of(inst):
    return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)


@pytest.mark.parametrize("Ly,Lx", [(3, 3), (4, 4), (3, 4)])
@pytest.mark.parametrize("D", [1, 2, 3, 4])
def test_q_is_normalised(Ly, Lx, D):
    inst = random_instance(Ly, Lx, 1.1, D, seed=Ly * 10 + Lx + D, field_scale=0.5)
    m = model_of(inst)
    env = bmps.build_envs(m, D)
    cfg = exact.all_configs(Ly, Lx)
    lq = sampler.eval_logq(m, env, cfg)['logq']
    assert abs(np.exp(lq).sum() - 1.0) < 1e-12


def test_untruncated_q_equals_boltzmann_4x4():
    inst = random_instance(4, 4, 0.9, 8, seed=21, field_scale=0.3)
    m = model_of(inst)
    env = bmps.build_envs(m, 8)
    cfg, _, _, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    lq = sampler.eval_logq(m, env, cfg)['logq']
    assert np.abs(lq - lp).max() < 1e-12


def test_untruncated_q_equals_boltzmann_8x8_sampled():
    Jh, Jv = uniform(8, 8, 1.0)
    m = ising.Model(Jh, Jv, None, 0.44)
    env = bmps.build_envs(m, 16)
    s = sampler.sample(m, env, 64, seed=210413264, step=3)
    lz = exact.transfer_logZ(Jh, Jv, None, 0.44)
    lp = exact.log_boltzmann(s['spins'], Jh, Jv, None, 0.44, lz)
    assert np.abs(s['logq'] - lp).max() < 1e-11


def test_beta_zero_uniform():
    inst = random_instance(5, 4, 0.0, 2, seed=3)
    m = model_of(inst)
    env = bmps.build_envs(m, 2)
    s = sampler.sample(m, env, 32, seed=5)
    np.testing.assert_allclose(s['logq'], -20 * np.log(2), rtol=0, atol=1e-12)


def test_global_flip_symmetry():
    # h = 0: the global flip is a +-1 gauge on every bond, truncation commutes
    inst = random_instance(8, 8, 1.0, 4, seed=4)
    m = model_of(inst)
    env = bmps.build_envs(m, 4)
    s = sampler.sample(m, env, 32, seed=11)
    back = sampler.eval_logq(m, env, -s['spins'])['logq']
    assert np.abs(back - s['logq']).max() < 1e-10
    # hence the first spin's marginal under q is exactly 1/2
    inst = random_instance(3, 4, 1.0, 1, seed=4)
    m = model_of(inst)
    env = bmps.build_envs(m, 1)
    cfg = exact.all_configs(3, 4)
    q = np.exp(sampler.eval_logq(m, env, cfg)['logq'])
    assert abs(q[cfg[:, 0, 0] == 1].sum() - 0.5) < 1e-13


def test_sample_mode_equals_eval_mode_bitwise():
    inst = random_instance(6, 5, 0.7, 3, seed=8, field_scale=0.2)
    m = model_of(inst)
    env = bmps.build_envs(m, 3)
    s = sampler.sample(m, env, 40, seed=123, step=9, first_id=77)
    ev = sampler.eval_logq(m, env, s['spins'])
    assert np.array_equal(ev['logq'], s['logq'])


def test_batch_composition_does_not_change_a_proposal():
    inst = random_instance(5, 5, 0.7, 2, seed=18)
    m = model_of(inst)
    env = bmps.build_envs(m, 2)
    a = sampler.sample(m, env, 10, seed=5, step=2, first_id=0)
    b = sampler.sample(m, env, 4, seed=5, step=2, first_id=6)
    assert np.array_equal(a['spins'][6:], b['spins'])
    assert np.array_equal(a['logq'][6:], b['logq'])


def test_gauge_invariance_of_logq():
    inst = random_instance(5, 6, 0.9, 2, seed=10, field_scale=0.3)
    m = model_of(inst)
    env = bmps.build_envs(m, 2)
    s = sampler.sample(m, env, 16, seed=1)
    rng = np.random.default_rng(3)
    m2 = model_of(inst)
    m2.set_gauge(random_orthogonal(rng, (5, 5)), random_orthogonal(rng, (4, 6)))
    env2 = bmps.build_envs(m2, 2)
    ev = sampler.eval_logq(m2, env2, s['spins'])
    assert np.abs(ev['logq'] - s['logq']).max() < 1e-11


def test_antiferro_maps_to_ferro():
    L, D = 10, 4
    Jh, Jv = uniform(L, L, 1.0)
    mf = ising.Model(Jh, Jv, None, 0.4407)
    ma = ising.Model(-Jh, -Jv, None, 0.4407)
    ef, ea = bmps.build_envs(mf, D), bmps.build_envs(ma, D)
    s = sampler.sample(ma, ea, 16, seed=2)
    chk = (1 - 2 * (np.add.outer(np.arange(L), np.arange(L)) % 2)).astype(np.int8)
    lf = sampler.eval_logq(mf, ef, s['spins'] * chk)['logq']
    assert np.abs(lf - s['logq']).max() < 1e-9


def row_contraction(m, env, r, above, row):
    """ln of the exact contraction of row r with the fixed row above, the env
    of the rows below, and row r's spins fixed (row given) or summed (None)."""
    F = env['env'][r + 1]
    state = np.ones((1, 1))   # [x (horizontal leg), a (env bond)]
    logscale = 0.0
    for c in range(m.Lx):
        T = m.site_tensor(r, c)                                  # [s,l,u,d,x]
        if above is not None:
            i = (1 - above[c]) // 2
            T = np.einsum('u,sludx->sldx', m.down_leg(r - 1, c)[i], T)
        else:
            T = T[:, :, 0]
        T = T[(1 - row[c]) // 2] if row is not None else T.sum(0)
        state = np.einsum('la,ldx,adb->xb', state, T, F[c])
        sc = np.abs(state).max()
        state /= sc
        logscale += np.log(sc)
    return logscale + np.log(state[0, 0])


def test_two_route_identity():
    # ln q(s) = sum_r [ln num_r - ln den_r]: every row's conditional is the
    # ratio of two exact row contractions against the same stored env
    inst = random_instance(5, 6, 1.0, 2, seed=31, field_scale=0.2)
    m = model_of(inst)
    env = bmps.build_envs(m, 2)
    s = sampler.sample(m, env, 6, seed=9)
    for b in range(6):
        sp = s['spins'][b]
        tot = 0.0
        for r in range(m.Ly):
            above = sp[r - 1] if r > 0 else None
            tot += row_contraction(m, env, r, above, sp[r]) - row_contraction(m, env, r, above, None)
        assert abs(tot - s['logq'][b]) < 1e-11


def test_empirical_frequencies_match_q():
    # 3x3 with D = 1 so that q != pi
    inst = random_instance(3, 3, 1.2, 1, seed=41, field_scale=0.3)
    m = model_of(inst)
    env = bmps.build_envs(m, 1)
    n = 200000
    s = sampler.sample(m, env, n, seed=2021)
    idx = (((1 - s['spins'].reshape(n, 9).astype(np.int64)) // 2) << np.arange(9)).sum(1)
    cnt = np.bincount(idx, minlength=512)
    q = np.exp(sampler.eval_logq(m, env, exact.all_configs(3, 3))['logq'])
    _, _, _, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    assert np.abs(q - np.exp(lp)).sum() > 1e-3          # truly approximate
    keep = q * n > 5
    stat = ((cnt[keep] - n * q[keep]) ** 2 / (n * q[keep])).sum()
    assert chi2_dist.sf(stat, keep.sum() - 1) > 1e-3


def test_negative_weights_are_clamped_and_q_stays_normalised():
    # Gaussian couplings at beta = 3 with D = 3: the truncated env makes some
    # conditional weights negative (App. A remark on positivity)
    inst = random_instance(4, 4, 3.0, 3, seed=17)
    m = model_of(inst)
    env = bmps.build_envs(m, 3)
    cfg = exact.all_configs(4, 4)
    ev = sampler.eval_logq(m, env, cfg)
    assert ev['clamps'].sum() > 0
    q = np.exp(ev['logq'])
    assert abs(q.sum() - 1.0) < 1e-12
    # both weights non-positive: the draw falls back to p+ = 1/2
    inst = random_instance(4, 5, 3.0, 3, seed=16)
    m = model_of(inst)
    env = bmps.build_envs(m, 3)
    s = sampler.sample(m, env, 50, seed=1)
    assert s['both_nonpos'].sum() > 0
    assert np.array_equal(sampler.eval_logq(m, env, s['spins'])['logq'], s['logq'])
