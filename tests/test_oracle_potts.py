"""Pins of the general-d (Potts) oracle, oracle/potts.py, against what the
mathematics fixes: the bond split reproduces W = exp(K delta) and is an SVD
split; two exact partition functions (enumeration, row transfer matrix)
agree with each other and with the untruncated environments; beta = 0; the
d = 2 model is the Ising model at half the coupling; sum_s q(s) = 1 for every
D and q = pi untruncated; sampled frequencies follow q; the MH transition
matrix satisfies detailed balance."""
import numpy as np
import pytest
from scipy import stats as sst

from oracle import bmps, potts, ising, sampler as isampler
from oracle.mh import mh_decide


def rand_couplings(Ly, Lx, seed, d=None, field=0.0, scale=1.0):
    rng = np.random.default_rng(seed)
    Jh = scale * rng.standard_normal((Ly, Lx - 1))
    Jv = scale * rng.standard_normal((Ly - 1, Lx))
    h = None if d is None or field == 0.0 else field * rng.standard_normal((Ly, Lx, d))
    return Jh, Jv, h


@pytest.mark.parametrize("d", [2, 3, 4, 5, 7])
def test_bond_split_reproduces_W_and_is_an_svd_split(d):
    K = np.array([-1.3, -0.2, 0.0, 0.7, 2.5, 6.0])
    P, Q = potts.bond_factors(K, d)
    W = np.exp(K[:, None, None] * np.eye(d)[None])
    np.testing.assert_allclose(np.einsum('ksm,kmt->kst', P, Q), W, rtol=1e-13, atol=1e-13)
    # the columns of P and the rows of Q are orthogonal with norms sqrt|lambda|
    # (an SVD split, App. A), lambda the eigenvalues of W
    lam = np.sort(np.abs(np.linalg.eigvalsh(W)), axis=1)
    PtP = np.einsum('ksm,ksn->kmn', P, P)
    QQt = np.einsum('kms,kns->kmn', Q, Q)
    for k in range(len(K)):
        np.testing.assert_allclose(PtP[k], np.diag(np.diag(PtP[k])), atol=1e-12)
        np.testing.assert_allclose(np.sort(np.diag(PtP[k])), lam[k], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(QQt[k], PtP[k], rtol=1e-12, atol=1e-12)


def test_energy_closed_forms():
    Ly, Lx = 4, 5
    Jh, Jv, _ = rand_couplings(Ly, Lx, 1)
    for d in (2, 3):
        same = np.full((1, Ly, Lx), d - 1, dtype=np.int8)
        assert potts.energy(same, Jh, Jv)[0] == pytest.approx(-(Jh.sum() + Jv.sum()), rel=1e-14)
        checker = ((np.arange(Ly)[:, None] + np.arange(Lx)[None, :]) % 2).astype(np.int8)[None]
        assert potts.energy(checker, Jh, Jv)[0] == 0.0
    h = np.random.default_rng(2).standard_normal((Ly, Lx, 3))
    s = np.random.default_rng(3).integers(0, 3, size=(1, Ly, Lx)).astype(np.int8)
    want = potts.energy(s, Jh, Jv) - sum(h[r, c, s[0, r, c]] for r in range(Ly) for c in range(Lx))
    assert potts.energy(s, Jh, Jv, h)[0] == pytest.approx(want[0], rel=1e-14)


@pytest.mark.parametrize("Ly,Lx,d", [(2, 3, 2), (3, 3, 3), (2, 4, 4), (3, 2, 5)])
def test_transfer_matrix_matches_enumeration(Ly, Lx, d):
    Jh, Jv, h = rand_couplings(Ly, Lx, 10 + d, d, field=0.4)
    _, _, lz, _ = potts.brute_force(Jh, Jv, h, 0.9, d)
    assert abs(potts.transfer_logZ(Jh, Jv, h, 0.9, d) - lz) <= 1e-12 * abs(lz)


@pytest.mark.parametrize("Ly,Lx,d,field", [(3, 5, 3, 0.0), (4, 4, 3, 0.5), (2, 6, 4, 0.3), (5, 3, 2, 0.0)])
def test_untruncated_environments_are_exact(Ly, Lx, d, field):
    Jh, Jv, h = rand_couplings(Ly, Lx, 20 + Ly, d, field=field)
    beta = 0.7
    m = potts.PottsModel(Jh, Jv, h, beta, d)
    lz = bmps.build_envs(m, d ** Lx)['logZ']
    ref = potts.transfer_logZ(Jh, Jv, h, beta, d)
    assert abs(lz - ref) <= 1e-12 * abs(ref)


def test_beta_zero():
    Ly, Lx, d = 5, 4, 3
    Jh, Jv, h = rand_couplings(Ly, Lx, 31, d, field=1.0)
    m = potts.PottsModel(Jh, Jv, h, 0.0, d)
    env = bmps.build_envs(m, 3)
    assert abs(env['logZ'] - Ly * Lx * np.log(d)) <= 1e-12 * Ly * Lx
    out = potts.sample(m, env, 16, seed=5)
    np.testing.assert_allclose(out['logq'], -Ly * Lx * np.log(d), rtol=1e-13)


@pytest.mark.parametrize("D", [2, 4, 64])
def test_d2_is_ising_at_half_coupling(D):
    # exp(K delta(s, s')) = exp(K/2) exp((K/2) s s') with value 0 <-> spin +1:
    # ln Z_Potts = ln Z_Ising(J/2) + beta sum J / 2, the same proposal law
    Ly, Lx = 6, 7
    Jh, Jv, _ = rand_couplings(Ly, Lx, 41)
    beta = 0.9
    mp = potts.PottsModel(Jh, Jv, None, beta, 2)
    mi = ising.Model(Jh / 2, Jv / 2, None, beta)
    ep, ei = bmps.build_envs(mp, D), bmps.build_envs(mi, D)
    shift = beta * (Jh.sum() + Jv.sum()) / 2
    assert abs(ep['logZ'] - (ei['logZ'] + shift)) <= 1e-12 * abs(ep['logZ'])
    a = potts.sample(mp, ep, 64, seed=7, step=3)
    b = isampler.sample(mi, ei, 64, seed=7, step=3)
    ok = (a['min_gap'] >= 1e-9) & (b['min_gap'] >= 1e-9)
    assert ok.sum() >= 56
    np.testing.assert_array_equal(1 - 2 * a['states'][ok].astype(int), b['spins'][ok])
    np.testing.assert_allclose(a['logq'][ok], b['logq'][ok], rtol=1e-12)
    # energies: H_Potts = H_Ising(J/2) - sum J / 2
    np.testing.assert_allclose(a['energy'], ising.energy(1 - 2 * a['states'].astype(int), Jh / 2, Jv / 2)
                               - (Jh.sum() + Jv.sum()) / 2, rtol=1e-13, atol=1e-12)


@pytest.mark.parametrize("D", [1, 2, 9])
def test_q_is_normalised_and_exact_when_untruncated(D):
    Ly, Lx, d = 3, 3, 3
    Jh, Jv, h = rand_couplings(Ly, Lx, 51, d, field=0.3)
    beta = 1.1
    m = potts.PottsModel(Jh, Jv, h, beta, d)
    env = bmps.build_envs(m, D)
    cfg, E, lz, lp = potts.brute_force(Jh, Jv, h, beta, d)
    ev = potts.eval_logq(m, env, cfg)
    assert abs(np.exp(ev['logq']).sum() - 1.0) <= 1e-12
    np.testing.assert_array_equal(ev['energy'], E)
    if D == 9:
        np.testing.assert_allclose(ev['logq'], lp, rtol=0, atol=1e-12)
    else:
        assert np.abs(ev['logq'] - lp).max() > 1e-3   # truncated: q differs from pi


def test_sampled_frequencies_follow_q():
    # 2x2, d = 3, D = 1 (q != pi): chi-square of 2e5 draws against q
    Ly, Lx, d = 2, 2, 3
    Jh, Jv, h = rand_couplings(Ly, Lx, 61, d, field=0.5)
    m = potts.PottsModel(Jh, Jv, h, 1.0, d)
    env = bmps.build_envs(m, 1)
    cfg = potts.all_configs(Ly, Lx, d)
    q = np.exp(potts.eval_logq(m, env, cfg)['logq'])
    n = 200000
    out = potts.sample(m, env, n, seed=2021, step=0)
    code = (out['states'].reshape(n, -1).astype(np.int64) * (d ** np.arange(Ly * Lx))[None, :]).sum(1)
    counts = np.bincount(code, minlength=d ** (Ly * Lx))
    # the sample's own ln q agrees with the evaluation of its configurations
    np.testing.assert_allclose(out['logq'], np.log(q[code]), rtol=1e-12)
    chi2 = ((counts - n * q) ** 2 / (n * q)).sum()
    p = sst.chi2.sf(chi2, len(q) - 1)
    assert p > 1e-3, (chi2, p)


def test_mh_transition_matrix_satisfies_detailed_balance():
    # Algorithm 1 with the prior q: T_ij = q_j min(1, exp(ln alpha)) (i != j)
    Ly, Lx, d = 2, 2, 3
    Jh, Jv, h = rand_couplings(Ly, Lx, 71, d, field=0.5)
    beta = 1.3
    m = potts.PottsModel(Jh, Jv, h, beta, d)
    env = bmps.build_envs(m, 1)
    cfg, E, lz, lp = potts.brute_force(Jh, Jv, h, beta, d)
    lq = potts.eval_logq(m, env, cfg)['logq']
    n = len(lq)
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing='ij')
    # the oracle's acceptance (u = 0 accepts iff ln alpha > -inf; the
    # probability is min(1, exp(ln alpha)))
    _, la = mh_decide(lq[i], E[i], lq[j], E[j], beta, np.zeros((n, n)))
    T = np.exp(lq)[None, :] * np.exp(np.minimum(0.0, la))
    T[np.arange(n), np.arange(n)] = 0.0
    T[np.arange(n), np.arange(n)] = 1.0 - T.sum(1)
    pi = np.exp(lp)
    F = pi[:, None] * T
    np.testing.assert_allclose(F, F.T, rtol=1e-10, atol=1e-15)
    np.testing.assert_allclose(pi @ T, pi, rtol=1e-12, atol=1e-15)


def test_chain_from_uniform_state():
    # a short chain runs, its energies are those of its states, and with
    # untruncated environments every move is accepted (q = pi)
    Ly, Lx, d = 3, 4, 3
    Jh, Jv, h = rand_couplings(Ly, Lx, 81, d, field=0.2)
    m = potts.PottsModel(Jh, Jv, h, 0.8, d)
    env = bmps.build_envs(m, 81)
    st = potts.init_state(m, env, 20)
    for t in range(5):
        acc = potts.mh_step(m, env, st, seed=9, t=t)
        assert acc.all()
        np.testing.assert_allclose(st['energy'], potts.energy(st['states'], Jh, Jv, h), rtol=1e-13)
