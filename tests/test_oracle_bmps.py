"""Pins of the boundary-MPS contraction (App. A) in the oracle."""
import numpy as np
import pytest

from oracle import bmps, exact, ising
from workloads import random_instance, uniform, fully_frustrated


def model_of(inst):
    return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)


@pytest.mark.parametrize("Ly,Lx,seed", [(4, 4, 11), (3, 5, 12), (5, 3, 13), (2, 6, 14)])
def test_untruncated_equals_brute_force(Ly, Lx, seed):
    inst = random_instance(Ly, Lx, 0.9, 64, seed=seed, field_scale=0.4)
    _, _, lz, _ = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    env = bmps.build_envs(model_of(inst), D=64)
    assert not any(env["trunc"])
    assert env['sign'] > 0
    assert abs(env['logZ'] - lz) < 1e-12 * abs(lz)


def test_untruncated_8x8_equals_transfer_matrix():
    Jh, Jv = uniform(8, 8, 1.0)
    m = ising.Model(Jh, Jv, None, 0.44)
    env = bmps.build_envs(m, 16)
    assert not any(env['trunc'])
    assert abs(env['logZ'] - exact.transfer_logZ(Jh, Jv, None, 0.44)) < 1e-12 * 60


def test_row_weight_beyond_fp64_range():
    # 3 x 128 ferromagnet at beta = 3: one row carries about e^765, past the
    # largest double; untruncated at D = 4, so ln Z~ is the exact value (the
    # transfer matrix runs along the transposed lattice, 3 spins wide)
    Ly, Lx, beta = 3, 128, 3.0
    Jh, Jv = uniform(Ly, Lx, 1.0)
    env = bmps.build_envs(ising.Model(Jh, Jv, None, beta), 4)
    assert not any(env['trunc'])
    lz = exact.transfer_logZ(Jv.T.copy(), Jh.T.copy(), None, beta)
    assert lz > 1800
    assert abs(env['logZ'] - lz) < 1e-12 * lz


def test_truncation_error_shrinks_with_D():
    inst = random_instance(8, 8, 1.0, 1, seed=5)
    lz = exact.transfer_logZ(inst.Jh, inst.Jv, None, inst.beta)
    errs = [abs(bmps.build_envs(model_of(inst), D)['logZ'] - lz) for D in (1, 2, 4, 16)]
    assert errs[0] > errs[2] and errs[1] > errs[2]
    assert errs[3] < 1e-12 * abs(lz)


@pytest.mark.parametrize("D", [1, 2, 8])
def test_beta_zero_gives_n_ln2(D):
    inst = random_instance(5, 6, 0.0, D, seed=2)
    env = bmps.build_envs(model_of(inst), D)
    assert abs(env['logZ'] - 30 * np.log(2)) < 1e-13 * 30


def test_strips_closed_form():
    K = 0.37
    for (Ly, Lx) in [(1, 9), (9, 1)]:
        Jh, Jv = uniform(Ly, Lx, 1.0)
        m = ising.Model(Jh, Jv, None, K)
        env = bmps.build_envs(m, 1)   # bond 1 suffices: a strip is exact at any D
        n = Ly * Lx
        assert abs(env['logZ'] - (np.log(2) + (n - 1) * np.log(2 * np.cosh(K)))) < 1e-13 * n


def test_antiferro_equals_ferro():
    # the sublattice spin flip maps J -> -J on the square lattice (Sec. 3,
    # "Observables"); in the network it is a +-1 gauge on the bond legs, so the
    # truncated contraction agrees too
    for L, D in [(12, 4), (16, 8)]:
        Jh, Jv = uniform(L, L, 1.0)
        f = bmps.build_envs(ising.Model(Jh, Jv, None, 0.4407), D)
        a = bmps.build_envs(ising.Model(-Jh, -Jv, None, 0.4407), D)
        assert abs(f['logZ'] - a['logZ']) < 1e-11 * abs(f['logZ'])


def random_orthogonal(rng, shape):
    th = rng.uniform(0, 2 * np.pi, size=shape)
    refl = rng.choice([-1.0, 1.0], size=shape)
    O = np.empty(shape + (2, 2))
    O[..., 0, 0] = np.cos(th)
    O[..., 0, 1] = -np.sin(th)
    O[..., 1, 0] = refl * np.sin(th)
    O[..., 1, 1] = refl * np.cos(th)
    return O


def test_gauge_invariance_of_logZ():
    inst = random_instance(6, 7, 0.8, 3, seed=9, field_scale=0.2)
    m = model_of(inst)
    ref = bmps.build_envs(m, 3)['logZ']
    rng = np.random.default_rng(1)
    m.set_gauge(random_orthogonal(rng, (6, 6)), random_orthogonal(rng, (5, 7)))
    got = bmps.build_envs(m, 3)['logZ']
    assert abs(got - ref) < 1e-12 * abs(ref)


def test_onsager_limit():
    # ln Z~ / N -> -beta f as L grows; open boundaries add O(1/L) terms, so
    # fit a + b/L + c/L^2 over L = 16, 32, 64
    Ls = np.array([16.0, 32.0, 64.0])
    for K, tol in [(0.3, 1e-6), (0.4407, 1e-3)]:
        y = []
        for L in Ls.astype(int):
            Jh, Jv = uniform(L, L, 1.0)
            y.append(bmps.build_envs(ising.Model(Jh, Jv, None, K), 16)['logZ'] / L ** 2)
        A = np.stack([np.ones(3), 1 / Ls, 1 / Ls ** 2], 1)
        a = np.linalg.solve(A, np.array(y))[0]
        bulk = exact.onsager_minus_beta_f(K)
        assert abs(a - bulk) < tol
        assert abs(y[2] - bulk) < abs(y[1] - bulk) < abs(y[0] - bulk)


def test_envs_are_right_canonical():
    inst = fully_frustrated(6, 1.0, 4)
    env = bmps.build_envs(model_of(inst), 4)
    for k in range(1, 6):
        for c in range(1, 6):
            E = env['env'][k][c]
            a = E.shape[0]
            G = E.reshape(a, -1) @ E.reshape(a, -1).T
            np.testing.assert_allclose(G, np.eye(a), atol=1e-12)
        assert abs(np.linalg.norm(env['env'][k][0]) - 1) < 1e-13
