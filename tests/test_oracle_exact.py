"""Pins of the exact references and of the energy (Eq. ising)."""
import numpy as np
from scipy.integrate import quad

from oracle import exact, ising
from workloads import random_instance, uniform


def test_energy_closed_forms():
    # all up: every bond contributes -J; checkerboard: every bond +J
    for L in (8, 64):
        Jh, Jv = uniform(L, L, 1.0)
        up = np.ones((1, L, L), dtype=np.int8)
        chk = (1 - 2 * ((np.add.outer(np.arange(L), np.arange(L))) % 2)).astype(np.int8)[None]
        assert ising.energy(up, Jh, Jv)[0] == -2 * L * (L - 1)
        assert ising.energy(chk, Jh, Jv)[0] == 2 * L * (L - 1)
    # a single flipped interior spin of the ferromagnet raises E by 2 * 4 bonds
    Jh, Jv = uniform(5, 5, 1.0)
    s = np.ones((1, 5, 5), dtype=np.int8)
    s[0, 2, 2] = -1
    assert ising.energy(s, Jh, Jv)[0] == -2 * 5 * 4 + 8
    # field term: all up in field h gives -h N
    h = np.full((5, 5), 0.25)
    assert np.isclose(ising.energy(np.ones((1, 5, 5)), Jh, Jv, h)[0], -40 - 0.25 * 25)


def test_energy_integer_for_pm_couplings():
    inst = random_instance(6, 7, 1.0, 4, seed=3, gaussian=False)
    rng = np.random.default_rng(0)
    s = rng.choice([-1, 1], size=(50, 6, 7)).astype(np.int8)
    E = ising.energy(s, inst.Jh, inst.Jv)
    assert np.all(E == np.round(E))


def test_bond_split_reproduces_weight():
    K = np.array([-1.3, -0.2, 0.0, 0.4407, 2.5])
    P, Q = ising.bond_factors(K)
    W = np.einsum('ksm,kmt->kst', P, Q)
    np.testing.assert_allclose(W, ising.bond_weight(K), rtol=1e-14, atol=1e-14)
    # W = [[e^K, e^-K], [e^-K, e^K]]  (App. A, Eq. transfMatrixFerro)
    np.testing.assert_allclose(W[:, 0, 0], np.exp(K), rtol=1e-14)
    np.testing.assert_allclose(W[:, 0, 1], np.exp(-K), rtol=1e-14)


def test_brute_force_vs_transfer_matrix():
    for (Ly, Lx, seed) in [(4, 4, 1), (3, 5, 2), (2, 7, 3), (5, 3, 4), (1, 6, 5), (6, 1, 6)]:
        inst = random_instance(Ly, Lx, 0.8, 4, seed=seed, field_scale=0.3)
        _, _, lz, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
        lt = exact.transfer_logZ(inst.Jh, inst.Jv, inst.h, inst.beta)
        assert abs(lz - lt) < 1e-12 * abs(lz)
        assert abs(np.log(np.exp(lp).sum())) < 1e-12


def test_strip_closed_form():
    # 1 x n chain, uniform J, h = 0:  Z = 2 (2 cosh K)^(n-1)
    n, beta = 9, 0.7
    Jh, Jv = uniform(1, n, 1.3)
    K = beta * 1.3
    lz = exact.transfer_logZ(Jh, Jv, None, beta)
    assert abs(lz - (np.log(2) + (n - 1) * np.log(2 * np.cosh(K)))) < 1e-12


def test_onsager_at_critical_point_and_high_temperature():
    Kc = 0.5 * np.log(1 + np.sqrt(2))
    catalan, _ = quad(lambda x: np.arctan(x) / x, 0, 1, epsabs=1e-15, epsrel=1e-15)
    assert abs(exact.onsager_minus_beta_f(Kc) - (0.5 * np.log(2) + 2 * catalan / np.pi)) < 1e-10
    # high-temperature (polygon) series: ln 2 + 2 ln cosh K + t^4 + 2 t^6
    # + 9/2 t^8 + 12 t^10 + O(t^12), t = tanh K
    K = 0.05
    t = np.tanh(K)
    series = (np.log(2) + 2 * np.log(np.cosh(K)) + t ** 4 + 2 * t ** 6
              + 4.5 * t ** 8 + 12 * t ** 10)
    assert abs(exact.onsager_minus_beta_f(K) - series) < 2e-13
