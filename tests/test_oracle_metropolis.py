"""Pins of the single-spin-flip Metropolis sweeps (oracle/metropolis.py).

The one-sweep transition matrix of a 2x2 lattice is built here from the
definition (each site of a colour flips independently with probability
min(1, exp(-beta (E(flipped) - E(current)))), the energies from Eq. (ising) by
direct evaluation, colour r + c even first) and checked to leave the
Boltzmann distribution invariant; the oracle's sweeps, started many times
from every configuration, must reproduce its rows within sampling error.  A
wrong sign, factor or neighbour term in the oracle's local field changes
those probabilities by far more than the tolerance.  Closed cases: beta = 0
flips every spin of every sweep; a deep ferromagnetic ground state never
moves.
"""
import itertools

import numpy as np

from oracle import metropolis, ising
from workloads import random_instance, ferro


def configs(Ly, Lx):
    return np.array([np.array(c).reshape(Ly, Lx)
                     for c in itertools.product([1, -1], repeat=Ly * Lx)], dtype=np.int8)


def exact_sweep_matrix(inst):
    """P[a, b]: probability that one checkerboard sweep takes configuration a
    to b, from the Metropolis rule with energy differences of Eq. (ising)."""
    Ly, Lx = inst.Ly, inst.Lx
    cf = configs(Ly, Lx)
    index = {c.tobytes(): k for k, c in enumerate(cf)}
    n = len(cf)

    def half_step(dist_in, colour):
        out = np.zeros((n, n))
        for a in range(n):
            for k0 in range(n):
                pk = dist_in[a, k0]
                if pk == 0.0:
                    continue
                s = cf[k0]
                sites = [(r, c) for r in range(Ly) for c in range(Lx) if (r + c) % 2 == colour]
                e0 = ising.energy(s, inst.Jh, inst.Jv, inst.h)
                probs = []
                for (r, c) in sites:   # same-colour sites share no bond
                    t = s.copy()
                    t[r, c] = -t[r, c]
                    dE = ising.energy(t, inst.Jh, inst.Jv, inst.h) - e0
                    probs.append(min(1.0, np.exp(-inst.beta * dE)))
                for pattern in itertools.product([0, 1], repeat=len(sites)):
                    t = s.copy()
                    w = pk
                    for f, (r, c), p in zip(pattern, sites, probs):
                        w *= p if f else 1.0 - p
                        if f:
                            t[r, c] = -t[r, c]
                    out[a, index[t.tobytes()]] += w
        return out

    P = half_step(np.eye(n), 0)
    return half_step(P, 1), cf


def test_exact_sweep_matrix_keeps_boltzmann():
    inst = random_instance(2, 2, 0.8, 4, seed=301, field_scale=0.4)
    P, cf = exact_sweep_matrix(inst)
    E = ising.energy(cf, inst.Jh, inst.Jv, inst.h)
    pi = np.exp(-inst.beta * (E - E.min()))
    pi /= pi.sum()
    np.testing.assert_allclose(P.sum(axis=1), 1.0, atol=1e-13)
    np.testing.assert_allclose(pi @ P, pi, atol=1e-13)


def test_oracle_sweep_frequencies_match_the_exact_matrix():
    inst = random_instance(2, 2, 0.8, 4, seed=301, field_scale=0.4)
    P, cf = exact_sweep_matrix(inst)
    model = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    index = {c.tobytes(): k for k, c in enumerate(cf)}
    N = 4000
    for a, start in enumerate(cf):
        spins = np.broadcast_to(start, (N, 2, 2)).copy()
        out, _ = metropolis.sweeps(model, spins, seed=77, step=a, nsweeps=1)
        freq = np.zeros(len(cf))
        for o in out:
            freq[index[o.tobytes()]] += 1.0
        freq /= N
        sigma = np.sqrt(P[a] * (1.0 - P[a]) / N)
        assert np.all(np.abs(freq - P[a]) <= 5.0 * sigma + 2e-3), (a, freq, P[a])


def test_beta_zero_flips_every_spin():
    inst = random_instance(5, 7, 0.0, 4, seed=302, field_scale=0.5)
    model = ising.Model(inst.Jh, inst.Jv, inst.h, 0.0)
    rng = np.random.default_rng(5)
    s0 = rng.choice([-1, 1], size=(6, 5, 7)).astype(np.int8)
    for nsw in (1, 2, 3):
        s, flips = metropolis.sweeps(model, s0, seed=3, step=0, nsweeps=nsw)
        np.testing.assert_array_equal(s, s0 if nsw % 2 == 0 else -s0)
        assert np.all(flips == nsw * 35)


def test_deep_ground_state_does_not_move():
    inst = ferro(6, 50.0, 4, Lx=5)
    model = ising.Model(inst.Jh, inst.Jv, None, inst.beta)
    s0 = np.ones((4, 6, 5), dtype=np.int8)
    s, flips = metropolis.sweeps(model, s0, seed=3, step=1, nsweeps=4)
    np.testing.assert_array_equal(s, s0)
    assert flips.sum() == 0


def test_uniform_counter_layout():
    # words of different sweeps, steps and chains are distinct draws; a site's
    # word is word i % 4 of block i // 4
    u0 = metropolis.sweep_uniforms(3, 13, seed=9, step=4, sweep=0)
    u1 = metropolis.sweep_uniforms(3, 13, seed=9, step=4, sweep=1)
    u2 = metropolis.sweep_uniforms(3, 13, seed=9, step=5, sweep=0)
    assert u0.shape == (3, 13)
    assert len(np.unique(np.concatenate([u0.ravel(), u1.ravel(), u2.ravel()]))) == 3 * 3 * 13
    assert np.all((u0 > 0) & (u0 < 1))
