"""Pins of the periodic-boundary step by frozen lines (oracle/periodic.py).

* The energy of the identified lattice: the partition function by brute force
  equals the closed form (2 cosh K)^N + (2 sinh K)^N of the Ising ring (both
  directions), and the trace of the product of row transfer matrices on a
  torus and a cylinder with random couplings and fields.
* The open model of a cut: with no truncation its ln q of every free
  configuration is the exact conditional log-probability of the periodic
  Boltzmann distribution given the frozen spins (brute force), which fixes the
  frozen-neighbour fields, the coupling map and the site map; its energy
  differs from the periodic energy by a constant.
* The step: started from 20000 exact Boltzmann samples of a 4x4 torus with
  D = 1 (acceptance below 1), three steps with different cuts leave the law of
  the energy Boltzmann (chi-square over 20 bins); the same test with the
  frozen-neighbour fields left out of the open model (a mistake planted in the
  oracle) fails it.  Without truncation every proposal is accepted and the
  frozen lines never move.
* Link overlaps: a configuration against itself counts every bond; one flipped
  site removes twice its degree.
"""
import itertools

import numpy as np
import pytest
from scipy.stats import chi2

from oracle import periodic
from oracle.bmps import build_envs
from oracle.sampler import eval_logq


def all_configs(Ly, Lx):
    return np.array([np.array(c).reshape(Ly, Lx)
                     for c in itertools.product([1, -1], repeat=Ly * Lx)], dtype=np.int8)


def couplings(rng, Ly, Lx, wrap_x, wrap_y, field=0.3):
    Jh = rng.normal(size=(Ly, Lx if wrap_x else Lx - 1))
    Jv = rng.normal(size=(Ly if wrap_y else Ly - 1, Lx))
    h = field * rng.normal(size=(Ly, Lx)) if field else None
    return Jh, Jv, h


def logsumexp(x):
    m = x.max()
    return m + np.log(np.exp(x - m).sum())


@pytest.mark.parametrize("along", ["x", "y"])
def test_ring_partition_function(along):
    N, J, beta = 9, 0.7, 0.9
    K = beta * J
    if along == "x":
        Ly, Lx, wx, wy = 1, N, True, False
        Jh, Jv = np.full((1, N), J), np.zeros((0, N))
    else:
        Ly, Lx, wx, wy = N, 1, False, True
        Jh, Jv = np.zeros((N, 0)), np.full((N, 1), J)
    cf = all_configs(Ly, Lx)
    Z = np.exp(-beta * periodic.energy(cf, Jh, Jv, None, wx, wy)).sum()
    exact = (2 * np.cosh(K)) ** N + (2 * np.sinh(K)) ** N
    assert Z == pytest.approx(exact, rel=1e-12)
    assert periodic.n_bonds(Lx, Ly, wx, wy) == N


def row_transfer_Z(Jh, Jv, h, beta, Ly, Lx, wrap_x, wrap_y):
    """Z as a product of row weights and row-to-row transfer matrices."""
    rows = all_configs(1, Lx)[:, 0, :].astype(np.float64)        # [2^Lx, Lx]
    nxt = np.roll(rows, -1, axis=1)
    M = np.eye(len(rows))
    for r in range(Ly):
        hb = np.zeros(Lx) if h is None else h[r]
        bonds = (Jh[r] * rows * nxt).sum(axis=1) if wrap_x else (Jh[r] * rows[:, :-1] * rows[:, 1:]).sum(axis=1)
        w = np.exp(beta * (bonds + rows @ hb))                   # row r's own weight
        M = M @ np.diag(w)
        if r < Ly - 1 or wrap_y:
            V = np.exp(beta * (rows * Jv[r]) @ rows.T)            # V[a, b] = exp(beta sum_c Jv a_c b_c)
            M = M @ V
    return np.trace(M) if wrap_y else M.sum()


@pytest.mark.parametrize("wrap_y", [True, False], ids=["torus", "cylinder"])
def test_partition_function_by_row_transfer(wrap_y):
    rng = np.random.default_rng(11)
    Ly, Lx, beta = 3, 4, 0.6
    Jh, Jv, h = couplings(rng, Ly, Lx, True, wrap_y)
    cf = all_configs(Ly, Lx)
    Z = np.exp(-beta * periodic.energy(cf, Jh, Jv, h, True, wrap_y)).sum()
    assert Z == pytest.approx(row_transfer_Z(Jh, Jv, h, beta, Ly, Lx, True, wrap_y), rel=1e-12)


CUT_CASES = [  # (Ly, Lx, wrap_x, wrap_y, cut_row, cut_col)
    (4, 4, True, True, 0, 0),
    (4, 4, True, True, 2, 1),
    (4, 4, True, True, 3, 3),
    (3, 5, True, False, 0, 4),
    (5, 3, False, True, 1, 0),
]


@pytest.mark.parametrize("case", range(len(CUT_CASES)))
def test_untruncated_cut_gives_the_exact_conditional(case):
    Ly, Lx, wx, wy, cr, cc = CUT_CASES[case]
    rng = np.random.default_rng(40 + case)
    Jh, Jv, h = couplings(rng, Ly, Lx, wx, wy)
    beta = 0.8
    for _ in range(3):
        s = rng.choice([-1, 1], size=(Ly, Lx)).astype(np.int8)
        model, rows, cols = periodic.cut_model(Jh, Jv, h, beta, s, cr, cc, wx, wy)
        assert (model.Ly, model.Lx) == (len(rows), len(cols))
        envs = build_envs(model, 8)
        free = all_configs(len(rows), len(cols))
        full = np.broadcast_to(s, (len(free), Ly, Lx)).copy()
        full[:, rows[:, None], cols[None, :]] = free
        E = periodic.energy(full, Jh, Jv, h, wx, wy)
        exact = -beta * E - logsumexp(-beta * E)
        ev = eval_logq(model, envs, free)
        np.testing.assert_allclose(ev["logq"], exact, rtol=0, atol=1e-10)
        # open energies differ from the periodic ones by a constant
        d = ev["energy"] - E
        np.testing.assert_allclose(d, d[0], rtol=0, atol=1e-12)


def boltzmann(Jh, Jv, h, beta, Ly, Lx, wx, wy):
    cf = all_configs(Ly, Lx)
    E = periodic.energy(cf, Jh, Jv, h, wx, wy)
    p = np.exp(-beta * (E - E.min()))
    return cf, p / p.sum()


def energy_chi2_pvalue(E, Ecf, p, nbins=20):
    """chi-square of the energies E against the exact law, in bins of about
    equal exact probability."""
    order = np.argsort(Ecf)
    cp = np.cumsum(p[order])
    edges = np.unique([Ecf[order][np.searchsorted(cp, q)] for q in np.arange(1, nbins) / nbins])
    bins = np.concatenate([[-np.inf], edges + 1e-9, [np.inf]])
    binp = np.histogram(Ecf, bins=bins, weights=p)[0]
    counts = np.histogram(E, bins=bins)[0]
    expect = binp * len(E)
    return chi2.sf(((counts - expect) ** 2 / expect).sum(), len(binp) - 1)


def run_stationarity():
    # 4x4 torus (open 3x3 after a cut) at D = 1: 20000 exact Boltzmann samples,
    # three steps with different cuts
    rng = np.random.default_rng(7)
    Ly, Lx, beta, D, N = 4, 4, 1.0, 1, 20000
    Jh, Jv, h = couplings(rng, Ly, Lx, True, True, field=0.4)
    cf, p = boltzmann(Jh, Jv, h, beta, Ly, Lx, True, True)
    Ecf = periodic.energy(cf, Jh, Jv, h, True, True)
    s = cf[rng.choice(len(cf), size=N, p=p)]
    inst = [dict(Jh=Jh, Jv=Jv, h=h, beta=beta, chains=N)]
    rates = []
    for t, (cr, cc) in enumerate([(0, 0), (1, 2), (3, 1)]):
        s, E, acc = periodic.step(inst, s, seed=5, t=t, cut_row=cr, cut_col=cc, D=D, wrap_x=True, wrap_y=True)
        rates.append(acc.mean())
    return energy_chi2_pvalue(E, Ecf, p), rates, s, E, (Jh, Jv, h)


def test_steps_keep_the_periodic_boltzmann_distribution():
    pval, rates, s, E, (Jh, Jv, h) = run_stationarity()
    assert min(rates) < 0.9 and max(rates) < 1.0, rates      # the truncation matters
    assert pval > 1e-4, pval
    np.testing.assert_allclose(E, periodic.energy(s, Jh, Jv, h, True, True), rtol=0, atol=1e-12)


def test_stationarity_test_catches_missing_frozen_fields(monkeypatch):
    real = periodic.cut_model

    def no_frozen_fields(Jh, Jv, h, beta, spins, cut_row, cut_col, wrap_x, wrap_y):
        m, rows, cols = real(Jh, Jv, h, beta, spins, cut_row, cut_col, wrap_x, wrap_y)
        base = np.asarray(h)[np.ix_(rows, cols)]
        return type(m)(m.Jh, m.Jv, base, m.beta), rows, cols

    monkeypatch.setattr(periodic, "cut_model", no_frozen_fields)
    pval, _, _, _, _ = run_stationarity()
    assert pval < 1e-6, pval


@pytest.mark.parametrize("wrap", [(True, True), (True, False), (False, True)], ids=["torus", "cyl_x", "cyl_y"])
def test_untruncated_steps_accept_everything_and_keep_frozen_lines(wrap):
    wx, wy = wrap
    rng = np.random.default_rng(3)
    Ly, Lx = 5, 4
    Jh, Jv, h = couplings(rng, Ly, Lx, wx, wy)
    C = 12
    s0 = rng.choice([-1, 1], size=(C, Ly, Lx)).astype(np.int8)
    inst = [dict(Jh=Jh[:], Jv=Jv, h=h, beta=0.7, chains=5), dict(Jh=-Jh, Jv=Jv, h=None, beta=0.4, chains=7)]
    s, E, acc = periodic.step(inst, s0, seed=1, t=0, cut_row=2, cut_col=1, D=16, wrap_x=wx, wrap_y=wy)
    assert acc.all()
    if wx:
        np.testing.assert_array_equal(s[:, :, 1], s0[:, :, 1])
    if wy:
        np.testing.assert_array_equal(s[:, 2, :], s0[:, 2, :])
    assert (s != s0).any()
    np.testing.assert_allclose(E[:5], periodic.energy(s[:5], Jh, Jv, h, wx, wy), atol=1e-12, rtol=0)
    np.testing.assert_allclose(E[5:], periodic.energy(s[5:], -Jh, Jv, None, wx, wy), atol=1e-12, rtol=0)


@pytest.mark.parametrize("wrap", [(True, True), (True, False)], ids=["torus", "cylinder"])
def test_link_overlap_counts(wrap):
    wx, wy = wrap
    rng = np.random.default_rng(2)
    Ly, Lx = 5, 6
    a = rng.choice([-1, 1], size=(Ly, Lx)).astype(np.int8)
    nb = periodic.n_bonds(Lx, Ly, wx, wy)
    assert periodic.link_overlap(a, a, wx, wy) == nb
    assert periodic.link_overlap(a, -a, wx, wy) == nb
    b = a.copy()
    b[0, 0] = -b[0, 0]          # corner: degree 4 on the torus, 3 on the cylinder
    deg = 4 if wy else 3
    assert periodic.link_overlap(a, b, wx, wy) == nb - 2 * deg
    b = a.copy()
    b[2, 3] = -b[2, 3]
    assert periodic.link_overlap(a, b, wx, wy) == nb - 8


def exact_sweep_matrix(Jh, Jv, h, beta, Ly, Lx, wx, wy):
    """One checkerboard Metropolis sweep on the identified lattice, from the
    rule min(1, exp(-beta dE)) with dE from the periodic energy directly."""
    cf = all_configs(Ly, Lx)
    index = {c.tobytes(): k for k, c in enumerate(cf)}
    n = len(cf)

    def half(P, colour):
        out = np.zeros((n, n))
        for a in range(n):
            for k0 in np.nonzero(P[a])[0]:
                s = cf[k0]
                sites = [(r, c) for r in range(Ly) for c in range(Lx) if (r + c) % 2 == colour]
                e0 = periodic.energy(s, Jh, Jv, h, wx, wy)
                probs = []
                for (r, c) in sites:
                    t = s.copy()
                    t[r, c] = -t[r, c]
                    probs.append(min(1.0, np.exp(-beta * (periodic.energy(t, Jh, Jv, h, wx, wy) - e0))))
                for pattern in itertools.product([0, 1], repeat=len(sites)):
                    t = s.copy()
                    w = P[a, k0]
                    for f, (r, c), p in zip(pattern, sites, probs):
                        w *= p if f else 1.0 - p
                        if f:
                            t[r, c] = -t[r, c]
                    out[a, index[t.tobytes()]] += w
        return out

    return half(half(np.eye(n), 0), 1), cf


def test_periodic_sweep_matrix_and_oracle_frequencies():
    # 2x4 cylinder along x: 256 states, the wrapping bonds in every sweep
    rng = np.random.default_rng(12)
    Ly, Lx, beta = 2, 4, 0.7
    Jh, Jv, h = couplings(rng, Ly, Lx, True, False, field=0.3)
    P, cf = exact_sweep_matrix(Jh, Jv, h, beta, Ly, Lx, True, False)
    _, p = boltzmann(Jh, Jv, h, beta, Ly, Lx, True, False)
    np.testing.assert_allclose(p @ P, p, atol=1e-13)
    index = {c.tobytes(): k for k, c in enumerate(cf)}
    N = 3000
    inst = [dict(Jh=Jh, Jv=Jv, h=h, beta=beta, chains=N)]
    for a in range(0, len(cf), 17):
        out, _ = periodic.sweeps(inst, np.broadcast_to(cf[a], (N, Ly, Lx)), seed=4, step=a, nsweeps=1,
                                 wrap_x=True, wrap_y=False)
        freq = np.bincount([index[o.tobytes()] for o in out], minlength=len(cf)) / N
        sigma = np.sqrt(P[a] * (1.0 - P[a]) / N)
        assert np.all(np.abs(freq - P[a]) <= 5.0 * sigma + 2e-3), a


def test_periodic_sweeps_keep_the_torus_energy_law():
    rng = np.random.default_rng(8)
    Ly, Lx, beta, N = 4, 4, 1.0, 20000
    Jh, Jv, h = couplings(rng, Ly, Lx, True, True, field=0.4)
    cf, p = boltzmann(Jh, Jv, h, beta, Ly, Lx, True, True)
    Ecf = periodic.energy(cf, Jh, Jv, h, True, True)
    s = cf[rng.choice(len(cf), size=N, p=p)]
    out, flips = periodic.sweeps([dict(Jh=Jh, Jv=Jv, h=h, beta=beta, chains=N)], s, seed=6, step=0, nsweeps=2,
                                 wrap_x=True, wrap_y=True)
    assert flips.sum() > 0
    assert energy_chi2_pvalue(periodic.energy(out, Jh, Jv, h, True, True), Ecf, p) > 1e-4
    # the local field against energy differences of single flips
    F = periodic.local_field(s[:50], Jh, Jv, h, True, True)
    E0 = periodic.energy(s[:50], Jh, Jv, h, True, True)
    for (r, c) in [(0, 0), (3, 3), (1, 2)]:
        t = s[:50].copy()
        t[:, r, c] = -t[:, r, c]
        dE = periodic.energy(t, Jh, Jv, h, True, True) - E0
        np.testing.assert_allclose(dE, 2.0 * s[:50, r, c] * F[:, r, c], atol=1e-12)
