"""Pins of the link overlap and of the equilibration test Eq. (Delta)
(oracle/stats.py).

The link overlap is checked against its definition bond by bond on small
lattices.  Delta is checked where it must vanish: with exact thermal averages
(brute-force enumeration of 3x3 lattices) averaged over Gaussian couplings,
the disorder average of Delta is zero within its sampling error, while a
dropped beta, a wrong sign or the plain (not squared) correlation miss zero by
many standard errors; and at beta = 0, where <s_i s_j> = 0 and <H> = 0 exactly,
Delta equals |E| beta / |V| = 0.
"""
import numpy as np

from oracle import stats, exact


def test_link_overlap_by_definition():
    rng = np.random.default_rng(3)
    for Ly, Lx in [(1, 5), (4, 1), (3, 4), (5, 5)]:
        a = rng.choice([-1, 1], size=(6, Ly, Lx))
        b = rng.choice([-1, 1], size=(6, Ly, Lx))
        ref = np.zeros(6, dtype=np.int64)
        for k in range(6):
            for r in range(Ly):
                for c in range(Lx):
                    if c + 1 < Lx:
                        ref[k] += a[k, r, c] * a[k, r, c + 1] * b[k, r, c] * b[k, r, c + 1]
                    if r + 1 < Ly:
                        ref[k] += a[k, r, c] * a[k + 0, r + 1, c] * b[k, r, c] * b[k, r + 1, c]
        np.testing.assert_array_equal(stats.link_overlap(a, b), ref)
    # a configuration with itself: every bond counts 1
    assert stats.link_overlap(a[:1], a[:1])[0] == 5 * 4 * 2


def exact_terms(Jh, Jv, beta):
    """<H> and sum_<ij> <s_i s_j>^2 of one instance by enumeration."""
    cfg, E, _, lp = exact.brute_force(Jh, Jv, None, beta)
    p = np.exp(lp)
    s = cfg.astype(np.float64)
    ch = (p[:, None, None] * s[:, :, :-1] * s[:, :, 1:]).sum(axis=0)
    cv = (p[:, None, None] * s[:, :-1, :] * s[:, 1:, :]).sum(axis=0)
    return float((p * E).sum()), float((ch ** 2).sum() + (cv ** 2).sum()), float(
        (ch).sum() + (cv).sum())


def test_delta_vanishes_on_the_gaussian_disorder_average():
    rng = np.random.default_rng(11)
    Ly = Lx = 3
    n_sites, n_bonds = Ly * Lx, Ly * (Lx - 1) + (Ly - 1) * Lx
    beta = 0.9
    d, d_nobeta, d_sign, d_plain = [], [], [], []
    for _ in range(1500):
        Jh = rng.normal(size=(Ly, Lx - 1))
        Jv = rng.normal(size=(Ly - 1, Lx))
        H, q2, q1 = exact_terms(Jh, Jv, beta)
        d.append(stats.delta(H, q2, beta, n_sites, n_bonds))
        d_nobeta.append(stats.delta(H, q2, 1.0, n_sites, n_bonds))
        d_sign.append(-H / n_sites + beta * (n_bonds - q2) / n_sites)
        d_plain.append(stats.delta(H, q1, beta, n_sites, n_bonds))
    for vals, zero in [(d, True), (d_nobeta, False), (d_sign, False), (d_plain, False)]:
        v = np.array(vals)
        m, se = v.mean(), v.std(ddof=1) / np.sqrt(len(v))
        if zero:
            assert abs(m) < 4 * se, (m, se)
        else:
            assert abs(m) > 8 * se, (m, se)


def test_delta_at_infinite_temperature():
    assert stats.delta(0.0, 0.0, 0.0, 9, 12) == 0.0
    rng = np.random.default_rng(2)
    Jh, Jv = rng.normal(size=(3, 2)), rng.normal(size=(2, 3))
    H, q2, _ = exact_terms(Jh, Jv, 0.0)
    assert abs(H) < 1e-12 and abs(q2) < 1e-12
