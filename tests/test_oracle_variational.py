"""Pins of the two-site variational compression (oracle/bmps.py:
fit_two_site, compress_variational).

Checked on dense state vectors built here (every MPS contracted to its full
vector), not through the oracle's own contractions:
* without truncation the fit returns the exact product (ln Z~ equals the
  successive-SVD value and the row-transfer-matrix value);
* with truncation, the distance ||X^ - psi|| after the sweeps is at most that
  of the successive-SVD start and does not grow from sweep to sweep;
* the converged psi is a stationary point of the distance: its derivative
  along a change of any one site tensor vanishes, and <psi|X^> = ||psi||^2
  (the residual is orthogonal to psi).
"""
import numpy as np
import pytest

from oracle import bmps, ising, exact
from workloads import random_instance


def dense(mps):
    v = np.ones((1, 1))
    for t in mps:
        v = np.einsum('pa,aub->pub', v, t).reshape(-1, t.shape[2])
    return v[:, 0]


def random_mps(rng, Lx, d, chi):
    dims = [1] + [min(chi, d ** min(c, Lx - c)) for c in range(1, Lx)] + [1]
    return [rng.normal(size=(dims[c], d, dims[c + 1])) for c in range(Lx)]


def test_untruncated_fit_is_exact():
    inst = random_instance(6, 5, 0.8, 64, seed=21, field_scale=0.3)
    m = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    a = bmps.build_envs(m, 64)
    b = bmps.build_envs(m, 64, fit_sweeps=2)
    assert b["logZ"] == pytest.approx(a["logZ"], abs=1e-11)
    assert b["logZ"] == pytest.approx(exact.transfer_logZ(inst.Jh, inst.Jv, inst.h, inst.beta), abs=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_fit_distance_beats_svd_and_does_not_grow(seed):
    rng = np.random.default_rng(seed)
    X = random_mps(rng, 7, 2, 8)
    Xh, _ = bmps.qr_sweep(X)
    x = dense(Xh)
    assert np.linalg.norm(x) == pytest.approx(1.0, abs=1e-12)
    D = 2
    phi, lm, _ = bmps.compress(Xh, D)
    phi[0] = phi[0] * np.exp(lm)
    d_prev = np.linalg.norm(x - dense(phi))
    d_svd = d_prev
    for sw in range(1, 5):
        psi = bmps.fit_two_site(Xh, phi, D, sw)
        d = np.linalg.norm(x - dense(psi))
        assert d <= d_prev + 1e-12
        d_prev = d
    assert d_prev < d_svd - 1e-6      # the fit improves on the SVD start here
    # compress_variational: the same fit, normalised, with ell = ln ||psi||
    env, ell, _ = bmps.compress_variational(Xh, D, 4)
    np.testing.assert_allclose(np.exp(ell) * dense(env), dense(psi), atol=1e-12)


def test_converged_fit_is_stationary():
    rng = np.random.default_rng(7)
    X = random_mps(rng, 6, 2, 8)
    Xh, _ = bmps.qr_sweep(X)
    x = dense(Xh)
    D = 2
    phi, lm, _ = bmps.compress(Xh, D)
    phi[0] = phi[0] * np.exp(lm)
    psi = bmps.fit_two_site(Xh, phi, D, 60)
    p = dense(psi)
    assert p @ x == pytest.approx(p @ p, abs=1e-10)
    r = x - p
    for c in range(len(psi)):
        for _ in range(3):
            delta = [t.copy() for t in psi]
            delta[c] = rng.normal(size=psi[c].shape)
            # derivative of ||x - psi||^2 along psi_c -> psi_c + eps delta_c
            assert abs(-2.0 * (r @ dense(delta))) < 1e-8
