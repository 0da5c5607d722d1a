"""Pins of the frozen-truncation derivative of ln Z~ in the oracle."""
import numpy as np
import pytest

from oracle import bmps, exact, grad, ising
from workloads import random_instance, fully_frustrated, uniform


def model_of(inst):
    return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)


def brute_derivatives(inst):
    cfg, E, lz, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    p = np.exp(lp)
    s = cfg.astype(float)
    b = inst.beta
    dJh = b * np.einsum('n,nij->ij', p, s[:, :, :-1] * s[:, :, 1:])
    dJv = b * np.einsum('n,nij->ij', p, s[:, :-1, :] * s[:, 1:, :])
    dH = np.einsum('n,nij->ij', p, s)           # d ln Z / d(beta h) = <s>
    return dJh, dJv, -np.dot(p, E), dH


@pytest.mark.parametrize("Ly,Lx,seed,field", [(4, 4, 1, 0.0), (3, 5, 2, 0.3), (5, 3, 3, 0.2),
                                               (2, 6, 4, 0.0), (4, 1, 5, 0.0), (1, 5, 6, 0.1)])
def test_untruncated_derivative_is_exact(Ly, Lx, seed, field):
    inst = random_instance(Ly, Lx, 0.8, 64, seed=seed, field_scale=field)
    m = model_of(inst)
    env = bmps.build_envs(m, 64)
    assert not any(env['trunc'])
    g = grad.grad_frozen(m, env)
    bh, bv, bb, bH = brute_derivatives(inst)
    np.testing.assert_allclose(g['dJh'], bh, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g['dJv'], bv, rtol=0, atol=1e-12)
    assert abs(g['dbeta'] - bb) < 1e-11
    np.testing.assert_allclose(g['dH'], bH, rtol=0, atol=1e-12)


def fd(model_fn, envs, eps=1e-5):
    return (grad.frozen_logZ(model_fn(+eps), envs) - grad.frozen_logZ(model_fn(-eps), envs)) / (2 * eps)


@pytest.mark.parametrize("mk,D", [
    (lambda: random_instance(4, 4, 0.8, 2, seed=7), 2),
    (lambda: random_instance(9, 10, 0.7, 4, seed=8), 4),
    (lambda: fully_frustrated(8, 1.0, 4), 4),
    (lambda: random_instance(7, 6, 0.9, 3, seed=9, field_scale=0.3), 3),
])
def test_truncated_derivative_matches_finite_differences(mk, D):
    inst = mk()
    m = model_of(inst)
    env = bmps.build_envs(m, D)
    assert any(env['trunc'])
    assert abs(grad.frozen_logZ(m, env) - env['logZ']) < 1e-11 * abs(env['logZ'])
    g = grad.grad_frozen(m, env)
    rng = np.random.default_rng(1)
    Ly, Lx = inst.Ly, inst.Lx
    for _ in range(6):
        r, c = rng.integers(Ly), rng.integers(Lx - 1)

        def mh(e, r=r, c=c):
            Jh = inst.Jh.copy()
            Jh[r, c] += e
            return ising.Model(Jh, inst.Jv, inst.h, inst.beta)
        assert abs(fd(mh, env) - g['dJh'][r, c]) < 2e-8
        r, c = rng.integers(Ly - 1), rng.integers(Lx)

        def mv(e, r=r, c=c):
            Jv = inst.Jv.copy()
            Jv[r, c] += e
            return ising.Model(inst.Jh, Jv, inst.h, inst.beta)
        assert abs(fd(mv, env) - g['dJv'][r, c]) < 2e-8

    def mb(e):
        return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta + e)
    assert abs(fd(mb, env) - g['dbeta']) < 1e-7


def test_derivative_with_row_weights_beyond_fp64_range():
    # 6 x 128 fully frustrated lattice at beta = 3 with D = 4: each row weighs
    # about e^400 and ln Z~ is about 2460.  The derivative must stay finite
    # and match central differences of the frozen contraction.  Rounding of
    # ln Z~ ~ 2460 limits the difference quotient: at eps = 1e-4 it is good to
    # a few 1e-7 (at 1e-5 the rounding term is ten times larger).
    inst = fully_frustrated(6, 3.0, 4, Lx=128)
    m = model_of(inst)
    env = bmps.build_envs(m, 4)
    assert any(env['trunc']) and env['logZ'] > 2000
    g = grad.grad_frozen(m, env)
    assert np.isfinite(g['dJh']).all() and np.isfinite(g['dJv']).all()
    rng = np.random.default_rng(2)
    for _ in range(4):
        r, c = rng.integers(inst.Ly), rng.integers(inst.Lx - 1)

        def mh(e, r=r, c=c):
            Jh = inst.Jh.copy()
            Jh[r, c] += e
            return ising.Model(Jh, inst.Jv, inst.h, inst.beta)
        assert abs(fd(mh, env, 1e-4) - g['dJh'][r, c]) < 5e-7
        r, c = rng.integers(inst.Ly - 1), rng.integers(inst.Lx)

        def mv(e, r=r, c=c):
            Jv = inst.Jv.copy()
            Jv[r, c] += e
            return ising.Model(inst.Jh, Jv, inst.h, inst.beta)
        assert abs(fd(mv, env, 1e-4) - g['dJv'][r, c]) < 5e-7


def test_beta_identity_without_field():
    # Z~_frozen depends on beta and J only through K = beta J: beta d_beta = sum J d_J
    inst = random_instance(8, 7, 0.9, 3, seed=12)
    m = model_of(inst)
    env = bmps.build_envs(m, 3)
    g = grad.grad_frozen(m, env)

    def mb(e):
        return ising.Model(inst.Jh, inst.Jv, None, inst.beta + e)
    lhs = inst.beta * fd(mb, env)
    rhs = (g['dJh'] * inst.Jh).sum() + (g['dJv'] * inst.Jv).sum()
    assert abs(lhs - rhs) < 1e-7 * max(1.0, abs(rhs))


def test_ferro_bond_correlation_symmetry():
    # the uniform ferromagnet is symmetric under left-right reflection; the
    # exact (untruncated) bond correlations must be too
    Jh, Jv = uniform(6, 6, 1.0)
    m = ising.Model(Jh, Jv, None, 0.44)
    env = bmps.build_envs(m, 64)
    g = grad.grad_frozen(m, env)
    np.testing.assert_allclose(g['dJh'], g['dJh'][:, ::-1], atol=1e-12)
    np.testing.assert_allclose(g['dJv'], g['dJv'][:, ::-1], atol=1e-12)
    assert np.all(g['dJh'] > 0) and np.all(g['dJh'] < 0.44)


def test_zero_coupling_is_rejected():
    inst = random_instance(3, 3, 0.5, 4, seed=1)
    Jh = inst.Jh.copy()
    Jh[0, 0] = 0.0
    m = ising.Model(Jh, inst.Jv, None, 0.5)
    env = bmps.build_envs(m, 4)
    with pytest.raises(ValueError):
        grad.grad_frozen(m, env)


# ---------------------------------------------------------------------------
# two-sided estimate (top-down upper boundary, bottom-up lower boundary)

@pytest.mark.parametrize("Ly,Lx,seed,field", [(4, 4, 21, 0.0), (3, 5, 22, 0.3), (5, 3, 23, 0.2),
                                               (4, 1, 24, 0.0), (1, 5, 25, 0.1)])
def test_two_sided_untruncated_is_exact(Ly, Lx, seed, field):
    inst = random_instance(Ly, Lx, 0.8, 64, seed=seed, field_scale=field)
    m = model_of(inst)
    env = bmps.build_envs(m, 64)
    g = grad.grad_two_sided(m, env)
    bh, bv, bb, bH = brute_derivatives(inst)
    np.testing.assert_allclose(g['dJh'], bh, rtol=0, atol=1e-12)
    np.testing.assert_allclose(g['dJv'], bv, rtol=0, atol=1e-12)
    assert abs(g['dbeta'] - bb) < 1e-11
    np.testing.assert_allclose(g['dH'], bH, rtol=0, atol=1e-12)


def test_two_sided_is_flip_equivariant():
    # upside down, the top-down and bottom-up boundaries trade places, so the
    # estimate of the flipped lattice is the flipped estimate (truncated, D 3)
    inst = random_instance(7, 6, 0.9, 3, seed=26, field_scale=0.2)
    m = model_of(inst)
    g = grad.grad_two_sided(m, bmps.build_envs(m, 3))
    mf = ising.Model(inst.Jh[::-1].copy(), inst.Jv[::-1].copy(), inst.h[::-1].copy(), inst.beta)
    gf = grad.grad_two_sided(mf, bmps.build_envs(mf, 3))
    np.testing.assert_allclose(gf['dJh'], g['dJh'][::-1], rtol=0, atol=1e-10)
    np.testing.assert_allclose(gf['dJv'], g['dJv'][::-1], rtol=0, atol=1e-10)
    np.testing.assert_allclose(gf['dH'], g['dH'][::-1], rtol=0, atol=1e-10)
    assert abs(gf['dbeta'] - g['dbeta']) < 1e-9


def test_two_sided_tracks_exact_derivative_on_frustrated_lattice():
    # 14x12 fully frustrated, beta 1, D 4 (truncated): exact derivatives by
    # central differences of the transfer-matrix ln Z.  The two-sided estimate
    # is within 0.01 on every bond checked (the frozen derivative of ln Z~ is
    # off by up to ~0.5 here: it differentiates the one-sided approximation)
    inst = fully_frustrated(14, 1.0, 4, Lx=12)
    m = model_of(inst)
    env = bmps.build_envs(m, 4)
    assert any(env['trunc'])
    g = grad.grad_two_sided(m, env)

    def exact_fd(kind, r, c, e=1e-4):
        vals = []
        for sgn in (1.0, -1.0):
            Jh, Jv = inst.Jh.copy(), inst.Jv.copy()
            (Jh if kind == 'h' else Jv)[r, c] += sgn * e
            vals.append(exact.transfer_logZ(Jh, Jv, None, inst.beta))
        return (vals[0] - vals[1]) / (2 * e)
    rng = np.random.default_rng(4)
    for _ in range(4):
        r, c = rng.integers(inst.Ly), rng.integers(inst.Lx - 1)
        assert abs(g['dJh'][r, c] - exact_fd('h', r, c)) < 1e-2
        r, c = rng.integers(inst.Ly - 1), rng.integers(inst.Lx)
        assert abs(g['dJv'][r, c] - exact_fd('v', r, c)) < 1e-2
