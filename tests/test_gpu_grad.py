"""Parity of tn_grad (frozen-truncation derivative of ln Z~) with the oracle.

The GPU builds its own environment; the frozen projectors are spans, so the
derivative is gauge invariant and comparable to the oracle's element by
element.  Tolerance: 1e-9 absolute on d ln Z~/dJ (entries are O(beta)),
1e-9 relative on d ln Z~/d beta.
"""
import numpy as np
import torch
import pytest

from oracle import bmps, exact, grad, ising
from workloads import random_instance, fully_frustrated, ea_pm, ferro

pytestmark = pytest.mark.gpu

CASES = [
    ("4x4 untruncated field", lambda: random_instance(4, 4, 0.8, 8, seed=1, field_scale=0.3), 8),
    ("3x5 untruncated", lambda: random_instance(3, 5, 0.7, 8, seed=2), 8),
    ("4x4 D2", lambda: random_instance(4, 4, 0.8, 2, seed=7), 2),
    ("9x10 D4", lambda: random_instance(9, 10, 0.7, 4, seed=8), 4),
    ("frustrated 8 D4", lambda: fully_frustrated(8, 1.0, 4), 4),
    ("ea 12 D8", lambda: ea_pm(12, 1.0, 8, seed=5), 8),
    ("ragged 11x7 D5 field", lambda: random_instance(11, 7, 0.6, 5, seed=9, field_scale=0.2), 5),
    ("strip 1x6", lambda: random_instance(1, 6, 0.6, 4, seed=10), 4),
    ("column 6x1", lambda: random_instance(6, 1, 0.6, 4, seed=11), 4),
    # ln Z~ beyond the fp64 exponent range: the upper state must stay rescaled
    ("ferro 20x12 beta3 D4", lambda: ferro(20, 3.0, 4, Lx=12), 4),
    ("frustrated 26x14 beta2 D6", lambda: fully_frustrated(26, 2.0, 6, Lx=14), 6),
    ("frustrated 6x128 beta3 D4", lambda: fully_frustrated(6, 3.0, 4, Lx=128), 4),
    ("frustrated 16x48 beta1 D8", lambda: fully_frustrated(16, 1.0, 8, Lx=48), 8),
]


@pytest.mark.parametrize("name,mk,D", CASES, ids=[c[0] for c in CASES])
def test_grad_matches_oracle(name, mk, D):
    from paper_2104_13264_amd import Sampler
    inst = mk()
    print(f"[grad] {name} Ly={inst.Ly} Lx={inst.Lx} D={D}", flush=True)
    m = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    env = bmps.build_envs(m, D)
    ref = grad.grad_frozen(m, env)
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, D)
    dJh, dJv, db = s.grad()
    dJh, dJv = dJh.cpu().numpy(), dJv.cpu().numpy()
    np.testing.assert_allclose(dJh, ref['dJh'], rtol=0, atol=1e-9)
    np.testing.assert_allclose(dJv, ref['dJv'], rtol=0, atol=1e-9)
    assert abs(db - ref['dbeta']) <= 1e-9 * max(1.0, abs(ref['dbeta']))
    s.close()


def test_untruncated_grad_is_bond_correlation():
    from paper_2104_13264_amd import Sampler
    inst = random_instance(4, 4, 0.9, 8, seed=3)
    cfg, E, lz, lp = exact.brute_force(inst.Jh, inst.Jv, None, inst.beta)
    p = np.exp(lp)
    sp = cfg.astype(float)
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, 8)
    dJh, dJv, db = s.grad()
    bh = inst.beta * np.einsum('n,nij->ij', p, sp[:, :, :-1] * sp[:, :, 1:])
    bv = inst.beta * np.einsum('n,nij->ij', p, sp[:, :-1, :] * sp[:, 1:, :])
    np.testing.assert_allclose(dJh.cpu().numpy(), bh, atol=1e-11)
    np.testing.assert_allclose(dJv.cpu().numpy(), bv, atol=1e-11)
    assert abs(db + np.dot(p, E)) < 1e-10
    s.close()


def test_grad_rejects_zero_coupling_and_installed_env():
    from paper_2104_13264_amd import Sampler, TNError
    inst = random_instance(3, 4, 0.5, 4, seed=1)
    Jh = inst.Jh.copy()
    Jh[1, 1] = 0.0
    s = Sampler()
    s.build_env(Jh, inst.Jv, None, 0.5, 4)
    with pytest.raises(TNError):
        s.grad()
    envs = s.get_env()
    t = Sampler()
    t.set_env(inst.Jh, inst.Jv, None, 0.5, 4, *envs[:3], envs[3])
    with pytest.raises(TNError):
        t.grad()
    s.close()
    t.close()


def test_autograd_function_matches_tn_grad_and_brute_force():
    from paper_2104_13264_amd import Sampler, log_z
    inst = random_instance(4, 4, 0.7, 8, seed=12)
    Jh = torch.tensor(inst.Jh, dtype=torch.float64, device='cuda', requires_grad=True)
    Jv = torch.tensor(inst.Jv, dtype=torch.float64, device='cuda', requires_grad=True)
    beta = torch.tensor(inst.beta, dtype=torch.float64, device='cuda', requires_grad=True)
    lz = log_z(Jh, Jv, beta, 8)
    gJh, gJv, gb = torch.autograd.grad(2.0 * lz, (Jh, Jv, beta))
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, 8)
    dJh, dJv, db = s.grad()
    assert torch.equal(gJh, 2.0 * dJh) and torch.equal(gJv, 2.0 * dJv)
    assert float(gb) == 2.0 * db
    # untruncated: d ln Z / d beta = -<E> exactly (brute force)
    cfg, E, _, lp = exact.brute_force(inst.Jh, inst.Jv, None, inst.beta)
    assert abs(float(gb) / 2.0 + float(np.dot(np.exp(lp), E))) < 1e-10
    # the two-sided estimator behind the same function: tn_grad_two_sided
    lz2 = log_z(Jh, Jv, beta, 8, estimator="two_sided")
    tJh, tJv, tb = torch.autograd.grad(lz2, (Jh, Jv, beta))
    eJh, eJv, eb = s.grad(two_sided=True)
    assert torch.equal(tJh, eJh) and torch.equal(tJv, eJv) and float(tb) == eb
    assert abs(float(tb) + float(np.dot(np.exp(lp), E))) < 1e-10
    with pytest.raises(ValueError):
        log_z(Jh, Jv, beta, 8, estimator="rebuilt")
    s.close()


TWO_SIDED_CASES = [
    ("4x4 untruncated field", lambda: random_instance(4, 4, 0.8, 8, seed=31, field_scale=0.3), 8),
    ("9x10 D4", lambda: random_instance(9, 10, 0.7, 4, seed=32), 4),
    ("ragged 11x7 D5 field", lambda: random_instance(11, 7, 0.6, 5, seed=33, field_scale=0.2), 5),
    ("frustrated 14x12 D4", lambda: fully_frustrated(14, 1.0, 4, Lx=12), 4),
    ("ea 12 D8", lambda: ea_pm(12, 1.0, 8, seed=34), 8),
    ("strip 1x6", lambda: random_instance(1, 6, 0.6, 4, seed=35), 4),
    ("column 6x1", lambda: random_instance(6, 1, 0.6, 4, seed=36), 4),
    ("frustrated 6x128 beta3 D4", lambda: fully_frustrated(6, 3.0, 4, Lx=128), 4),
]


@pytest.mark.parametrize("name,mk,D", TWO_SIDED_CASES, ids=[c[0] for c in TWO_SIDED_CASES])
def test_two_sided_matches_oracle(name, mk, D):
    # same tolerances as the frozen derivative: fp64 contractions on both
    # sides, the top-down boundary built by the upside-down build on the GPU
    # and by a top-down recursion in the oracle (equal up to a +-1 leg gauge)
    from paper_2104_13264_amd import Sampler
    inst = mk()
    print(f"[grad two-sided] {name} Ly={inst.Ly} Lx={inst.Lx} D={D}", flush=True)
    m = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    ref = grad.grad_two_sided(m, bmps.build_envs(m, D))
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, D)
    for _ in range(2):      # the second call reuses the upside-down build
        dJh, dJv, db = s.grad(two_sided=True)
        np.testing.assert_allclose(dJh.cpu().numpy(), ref['dJh'], rtol=0, atol=1e-9)
        np.testing.assert_allclose(dJv.cpu().numpy(), ref['dJv'], rtol=0, atol=1e-9)
        assert abs(db - ref['dbeta']) <= 1e-9 * max(1.0, abs(ref['dbeta']))
    s.close()


def test_two_sided_follows_a_new_instance():
    from paper_2104_13264_amd import Sampler
    a = random_instance(5, 6, 0.7, 3, seed=37)
    b = random_instance(5, 6, 0.9, 3, seed=38)
    s = Sampler()
    s.build_env(a.Jh, a.Jv, None, a.beta, 3)
    s.grad(two_sided=True)
    s.build_env(b.Jh, b.Jv, None, b.beta, 3)
    dJh, _, _ = s.grad(two_sided=True)
    m = ising.Model(b.Jh, b.Jv, None, b.beta)
    ref = grad.grad_two_sided(m, bmps.build_envs(m, 3))
    np.testing.assert_allclose(dJh.cpu().numpy(), ref['dJh'], rtol=0, atol=1e-9)
    s.close()
