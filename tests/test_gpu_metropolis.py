"""Metropolis sweeps on the GPU (tn_metropolis_sweeps) against the oracle.

Spins bitwise equal to the oracle's sweeps under the shared Philox stream
(both decide u < exp(-(beta dE)) in FP64 from the same expressions; a draw
within 1e-12 of its threshold would fail the test, and none is expected),
flip counts equal, ln q and E of the new states bitwise those tn_eval_logq
gives them, ln q within 1e-9 of the oracle's eval mode on FP64 paths (FP32:
1e-5 where the states are not deep in the tails of q), energies exact for +-1
couplings.  An interleaved run of TNMH steps and sweeps follows the oracle's
chain bitwise.
"""
import numpy as np
import pytest
import torch

from oracle import metropolis, mh
from oracle.metropolis import sweep_uniforms, local_field
from workloads import random_instance, ea_pm
from bridge import model_of, gpu_sampler_with_oracle_env, TOL_LOGZ_FP64, TOL_LOGQ_FP32

pytestmark = pytest.mark.gpu

FP64, FP32, BF16 = 0, 1, 2


def log(msg):
    print(msg, flush=True)


def min_gap(model, spins, seed, step, nsweeps):
    """Smallest |u - exp(-(beta dE))| over the oracle's decisions."""
    s = np.array(spins, dtype=np.float64)
    chains, Ly, Lx = s.shape
    rr, cc = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    gap = np.full(chains, np.inf)
    for k in range(nsweeps):
        u = sweep_uniforms(chains, Ly * Lx, seed, step, k).reshape(chains, Ly, Lx)
        for col in (0, 1):
            F = local_field(s, model.Jh, model.Jv, model.h)
            thr = np.exp(-(model.beta * ((2.0 * s) * F)))
            m = ((rr + cc) & 1) == col
            g = np.where(m[None], np.abs(u - thr), np.inf)
            gap = np.minimum(gap, g.reshape(chains, -1).min(axis=1))
            s = np.where((u < thr) & m[None], -s, s)
    return gap


CASES = [  # (instance, D, precision, chains, sweeps)
    (random_instance(7, 9, 0.7, 8, seed=401, field_scale=0.3), 8, FP64, 37, 3),
    (ea_pm(10, 1.0, 12, seed=402), 12, FP32, 64, 2),
    (ea_pm(12, 3.0, 16, seed=403), 16, FP64, 130, 5),
    (ea_pm(12, 3.0, 16, seed=403), 16, FP32, 130, 5),   # atypical states: ln q vs eval only
    (random_instance(1, 11, 0.9, 4, seed=404, field_scale=0.5), 4, FP64, 9, 4),   # one row
    (random_instance(13, 1, 0.9, 4, seed=405, field_scale=0.5), 4, FP32, 9, 4),   # one column
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_sweeps_match_oracle(case):
    inst, D, prec, C, nsw = CASES[case]
    log(f"[metro] {inst.name} {inst.Ly}x{inst.Lx} D={D} prec={prec} chains={C} sweeps={nsw}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, prec)
    m = model_of(inst)
    rng = np.random.default_rng(case)
    s0 = rng.choice([-1, 1], size=(C, inst.Ly, inst.Lx)).astype(np.int8)
    state = s.init_state(C, torch.as_tensor(s0))
    s.stats(reset=True)
    seed, step = 1234 + case, 17
    s.metropolis_sweeps(state, nsw, seed, step)
    ref, flips = metropolis.sweeps(m, s0, seed, step, nsw)
    ok = min_gap(m, s0, seed, step, nsw) >= 1e-12
    assert ok.all()
    got = state["spins"].cpu().numpy()
    np.testing.assert_array_equal(got, ref)
    assert s.stats()["metropolis_flips"] == int(flips.sum())
    # the new states' ln q and E are those tn_eval_logq gives them (the
    # arithmetic the proposals are drawn with), bitwise
    lq2, E2 = s.eval_logq(state["spins"])
    assert torch.equal(lq2, state["logq"]) and torch.equal(E2, state["energy"])
    ev = mh.init_state(m, envs, C, ref)
    np.testing.assert_allclose(state["energy"].cpu().numpy(), ev["energy"], rtol=1e-13, atol=1e-12)
    # against the FP64 oracle: FP64 paths always; FP32 where the states are
    # not far in the tails of q (sweeps from random spins at beta = 3 give
    # configurations whose small conditionals FP32 resolves only to ~1e-3)
    if prec == FP64 or inst.beta <= 1.0:
        tol = TOL_LOGZ_FP64 if prec == FP64 else TOL_LOGQ_FP32
        np.testing.assert_allclose(state["logq"].cpu().numpy(), ev["logq"], rtol=tol, atol=0)
    s.close()


def test_interleaved_chain_matches_oracle():
    # +-J spin glass at beta 2, D 8: TNMH steps with one sweep after each
    inst = ea_pm(8, 2.0, 8, seed=406)
    D, C, steps = 8, 48, 6
    log(f"[metro] interleaved ea_pm 8x8 D={D} chains={C} steps={steps}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, FP64)
    m = model_of(inst)
    state = s.init_state(C)
    ref = mh.init_state(m, envs, C)
    seed = 99
    for t in range(steps):
        s.mh_step(state, seed, t)
        acc, _, _ = mh.mh_step(m, envs, ref, seed, t)
        assert np.array_equal(state["accepted"].cpu().numpy().astype(bool), acc)
        s.metropolis_sweeps(state, 1, seed, t)
        metropolis.interleave(m, envs, ref, seed, t, 1)
        np.testing.assert_array_equal(state["spins"].cpu().numpy(), ref["spins"])
        np.testing.assert_array_equal(state["energy"].cpu().numpy(), ref["energy"])
        np.testing.assert_allclose(state["logq"].cpu().numpy(), ref["logq"], rtol=TOL_LOGZ_FP64, atol=0)
    s.close()


def test_beta_zero_flips_everything_and_no_sweeps_is_a_noop():
    from paper_2104_13264_amd import Sampler, TNError
    inst = random_instance(6, 8, 0.0, 4, seed=407, field_scale=0.3)
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, inst.h, 0.0, 4, FP32)
    state = s.init_state(5)
    before = state["spins"].clone()
    s.metropolis_sweeps(state, 0, 1, 0)
    assert torch.equal(state["spins"], before)
    s.metropolis_sweeps(state, 3, 1, 0)
    assert torch.equal(state["spins"], -before)
    with pytest.raises(TNError):
        s.metropolis_sweeps(state, 1 << 18, 1, 0)
    s.close()
