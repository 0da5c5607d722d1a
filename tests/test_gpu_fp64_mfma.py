"""The batched FP64 sampler (TN_FP64_MFMA: the team kernel with fp64
operands and vectors on the fp64 matrix cores) against the oracle.

With the oracle's environments installed on the GPU (tn_set_env), so that
only the sampler's arithmetic is compared:
* proposals bitwise equal to the oracle's draws off-threshold (draws within
  1e-6 of a threshold excluded), ln q within 1e-9 relative, energies bitwise
  for +-1 couplings, over both bond classes (D <= 16, D <= 32), fields,
  strips, columns and a 256-wide lattice; eval mode bitwise sample mode;
* an MH chain of Algorithm 1 bitwise the oracle's chain (8x8, D = 8);
* the low-temperature instance where FP32 operands cannot resolve the
  conditionals (+-J 32x32, T = 0.212, D = 16, chains from a draw of the
  proposal law): ln q within the instance's own conditioning of the oracle
  (ten times the largest relative change of the oracle's ln q under one-ulp
  changes of the environment, at least 1e-9), and the acceptance within 1%
  absolute of the plain FP64 path's; the FP32 path's ln q error on the same
  proposals is measured and pinned as the reason for this path.
The batched FP64 sampler refuses D > 32 and the batched-instance build.
"""
import numpy as np
import pytest
import torch

from oracle import bmps, mh, sampler
from workloads import random_instance, ferro, ea_pm, SEED
from bridge import model_of, pack_envs, TOL_LOGZ_FP64, TOL_LOGQ_FP32, NEAR_FP64

pytestmark = pytest.mark.gpu

FP64, FP32, BF16, FP64M = 0, 1, 2, 3


def log(msg):
    print(msg, flush=True)


def with_oracle_env(inst, D, prec, envs=None):
    from paper_2104_13264_amd import Sampler
    envs = envs if envs is not None else bmps.build_envs(model_of(inst), D)
    env, dims, ell = pack_envs(envs, D)
    s = Sampler()
    s.set_env(inst.Jh, inst.Jv, inst.h, inst.beta, D, env, dims, ell, envs['logZ'], prec)
    return s, envs


CASES = [
    ("ferro 8x8 D8", lambda: ferro(8, 0.44, 8), 8),
    ("random 7x9 D6 field", lambda: random_instance(7, 9, 0.7, 6, seed=91, field_scale=0.3), 6),
    ("ea 12x12 D16 beta1", lambda: ea_pm(12, 1.0, 16, seed=92), 16),
    ("random 16x16 D24", lambda: random_instance(16, 16, 0.5, 24, seed=93), 24),
    ("random 10x12 D32 field", lambda: random_instance(10, 12, 0.6, 32, seed=94, field_scale=0.2), 32),
    ("strip 1x9 D4", lambda: random_instance(1, 9, 0.8, 4, seed=95), 4),
    ("column 6x1 D2", lambda: random_instance(6, 1, 0.8, 2, seed=96), 2),
    ("wide 3x256 D16", lambda: random_instance(3, 256, 0.6, 16, seed=97), 16),
]


@pytest.mark.parametrize("name,mk,D", CASES, ids=[c[0] for c in CASES])
def test_fp64_mfma_matches_oracle(name, mk, D):
    inst = mk()
    log(f"[fp64m] {name} Ly={inst.Ly} Lx={inst.Lx} D={D}")
    s, envs = with_oracle_env(inst, D, FP64M)
    m = model_of(inst)
    B, seed, step, first = 45, 777, 2, 3
    want = sampler.sample(m, envs, B, seed, step=step, first_id=first)
    sp, lq, E = s.sample(B, seed, step=step, first_id=first)
    ok = want["min_gap"] >= NEAR_FP64
    assert ok.sum() >= B - 4
    sp_n, lq_n, E_n = sp.cpu().numpy(), lq.cpu().numpy(), E.cpu().numpy()
    assert np.array_equal(sp_n[ok], want["spins"][ok])
    assert np.all(np.abs(lq_n[ok] - want["logq"][ok]) <= TOL_LOGZ_FP64 * np.abs(want["logq"][ok]))
    np.testing.assert_allclose(E_n[ok], want["energy"][ok], rtol=1e-13, atol=1e-12)
    lq2, E2 = s.eval_logq(sp)
    assert torch.equal(lq2, lq) and torch.equal(E2, E)
    # the no-allocation entry point draws the same proposals
    b = s.sample_noalloc(B, seed, step=step, first_id=first)
    assert torch.equal(b[0], sp) and torch.equal(b[1], lq)
    s.close()


def test_fp64_mfma_chain_follows_the_oracle():
    inst = ferro(8, 0.44, 8)
    s, envs = with_oracle_env(inst, 8, FP64M)
    m = model_of(inst)
    C, steps = 64, 30
    st = s.init_state(C)
    ost = mh.init_state(m, envs, C)
    np.testing.assert_allclose(st["logq"].cpu().numpy(), ost["logq"], rtol=TOL_LOGZ_FP64)
    compared = 0
    for t in range(steps):
        s.mh_step(st, SEED, t)
        acc, _, _ = mh.mh_step(m, envs, ost, SEED, t)
        if s.stats()["near_threshold"]:
            log(f"[fp64m] near-threshold draw at step {t}: comparison stops")
            break
        assert np.array_equal(st["accepted"].cpu().numpy().astype(bool), acc)
        assert np.array_equal(st["spins"].cpu().numpy(), ost["spins"])
        compared += 1
    assert compared >= 20
    s.close()


def env_spread(m, envs, spins, logq, seed=5):
    """|change of the oracle's ln q| of the given configurations when every
    environment entry moves by one ulp (random sign): the conditioning of the
    sampler's arithmetic on this instance."""
    rng = np.random.default_rng(seed)
    pert = dict(envs)
    pert["env"] = [None if k is None else
                   [E * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=E.shape)) for E in k]
                   for k in envs["env"]]
    ev = sampler.eval_logq(m, pert, spins)
    return np.abs(ev["logq"] - logq)


def test_low_temperature_instance():
    # +-J 32x32 at T = 0.212, D = 16 (the setting of the paper's interleaving
    # experiment); one environment (the oracle's) for all precisions.  The
    # chains start from a draw of the proposal law (q > 0 by construction: the
    # all-up state can be a zero of the clamped FP64 law, a state no move
    # leaves)
    inst = ea_pm(32, 1.0 / 0.212, 16, SEED + 7)
    envs = bmps.build_envs(model_of(inst), 16)
    m = model_of(inst)
    C = 1024
    s0, _ = with_oracle_env(inst, 16, FP64M, envs)
    start, _, _ = s0.sample(C, SEED, step=999)
    s0.close()
    out = {}
    for prec, name in ((FP64M, "fp64_mfma"), (FP64, "fp64"), (FP32, "fp32")):
        s, _ = with_oracle_env(inst, 16, prec, envs)
        sp, lq, _ = s.sample(256, SEED, step=5)
        sp_n, lq_n = sp.cpu().numpy(), lq.cpu().numpy()
        ev = sampler.eval_logq(m, envs, sp_n)
        with np.errstate(invalid="ignore"):
            rel = np.abs(lq_n - ev["logq"]) / np.abs(ev["logq"])
        st = s.init_state(C, spins=start)
        s.stats(reset=True)
        for t in range(20):
            s.mh_step(st, SEED, t)
        stt = s.stats()
        acc = stt["accepted"] / stt["proposed"]
        out[name] = (sp_n, lq_n, ev, rel, acc)
        bad = ~(rel <= TOL_LOGQ_FP32)
        log(f"[fp64m] T=0.212 {name}: ln q rel max {np.nanmax(rel):.2e} median {np.nanmedian(rel):.2e}; "
            f"{int(bad.sum())}/256 miss 1e-5 ({int(np.isinf(ev['logq']).sum())} have zero oracle probability); "
            f"acceptance {acc:.5f}")
        s.close()
    # FP64 on the matrix cores: ln q within ten times the instance's
    # conditioning, the largest relative change of the oracle's ln q over all
    # proposals when the environment moves by one ulp (at least 1e-9): at this
    # temperature a row's conditional sums cancel by several orders, and
    # rounding of the order-of-operations alone moves ln q by that much
    sp_m, lq_m, ev_m, rel_m, acc_m = out["fp64_mfma"]
    cond = float(np.max(env_spread(m, envs, sp_m, ev_m["logq"]) / np.abs(ev_m["logq"])))
    tol_rel = max(TOL_LOGZ_FP64, 10.0 * cond)
    log(f"[fp64m] conditioning: one-ulp relative spread max {cond:.2e}; bound {tol_rel:.2e}")
    assert np.all(np.abs(lq_m - ev_m["logq"]) <= tol_rel * np.abs(ev_m["logq"]))
    # the same MH chains accept as often as with the plain FP64 sampler
    assert abs(acc_m - out["fp64"][4]) <= 0.01
    # FP32 operands do not resolve this instance's small conditional weights:
    # a good part of its proposals miss 1e-5 (some have zero probability under
    # the FP64 law), the reason for the FP64 path
    rel_f = out["fp32"][3]
    assert (~(rel_f <= TOL_LOGQ_FP32)).sum() >= 25


def test_fp64_mfma_refusals():
    from paper_2104_13264_amd import Sampler, TNError
    inst = random_instance(6, 7, 0.5, 40, seed=98)
    s = Sampler()
    with pytest.raises(TNError):
        s.build_env(inst.Jh, inst.Jv, None, inst.beta, 40, FP64M)
    with pytest.raises(TNError):
        s.build_env_multi([dict(Jh=inst.Jh, Jv=inst.Jv, h=None, beta=inst.beta, D=8, chains=4)], FP64M)
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, 8, FP64M)
    sp, lq, _ = s.sample(16, 1)
    assert torch.isfinite(lq).all()
    s.close()
