"""Parity at the benchmarked configuration: 64x64 open ferromagnet, J = +1,
beta = 0.4407, D = 32, 4096 chains (Sec. 2 Eqs. mh-acc, tns-prior; App. A
Eq. proba-ratio-apx).

* The batched FP32 sampler in the launch shape the benchmark times (the
  autotuner's choice for 20 MH steps of 4096 chains, as the benchmark tunes
  it: one launch of 81920 proposals): ln q of 640 proposals spread over every
  step within 1e-5 relative of the oracle's evaluation of the same
  configurations, energies bitwise, spins equal to the oracle's own draws
  wherever the oracle's draw was farther than 1e-4 from its threshold.
* The batched BF16 sampler in its tuned launch shape: ln q of 160 proposals
  within the BF16 bound (8 * 2^-8 * sqrt(2 Lx Ly)) of the oracle's evaluation,
  and the eval mode of every proposal of the launch bitwise its sample mode.
* The plain FP64 path: 64 proposals of a 4096-proposal batch bitwise equal
  to the oracle's draws of the same proposal ids (draws within 1e-6 of a
  threshold excluded and counted), ln q within 1e-9 relative.
* Acceptance of Algorithm 1 over 256 chains x 20 steps from all-up: the FP32
  chain within 1% absolute of the oracle's chain, the FP64 chain too.
"""
import numpy as np
import pytest

from oracle import bmps, mh, sampler
from workloads import ferro_64, SEED
from bridge import model_of, TOL_LOGZ_FP64, TOL_LOGQ_FP32, NEAR_FP64

pytestmark = pytest.mark.gpu

FP64, FP32, BF16 = 0, 1, 2


def log(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def c2():
    inst = ferro_64()
    log("[c2] oracle build 64x64 D32")
    return inst, model_of(inst), bmps.build_envs(model_of(inst), inst.D)


def test_fp32_launch_shape_of_the_benchmark(c2):
    from paper_2104_13264_amd import Sampler
    inst, m, ref = c2
    C, nsteps = inst.chains, 20
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, None, inst.beta, inst.D, FP32)
    assert abs(lz - ref["logZ"]) <= TOL_LOGZ_FP64 * abs(ref["logZ"])
    v, m_steps = s.autotune(C, max_steps=nsteps)
    log(f"[c2] fp32: {C} chains x {nsteps} steps, tuned variant {v}, {m_steps} steps per launch")
    sp, lq, E = s.sample_steps(C, nsteps, SEED, step0=0)
    sp, lq, E = sp.cpu().numpy(), lq.cpu().numpy(), E.cpu().numpy()
    ids = np.arange(0, C, 128)            # 32 chains per step, every step: 640 proposals
    got_sp = sp[:, ids].reshape(-1, inst.Ly, inst.Lx)
    got_lq = lq[:, ids].reshape(-1)
    got_E = E[:, ids].reshape(-1)
    log(f"[c2] oracle eval of {got_sp.shape[0]} proposals")
    ev = sampler.eval_logq(m, ref, got_sp)
    rel = np.abs(got_lq - ev["logq"]) / np.abs(ev["logq"])
    log(f"[c2] fp32 ln q rel: max {rel.max():.2e} median {np.median(rel):.2e}")
    assert np.all(rel <= TOL_LOGQ_FP32)
    assert np.array_equal(got_E, ev["energy"])
    # the oracle's own draws of the same proposals (ids, steps)
    same = far = 0
    for t in range(nsteps):
        want = sampler.sample(m, ref, len(ids), SEED, step=t, ids=ids)
        ok = want["min_gap"] >= 1e-4
        far += int(ok.sum())
        same += int(np.all(sp[t, ids][ok] == want["spins"][ok], axis=(1, 2)).sum())
    log(f"[c2] fp32 spins equal to the oracle's on {same}/{far} proposals drawn >= 1e-4 from every threshold")
    assert far >= 128 and same == far
    s.close()


def test_bf16_launch_shape_full_size(c2):
    import torch
    from paper_2104_13264_amd import Sampler
    inst, m, ref = c2
    C, nsteps = inst.chains, 20
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, inst.D, BF16)
    v, m_steps = s.autotune(C, max_steps=nsteps)
    log(f"[c2] bf16: {C} chains x {nsteps} steps, tuned variant {v}, {m_steps} steps per launch")
    sp, lq, E = s.sample_steps(C, nsteps, SEED, step0=0)
    lq2, E2 = s.eval_logq(sp.reshape(-1, inst.Ly, inst.Lx))
    assert torch.equal(lq2, lq.reshape(-1)) and torch.equal(E2, E.reshape(-1))
    sp, lq = sp.cpu().numpy(), lq.cpu().numpy()
    ids = np.arange(0, C, 512)            # 8 chains per step, every step: 160 proposals
    got_sp = sp[:, ids].reshape(-1, inst.Ly, inst.Lx)
    ev = sampler.eval_logq(m, ref, got_sp)
    dev = np.abs(lq[:, ids].reshape(-1) - ev["logq"])
    bound = 8 * 2.0 ** -8 * np.sqrt(2 * inst.Lx * inst.Ly)
    log(f"[c2] bf16 |ln q - oracle|: mean {dev.mean():.3e} max {dev.max():.3e} (bound {bound:.3e})")
    assert np.all(np.isfinite(lq)) and dev.max() <= bound
    s.close()


def test_fp64_plain_path_full_size(c2):
    from paper_2104_13264_amd import Sampler
    inst, m, ref = c2
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, None, inst.beta, inst.D, FP64)
    assert abs(lz - ref["logZ"]) <= TOL_LOGZ_FP64 * abs(ref["logZ"])
    log("[c2] fp64: 4096 proposals, 64 compared")
    sp, lq, E = s.sample(inst.chains, SEED, step=7)
    ids = np.arange(0, inst.chains, 64)
    want = sampler.sample(m, ref, len(ids), SEED, step=7, ids=ids)
    ok = want["min_gap"] >= NEAR_FP64
    log(f"[c2] fp64: {int((~ok).sum())} of {len(ids)} proposals drew within 1e-6 of a threshold")
    got_sp = sp.cpu().numpy()[ids]
    assert np.array_equal(got_sp[ok], want["spins"][ok])
    got_lq = lq.cpu().numpy()[ids]
    assert np.all(np.abs(got_lq[ok] - want["logq"][ok]) <= TOL_LOGZ_FP64 * np.abs(want["logq"][ok]))
    assert np.array_equal(E.cpu().numpy()[ids][ok], want["energy"][ok])
    assert ok.sum() >= 48
    s.close()


@pytest.mark.timeout(900)
def test_acceptance_against_the_oracle_chain(c2):
    from paper_2104_13264_amd import Sampler
    inst, m, ref = c2
    chains, steps = 256, 20
    log(f"[c2] oracle chain: {chains} chains x {steps} steps")
    _, acc_ref, _ = mh.run_chain(m, ref, chains, steps, SEED)
    a_ref = float(acc_ref.mean())
    for prec, name in ((FP32, "fp32"), (FP64, "fp64")):
        s = Sampler()
        s.build_env(inst.Jh, inst.Jv, None, inst.beta, inst.D, prec)
        st = s.init_state(chains)
        acc = []
        for t in range(steps):
            s.mh_step(st, SEED, t)
            acc.append(st["accepted"].cpu().numpy().astype(bool))
        a = float(np.mean(acc))
        log(f"[c2] acceptance {name} {a:.5f} oracle {a_ref:.5f}")
        assert abs(a - a_ref) <= 0.01
        s.close()
