"""Parity of the HIP path (through the C ABI) against the oracle.

Environment build: ln Z~ within 1e-9 relative (fp64 QR/SVD on both sides;
raw env tensors are gauge dependent and never compared).
Plain fp64 sampler: spins bit-exact under the shared Philox stream except
proposals with a draw within 1e-6 of its threshold (counted), ln q within
1e-9 relative, energies bit-exact for +-1 couplings.
Batched fp32 sampler: ln q of the drawn spins within 1e-5 relative of the
oracle's fp64 evaluation of the same spins; identical draws wherever the
oracle's draw was farther from its threshold than the fp32 error.
"""
import numpy as np
import pytest
import torch

from oracle import bmps, exact, mh, sampler
from workloads import (random_instance, ferro, fully_frustrated, antiferro, ea_pm,
                       small_ferro_8, ferro_64, SEED)
from bridge import (model_of, pack_envs, gpu_sampler_with_oracle_env, TOL_LOGZ_FP64,
                    TOL_LOGQ_FP32, NEAR_FP64)

pytestmark = pytest.mark.gpu

FP64, FP32, BF16 = 0, 1, 2


def log(msg):
    print(msg, flush=True)


ENV_CASES = [
    ("4x4 exact", lambda: random_instance(4, 4, 0.9, 8, seed=1, field_scale=0.3), 8),
    ("4x4 D2", lambda: random_instance(4, 4, 0.9, 2, seed=2, field_scale=0.3), 2),
    ("ragged 9x11 D5", lambda: random_instance(9, 11, 0.7, 5, seed=3, field_scale=0.2), 5),
    ("ferro 16 D8", lambda: ferro(16, 0.4407, 8), 8),
    ("frustrated 12 D6", lambda: fully_frustrated(12, 1.0, 6), 6),
    ("ea 14 D20", lambda: ea_pm(14, 1.0, 20, seed=7), 20),
    ("strip 1x9", lambda: random_instance(1, 9, 0.8, 4, seed=4), 4),
    ("column 7x1", lambda: random_instance(7, 1, 0.8, 4, seed=5), 4),
    ("beta0 6x5", lambda: random_instance(6, 5, 0.0, 3, seed=6), 3),
    ("ea 10 D40", lambda: ea_pm(10, 0.7, 40, seed=8), 40),
    # row weights past the fp64 range (e^400 .. e^765 a row)
    ("ferro 3x128 beta3 D4", lambda: ferro(3, 3.0, 4, Lx=128), 4),
    ("frustrated 6x128 beta3 D4", lambda: fully_frustrated(6, 3.0, 4, Lx=128), 4),
]


@pytest.mark.parametrize("name,mk,D", ENV_CASES, ids=[c[0] for c in ENV_CASES])
def test_env_build_logZ(name, mk, D):
    from paper_2104_13264_amd import Sampler
    inst = mk()
    log(f"[env] {name} Ly={inst.Ly} Lx={inst.Lx} D={D}")
    ref = bmps.build_envs(model_of(inst), D)
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, D, FP64)
    assert abs(lz - ref['logZ']) <= TOL_LOGZ_FP64 * abs(ref['logZ']) + 1e-12
    st = s.stats()
    assert st['clamps'] == 0
    s.close()


SAMPLER_CASES = [
    ("4x4 D2 field", lambda: random_instance(4, 4, 0.9, 2, seed=11, field_scale=0.3), 2, 37),
    ("ragged 9x11 D5", lambda: random_instance(9, 11, 0.7, 5, seed=12, field_scale=0.2), 5, 53),
    ("ferro 16 D8", lambda: ferro(16, 0.4407, 8), 8, 40),
    ("ea 12 D20", lambda: ea_pm(12, 1.0, 20, seed=13), 20, 33),
    ("frustrated 10 D33", lambda: fully_frustrated(10, 1.0, 33), 33, 21),
    ("strip 1x9", lambda: random_instance(1, 9, 0.8, 4, seed=14), 4, 17),
    ("column 7x1", lambda: random_instance(7, 1, 0.8, 4, seed=15), 4, 17),
    ("ea 12 D64", lambda: ea_pm(12, 1.0, 64, seed=16), 64, 19),
    ("frustrated 6x128 beta3 D4", lambda: fully_frustrated(6, 3.0, 4, Lx=128), 4, 9),
    # the widest lattice (largest LDS tables of the batched kernels)
    ("wide 3x256 D32", lambda: random_instance(3, 256, 0.6, 32, seed=17, field_scale=0.1), 32, 40),
    ("wide 2x256 D64", lambda: random_instance(2, 256, 0.6, 64, seed=18), 64, 20),
]


@pytest.mark.parametrize("name,mk,D,B", SAMPLER_CASES, ids=[c[0] for c in SAMPLER_CASES])
def test_fp64_sampler_matches_oracle(name, mk, D, B):
    inst = mk()
    log(f"[fp64 sampler] {name} Ly={inst.Ly} Lx={inst.Lx} D={D} B={B}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, FP64)
    m = model_of(inst)
    seed, step, first = 987654321, 5, 11
    ref = sampler.sample(m, envs, B, seed, step=step, first_id=first)
    sp, lq, E = s.sample(B, seed, step=step, first_id=first)
    sp, lq, E = sp.cpu().numpy(), lq.cpu().numpy(), E.cpu().numpy()
    ok = ref['min_gap'] >= NEAR_FP64
    log(f"  near-threshold proposals excluded: {(~ok).sum()}")
    assert np.array_equal(sp[ok], ref['spins'][ok])
    assert np.all(np.abs(lq[ok] - ref['logq'][ok]) <= TOL_LOGZ_FP64 * np.abs(ref['logq'][ok]) + 1e-12)
    if inst.h is None and np.all(np.abs(inst.Jh) == 1) and np.all(np.abs(inst.Jv) == 1):
        assert np.array_equal(E[ok], ref['energy'][ok])
    else:
        np.testing.assert_allclose(E[ok], ref['energy'][ok], rtol=1e-12, atol=1e-12)
    # eval mode on the GPU's own draws reproduces its ln q bitwise
    lq2, E2 = s.eval_logq(torch.as_tensor(sp, device='cuda'))
    assert np.array_equal(lq2.cpu().numpy(), lq)
    # eval mode on arbitrary spins agrees with the oracle's eval
    rng = np.random.default_rng(3)
    rnd = rng.choice([-1, 1], size=(B, inst.Ly, inst.Lx)).astype(np.int8)
    lq3, _ = s.eval_logq(torch.as_tensor(rnd, device='cuda'))
    ev = sampler.eval_logq(m, envs, rnd)['logq']
    fin = np.isfinite(ev)
    np.testing.assert_allclose(lq3.cpu().numpy()[fin], ev[fin], rtol=TOL_LOGZ_FP64, atol=1e-12)
    s.close()


@pytest.mark.parametrize("name,mk,D,B", SAMPLER_CASES, ids=[c[0] for c in SAMPLER_CASES])
def test_fp32_sampler_matches_oracle(name, mk, D, B):
    inst = mk()
    log(f"[fp32 sampler] {name} Ly={inst.Ly} Lx={inst.Lx} D={D} B={B}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, FP32)
    m = model_of(inst)
    seed, step, first = 4242, 3, 100
    sp, lq, E = s.sample(B, seed, step=step, first_id=first)
    sp, lq, E = sp.cpu().numpy(), lq.cpu().numpy(), E.cpu().numpy()
    ev = sampler.eval_logq(m, envs, sp)
    np.testing.assert_allclose(lq, ev['logq'], rtol=TOL_LOGQ_FP32, atol=1e-9)
    np.testing.assert_allclose(E, ev['energy'], rtol=1e-13, atol=1e-12)
    ref = sampler.sample(m, envs, B, seed, step=step, first_id=first)
    same = np.all(sp == ref['spins'], axis=(1, 2))
    far = ref['min_gap'] >= 1e-4
    log(f"  identical proposals {same.sum()}/{B}; far-from-threshold {far.sum()}")
    assert np.all(same[far])
    lq2, _ = s.eval_logq(torch.as_tensor(sp, device='cuda'))
    assert np.array_equal(lq2.cpu().numpy(), lq)
    s.close()


def test_gpu_env_feeds_sampler():
    # the GPU-built environment gives the same ln q as the oracle's, on the
    # oracle's draws (gauge-invariant comparison)
    from paper_2104_13264_amd import Sampler
    inst = random_instance(10, 12, 0.8, 6, seed=21, field_scale=0.1)
    m = model_of(inst)
    envs = bmps.build_envs(m, 6)
    ref = sampler.sample(m, envs, 29, seed=77)
    for prec, tol in [(FP64, TOL_LOGZ_FP64), (FP32, TOL_LOGQ_FP32)]:
        s = Sampler()
        s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 6, prec)
        lq, E = s.eval_logq(torch.as_tensor(ref['spins'], device='cuda'))
        np.testing.assert_allclose(lq.cpu().numpy(), ref['logq'], rtol=tol, atol=1e-12)
        s.close()


def test_env_roundtrip_get_set():
    from paper_2104_13264_amd import Sampler
    inst = random_instance(6, 7, 0.8, 4, seed=31)
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 4, FP64)
    env, dims, ell, lz2 = s.get_env()
    assert lz2 == lz
    a = s.sample(19, 5)
    t = Sampler()
    t.set_env(inst.Jh, inst.Jv, inst.h, inst.beta, 4, env, dims, ell, lz)
    b = t.sample(19, 5)
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    s.close()
    t.close()


def test_mh_chain_small_ferro_matches_oracle():
    # 8x8 ferromagnet, beta 0.44, D 8, one chain of 1000 proposals from all up
    inst = small_ferro_8()
    log("[mh] 8x8 ferro D8 1 chain x 1000 steps")
    s, envs = gpu_sampler_with_oracle_env(inst, inst.D, FP64)
    m = model_of(inst)
    st_ref, acc_ref, E_ref = mh.run_chain(m, envs, 1, 1000, inst.seed)
    state = s.init_state(1)
    acc = []
    E = []
    for t in range(1000):
        s.mh_step(state, inst.seed, t)
        acc.append(int(state['accepted'][0]))
        E.append(float(state['energy'][0]))
    acc = np.array(acc, dtype=bool)
    assert np.array_equal(acc, acc_ref[:, 0])
    assert np.array_equal(np.array(E), E_ref[:, 0])
    assert np.array_equal(state['spins'].cpu().numpy(), st_ref['spins'])
    st = s.stats()
    assert st['proposed'] == 1000 and st['accepted'] == acc.sum()
    s.close()


def test_mh_fp32_chains_track_oracle_acceptance():
    inst = ferro(16, 0.4407, 8)
    s, envs = gpu_sampler_with_oracle_env(inst, 8, FP32)
    m = model_of(inst)
    chains, steps = 64, 20
    state = s.init_state(chains)
    st_ref = mh.init_state(m, envs, chains)
    ga, oa = 0, 0
    for t in range(steps):
        s.mh_step(state, SEED, t)
        acc, _, _ = mh.mh_step(m, envs, st_ref, SEED, t)
        ga += int(state['accepted'].sum())
        oa += int(acc.sum())
    assert abs(ga - oa) <= 0.01 * chains * steps + 2


def test_untruncated_gpu_accepts_everything():
    from paper_2104_13264_amd import Sampler
    inst = random_instance(4, 4, 0.9, 8, seed=41, field_scale=0.2)
    cfg, _, _, lp = exact.brute_force(inst.Jh, inst.Jv, inst.h, inst.beta)
    for prec, tol in [(FP64, 1e-11), (FP32, 1e-5)]:
        s = Sampler()
        s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 8, prec)
        lq, _ = s.eval_logq(torch.as_tensor(cfg, device='cuda'))
        np.testing.assert_allclose(lq.cpu().numpy(), lp, rtol=0, atol=tol * 20)
        state = s.init_state(64)
        for t in range(5):
            s.mh_step(state, 9, t)
            if prec == FP64:
                assert bool(state['accepted'].all())
        s.close()


def test_negative_weight_clamps_counted():
    inst = random_instance(4, 5, 3.0, 3, seed=16)
    s, envs = gpu_sampler_with_oracle_env(inst, 3, FP64)
    m = model_of(inst)
    ref = sampler.sample(m, envs, 50, seed=1)
    sp, lq, _ = s.sample(50, 1)
    st = s.stats()
    ok = ref['min_gap'] >= NEAR_FP64
    assert np.array_equal(sp.cpu().numpy()[ok], ref['spins'][ok])
    assert st['clamps'] >= ref['clamps'][ok].sum() > 0
    assert st['both_nonpos'] >= ref['both_nonpos'][ok].sum()
    s.close()


def test_empty_batch_and_errors():
    from paper_2104_13264_amd import Sampler, TNError
    s = Sampler()
    with pytest.raises(TNError):
        s._check(__import__('paper_2104_13264_amd').lib().tn_sample(
            s._ctx, 1, 0, 0, 0, None, None, None))
    inst = random_instance(3, 3, 0.5, 2, seed=1)
    with pytest.raises(TNError):
        s.build_env(inst.Jh, inst.Jv, None, inst.beta, 0)
    with pytest.raises(TNError):
        s.build_env(inst.Jh, inst.Jv, None, float('nan'), 2)
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, 2)
    sp, lq, E = s.sample(0, 1)
    assert sp.shape[0] == 0
    s.close()


def test_full_size_ferro64_sampled_parity():
    # 64x64 ferromagnet at beta 0.4407 with D 32, 4096 proposals in one launch
    # (the benchmarked configuration); 16 sampled proposals checked one by one
    from paper_2104_13264_amd import Sampler
    inst = ferro_64()
    log("[full] 64x64 D32 build + 4096 proposals")
    ref_env = bmps.build_envs(model_of(inst), 32)
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, None, inst.beta, 32, FP32)
    log(f"  env build {s.stats()['env_build_ms']:.1f} ms, ln Z~ {lz!r} vs {ref_env['logZ']!r}")
    assert abs(lz - ref_env['logZ']) <= TOL_LOGZ_FP64 * abs(ref_env['logZ'])
    sp, lq, E = s.sample(4096, SEED, step=0)
    pick = np.arange(0, 4096, 257)
    sps = sp.cpu().numpy()[pick]
    ev = sampler.eval_logq(model_of(inst), ref_env, sps)
    np.testing.assert_allclose(lq.cpu().numpy()[pick], ev['logq'], rtol=TOL_LOGQ_FP32)
    assert np.array_equal(E.cpu().numpy()[pick], ev['energy'])
    s.close()


@pytest.mark.parametrize("prec", [FP64, FP32, BF16], ids=["fp64", "fp32", "bf16"])
def test_sample_steps_equals_per_step_sampling(prec):
    # proposals of several MH steps in one launch are bitwise the per-step ones
    # (ragged chain count: the steps split inside a 16-proposal workgroup)
    inst = random_instance(7, 9, 0.6, 6, seed=51, field_scale=0.2)
    log(f"[steps] 7x9 D6 prec {prec}")
    s, envs = gpu_sampler_with_oracle_env(inst, 6, prec)
    chains, nsteps, seed, step0, first = 37, 3, 99, 11, 5
    sp, lq, E = s.sample_steps(chains, nsteps, seed, step0=step0, first_id=first)
    for t in range(nsteps):
        a, b, c = s.sample(chains, seed, step=step0 + t, first_id=first)
        assert torch.equal(sp[t], a)
        assert torch.equal(lq[t], b)
        assert torch.equal(E[t], c)
    s.close()


@pytest.mark.parametrize("prec", [FP64, FP32], ids=["fp64", "fp32"])
def test_mh_run_equals_mh_steps(prec):
    inst = random_instance(6, 8, 0.7, 5, seed=52)
    log(f"[mh_run] 6x8 D5 prec {prec}")
    s, envs = gpu_sampler_with_oracle_env(inst, 5, prec)
    chains, nsteps, seed = 45, 7, 123
    st1 = s.init_state(chains)
    st2 = s.init_state(chains)
    acc, es = s.mh_run(st1, seed, 3, nsteps)
    for t in range(nsteps):
        s.mh_step(st2, seed, 3 + t)
        assert torch.equal(acc[t], st2['accepted'])
        assert torch.equal(es[t], st2['energy'])
    for k in ("spins", "logq", "energy"):
        assert torch.equal(st1[k], st2[k])
    s.close()


def test_sample_steps_rejects_bad_sizes():
    from paper_2104_13264_amd import TNError
    inst = random_instance(3, 4, 0.5, 4, seed=53)
    s, _ = gpu_sampler_with_oracle_env(inst, 4, FP32)
    with pytest.raises(TNError):
        s.sample_steps(8, 0, 1)
    s.close()


def test_incremental_build_equals_one_call():
    from paper_2104_13264_amd import Sampler, TNError
    inst = random_instance(9, 8, 0.7, 6, seed=54, field_scale=0.1)
    a = Sampler()
    lza = a.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 6, FP32)
    b = Sampler()
    seen = []
    lzb = b.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 6, FP32,
                      progress=lambda done, tot: seen.append((done, tot)), rows_per_call=3)
    assert lza == lzb and seen[-1] == (8, 8) and len(seen) == 3
    for x, y in zip(a.get_env()[:3], b.get_env()[:3]):
        assert np.array_equal(x, y)
    pa, pb = a.sample(20, 3), b.sample(20, 3)
    for x, y in zip(pa, pb):
        assert torch.equal(x, y)
    # calls on a context whose build is open fail
    from paper_2104_13264_amd.tnmh import lib, _ptr, _dev64
    Jh, Jv = _dev64(inst.Jh, b.device), _dev64(inst.Jv, b.device)
    assert lib().tn_build_env_begin(b._ctx, 8, 9, _ptr(Jh), _ptr(Jv), None, 0.7, 6, FP32) == 0
    with pytest.raises(TNError):
        b.sample(4, 1)
    a.close()
    b.close()


BF16_CASES = [
    ("ragged 9x11 D5", lambda: random_instance(9, 11, 0.7, 5, seed=12, field_scale=0.2), 5, 53),
    ("ea 12 D20", lambda: ea_pm(12, 1.0, 20, seed=13), 20, 33),
    ("frustrated 10 D33", lambda: fully_frustrated(10, 1.0, 33), 33, 21),
    ("ea 12 D64", lambda: ea_pm(12, 1.0, 64, seed=16), 64, 19),
    ("wide 3x256 D32", lambda: random_instance(3, 256, 0.6, 32, seed=17, field_scale=0.1), 32, 40),
    ("wide 2x256 D64", lambda: random_instance(2, 256, 0.6, 64, seed=18), 64, 20),
]


@pytest.mark.parametrize("name,mk,D,B", BF16_CASES, ids=[c[0] for c in BF16_CASES])
def test_bf16_sampler_against_oracle(name, mk, D, B):
    # BF16 operands (8 significant bits, unit roundoff u = 2^-8) with fp32
    # accumulation: every column step rounds the carried row vector and the
    # environment tiles once, so over the 2*Lx*Ly roundings along a
    # configuration the ln q error behaves like u*sqrt(2*Lx*Ly) when the
    # rounding errors are independent; the bound below allows 8 times that.
    # What must hold exactly: ln q of a drawn configuration is the value the
    # BF16 arithmetic gives when it evaluates that configuration again.
    inst = mk()
    log(f"[bf16 sampler] {name} Ly={inst.Ly} Lx={inst.Lx} D={D} B={B}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, BF16)
    m = model_of(inst)
    sp, lq, E = s.sample(B, 777, step=2, first_id=9)
    lq2, E2 = s.eval_logq(sp)
    assert torch.equal(lq2, lq) and torch.equal(E2, E)
    sp, lq, E = sp.cpu().numpy(), lq.cpu().numpy(), E.cpu().numpy()
    ev = sampler.eval_logq(m, envs, sp)
    np.testing.assert_allclose(E, ev['energy'], rtol=1e-13, atol=1e-12)
    bound = 8 * 2.0 ** -8 * np.sqrt(2 * inst.Lx * inst.Ly)
    dev = np.abs(lq - ev['logq'])
    log(f"  max |ln q_bf16 - ln q_fp64| {dev.max():.3e} (mean {dev.mean():.3e}, bound {bound:.3e})")
    assert np.all(np.isfinite(lq)) and dev.max() <= bound
    s.close()


@pytest.mark.parametrize("prec", [FP64, FP32, BF16], ids=["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("D", [8, 24, 40, 64])
def test_beta0_spins_follow_the_philox_stream(prec, D):
    # at beta = 0 both spins of every site weigh exactly the same in any
    # precision, so p+ = 1/2 exactly and every spin is fixed by its random word
    # alone: the batched kernels of every bond class (the row's words drawn in
    # LDS or as the row goes) must reproduce the oracle's spins bit for bit,
    # with ln q = N ln(1/2)
    inst = random_instance(9, 11, 0.0, D, seed=61)
    log(f"[beta0] 9x11 D={D} prec {prec}")
    s, envs = gpu_sampler_with_oracle_env(inst, D, prec)
    B, seed, step, first = 70, 31, 5, 3
    sp, lq, _ = s.sample(B, seed, step=step, first_id=first)
    ref = sampler.sample(model_of(inst), envs, B, seed, step=step, first_id=first)
    assert np.array_equal(sp.cpu().numpy(), ref['spins'])
    np.testing.assert_allclose(lq.cpu().numpy(), 99 * np.log(0.5), rtol=1e-12)
    steps = s.sample_steps(B, 3, seed, step0=step, first_id=first)
    for t in range(3):
        r = sampler.sample(model_of(inst), envs, B, seed, step=step + t, first_id=first)
        assert np.array_equal(steps[0][t].cpu().numpy(), r['spins'])
    s.close()
