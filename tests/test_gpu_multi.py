"""Batched uneven instances (tn_build_env_multi, tn_mh_step_multi) and HIP
graph replay (tn_graph_begin / tn_graph_end_and_replay).

ln Z~ of every instance within 1e-9 relative of the oracle; batched MH steps
bitwise the per-instance steps on the same environments; graph replays
bitwise the eager steps, every replay checked.
"""
import numpy as np
import pytest
import torch

from oracle import bmps
from workloads import random_instance, ea_pm, ferro
from bridge import model_of, TOL_LOGZ_FP64

pytestmark = pytest.mark.gpu

FP64, FP32, BF16 = 0, 1, 2


def log(msg):
    print(msg, flush=True)


def mixed_instances():
    # uneven sizes, bond caps in all four 16-wide classes, betas, fields, chains
    out = [
        (random_instance(6, 9, 0.7, 5, seed=61, field_scale=0.2), 5, 37),
        (ea_pm(10, 1.0, 12, seed=62), 12, 21),
        (random_instance(9, 7, 0.5, 24, seed=63), 24, 16),
        (ferro(8, 0.4407, 40), 40, 9),
        (ea_pm(7, 2.0, 50, seed=64), 50, 18),
    ]
    return out


def as_dicts(items):
    return [dict(Jh=i.Jh, Jv=i.Jv, h=i.h, beta=i.beta, D=D, chains=C) for i, D, C in items]


def clone(st):
    return {k: v.clone() for k, v in st.items()}


@pytest.mark.parametrize("prec", [FP32, FP64, BF16], ids=["fp32", "fp64", "bf16"])
def test_multi_env_matches_oracle_and_steps_match_single(prec):
    from paper_2104_13264_amd import Sampler
    items = mixed_instances()
    log(f"[multi] {len(items)} instances prec {prec}")
    s = Sampler()
    lz = s.build_env_multi(as_dicts(items), prec)
    for (inst, D, C), z in zip(items, lz):
        ref = bmps.build_envs(model_of(inst), D)['logZ']
        assert abs(z - ref) <= TOL_LOGZ_FP64 * abs(ref), (inst.Ly, inst.Lx, D, z, ref)
    subs = [s.instance(i) for i in range(len(items))]
    sa = [sub.init_state(C) for sub, (_, _, C) in zip(subs, items)]
    sb = [clone(x) for x in sa]
    seed = 7
    for t in range(4):
        s.mh_step_multi(sa, seed, t)
        for sub, st in zip(subs, sb):
            sub.mh_step(st, seed, t)
        for x, y in zip(sa, sb):
            for k in ("spins", "logq", "energy", "accepted"):
                assert torch.equal(x[k], y[k])
    s.close()


def test_multi_graph_replays_match_eager():
    from paper_2104_13264_amd import Sampler
    items = mixed_instances()[:3]
    stream = torch.cuda.Stream()
    s = Sampler(stream=stream)
    s.build_env_multi(as_dicts(items), FP32)
    subs = [s.instance(i) for i in range(len(items))]
    with torch.cuda.stream(stream):
        ga = [sub.init_state(C) for sub, (_, _, C) in zip(subs, items)]
        ea = [clone(x) for x in ga]
    stream.synchronize()
    seed, t = 11, 0
    # eager first call with the same buffers (allocations happen here)
    s.mh_step_multi(ga, seed, t)
    s.mh_step_multi(ea, seed, t)
    t += 1
    for cycle, (nstep, nrep) in enumerate([(2, 1), (1, 1), (2, 3)]):
        log(f"[graph] cycle {cycle}: {nstep} captured steps x {nrep} replays")
        s.graph_begin()
        for j in range(nstep):
            s.mh_step_multi(ga, seed, t + j)
        s.graph_end_and_replay(nrep)
        for j in range(nstep * nrep):
            s.mh_step_multi(ea, seed, t + j)
        stream.synchronize()
        for x, y in zip(ga, ea):
            for k in ("spins", "logq", "energy", "accepted"):
                assert torch.equal(x[k], y[k])
        t += nstep * nrep
    s.close()


def test_single_instance_graph_replay_matches_eager():
    from paper_2104_13264_amd import Sampler
    inst = random_instance(8, 8, 0.6, 8, seed=65)
    stream = torch.cuda.Stream()
    s = Sampler(stream=stream)
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 8, FP32)
    with torch.cuda.stream(stream):
        a = s.init_state(50)
        b = clone(a)
    stream.synchronize()
    s.mh_step(a, 3, 0)
    s.mh_step(b, 3, 0)
    for rep in range(2):
        s.graph_begin()
        s.mh_step(a, 3, 1 + 3 * rep)
        s.graph_end_and_replay(3)
        for j in range(3):
            s.mh_step(b, 3, 1 + 3 * rep + j)
        stream.synchronize()
        for k in ("spins", "logq", "energy", "accepted"):
            assert torch.equal(a[k], b[k])
    s.close()


def test_graph_capture_refuses_allocation():
    from paper_2104_13264_amd import Sampler, TNError
    inst = random_instance(5, 6, 0.6, 4, seed=66)
    stream = torch.cuda.Stream()
    s = Sampler(stream=stream)
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 4, FP32)
    with torch.cuda.stream(stream):
        a = s.init_state(20)
    stream.synchronize()
    s.graph_begin()
    with pytest.raises(TNError):
        s.mh_step(a, 1, 0)   # first call: its buffers would be allocated
    s.graph_end_and_replay(0)   # closes the (empty) capture
    with pytest.raises(TNError):
        s.graph_end_and_replay(1)   # no capture open
    s.mh_step(a, 1, 0)   # eager works again
    stream.synchronize()
    s.close()


def test_graph_capture_refuses_calls_other_than_mh_steps():
    # Only MH steps may be captured: the other calls' random streams would not
    # follow the replays' step shift, or they synchronise or allocate.  Each
    # is refused (TN_ESTATE) without enqueuing work, and the captured steps
    # still replay bitwise like the eager ones.  The calls go straight to the
    # C ABI with buffers allocated before the capture.
    import ctypes
    from paper_2104_13264_amd import Sampler
    from paper_2104_13264_amd.tnmh import lib, _ptr, _Stats
    TN_ESTATE = -6
    inst = random_instance(6, 7, 0.6, 4, seed=67)
    stream = torch.cuda.Stream()
    s = Sampler(stream=stream)
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 4, FP32)
    C = 24
    with torch.cuda.stream(stream):
        a = s.init_state(C)
        b = clone(a)
        sp, lq, E = s.empty_batch(2 * C)
        q = torch.empty(C, dtype=torch.int32, device=s.device)
        acc = torch.empty(2 * C, dtype=torch.uint8, device=s.device)
        dJh = torch.empty((inst.Ly, inst.Lx - 1), dtype=torch.float64, device=s.device)
        dJv = torch.empty((inst.Ly - 1, inst.Lx), dtype=torch.float64, device=s.device)
    stream.synchronize()
    s.mh_step(a, 5, 0)
    s.mh_step(b, 5, 0)
    L, ctx = lib(), s._ctx
    st = (_ptr(b["spins"]), _ptr(b["logq"]), _ptr(b["energy"]))
    db = ctypes.c_double()
    stats = _Stats()
    refused = {
        "tn_sample": lambda: L.tn_sample(ctx, C, 5, 9, 0, _ptr(sp), _ptr(lq), _ptr(E)),
        "tn_sample_steps": lambda: L.tn_sample_steps(ctx, C, 2, 5, 9, 0, _ptr(sp), _ptr(lq), _ptr(E)),
        "tn_eval_logq": lambda: L.tn_eval_logq(ctx, C, _ptr(a["spins"]), _ptr(lq), _ptr(E)),
        "tn_mh_accept": lambda: L.tn_mh_accept(ctx, C, 5, 9, _ptr(sp), _ptr(lq), _ptr(E), *st, _ptr(acc)),
        "tn_mh_run": lambda: L.tn_mh_run(ctx, C, 2, 5, 9, *st, _ptr(acc), None),
        "tn_metropolis_sweeps": lambda: L.tn_metropolis_sweeps(ctx, C, 1, 5, 9, *st),
        "tn_link_overlap": lambda: L.tn_link_overlap(ctx, C, _ptr(a["spins"]), _ptr(b["spins"]), _ptr(q)),
        "tn_stats": lambda: L.tn_stats(ctx, ctypes.byref(stats), 0),
        "tn_grad": lambda: L.tn_grad(ctx, _ptr(dJh), _ptr(dJv), ctypes.byref(db)),
    }
    s.graph_begin()
    s.mh_step(a, 5, 1)
    codes = {name: call() for name, call in refused.items()}
    s.graph_end_and_replay(2)
    log(f"[graph] return codes while capturing: {codes}")
    assert all(rc == TN_ESTATE for rc in codes.values()), codes
    for j in range(2):
        s.mh_step(b, 5, 1 + j)
    stream.synchronize()
    for k in ("spins", "logq", "energy", "accepted"):
        assert torch.equal(a[k], b[k])
    s.close()


def test_multi_step_refuses_fp64_mfma_instance():
    # An instance switched to FP64 operands on the matrix cores has no batched
    # sampler group: the step and its tuner refuse it instead of running a
    # group's kernel on its operand layout; switched back, the step works.
    from paper_2104_13264_amd import Sampler, TNError, FP64_MFMA
    items = [random_instance(5, 6, 0.6, 8, seed=68), random_instance(6, 5, 0.7, 8, seed=69)]
    s = Sampler()
    s.build_env_multi([dict(Jh=i.Jh, Jv=i.Jv, h=i.h, beta=i.beta, D=8, chains=16) for i in items], FP32)
    subs = [s.instance(k) for k in range(len(items))]
    st = [sub.init_state(16) for sub in subs]
    subs[1].set_precision(FP64_MFMA)
    with pytest.raises(TNError):
        s.mh_step_multi(st, 3, 0)
    with pytest.raises(TNError):
        s.autotune_multi()
    subs[1].set_precision(FP32)
    s.mh_step_multi(st, 3, 0)
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(x["logq"]).all()) for x in st)
    s.close()
