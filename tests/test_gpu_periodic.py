"""Periodic boundaries by frozen lines on the GPU (tn_periodic_*) against the
oracle.

* FP64: chains on a torus and on cylinders along x and y, several instances
  of uneven chain counts, with and without fields, follow the oracle's chains
  step by step: spins and accept flags bitwise (draws within ~1e-15 of a
  threshold could differ; none is expected), periodic energies to 1e-12.
* FP32 / BF16: two steps of every chain equal what the open-boundary entry
  points give on the chain's open model (couplings and fields from the
  oracle's cut, built by tn_build_env; proposal id j and instance m; the
  oracle's acceptance rule on their ln q and energies), bitwise, also on a
  32x32 torus with 2 x 30 chains sampled at a few chains; the frozen lines
  never move.
* No truncation: every proposal accepted.  Energies and link overlaps of the
  periodic lattice exact against the oracle.  Errors: a step before set-up, a
  cut out of range, a wrapped direction of two sites.
"""
import numpy as np
import pytest
import torch

from oracle import periodic
from oracle.mh import accept_uniforms, mh_decide
from workloads import periodic_couplings

pytestmark = pytest.mark.gpu

FP64, FP32, BF16 = 0, 1, 2


def log(msg):
    print(msg, flush=True)


def instances(Ly, Lx, wx, wy, chains, seed, beta=(0.9, 0.5)):
    out = []
    for k, C in enumerate(chains):
        c = periodic_couplings(Ly, Lx, wx, wy, seed + k, gaussian=(k % 2 == 0),
                               field_scale=0.4 if k % 2 == 0 else 0.0)
        out.append(dict(c, beta=beta[k % len(beta)], chains=C))
    return out


def cuts(t, Ly, Lx):
    return (3 * t + 1) % Ly, (5 * t + 2) % Lx


FP64_CASES = [  # (Ly, Lx, wrap_x, wrap_y, D, chains per instance)
    (7, 8, True, True, 4, (5, 7)),
    (6, 9, True, False, 3, (4, 1, 6)),
    (9, 5, False, True, 4, (8,)),
]


@pytest.mark.parametrize("case", range(len(FP64_CASES)))
def test_fp64_chains_follow_the_oracle(case):
    from paper_2104_13264_amd import Sampler
    Ly, Lx, wx, wy, D, chains = FP64_CASES[case]
    log(f"[periodic] fp64 {Ly}x{Lx} wrap=({wx},{wy}) D={D} chains={chains}")
    inst = instances(Ly, Lx, wx, wy, chains, seed=500 + 10 * case)
    T = sum(chains)
    rng = np.random.default_rng(case)
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=(T, Ly, Lx))
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, wx, wy, D, FP64)
    spins = torch.as_tensor(s0, device=s.device).contiguous()
    ref = s0.copy()
    seed = 77 + case
    for t in range(4):
        cr, cc = cuts(t, Ly, Lx)
        E, acc = s.periodic_step(spins, seed, t, cr, cc)
        ref, Eref, accref = periodic.step(inst, ref, seed, t, cr, cc, D, wx, wy)
        np.testing.assert_array_equal(acc.cpu().numpy().astype(bool), accref)
        np.testing.assert_array_equal(spins.cpu().numpy(), ref)
        np.testing.assert_allclose(E.cpu().numpy(), Eref, rtol=1e-13, atol=1e-12)
    st = s.stats()
    assert st["proposed"] == 4 * T
    s.close()


def open_context_step(inst, spins, m, j, seed, t, cr, cc, D, prec, wx, wy):
    """Chain j of instance m after one step, from the open-boundary entry
    points on the chain's open model and the oracle's acceptance rule."""
    from paper_2104_13264_amd import Sampler
    it = inst[m]
    model, rows, cols = periodic.cut_model(it["Jh"], it["Jv"], it.get("h"), it["beta"], spins, cr, cc, wx, wy)
    o = Sampler()
    o.build_env(model.Jh, model.Jv, model.h, model.beta, D, prec)
    o.set_instance(m)
    cur = torch.as_tensor(spins[np.ix_(rows, cols)][None], device=o.device).contiguous()
    lq_c, E_c = o.eval_logq(cur)
    sp, lq_p, E_p = o.sample(1, seed, step=t, first_id=j)
    u = accept_uniforms(it["chains"], seed, t, inst=m)[j:j + 1]
    ok, _ = mh_decide(lq_c.cpu().numpy(), E_c.cpu().numpy(), lq_p.cpu().numpy(), E_p.cpu().numpy(),
                      model.beta, u)
    out = spins.copy()
    if ok[0]:
        out[np.ix_(rows, cols)] = sp.cpu().numpy()[0]
    o.close()
    return out, bool(ok[0])


BATCHED_CASES = [  # (Ly, Lx, wrap_x, wrap_y, D, precision, chains, chains checked per instance)
    (8, 9, True, True, 16, FP32, (6, 3), None),
    (7, 10, True, False, 24, BF16, (5,), None),
    (10, 6, False, True, 40, FP32, (4, 2), None),
    (32, 32, True, True, 16, FP32, (30, 30), (0, 17, 29)),
]


@pytest.mark.parametrize("case", range(len(BATCHED_CASES)))
def test_batched_step_equals_open_contexts(case):
    from paper_2104_13264_amd import Sampler
    Ly, Lx, wx, wy, D, prec, chains, check = BATCHED_CASES[case]
    log(f"[periodic] batched {Ly}x{Lx} wrap=({wx},{wy}) D={D} prec={prec} chains={chains}")
    inst = instances(Ly, Lx, wx, wy, chains, seed=600 + 10 * case, beta=(1.2, 0.7))
    T = sum(chains)
    rng = np.random.default_rng(100 + case)
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=(T, Ly, Lx))
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, wx, wy, D, prec)
    spins = torch.as_tensor(s0, device=s.device).contiguous()
    seed = 31 + case
    # two steps: the first builds every chain's operands one chain at a time
    # (allocating them), later steps in one batched launch pair
    for t in (5, 6):
        before = spins.cpu().numpy()
        cr, cc = cuts(case + t, Ly, Lx)
        E, acc = s.periodic_step(spins, seed, t, cr, cc)
        got = spins.cpu().numpy()
        acc = acc.cpu().numpy()
        if wx:
            np.testing.assert_array_equal(got[:, :, cc], before[:, :, cc])
        if wy:
            np.testing.assert_array_equal(got[:, cr, :], before[:, cr, :])
        g0 = 0
        for m, C in enumerate(chains):
            np.testing.assert_allclose(
                E.cpu().numpy()[g0:g0 + C],
                periodic.energy(got[g0:g0 + C], inst[m]["Jh"], inst[m]["Jv"], inst[m].get("h"), wx, wy),
                rtol=1e-13, atol=1e-12)
            for j in (check if check is not None else range(C)):
                want, ok = open_context_step(inst, before[g0 + j], m, j, seed, t, cr, cc, D, prec, wx, wy)
                assert bool(acc[g0 + j]) == ok, (t, m, j)
                np.testing.assert_array_equal(got[g0 + j], want, err_msg=f"step {t} instance {m} chain {j}")
            g0 += C
        assert 0 < acc.sum()
    s.close()


def test_untruncated_steps_accept_everything():
    from paper_2104_13264_amd import Sampler
    Ly, Lx = 5, 4
    inst = instances(Ly, Lx, True, True, (6, 3), seed=700)
    log("[periodic] untruncated 5x4 torus D=16")
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, True, True, 16, FP64)
    rng = np.random.default_rng(9)
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=(9, Ly, Lx))
    spins = torch.as_tensor(s0, device=s.device).contiguous()
    for t in range(3):
        _, acc = s.periodic_step(spins, 3, t, *cuts(t, Ly, Lx))
        assert acc.cpu().numpy().all()
    assert (spins.cpu().numpy() != s0).any()
    s.close()


@pytest.mark.parametrize("wrap", [(True, True), (True, False), (False, True)], ids=["torus", "cyl_x", "cyl_y"])
def test_energy_and_link_overlap(wrap):
    from paper_2104_13264_amd import Sampler
    wx, wy = wrap
    Ly, Lx = 11, 13
    inst = instances(Ly, Lx, wx, wy, (4, 5), seed=800)
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, wx, wy, 4, FP32)
    rng = np.random.default_rng(1)
    a = rng.choice(np.array([-1, 1], dtype=np.int8), size=(9, Ly, Lx))
    b = rng.choice(np.array([-1, 1], dtype=np.int8), size=(9, Ly, Lx))
    E = s.periodic_energy(torch.as_tensor(a, device=s.device)).cpu().numpy()
    np.testing.assert_allclose(E[:4], periodic.energy(a[:4], inst[0]["Jh"], inst[0]["Jv"], inst[0]["h"], wx, wy),
                               rtol=1e-13, atol=1e-12)
    np.testing.assert_array_equal(E[4:], periodic.energy(a[4:], inst[1]["Jh"], inst[1]["Jv"], None, wx, wy))
    q = s.periodic_link_overlap(torch.as_tensor(a, device=s.device), torch.as_tensor(b, device=s.device))
    np.testing.assert_array_equal(q.cpu().numpy(), periodic.link_overlap(a, b, wx, wy))
    s.close()


def test_errors():
    from paper_2104_13264_amd import Sampler, TNError
    s = Sampler()
    spins = torch.ones((2, 4, 4), dtype=torch.int8, device=s.device)
    with pytest.raises(TNError):
        s.periodic_step(spins, 1, 0, 0, 0)
    with pytest.raises(TNError):
        s.periodic_setup(instances(4, 2, True, False, (2,), seed=1), 2, 4, True, False, 4, FP32)
    s.periodic_setup(instances(4, 4, True, True, (2,), seed=1), 4, 4, True, True, 4, FP32)
    with pytest.raises(TNError):
        s.periodic_step(spins, 1, 0, 4, 0)
    with pytest.raises(TNError):
        s.periodic_step(spins, 1, 0, 0, -1)
    s.periodic_step(spins, 1, 0, 3, 3)
    s.close()


@pytest.mark.parametrize("wrap", [(True, True), (True, False), (False, True)], ids=["torus", "cyl_x", "cyl_y"])
def test_periodic_sweeps_match_oracle(wrap):
    from paper_2104_13264_amd import Sampler
    wx, wy = wrap
    Ly, Lx = 10, 12
    inst = instances(Ly, Lx, wx, wy, (5, 8), seed=900, beta=(1.3, 0.6))
    log(f"[periodic] sweeps {Ly}x{Lx} wrap=({wx},{wy})")
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, wx, wy, 4, FP32)
    rng = np.random.default_rng(21)
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=(13, Ly, Lx))
    spins = torch.as_tensor(s0, device=s.device).contiguous()
    s.stats(reset=True)
    E = s.periodic_sweeps(spins, 3, 55, 7)
    ref, flips = periodic.sweeps(inst, s0, 55, 7, 3, wx, wy)
    np.testing.assert_array_equal(spins.cpu().numpy(), ref)
    assert s.stats()["metropolis_flips"] == int(flips.sum())
    g0 = 0
    for it in inst:
        C = it["chains"]
        np.testing.assert_allclose(E.cpu().numpy()[g0:g0 + C],
                                   periodic.energy(ref[g0:g0 + C], it["Jh"], it["Jv"], it.get("h"), wx, wy),
                                   rtol=1e-13, atol=1e-12)
        g0 += C
    s.close()


def test_periodic_sweeps_refuse_odd_wrapped_lengths():
    from paper_2104_13264_amd import Sampler, TNError
    s = Sampler()
    s.periodic_setup(instances(6, 5, True, False, (2,), seed=3), 5, 6, True, False, 4, FP32)
    spins = torch.ones((2, 6, 5), dtype=torch.int8, device=s.device)
    with pytest.raises(TNError):
        s.periodic_sweeps(spins, 1, 1, 0)
    s.close()


EDGE_CASES = [  # (Ly, Lx, wrap_x, wrap_y, D, precision, chains per instance)
    (3, 3, True, True, 2, FP64, (4, 0, 3)),      # smallest torus (open 2x2), an instance without chains
    (5, 4, True, False, 2, FP64, (0, 5)),        # the first instance without chains
    (2, 257, True, False, 4, FP32, (3,)),        # widest open lattice: 256 columns
]


@pytest.mark.parametrize("case", range(len(EDGE_CASES)))
def test_edge_shapes(case):
    from paper_2104_13264_amd import Sampler
    Ly, Lx, wx, wy, D, prec, chains = EDGE_CASES[case]
    log(f"[periodic] edge {Ly}x{Lx} wrap=({wx},{wy}) D={D} prec={prec} chains={chains}")
    inst = instances(Ly, Lx, wx, wy, chains, seed=950 + case, beta=(1.1, 0.6))
    T = sum(chains)
    rng = np.random.default_rng(30 + case)
    s0 = rng.choice(np.array([-1, 1], dtype=np.int8), size=(T, Ly, Lx))
    s = Sampler()
    s.periodic_setup(inst, Lx, Ly, wx, wy, D, prec)
    spins = torch.as_tensor(s0, device=s.device).contiguous()
    ref = s0.copy()
    for t in range(2):
        cr, cc = cuts(t, Ly, Lx)
        before = spins.cpu().numpy()
        E, acc = s.periodic_step(spins, 13, t, cr, cc)
        got = spins.cpu().numpy()
        if prec == FP64:
            ref, Eref, accref = periodic.step(inst, ref, 13, t, cr, cc, D, wx, wy)
            np.testing.assert_array_equal(got, ref)
            np.testing.assert_array_equal(acc.cpu().numpy().astype(bool), accref)
            np.testing.assert_allclose(E.cpu().numpy(), Eref, rtol=1e-13, atol=1e-12)
        else:
            for j in range(T):
                want, ok = open_context_step(inst, before[j], 0, j, 13, t, cr, cc, D, prec, wx, wy)
                assert bool(acc.cpu().numpy()[j]) == ok
                np.testing.assert_array_equal(got[j], want)
    s.close()
