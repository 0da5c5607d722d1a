"""The frozen contraction at other couplings (tn_logz_frozen) and the check of
tn_grad by central finite differences of it.

* ln Z~_frozen at perturbed couplings, fields and beta within 1e-9 relative of
  the oracle's frozen_logZ (oracle/grad.py), whose projectors come from the
  oracle's own build, on builds without degenerate cuts; at the build's
  couplings it equals ln Z~ (also with degenerate cuts, where the projectors
  themselves are picked by rounding).
* The differentiation workload: 128 x 128 fully frustrated lattice (one
  negative bond per plaquette), beta = 1, D = 32.  d ln Z~/dJ from tn_grad on
  32 bonds picked by Philox against central differences of ln Z~_frozen with
  step 1e-4 (64 evaluations in one batched build), and d ln Z~/d beta the
  same way: relative error below 1e-6.
"""
import numpy as np
import pytest

from oracle import bmps, grad, ising
from oracle.philox import philox4x32_10, seed_key
from workloads import random_instance, fully_frustrated, ea_pm, SEED

pytestmark = pytest.mark.gpu


def log(msg):
    print(msg, flush=True)


CASES = [
    ("9x10 D4", lambda: random_instance(9, 10, 0.7, 4, seed=8), 4),
    ("12x16 D8 field", lambda: random_instance(12, 16, 0.6, 8, seed=81, field_scale=0.3), 8),
    ("ea 12 D8 beta1", lambda: ea_pm(12, 1.0, 8, seed=5), 8),
    ("frustrated 6x128 beta3 D4", lambda: fully_frustrated(6, 3.0, 4, Lx=128), 4),
    ("11x9 D40", lambda: random_instance(11, 9, 0.5, 40, seed=83), 40),
]


@pytest.mark.parametrize("name,mk,D", CASES, ids=[c[0] for c in CASES])
def test_frozen_contraction_matches_oracle(name, mk, D):
    from paper_2104_13264_amd import Sampler
    inst = mk()
    log(f"[frozen] {name} Ly={inst.Ly} Lx={inst.Lx} D={D}")
    m = ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)
    env = bmps.build_envs(m, D)
    assert sum(env["degenerate"]) == 0   # the frozen projectors are defined by the build
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, D)
    rng = np.random.default_rng(7)
    sets = [(inst.Jh, inst.Jv, inst.h, inst.beta)]
    for k in range(3):
        Jh = inst.Jh + 0.05 * rng.standard_normal(inst.Jh.shape)
        Jv = inst.Jv + 0.05 * rng.standard_normal(inst.Jv.shape)
        h = None if inst.h is None else inst.h + 0.05 * rng.standard_normal(inst.h.shape)
        sets.append((Jh, Jv, h, inst.beta * (1.0 + 0.02 * (k - 1))))
    got = s.logz_frozen(sets)
    assert abs(got[0] - lz) <= 1e-12 * abs(lz), (got[0], lz)
    for (Jh, Jv, h, beta), g in zip(sets, got):
        want = grad.frozen_logZ(ising.Model(Jh, Jv, h, beta), env)
        log(f"  ln Z~_frozen {g!r} oracle {want!r}")
        assert abs(g - want) <= 1e-9 * abs(want)
    # a second call with fewer sets reuses the evaluation contexts
    again = s.logz_frozen(sets[1:3])
    assert again == got[1:3]
    s.close()


def test_frozen_contraction_with_degenerate_cuts():
    # +-J couplings at beta = 2: tied singular values at the cuts (counted by
    # the oracle), where rounding picks the kept vectors and so the frozen
    # projectors; the frozen contraction is then defined only at the build's
    # own couplings, where it equals ln Z~ whichever vectors were kept.
    from paper_2104_13264_amd import Sampler
    inst = ea_pm(14, 2.0, 12, seed=82)
    env = bmps.build_envs(ising.Model(inst.Jh, inst.Jv, None, inst.beta), 12)
    assert sum(env["degenerate"]) > 0
    s = Sampler()
    lz = s.build_env(inst.Jh, inst.Jv, None, inst.beta, 12)
    got = s.logz_frozen([(inst.Jh, inst.Jv, None, inst.beta)])[0]
    log(f"[frozen] degenerate cuts: oracle {sum(env['degenerate'])}, gpu {s.stats()['degenerate_cuts']}; "
        f"ln Z~ {lz!r} frozen {got!r} oracle {env['logZ']!r}")
    assert abs(got - lz) <= 1e-12 * abs(lz)
    assert abs(got - env["logZ"]) <= 1e-9 * abs(env["logZ"])
    s.close()


def pick_bonds(n, nbonds, seed):
    """n distinct bond indices from Philox4x32-10 (key seed, counter
    (k, 0, 0, 3)), word 0 modulo the bond count."""
    out, k = [], 0
    while len(out) < n:
        ctr = np.array([[k, 0, 0, 3]], dtype=np.uint64)
        b = int(philox4x32_10(ctr, seed_key(seed)[None, :])[0, 0]) % nbonds
        if b not in out:
            out.append(b)
        k += 1
    return out


@pytest.mark.timeout(900)
def test_grad_by_central_differences_at_128():
    from paper_2104_13264_amd import Sampler
    L, beta, D, step = 128, 1.0, 32, 1e-4
    inst = fully_frustrated(L, beta, D)
    s = Sampler()
    log("[frozen] 128x128 fully frustrated D32: build")
    lz = s.build_env(inst.Jh, inst.Jv, None, beta, D)
    log(f"[frozen] ln Z~ {lz!r}; frozen derivative")
    dJh, dJv, db = s.grad()
    dJh, dJv = dJh.cpu().numpy(), dJv.cpu().numpy()
    nh = inst.Jh.size
    bonds = pick_bonds(32, nh + inst.Jv.size, SEED)
    sets, exact = [], []
    for b in bonds:
        for sg in (1.0, -1.0):
            Jh, Jv = inst.Jh.copy(), inst.Jv.copy()
            if b < nh:
                Jh.flat[b] += sg * step
            else:
                Jv.flat[b - nh] += sg * step
            sets.append((Jh, Jv, None, beta))
        exact.append(dJh.flat[b] if b < nh else dJv.flat[b - nh])
    for sg in (1.0, -1.0):
        sets.append((inst.Jh, inst.Jv, None, beta + sg * step))
    log(f"[frozen] {len(sets)} frozen contractions in one batched build")
    vals = s.logz_frozen(sets)
    fd = [(vals[2 * i] - vals[2 * i + 1]) / (2 * step) for i in range(len(bonds))]
    rel = [abs(f - e) / abs(e) for f, e in zip(fd, exact)]
    fdb = (vals[-2] - vals[-1]) / (2 * step)
    relb = abs(fdb - db) / abs(db)
    for b, f, e, r in zip(bonds, fd, exact, rel):
        log(f"  bond {b}: tn_grad {e:.10f} central difference {f:.10f} rel {r:.2e}")
    log(f"  beta: tn_grad {db:.6f} central difference {fdb:.6f} rel {relb:.2e}")
    assert max(rel) < 1e-6 and relb < 1e-6
    s.close()
