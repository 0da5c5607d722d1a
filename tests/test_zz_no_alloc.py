"""tn_sample_noalloc (the sampler for callers that cannot allocate) against
tn_sample through the C ABI: bitwise the same proposals, ln q and energies on
two calls in a row, the second with a smaller batch (the fixed scratch keeps
the first call's contents), in FP32 at the largest batch that fits (4096
proposals of the 64x64, D = 32 lattice: exactly its 64 MiB) and in FP64; a
batch above the fixed size is refused with TN_EINVAL and nothing written."""
import numpy as np
import pytest
import torch

from workloads import random_instance, ferro_64, SEED

pytestmark = pytest.mark.gpu

FP64, FP32 = 0, 1
TN_EINVAL = -1


def log(msg):
    print(msg, flush=True)


def compare(s, batch, seed, step, first_id):
    from paper_2104_13264_amd.tnmh import lib, _ptr
    a = s.empty_batch(batch)
    b = s.empty_batch(batch)
    for t in b:
        t.fill_(0)
    s.sample(batch, seed, step=step, first_id=first_id, out=a)
    rc = lib().tn_sample_noalloc(s._ctx, batch, seed, step, first_id, _ptr(b[0]), _ptr(b[1]), _ptr(b[2]))
    assert rc == 0, lib().tn_last_error(s._ctx)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("prec,name,mk,calls", [
    (FP32, "ferro 64x64 D32", lambda: (ferro_64(), 32), [(4096, 0, 0), (1000, 3, 17)]),
    (FP64, "random 12x16 D8", lambda: (random_instance(12, 16, 0.7, 8, seed=71, field_scale=0.2), 8),
     [(4000, 1, 0), (333, 2, 5)]),
], ids=["fp32", "fp64"])
def test_noalloc_sampler_matches_tn_sample(prec, name, mk, calls):
    from paper_2104_13264_amd import Sampler
    inst, D = mk()
    log(f"[noalloc] {name} prec {prec}: calls {calls}")
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, D, prec)
    for batch, step, first_id in calls:
        compare(s, batch, SEED, step, first_id)
    s.close()


def test_noalloc_refuses_a_batch_above_its_scratch():
    from paper_2104_13264_amd import Sampler
    from paper_2104_13264_amd.tnmh import lib, _ptr
    inst = ferro_64()
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, inst.h, inst.beta, 32, FP32)
    batch = 4097                         # one more team than 64 MiB holds
    sp, lq, E = s.empty_batch(batch)
    lq.fill_(7.0)
    rc = lib().tn_sample_noalloc(s._ctx, batch, SEED, 0, 0, _ptr(sp), _ptr(lq), _ptr(E))
    msg = lib().tn_last_error(s._ctx).decode()
    log(f"[noalloc] refused: rc {rc}, {msg}")
    assert rc == TN_EINVAL and "scratch" in msg
    torch.cuda.synchronize()
    assert bool((lq == 7.0).all())
    compare(s, 64, SEED, 1, 0)           # the context still samples
    s.close()
