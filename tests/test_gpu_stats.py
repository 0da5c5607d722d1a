"""Link overlaps on the GPU (tn_link_overlap) against the oracle: exact
integers, bitwise, on strips, columns, odd shapes and the widest lattice."""
import numpy as np
import pytest
import torch

from oracle import stats
from workloads import random_instance, random_spins

pytestmark = pytest.mark.gpu

FP32 = 1


@pytest.mark.parametrize("shape", [(1, 9), (7, 1), (5, 7), (32, 32), (3, 256)])
def test_link_overlap_matches_oracle(shape):
    from paper_2104_13264_amd import Sampler
    Ly, Lx = shape
    print(f"[stats] link overlap {Ly}x{Lx}", flush=True)
    inst = random_instance(Ly, Lx, 0.5, 4, seed=501)
    s = Sampler()
    s.build_env(inst.Jh, inst.Jv, None, inst.beta, 4, FP32)
    a = random_spins(37, Ly, Lx, seed=1)
    b = random_spins(37, Ly, Lx, seed=2)
    q = s.link_overlap(torch.as_tensor(a), torch.as_tensor(b)).cpu().numpy()
    np.testing.assert_array_equal(q, stats.link_overlap(a, b))
    q0 = s.link_overlap(torch.as_tensor(a[:3]), torch.as_tensor(a[:3])).cpu().numpy()
    assert np.all(q0 == Ly * (Lx - 1) + (Ly - 1) * Lx)
    s.close()
