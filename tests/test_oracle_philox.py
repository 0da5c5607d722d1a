"""Pin of the oracle's Philox4x32-10 (Salmon et al., SC'11) against rocRAND's
independent implementation, compiled from its public header and run on the
host.  Plus the (0,1) mapping and basic uniformity."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle.philox import philox4x32_10, to_uniform, seed_key

HELPER = os.path.join(os.path.dirname(__file__), "helpers", "philox_rocrand.cpp")


@pytest.fixture(scope="module")
def rocrand_exe(tmp_path_factory):
    hdr = "/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"
    if not os.path.exists(hdr) or shutil.which("g++") is None:
        pytest.skip("rocRAND header or g++ unavailable")
    out = str(tmp_path_factory.mktemp("philox") / "philox_rr")
    subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                    HELPER, "-o", out], check=True, capture_output=True)
    return out


def test_philox_matches_rocrand(rocrand_exe):
    rng = np.random.default_rng(7)
    n = 2000
    keys = rng.integers(0, 2 ** 32, size=(n, 2), dtype=np.uint64)
    ctrs = rng.integers(0, 2 ** 32, size=(n, 4), dtype=np.uint64)
    # edge words and the counter layouts used by the method
    keys[:4] = [[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [210413264, 0], [1, 0]]
    ctrs[:4] = [[0, 0, 0, 0], [0xFFFFFFFF] * 4, [17, 4095, 199, 0], [0, 3, 7, 1]]
    lines = "\n".join(" ".join(str(int(v)) for v in np.concatenate([k, c]))
                      for k, c in zip(keys, ctrs))
    res = subprocess.run([rocrand_exe], input=lines, capture_output=True,
                         text=True, check=True)
    ref = np.array([[int(w) for w in ln.split()] for ln in res.stdout.strip().splitlines()],
                   dtype=np.uint64)
    got = philox4x32_10(ctrs, keys)
    assert got.shape == ref.shape
    np.testing.assert_array_equal(got, ref)


def test_uniform_mapping_open_interval():
    u = to_uniform(np.array([0, 2 ** 32 - 1], dtype=np.uint64))
    assert u[0] == 0.5 * 2.0 ** -32 and 0.0 < u[0]
    assert u[1] == 1.0 - 0.5 * 2.0 ** -32 and u[1] < 1.0


def test_uniformity_and_word_independence():
    ctr = np.zeros((1 << 16, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(1 << 16)
    w = philox4x32_10(ctr, seed_key(210413264)[None, :])
    u = to_uniform(w)
    # each word: mean 1/2, variance 1/12 within 5 sigma
    n = u.shape[0]
    assert np.all(np.abs(u.mean(0) - 0.5) < 5 * np.sqrt(1 / 12 / n))
    # 16-bin chi^2 per word (15 dof; 99.99% quantile ~ 44)
    for j in range(4):
        cnt = np.bincount((u[:, j] * 16).astype(int), minlength=16)
        chi2 = ((cnt - n / 16) ** 2 / (n / 16)).sum()
        assert chi2 < 44
    # words of one block are uncorrelated
    cc = np.corrcoef(u.T)
    assert np.all(np.abs(cc - np.eye(4)) < 5 / np.sqrt(n))
