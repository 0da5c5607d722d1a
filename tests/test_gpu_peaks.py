"""Peak probes (tn_peak_probe): each probe runs its unit and reports a rate
that is positive and not above the published MI355X figure (a rate above the
hardware's means the probe miscounts its work); bad arguments are refused."""
import pytest

pytestmark = pytest.mark.gpu

PUBLISHED = {  # flop/s or byte/s
    "mfma_f32": 157.3e12, "mfma_bf16": 2.5e15, "mfma_f64": 78.6e12, "fma_f64": 78.6e12,
    "hbm_read": 8.0e12, "hbm_copy": 8.0e12,
}
AMOUNT = {"mfma_f32": 2000, "mfma_bf16": 4000, "mfma_f64": 1000, "fma_f64": 10000,
          "hbm_read": 1 << 30, "hbm_copy": 1 << 29}


@pytest.mark.parametrize("kind", list(PUBLISHED))
def test_probe_rate_is_plausible(kind):
    from paper_2104_13264_amd import peak_probe
    sec, work = peak_probe(kind, AMOUNT[kind])
    rate = work / sec
    print(f"[peaks] {kind}: {rate:.4g} per s ({rate / PUBLISHED[kind]:.3f} of published)", flush=True)
    assert sec > 0 and work > 0
    assert rate <= 1.05 * PUBLISHED[kind]


def test_probe_arguments():
    from paper_2104_13264_amd import lib
    import ctypes
    s, w = ctypes.c_double(), ctypes.c_double()
    L = lib()
    assert L.tn_peak_probe(99, 10, ctypes.byref(s), ctypes.byref(w)) != 0    # unknown kind
    assert L.tn_peak_probe(0, 0, ctypes.byref(s), ctypes.byref(w)) != 0     # amount < 1
    assert L.tn_peak_probe(4, 1000, ctypes.byref(s), ctypes.byref(w)) != 0  # bytes not a multiple of 16
    assert L.tn_peak_probe(0, 10, None, ctypes.byref(w)) != 0               # NULL output
