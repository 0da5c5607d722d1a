"""Seeded synthetic Ising instances shared by the tests, the benchmark and the
smoke check.  This module holds input generation only: couplings, fields,
initial configurations and run sizes.  It contains none of the method's
arithmetic and imports neither the oracle nor the HIP package.

The paper's experiments use ferromagnetic, antiferromagnetic, J'-J (fully
frustrated) and disordered square lattices with open boundaries (Sec. 3,
"Role of the bond dimension"); the named workloads below follow those families
at the sizes the benchmarks quote.
"""
from dataclasses import dataclass, field

import numpy as np

SEED = 210413264


@dataclass
class Instance:
    name: str
    Jh: np.ndarray            # [Ly][Lx-1] float64
    Jv: np.ndarray            # [Ly-1][Lx] float64
    h: object                 # None or [Ly][Lx] float64
    beta: float
    D: int
    chains: int = 1
    steps: int = 1
    seed: int = SEED
    extra: dict = field(default_factory=dict)

    @property
    def Ly(self):
        return self.Jv.shape[0] + 1

    @property
    def Lx(self):
        return self.Jh.shape[1] + 1


def uniform(Ly, Lx, J):
    return (np.full((Ly, Lx - 1), float(J)), np.full((Ly - 1, Lx), float(J)))


def ferro(L, beta, D, chains=1, steps=1, name=None, Lx=None):
    Lx = L if Lx is None else Lx
    Jh, Jv = uniform(L, Lx, 1.0)
    return Instance(name or f"ferro{L}x{Lx}", Jh, Jv, None, beta, D, chains, steps)


def antiferro(L, beta, D, chains=1, steps=1):
    Jh, Jv = uniform(L, L, -1.0)
    return Instance(f"antiferro{L}", Jh, Jv, None, beta, D, chains, steps)


def fully_frustrated(L, beta, D, Lx=None):
    """|J| = 1; horizontal bonds +1; vertical bonds -1 in odd (0-indexed)
    columns, so every plaquette holds exactly one negative bond."""
    Lx = L if Lx is None else Lx
    Jh = np.ones((L, Lx - 1))
    Jv = np.ones((L - 1, Lx))
    Jv[:, 1::2] = -1.0
    return Instance(f"fullyfrustrated{L}x{Lx}", Jh, Jv, None, beta, D)


def ea_pm(L, beta, D, seed, chains=1, steps=1):
    """Edwards-Anderson +-J instance: iid J = +-1 with p = 1/2, from numpy's
    PCG64 stream seeded with `seed`."""
    rng = np.random.default_rng(seed)
    Jh = rng.choice([-1.0, 1.0], size=(L, L - 1))
    Jv = rng.choice([-1.0, 1.0], size=(L - 1, L))
    return Instance(f"ea_pm{L}_s{seed}", Jh, Jv, None, beta, D, chains, steps)


def ea_gauss(L, beta, D, seed, chains=1, steps=1):
    """Edwards-Anderson instance with iid standard Gaussian couplings from
    numpy's PCG64 stream seeded with `seed`, no field."""
    rng = np.random.default_rng(seed)
    Jh = rng.normal(size=(L, L - 1))
    Jv = rng.normal(size=(L - 1, L))
    return Instance(f"ea_gauss{L}_s{seed}", Jh, Jv, None, beta, D, chains, steps)


def random_instance(Ly, Lx, beta, D, seed, field_scale=0.0, gaussian=True):
    """Small random instance for parity tests (Gaussian or +-1 couplings)."""
    rng = np.random.default_rng(seed)
    if gaussian:
        Jh = rng.normal(size=(Ly, Lx - 1))
        Jv = rng.normal(size=(Ly - 1, Lx))
    else:
        Jh = rng.choice([-1.0, 1.0], size=(Ly, Lx - 1))
        Jv = rng.choice([-1.0, 1.0], size=(Ly - 1, Lx))
    h = rng.normal(size=(Ly, Lx)) * field_scale if field_scale else None
    return Instance(f"random{Ly}x{Lx}_s{seed}", Jh, Jv, h, beta, D)


# --- named workloads -------------------------------------------------------

def small_ferro_8():
    """8x8 ferromagnet, beta = 0.44, D = 8; one chain of 1000 proposals."""
    return ferro(8, 0.44, 8, chains=1, steps=1000, name="ferro8_D8")


def ferro_64():
    """64x64 ferromagnet at beta = 0.4407, D = 32; 4096 chains x 200 steps
    (one proposal per chain per step)."""
    return ferro(64, 0.4407, 32, chains=4096, steps=200, name="ferro64_D32")


def ea_mix(n=64):
    """64 +-J spin-glass instances of mixed size: L in {16,24,32,48} (16 each),
    beta in {1,2,3} by instance index mod 3, D = 16/32/32/64 for L =
    16/24/32/48; 1024 proposals per instance per step."""
    sizes = [16, 24, 32, 48]
    Ds = {16: 16, 24: 32, 32: 32, 48: 64}
    out = []
    for i in range(n):
        L = sizes[i // (n // 4)] if n >= 4 else sizes[i % 4]
        beta = [1.0, 2.0, 3.0][i % 3]
        out.append(ea_pm(L, beta, Ds[L], SEED + i, chains=1024, steps=200))
    return out


def frustrated_128():
    """128x128 fully frustrated lattice, beta = 1, D = 32 (gradient workload)."""
    return fully_frustrated(128, 1.0, 32)


def antiferro_256():
    """256x256 antiferromagnet, beta = 0.4407, D = 64; 16384 proposals/step."""
    return antiferro(256, 0.4407, 64, chains=16384, steps=20)


def ea_gauss_set(n=64, L=32, T=0.212, D=16, chains=30):
    """n Gaussian EA instances at temperature T (the setting of the paper's
    equilibration test, Fig. hb b: 32x32 open, T = 0.212, D = 16, 30 chains
    per instance), seeds SEED + 1000 + i."""
    return [ea_gauss(L, 1.0 / T, D, SEED + 1000 + i, chains=chains) for i in range(n)]


def periodic_couplings(Ly, Lx, wrap_x, wrap_y, seed, gaussian=True, field_scale=0.0):
    """Couplings of a lattice wrapped along x and/or y (Jh [Ly][Lx] when wrapped
    along x, else [Ly][Lx-1]; Jv [Ly][Lx] when wrapped along y, else
    [Ly-1][Lx]): iid standard Gaussian or +-1 from numpy's PCG64 stream, with
    an optional Gaussian field."""
    rng = np.random.default_rng(seed)
    sh = (Ly, Lx if wrap_x else Lx - 1)
    sv = (Ly if wrap_y else Ly - 1, Lx)
    if gaussian:
        Jh, Jv = rng.normal(size=sh), rng.normal(size=sv)
    else:
        Jh, Jv = rng.choice([-1.0, 1.0], size=sh), rng.choice([-1.0, 1.0], size=sv)
    h = rng.normal(size=(Ly, Lx)) * field_scale if field_scale else None
    return dict(Jh=Jh, Jv=Jv, h=h)


def ea_gauss_torus_set(n=64, L=32, T=0.212, chains=30):
    """n Gaussian EA instances on the L x L torus at temperature T (the
    periodic counterpart of ea_gauss_set), seeds SEED + 2000 + i; dicts for
    Sampler.periodic_setup."""
    return [dict(periodic_couplings(L, L, True, True, SEED + 2000 + i), beta=1.0 / T, chains=chains)
            for i in range(n)]


def random_spins(chains, Ly, Lx, seed):
    """Independent uniform +-1 configurations (an easy starting distribution)."""
    rng = np.random.default_rng(seed)
    return rng.choice(np.array([-1, 1], dtype=np.int8), size=(chains, Ly, Lx))


def all_up(chains, Ly, Lx):
    return np.ones((chains, Ly, Lx), dtype=np.int8)
