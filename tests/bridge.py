"""Test helpers: pack oracle environments into the C-ABI host layout, open a
GPU sampler, compare draws.  Used only by the tests."""
import numpy as np

from oracle import bmps, ising

TOL_LOGZ_FP64 = 1e-9      # relative, ln Z~ and ln q, fp64 paths
TOL_LOGQ_FP32 = 1e-5      # relative, ln q, fp32 path
NEAR_FP64 = 1e-6          # |u - p+| below which an fp64 draw may diverge


def model_of(inst):
    return ising.Model(inst.Jh, inst.Jv, inst.h, inst.beta)


def pack_envs(envs, D):
    """Oracle env list -> (env [(Ly-1)][Lx][D][2][D], dims [(Ly-1)][Lx+1], ell)."""
    env = envs['env']
    Ly = len(env) - 1
    Lx = len(env[Ly])
    out = np.zeros((max(Ly - 1, 0), Lx, D, 2, D))
    dims = np.ones((max(Ly - 1, 0), Lx + 1), dtype=np.int32)
    for k in range(1, Ly):
        for c in range(Lx):
            E = env[k][c]
            a, u, b = E.shape
            out[k - 1, c, :a, :u, :b] = E
            dims[k - 1, c] = a
        dims[k - 1, Lx] = 1
    return out, dims, envs['ell'][1:Ly].copy()


def gpu_sampler_with_oracle_env(inst, D, prec):
    from paper_2104_13264_amd import Sampler
    envs = bmps.build_envs(model_of(inst), D)
    env, dims, ell = pack_envs(envs, D)
    s = Sampler()
    s.set_env(inst.Jh, inst.Jv, inst.h, inst.beta, D, env, dims, ell, envs['logZ'], prec)
    return s, envs


def divergence_mask(oracle_run, near):
    """Proposals whose every draw was farther than `near` from its threshold."""
    return oracle_run['min_gap'] >= near
