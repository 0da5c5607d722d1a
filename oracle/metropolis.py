"""Single-spin-flip Metropolis sweeps interleaved with TNMH steps (oracle, FP64).

Sec. 3 (discussion of Fig. hb and Table hb) reports that spin-flip Metropolis
sweeps between TNMH moves rescue chains that the approximate prior alone
leaves stuck in disordered instances.  The paper does not fix the sweep order
or its random numbers; the readings adopted here are:
  * a sweep visits every site once in checkerboard order: all sites with
    r + c even, then all with r + c odd.  Sites of one colour share no bond, so
    one colour is updated at once (equal to any order within the colour);
  * at site i with spin s the local field is
        F = h_i + J_left s_left + J_right s_right + J_up s_up + J_down s_down,
    summed in that order (missing neighbours of the open boundary add
    nothing); flipping changes the energy of Eq. (ising) by dE = 2 s F and is
    accepted iff u < exp(-(beta dE)), the Metropolis rule min(1, e^{-beta dE});
  * u is word i % 4 of Philox4x32-10 (key = seed) at counter
    (sweep * 2^14 + i // 4, chain, step, inst << 2 | 2), mapped to (0, 1) as in
    oracle.philox; stream 2 keeps these words apart from the proposals (0) and
    the acceptance (1).
After the sweeps a chain's ln q and energy are those of its new configuration
(eval mode of the sampler), which the next TNMH step needs.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .philox import philox4x32_10, seed_key, to_uniform
from .sampler import eval_logq
from .ising import energy


def sweep_uniforms(chains, nsite, seed, step, sweep, inst=0):
    """u[chain, site] of one sweep."""
    nblk = (nsite + 3) // 4
    ctr = np.zeros((chains, nblk, 4), dtype=np.uint64)
    ctr[:, :, 0] = (np.uint64(sweep) << np.uint64(14)) | np.arange(nblk, dtype=np.uint64)[None, :]
    ctr[:, :, 1] = np.arange(chains, dtype=np.uint64)[:, None]
    ctr[:, :, 2] = np.uint64(step)
    ctr[:, :, 3] = np.uint64((inst << 2) | 2)
    w = philox4x32_10(ctr, seed_key(seed)[None, None, :])      # [chains, nblk, 4]
    return to_uniform(w.reshape(chains, 4 * nblk)[:, :nsite])


def local_field(s, Jh, Jv, h):
    """F[..., r, c] = h + J_left s_left + J_right s_right + J_up s_up + J_down s_down,
    with the terms added in this order (zero where the neighbour is missing)."""
    Ly, Lx = s.shape[-2:]
    left = np.zeros(s.shape)
    right = np.zeros(s.shape)
    up = np.zeros(s.shape)
    down = np.zeros(s.shape)
    left[..., :, 1:] = Jh * s[..., :, :-1]
    right[..., :, :-1] = Jh * s[..., :, 1:]
    up[..., 1:, :] = Jv * s[..., :-1, :]
    down[..., :-1, :] = Jv * s[..., 1:, :]
    F = np.zeros(s.shape) if h is None else np.broadcast_to(np.asarray(h, dtype=np.float64), s.shape).copy()
    return (((F + left) + right) + up) + down


def sweeps(model, spins, seed, step, nsweeps, inst=0):
    """nsweeps checkerboard Metropolis sweeps of spins [chains, Ly, Lx] (a new
    array is returned) and the number of accepted flips per chain."""
    s = np.array(spins, dtype=np.float64)
    chains, Ly, Lx = s.shape
    rr, cc = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    colour = (rr + cc) & 1
    Jh = np.asarray(model.Jh, dtype=np.float64)
    Jv = np.asarray(model.Jv, dtype=np.float64)
    flips = np.zeros(chains, dtype=np.int64)
    for k in range(nsweeps):
        u = sweep_uniforms(chains, Ly * Lx, seed, step, k, inst).reshape(chains, Ly, Lx)
        for col in (0, 1):
            F = local_field(s, Jh, Jv, model.h)
            dE = (2.0 * s) * F
            flip = (u < np.exp(-(model.beta * dE))) & (colour == col)[None]
            s = np.where(flip, -s, s)
            flips += flip.sum(axis=(1, 2))
    return s.astype(np.int8), flips


def interleave(model, envs, state, seed, step, nsweeps, inst=0):
    """The sweeps applied to a TNMH chain state (dict of spins, logq, energy),
    with ln q and the energy of the new configurations (updated in place)."""
    new, flips = sweeps(model, state["spins"], seed, step, nsweeps, inst)
    ev = eval_logq(model, envs, new)
    state["spins"] = new
    state["logq"] = ev["logq"]
    state["energy"] = energy(new, model.Jh, model.Jv, model.h)
    return flips
