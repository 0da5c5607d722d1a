"""TNMH Markov chain (oracle, FP64): Algorithm 1 with Eqs. (mh-acc), (tns-prior).

The prior is the independence proposal g(w'|w) = pi~(w') (Eq. tns-prior), so
the acceptance of Eq. (mh-acc) becomes
    min{1, [q(w) / q(w')] * exp(-beta (H(w') - H(w)))}.
Readings adopted:
  * The ratio is taken in the log domain in FP64:
        ln alpha = (ln q(w) - ln q(w')) - beta (E(w') - E(w)),
    and the move is accepted iff u < exp(min(0, ln alpha)).
  * u = Philox4x32-10(key = seed, counter = (0, chain, t, inst << 2 | 1))
    word 0 mapped to (0,1); the proposal of chain j at step t is drawn with
    id = j and step = t (oracle.sampler).
  * The garbled conditional notation of the acceptance line of Algorithm 1 is
    read as q(w)/q(w') by Eq. (tns-prior) and the reversibility argument of
    Sec. 2 (properties of the chain).
  * The initial state is the all-up configuration unless given; its ln q comes
    from the eval mode of the sampler (Algorithm 1 allows any initial law).

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .philox import philox4x32_10, seed_key, to_uniform
from .sampler import sample, eval_logq
from .ising import energy


def accept_uniforms(chains, seed, step, inst=0):
    ctr = np.zeros((chains, 4), dtype=np.uint64)
    ctr[:, 1] = np.arange(chains, dtype=np.uint64)
    ctr[:, 2] = np.uint64(step)
    ctr[:, 3] = np.uint64((inst << 2) | 1)
    return to_uniform(philox4x32_10(ctr, seed_key(seed)[None, :])[:, 0])


def mh_decide(logq_cur, E_cur, logq_prop, E_prop, beta, u):
    """Eq. (mh-acc) with the prior of Eq. (tns-prior); returns accept flags."""
    log_alpha = (logq_cur - logq_prop) - beta * (E_prop - E_cur)
    return u < np.exp(np.minimum(0.0, log_alpha)), log_alpha


def init_state(model, envs, chains, spins=None):
    if spins is None:
        spins = np.ones((chains, model.Ly, model.Lx), dtype=np.int8)
    ev = eval_logq(model, envs, spins)
    return dict(spins=np.array(spins, dtype=np.int8), logq=ev['logq'],
                energy=energy(spins, model.Jh, model.Jv, model.h))


def mh_step(model, envs, state, seed, t, inst=0):
    """One step of Algorithm 1 for every chain in `state` (updated in place)."""
    chains = state['spins'].shape[0]
    prop = sample(model, envs, chains, seed, step=t, first_id=0, inst=inst)
    u = accept_uniforms(chains, seed, t, inst)
    acc, log_alpha = mh_decide(state['logq'], state['energy'], prop['logq'],
                               prop['energy'], model.beta, u)
    state['spins'][acc] = prop['spins'][acc]
    state['logq'][acc] = prop['logq'][acc]
    state['energy'][acc] = prop['energy'][acc]
    return acc, prop, log_alpha


def run_chain(model, envs, chains, steps, seed, inst=0, spins=None):
    """Run Algorithm 1; returns the state, accept flags [steps, chains] and the
    energy series [steps, chains] (after each step)."""
    state = init_state(model, envs, chains, spins)
    acc_all = np.zeros((steps, chains), dtype=bool)
    E_series = np.zeros((steps, chains))
    for t in range(steps):
        acc, _, _ = mh_step(model, envs, state, seed, t, inst)
        acc_all[t] = acc
        E_series[t] = state['energy']
    return state, acc_all, E_series
