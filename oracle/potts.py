"""q-state Potts models: general local dimension d (oracle, FP64).

App. A writes the partition function of any nearest-neighbour Hamiltonian
whose local variables take values in a finite set of size d as a contraction
of d x d bond matrices W_ij(s, s') = exp(-beta phi_ij(s, s'))
(Eq. pf_bond_description), splits each W into two site factors by its SVD and
groups the factors into site tensors (Eq. tensor-general); Sec. 2 notes that
the sampler carries over to other nearest-neighbour models such as the Potts
model unchanged.  The model here:

    H(s) = - sum_<ij> J_ij delta(s_i, s_j) - sum_i h_i(s_i),   s_i in 0..d-1

with Jh [Ly][Lx-1], Jv [Ly-1][Lx] as for Ising and h [Ly][Lx][d] (None: 0).

Readings adopted:
  * Bond split.  With K = beta J, W = exp(K delta) = (e^K - 1) I + 1 1^T: its
    eigenvectors are e_0 = (1, .., 1) / sqrt(d) (eigenvalue e^K - 1 + d) and
    any orthonormal basis of the complement of e_0 (eigenvalue e^K - 1).  The
    basis taken is Helmert's: for m = 1..d-1, e_m(s) = 1/sqrt(m(m+1)) for
    s < m, -m/sqrt(m(m+1)) for s = m, 0 for s > m.  The square-root split of
    App. A, with the eigenvalue's sign on the second factor:
        P(s, mu) = e_mu(s) sqrt|lambda_mu|,
        Q(mu, s') = sign(lambda_mu) sqrt|lambda_mu| e_mu(s'),
    so that sum_mu P(s, mu) Q(mu, s') = W(s, s') exactly.  P belongs to the
    left/top site of the bond and Q to the right/bottom one, as for Ising.
    Any other basis is an orthogonal gauge on the bond (outputs unchanged).
  * Site tensor T[s, l, u, dn, x] = exp(beta h(s)) Q_left(l, s) P_right(s, x)
    Q_up(u, s) P_down(s, dn) (Eq. tensor-general with the field as a site
    factor); the environments are those of oracle.bmps, which contracts any
    model that provides these tensors.
  * Sequential sampler (Sec. 2, Eqs. bayes, pi-approx; App. A
    Eq. proba-ratio-apx): snake order as for Ising; the conditional of a site
    is the categorical law of its d weights, each a contraction of the same
    stored environment, normalised by their sum.  The draw takes the smallest
    value k with u * (w_0 + .. + w_{d-1}) < w_0 + .. + w_k (u from the same
    Philox stream and counters as the Ising sampler); for d = 2 that is the
    Ising rule with value 0 <-> spin +1.  Negative weights are clamped to 0
    and counted; if no weight is positive (or the sum is not finite) the draw
    is uniform over the d values and counted.
  * The acceptance is Algorithm 1's, with these energies.

Test infrastructure only (see the package docstring).  Pinned by
tests/test_oracle_potts.py.
"""
import numpy as np

from . import bmps
from .sampler import site_uniforms, _pow2_rescale
from .mh import accept_uniforms, mh_decide


def energy(states, Jh, Jv, h=None):
    """H(s) = -sum J delta(s_i, s_j) - sum_i h_i(s_i) per configuration.
    states: int array [..., Ly, Lx] with values 0..d-1."""
    s = np.asarray(states)
    e = -(np.asarray(Jh) * (s[..., :, :-1] == s[..., :, 1:])).sum(axis=(-1, -2))
    e = e - (np.asarray(Jv) * (s[..., :-1, :] == s[..., 1:, :])).sum(axis=(-1, -2))
    if h is not None:
        h = np.asarray(h)
        Ly, Lx = s.shape[-2], s.shape[-1]
        r = np.arange(Ly)[:, None]
        c = np.arange(Lx)[None, :]
        e = e - h[r, c, s].sum(axis=(-1, -2))
    return np.asarray(e, dtype=np.float64)


def helmert(d):
    """Orthonormal basis e_mu(s) as a d x d matrix B[s, mu] (column 0 uniform)."""
    B = np.zeros((d, d))
    B[:, 0] = 1.0 / np.sqrt(d)
    for m in range(1, d):
        a = 1.0 / np.sqrt(m * (m + 1.0))
        B[:m, m] = a
        B[m, m] = -m * a
    return B


def bond_factors(K, d):
    """P [..., d(s), d(mu)] and Q [..., d(mu), d(s)] with P Q = exp(K delta)."""
    K = np.asarray(K, dtype=np.float64)
    B = helmert(d)
    lam = np.empty(K.shape + (d,))
    lam[..., 0] = np.expm1(K) + d
    lam[..., 1:] = np.expm1(K)[..., None]
    root = np.sqrt(np.abs(lam))
    P = B * root[..., None, :]                                  # [.., s, mu]
    Q = (np.sign(lam) * root)[..., :, None] * B.T               # [.., mu, s]
    return P, Q


class PottsModel:
    """A 2D q-state Potts instance with open boundaries and its bond factors
    (the interface oracle.bmps contracts)."""

    def __init__(self, Jh, Jv, h, beta, d):
        self.Jh = np.asarray(Jh, dtype=np.float64)
        self.Jv = np.asarray(Jv, dtype=np.float64)
        self.Ly = self.Jv.shape[0] + 1
        self.Lx = self.Jh.shape[1] + 1
        self.d = int(d)
        assert self.Jh.shape == (self.Ly, self.Lx - 1)
        assert self.Jv.shape == (self.Ly - 1, self.Lx)
        self.h = None if h is None else np.asarray(h, dtype=np.float64)
        assert self.h is None or self.h.shape == (self.Ly, self.Lx, self.d)
        self.beta = float(beta)
        self.Ph, self.Qh = bond_factors(self.beta * self.Jh, self.d)
        self.Pv, self.Qv = bond_factors(self.beta * self.Jv, self.d)

    @property
    def n_sites(self):
        return self.Lx * self.Ly

    def field(self, r, c):
        """h_{r,c}(s) for every value s."""
        return np.zeros(self.d) if self.h is None else self.h[r, c]

    def left_leg(self, r, c):   # [l, s]
        return self.Qh[r, c - 1] if c > 0 else np.ones((1, self.d))

    def right_leg(self, r, c):  # [s, x]
        return self.Ph[r, c] if c < self.Lx - 1 else np.ones((self.d, 1))

    def up_leg(self, r, c):     # [u, s]
        return self.Qv[r - 1, c] if r > 0 else np.ones((1, self.d))

    def down_leg(self, r, c):   # [s, dn]
        return self.Pv[r, c] if r < self.Ly - 1 else np.ones((self.d, 1))

    def site_tensor(self, r, c):
        """Eq. (tensor-general), one slice per value s: T[s, l, u, dn, x]."""
        f = np.exp(self.beta * self.field(r, c))
        return np.einsum('s,ls,sx,us,sd->sludx', f, self.left_leg(r, c),
                         self.right_leg(r, c), self.up_leg(r, c),
                         self.down_leg(r, c))


def build_envs(model, D):
    """Bottom-up environments and ln Z~ (oracle.bmps, successive SVD)."""
    return bmps.build_envs(model, D)


def run_rows(model, envs, batch, seed=0, step=0, first_id=0, inst=0,
             states=None, near=1e-6, ids=None):
    """Sample (states None) or evaluate (states [B,Ly,Lx] given) proposals.

    Returns dict(states int8 [B,Ly,Lx], logq [B], energy [B], clamps [B],
                 both_nonpos [B], near [B], min_gap [B]); min_gap is the
    smallest distance of u to a threshold (w_0 + .. + w_k) / sum, k < d-1.
    """
    Ly, Lx, beta, d = model.Ly, model.Lx, model.beta, model.d
    env = envs['env']
    B = batch
    eval_mode = states is not None
    if eval_mode:
        out = np.asarray(states, dtype=np.int8).copy()
    else:
        out = np.zeros((B, Ly, Lx), dtype=np.int8)
        if ids is None:
            ids = first_id + np.arange(B)
        u_all = site_uniforms(Ly * Lx, ids, seed, step, inst)
    logq = np.zeros(B)
    clamps = np.zeros(B, dtype=np.int64)
    both = np.zeros(B, dtype=np.int64)
    nnear = np.zeros(B, dtype=np.int64)
    min_gap = np.full(B, np.inf)
    rows_b = np.arange(B)

    for r in range(Ly):
        F = env[r + 1]
        # G_c(s) = sum_dn P_down(s, dn) F_c[:, dn, :]
        G = [np.einsum('sd,adb->sab', model.down_leg(r, c), F[c]) for c in range(Lx)]
        # the field and the vertical bond to the fixed value above
        v = np.empty((B, Lx, d))
        for c in range(Lx):
            f = np.exp(beta * model.field(r, c))                  # [d]
            if r > 0:
                W = model.down_leg(r - 1, c) @ model.up_leg(r, c)  # [s', s]
                v[:, c, :] = f[None, :] * W[out[:, r - 1, c], :]
            else:
                v[:, c, :] = f[None, :]
        if r % 2 == 0:
            env_side = [None] * Lx
            env_side[Lx - 1] = np.ones((B, 1, 1))                  # [b, x', a]
            for c in range(Lx - 1, 0, -1):
                Gc = G[c]
                ns, Dl, Dr = Gc.shape
                Xp = env_side[c].shape[1]
                t = (env_side[c].reshape(B * Xp, Dr) @ Gc.reshape(ns * Dl, Dr).T)
                t = t.reshape(B, Xp, ns, Dl)
                y = np.einsum('sx,bxsa->bsa', model.right_leg(r, c), t)
                nr = np.einsum('xs,bs,bsa->bxa', model.left_leg(r, c), v[:, c, :], y)
                env_side[c - 1] = _pow2_rescale(nr, (1, 2))
            order = range(Lx)
        else:
            env_side = [None] * Lx
            env_side[0] = np.ones((B, 1, 1))
            for c in range(0, Lx - 1):
                Gc = G[c]
                ns, Dl, Dr = Gc.shape
                Xl = env_side[c].shape[1]
                t = (env_side[c].reshape(B * Xl, Dl) @ Gc.transpose(1, 0, 2).reshape(Dl, ns * Dr))
                t = t.reshape(B, Xl, ns, Dr)
                y = np.einsum('xs,bxsa->bsa', model.left_leg(r, c), t)
                nl = np.einsum('sx,bs,bsa->bxa', model.right_leg(r, c), v[:, c, :], y)
                env_side[c + 1] = _pow2_rescale(nl, (1, 2))
            order = range(Lx - 1, -1, -1)
        lam = np.ones((B, 1))
        prev = None
        for c in order:
            Gc = G[c]
            ns, Dl, Dr = Gc.shape
            if r % 2 == 0:
                lg = (lam @ Gc.transpose(1, 0, 2).reshape(Dl, ns * Dr)).reshape(B, ns, Dr)
                z = np.einsum('bsa,bxa->bsx', lg, env_side[c])
                w = v[:, c, :] * np.einsum('sx,bsx->bs', model.right_leg(r, c), z)
                if prev is not None:
                    W = model.right_leg(r, c - 1) @ model.left_leg(r, c)   # [s', s]
            else:
                lg = np.einsum('sab,zb->zsa', Gc, lam)
                z = np.einsum('bsa,bxa->bsx', lg, env_side[c])
                w = v[:, c, :] * np.einsum('xs,bsx->bs', model.left_leg(r, c), z)
                if prev is not None:
                    W = (model.right_leg(r, c) @ model.left_leg(r, c + 1)).T   # [s', s]
            if prev is not None:
                w = w * W[out[:, r, prev], :]
            neg = w < 0
            clamps += neg.sum(axis=1)
            w = np.where(neg, 0.0, w)
            # cumulative weights, summed in value order; the total is the last
            cum = np.cumsum(w, axis=1)
            tot = cum[:, -1]
            bad = ~(np.isfinite(tot) & (tot > 0))
            both += bad
            w = np.where(bad[:, None], 1.0, w)                   # uniform law
            cum = np.where(bad[:, None], np.cumsum(w, axis=1), cum)
            tot = cum[:, -1]
            if eval_mode:
                s = out[:, r, c].astype(np.int64)
            else:
                ut = u_all[:, r * Lx + c] * tot
                s = np.argmax(ut[:, None] < cum, axis=1)          # first k with u tot < cum_k
                gap = np.abs(ut[:, None] - cum[:, :d - 1]) / tot[:, None]
                g = gap.min(axis=1) if d > 1 else np.full(B, np.inf)
                nnear += g < near
                min_gap = np.minimum(min_gap, g)
                out[:, r, c] = s
            with np.errstate(divide='ignore'):
                logq += np.log(w[rows_b, s] / tot)
            lam = _pow2_rescale(lg[rows_b, s, :], (1,))
            prev = c
    E = energy(out, model.Jh, model.Jv, model.h)
    return dict(states=out, logq=logq, energy=E, clamps=clamps,
                both_nonpos=both, near=nnear, min_gap=min_gap)


def sample(model, envs, batch, seed, step=0, first_id=0, inst=0, ids=None):
    """Draw `batch` proposals; proposal j uses id = first_id + j (or ids[j])."""
    return run_rows(model, envs, batch, seed, step, first_id, inst, ids=ids)


def eval_logq(model, envs, states):
    """ln q(s) of given configurations by the same arithmetic (eval mode)."""
    states = np.asarray(states)
    return run_rows(model, envs, states.shape[0], states=states)


def mh_step(model, envs, state, seed, t, inst=0):
    """One step of Algorithm 1 (Eqs. mh-acc, tns-prior) for every chain of
    `state` (dict states, logq, energy; updated in place)."""
    chains = state['states'].shape[0]
    prop = sample(model, envs, chains, seed, step=t, first_id=0, inst=inst)
    u = accept_uniforms(chains, seed, t, inst)
    acc, _ = mh_decide(state['logq'], state['energy'], prop['logq'], prop['energy'],
                       model.beta, u)
    for k in ('states', 'logq', 'energy'):
        state[k][acc] = prop[k][acc]
    return acc


def init_state(model, envs, chains, states=None):
    if states is None:
        states = np.zeros((chains, model.Ly, model.Lx), dtype=np.int8)
    ev = eval_logq(model, envs, states)
    return dict(states=np.array(states, dtype=np.int8), logq=ev['logq'],
                energy=energy(states, model.Jh, model.Jv, model.h))


# ---------------------------------------------------------------------------
# exact references, independent of the tensor-network code

def all_configs(Ly, Lx, d):
    """All d^(Ly*Lx) configurations (site i is digit i of the index in base d)."""
    N = Ly * Lx
    n = np.arange(d ** N, dtype=np.int64)
    digits = (n[:, None] // (d ** np.arange(N, dtype=np.int64))[None, :]) % d
    return digits.reshape(-1, Ly, Lx).astype(np.int8)


def brute_force(Jh, Jv, h, beta, d):
    """(configs, energies, ln Z, ln pi) by enumeration of every configuration."""
    Ly, Lx = np.asarray(Jv).shape[0] + 1, np.asarray(Jh).shape[1] + 1
    cfg = all_configs(Ly, Lx, d)
    E = energy(cfg, Jh, Jv, h)
    a = -beta * E
    amax = a.max()
    logZ = amax + np.log(np.exp(a - amax).sum())
    return cfg, E, logZ, a - logZ


def transfer_logZ(Jh, Jv, h, beta, d):
    """Exact ln Z by the row transfer matrix over the d^Lx values of a row,
    one column replaced at a time (weight exp(beta Jv delta(s_old, s_new)),
    summed over s_old), with the row's own bonds and fields diagonal."""
    Jh = np.asarray(Jh, dtype=np.float64)
    Jv = np.asarray(Jv, dtype=np.float64)
    Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
    n = np.arange(d ** Lx, dtype=np.int64)
    s = (n[:, None] // (d ** np.arange(Lx, dtype=np.int64))[None, :]) % d   # [state, c]

    def diag(r):
        e = (Jh[r][None, :] * (s[:, :-1] == s[:, 1:])).sum(1)
        if h is not None:
            e = e + np.asarray(h)[r][np.arange(Lx)[None, :], s].sum(1)
        return beta * e

    a = diag(0)
    m = a.max()
    vec = np.exp(a - m)
    logscale = m
    for r in range(1, Ly):
        for c in range(Lx):
            stride = d ** c
            digit = s[:, c]
            base = n - digit * stride                   # the state with column c zeroed
            new = np.zeros_like(vec)
            K = beta * Jv[r - 1, c]
            for so in range(d):
                src = vec[base + so * stride]          # state with the old value so at column c
                new += src * np.exp(K * (digit == so))
            vec = new
        a = np.log(vec) + diag(r)
        m = a.max()
        vec = np.exp(a - m)
        logscale += m
    return logscale + np.log(vec.sum())
