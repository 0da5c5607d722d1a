"""Sequential sampler and proposal probability (oracle, FP64).

Sec. 2, Eqs. (bayes) and (pi-approx): the configuration is drawn site by site,
each spin from the conditional pi~_k(s_k | s_1..s_{k-1}) = Z~(..s_k) / Z~(..),
and q(s) = pi~(s) is the product of the conditionals actually used.  App. A
Eq. (proba-ratio-apx) and the fixed-spin tensor give both contractions; App. A
notes that with the boundary tensors stored the whole update costs time linear
in the lattice size, i.e. partial contractions are cached.

Readings adopted:
  * Site order is the snake (boustrophedon) labelling: row 0 first, even
    rows left to right, odd rows right to left (the labelling figure of the
    paper is not available; the within-row order does not change q, since every
    row is contracted exactly, but it fixes which random number meets which
    site).  Before sampling a row, the environments of its free columns are
    contracted from the far end towards the row's starting column.
  * For row r, the fixed rows above reduce to a product state: the fixed spin
    s' above column c enters through its down leg contracted with the up leg of
    (r,c), v_c(s) = exp(beta h s) sum_u P(s',u) Q(u,s).  The rows below are the
    stored env r+1.  The conditional of column c is the ratio of two exact
    contractions of row r with that env, normalised over s in {+1,-1}; in a
    rightward row
        w(s) = v_c(s) hf(s) sum_x' R(s,x') [(Lam G_c(s)) . rho_c[x']]
        G_c(s) = sum_d D(s,d) env_{r+1,c}[:, d, :]
    with rho_c the environment of the free columns c+1.. (horizontal leg x' and
    env bond), Lam the environment of the fixed columns ..c-1 and hf(s) the
    horizontal bond to the fixed neighbour; a leftward row is the mirror image
    (free columns ..c-1 contracted from the left, Lam <- G_c(s) Lam).
  * Negative weights (ill-conditioning, App. A remark on positivity) are
    clamped to 0 and counted; if both weights are <= 0 (or not finite) the
    draw uses p+ = 1/2 and is counted.
  * Random numbers: u = Philox4x32-10(key = seed,
    counter = (i // 4, id, step, inst << 2 | 0)) word i % 4 mapped to (0,1)
    (see oracle.philox), i = r*Lx + c; the spin is +1 iff u < p+.
  * Partial results are rescaled by exact powers of two after every column.

Eval mode takes the spins as given and follows the same arithmetic.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .philox import philox4x32_10, seed_key, to_uniform
from .ising import SPIN, energy


def site_uniforms(n_sites, ids, seed, step, inst=0, stream=0):
    """Uniforms u[b, i] for sites i of proposals with the given ids."""
    ids = np.asarray(ids, dtype=np.uint64)
    nblk = (n_sites + 3) // 4
    ctr = np.zeros((ids.shape[0], nblk, 4), dtype=np.uint64)
    ctr[:, :, 0] = np.arange(nblk, dtype=np.uint64)[None, :]
    ctr[:, :, 1] = ids[:, None]
    ctr[:, :, 2] = np.uint64(step)
    ctr[:, :, 3] = np.uint64((inst << 2) | stream)
    words = philox4x32_10(ctr, seed_key(seed)[None, None, :])
    return to_uniform(words.reshape(ids.shape[0], nblk * 4)[:, :n_sites])


def _pow2_rescale(x, axes):
    """Divide by 2^e with e the binary exponent of max|x| (exact in FP)."""
    m = np.abs(x).max(axis=axes, keepdims=True)
    _, e = np.frexp(m)
    return np.ldexp(x, -e)


def run_rows(model, envs, batch, seed=0, step=0, first_id=0, inst=0,
             spins=None, near=1e-6, ids=None):
    """Sample (spins None) or evaluate (spins [B,Ly,Lx] given) proposals.

    Returns dict(spins int8 [B,Ly,Lx], logq [B], energy [B],
                 clamps [B], both_nonpos [B], near [B], min_gap [B]).
    """
    Ly, Lx, beta = model.Ly, model.Lx, model.beta
    env = envs['env']
    B = batch
    eval_mode = spins is not None
    if eval_mode:
        out = np.asarray(spins, dtype=np.int8).copy()
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
        G = [np.einsum('sd,adb->sab', model.down_leg(r, c), F[c]) for c in range(Lx)]
        # vertical factor from the fixed spin above (and the field)
        v = np.empty((B, Lx, 2))
        for c in range(Lx):
            f = np.exp(beta * model.field(r, c) * SPIN)          # [2]
            if r > 0:
                W = model.down_leg(r - 1, c) @ model.up_leg(r, c)  # [s', s]
                idx = (1 - out[:, r - 1, c]) // 2
                v[:, c, :] = f[None, :] * W[idx, :]
            else:
                v[:, c, :] = f[None, :]
        if r % 2 == 0:
            # rightward row: environments of the free columns to the right
            env_side = [None] * Lx
            env_side[Lx - 1] = np.ones((B, 1, 1))                  # [b, x', a]
            for c in range(Lx - 1, 0, -1):
                Gc = G[c]                                         # [2, Dl, Dr]
                ns, Dl, Dr = Gc.shape
                Xp = env_side[c].shape[1]
                t = (env_side[c].reshape(B * Xp, Dr) @ Gc.reshape(ns * Dl, Dr).T)
                t = t.reshape(B, Xp, ns, Dl)                      # [b,x',s,a]
                y = np.einsum('sx,bxsa->bsa', model.right_leg(r, c), t)
                nr = np.einsum('xs,bs,bsa->bxa', model.left_leg(r, c), v[:, c, :], y)
                env_side[c - 1] = _pow2_rescale(nr, (1, 2))
            order = range(Lx)
        else:
            # leftward row: environments of the free columns to the left
            env_side = [None] * Lx
            env_side[0] = np.ones((B, 1, 1))                      # [b, x, a]
            for c in range(0, Lx - 1):
                Gc = G[c]
                ns, Dl, Dr = Gc.shape
                Xl = env_side[c].shape[1]
                t = (env_side[c].reshape(B * Xl, Dl) @ Gc.transpose(1, 0, 2).reshape(Dl, ns * Dr))
                t = t.reshape(B, Xl, ns, Dr)                      # [b,x,s,a']
                y = np.einsum('xs,bxsa->bsa', model.left_leg(r, c), t)
                nl = np.einsum('sx,bs,bsa->bxa', model.right_leg(r, c), v[:, c, :], y)
                env_side[c + 1] = _pow2_rescale(nl, (1, 2))
            order = range(Lx - 1, -1, -1)
        # sampling sweep in the row's direction, column by column
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
                lg = np.einsum('sab,zb->zsa', Gc, lam)            # G_c(s) Lam
                z = np.einsum('bsa,bxa->bsx', lg, env_side[c])
                w = v[:, c, :] * np.einsum('xs,bsx->bs', model.left_leg(r, c), z)
                if prev is not None:
                    W = (model.right_leg(r, c) @ model.left_leg(r, c + 1)).T   # [s', s]
            if prev is not None:
                idx = (1 - out[:, r, prev]) // 2
                w = w * W[idx, :]
            neg = w < 0
            clamps += neg.sum(axis=1)
            w = np.where(neg, 0.0, w)
            tot = w[:, 0] + w[:, 1]
            bad = ~(np.isfinite(tot) & (tot > 0))
            both += bad
            with np.errstate(invalid='ignore', divide='ignore'):
                pplus = np.where(bad, 0.5, w[:, 0] / np.where(bad, 1.0, tot))
            if eval_mode:
                s = out[:, r, c]
            else:
                u = u_all[:, r * Lx + c]
                gap = np.abs(u - pplus)
                nnear += gap < near
                min_gap = np.minimum(min_gap, gap)
                s = np.where(u < pplus, 1, -1).astype(np.int8)
                out[:, r, c] = s
            ps = np.where(s == 1, pplus, 1.0 - pplus)
            with np.errstate(divide='ignore'):
                logq += np.log(ps)
            idx = (1 - s) // 2
            lam = _pow2_rescale(lg[rows_b, idx, :], (1,))
            prev = c
    E = energy(out, model.Jh, model.Jv, model.h)
    return dict(spins=out, logq=logq, energy=E, clamps=clamps,
                both_nonpos=both, near=nnear, min_gap=min_gap)


def sample(model, envs, batch, seed, step=0, first_id=0, inst=0, ids=None):
    """Draw `batch` proposals; proposal j uses id = first_id + j (or ids[j])."""
    return run_rows(model, envs, batch, seed, step, first_id, inst, ids=ids)


def eval_logq(model, envs, spins):
    """ln q(s) of given configurations by the same arithmetic (eval mode)."""
    spins = np.asarray(spins)
    return run_rows(model, envs, spins.shape[0], spins=spins)
