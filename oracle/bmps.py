"""Approximate contraction by boundary MPS (App. A, oracle, FP64).

The paper writes Z = <bot| TM_{L-1} ... TM_2 |top> (Eq. braket-top-tm-bot) and
contracts it row by row: the row MPO is applied to the current boundary MPS
(bond dimension grows by the MPO bond d = 2) and the product is compressed
back to bond dimension D by "successive SVD" (App. A, Fig. mpoMpsRenormalisation).

Readings adopted (the paper gives no more detail):
  * Direction: the recursion runs bottom-up, so that the sequential sampler can
    start at row 0 with the environment of all rows below already stored.
    Env k (k = 1..Ly-1) approximates rows k..Ly-1 with their up legs open; its
    physical index is the leg of the vertical bond (k-1,c)-(k,c).
  * Successive SVD: a left-to-right QR sweep makes the product left-canonical,
    then a right-to-left sweep of SVDs keeps the chi = min(D, rows, cols)
    largest singular values at every bond (no threshold), absorbing U S into
    the left neighbour.  Each stored env is right-orthonormal with its centre
    at column 0 and unit norm; the removed norms give ell_k.
  * ln Z~ = sum_k ell_k + ln <top|env_1>.

Each env tensor is stored as E[a, u, b] (left bond, physical leg, right bond).

Test infrastructure only (see the package docstring).
"""
import numpy as np


def trivial_env(Lx):
    """The empty boundary below the last row: bond 1, physical leg of dim 1."""
    return [np.ones((1, 1, 1)) for _ in range(Lx)]


def apply_row(model, k, env_below):
    """MPO-MPS product of App. A Fig. mpoMpsRenormalisation (b).

    X_c[(a,l), u, (b,x)] = sum_d E_c[a,d,b] M_c[l,u,d,x],  M = sum_s T[s].
    """
    X = []
    for c in range(model.Lx):
        M = model.site_tensor(k, c).sum(axis=0)           # [l,u,d,x]
        E = env_below[c]                                   # [a,d,b]
        Xc = np.einsum('adb,ludx->alubx', E, M)
        a, l, u, b, x = Xc.shape
        X.append(Xc.reshape(a * l, u, b * x))
    return X


def compress(X, D):
    """Successive-SVD compression of an MPS to bond D (App. A; reading above).

    Returns (tensors, ln of the removed norm, list of truncated bonds).  A bond
    c (between columns c-1 and c) is "truncated" when chi < min(rows, cols) of
    the SVD taken at column c.
    """
    X = [x.copy() for x in X]
    Lx = len(X)
    # left-to-right QR sweep: X_c <- Q, X_{c+1} <- R X_{c+1}; the carried
    # factor is brought back to unit norm at every step and its norm logged
    # (a row's weight can pass the fp64 range before the sweep ends)
    lognorm = 0.0
    for c in range(Lx - 1):
        a, u, b = X[c].shape
        q, r = np.linalg.qr(X[c].reshape(a * u, b))
        X[c] = q.reshape(a, u, q.shape[1])
        X[c + 1] = np.einsum('ij,jub->iub', r, X[c + 1])
        s = np.linalg.norm(X[c + 1])
        if s > 0.0:
            X[c + 1] = X[c + 1] / s
            lognorm += np.log(s)
    n = np.linalg.norm(X[Lx - 1])
    X[Lx - 1] = X[Lx - 1] / n
    lognorm += np.log(n)
    truncated = []
    # right-to-left SVD sweep with truncation to D
    for c in range(Lx - 1, 0, -1):
        a, u, b = X[c].shape
        U, S, Vt = np.linalg.svd(X[c].reshape(a, u * b), full_matrices=False)
        chi = min(D, S.shape[0])
        if chi < S.shape[0]:
            truncated.append(c)
        X[c] = Vt[:chi].reshape(chi, u, b)
        X[c - 1] = np.einsum('aub,bk->auk', X[c - 1], U[:, :chi] * S[:chi])
    m = np.linalg.norm(X[0])
    X[0] = X[0] / m
    return X, lognorm + np.log(m), truncated


def row_overlap(model, r, env_below):
    """ln of the exact contraction of row r (its up legs absent, i.e. r = 0, or
    closed) with the boundary MPS below, left to right with log-scaling.
    Returns (ln |value|, sign)."""
    v = np.ones((1, 1))                                    # [l, a]
    logscale = 0.0
    for c in range(model.Lx):
        M = model.site_tensor(r, c).sum(axis=0)            # [l,u,d,x], u dim 1
        v = np.einsum('la,ludx,adb->xb', v, M, env_below[c])
        s = np.abs(v).max()
        v = v / s
        logscale += np.log(s)
    val = v[0, 0]
    return logscale + np.log(abs(val)), np.sign(val)


def build_envs(model, D):
    """Bottom-up boundary-MPS environments and ln Z~.

    Returns a dict with
        env[k]   list over columns of E[a,u,b], k = 1..Ly (env[Ly] trivial)
        ell[k]   ln of the norm removed at step k
        trunc[k] truncated bonds of step k
        logZ     sum_k ell_k + ln <top|env_1>
        sign     sign of <top|env_1> (Z~ <= 0 breaks irreducibility, App. A)
    """
    Ly, Lx = model.Ly, model.Lx
    env = [None] * (Ly + 1)
    ell = np.zeros(Ly + 1)
    trunc = [[] for _ in range(Ly + 1)]
    env[Ly] = trivial_env(Lx)
    for k in range(Ly - 1, 0, -1):
        X = apply_row(model, k, env[k + 1])
        env[k], ell[k], trunc[k] = compress(X, D)
    lo, sign = row_overlap(model, 0, env[1])
    return dict(env=env, ell=ell, trunc=trunc, logZ=ell.sum() + lo, sign=sign,
                D=D)
