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
    largest singular values at every bond, absorbing U S into the left
    neighbour.  Each stored env is right-orthonormal on its nonzero rows, with
    its centre at column 0 and unit norm; the removed norms give ell_k.
  * Numerically zero singular values: a kept singular value s of the matrix
    M with s <= n eps ||M||_F, n the dimension of the factor kept orthonormal
    (u b for the successive SVD's right factor; in the fit a u on a
    left-to-right pass, v b on a right-to-left one), is not resolved in FP64:
    its vectors are rounding noise.
    Such a triplet is kept as zeros (its rows and columns of both factors set
    to 0; the bond keeps its dimension).  Keeping the library's noise vectors
    instead lets later rows amplify them: on a +-J 32x32 lattice at beta = 3,
    D = 32, ln Z~ then moves by O(1) under one-ulp changes of the couplings,
    while with the zeros it moves by 1e-12 relative.
  * ln Z~ = sum_k ell_k + ln <top|env_1>.
  * Two-site variational compression (the alternative App. A names for the
    Gaussian-disorder runs, after Schollwoeck's review): starting from the
    successive-SVD result, sweeps of two-site updates fit the bond-D MPS psi
    to the normalised product X^ (the left-canonical output of the QR sweep):
    with the blocks of psi left and right of sites (c, c+1) orthonormal, the
    two-site tensor that minimises ||X^ - psi|| is the contraction
    Theta = L_c X^_c X^_{c+1} R_{c+2} of X^ with those blocks; its SVD,
    truncated to D, gives the new psi_c, psi_{c+1} (left-canonical psi_c on a
    left-to-right pass, right-canonical psi_{c+1} on a right-to-left pass).
    One sweep is a left-to-right and a right-to-left pass; after the last one
    psi is right-orthonormal with its centre at column 0, and
    ell_k = ln ||X|| (removed by the QR sweep) + ln ||psi||.

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


def qr_sweep(X):
    """Left-to-right QR sweep: X becomes left-canonical with a unit-norm last
    tensor; returns (tensors, ln of the removed norm)."""
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
    return X, lognorm


def degenerate_cut(S, chi):
    """A truncation that keeps chi of the descending singular values S is
    degenerate when the last kept and the first dropped one are tied to
    1e-12 of the largest: which vectors are kept is then decided by rounding
    (reading: parity is not defined for such a cut; it is counted)."""
    return chi < S.shape[0] and (S[chi - 1] - S[chi]) < 1e-12 * S[0]


EPS = 2.220446049250313e-16


def resolved(S, chi, n, fro):
    """1 for each of the chi kept singular values that FP64 resolves, 0 for
    the numerically zero ones (s <= n eps ||M||_F; reading above)."""
    return (S[:chi] > n * EPS * fro).astype(np.float64)


def compress(X, D, degen=None):
    """Successive-SVD compression of an MPS to bond D (App. A; reading above).

    Returns (tensors, ln of the removed norm, list of truncated bonds).  A bond
    c (between columns c-1 and c) is "truncated" when chi < min(rows, cols) of
    the SVD taken at column c.  degen (a list, optional) receives one entry per
    degenerate cut.
    """
    X, lognorm = qr_sweep(X)
    Lx = len(X)
    truncated = []
    # right-to-left SVD sweep with truncation to D
    for c in range(Lx - 1, 0, -1):
        a, u, b = X[c].shape
        M = X[c].reshape(a, u * b)
        U, S, Vt = np.linalg.svd(M, full_matrices=False)
        chi = min(D, S.shape[0])
        if chi < S.shape[0]:
            truncated.append(c)
        if degen is not None and degenerate_cut(S, chi):
            degen.append(c)
        k = resolved(S, chi, u * b, np.linalg.norm(M))
        X[c] = (Vt[:chi] * k[:, None]).reshape(chi, u, b)
        X[c - 1] = np.einsum('aub,bk->auk', X[c - 1], U[:, :chi] * (S[:chi] * k))
    m = np.linalg.norm(X[0])
    X[0] = X[0] / m
    return X, lognorm + np.log(m), truncated


def fit_two_site(Xh, psi, D, sweeps, degen=None):
    """Two-site variational sweeps fitting psi (right-canonical, centre at
    column 0) to Xh; returns the fitted, unnormalised psi (right-canonical,
    centre at column 0).  degen (a list, optional) receives one entry per
    degenerate two-site cut."""
    Lx = len(Xh)
    psi = [p.copy() for p in psi]
    if Lx == 1:                       # one site: the fit is Xh itself
        return [Xh[0].copy()]
    one = np.ones((1, 1))

    # Each contraction is written as the one sum it defines; numpy picks the
    # order in which its pairs are multiplied (optimize=True).
    def right_env(c, R):              # R_c[b_psi, B] from R_{c+1}
        return np.einsum('aub,AuB,bB->aA', psi[c], Xh[c], R, optimize=True)

    def left_env(c, L):               # L_{c+1}[a_psi, A] from L_c
        return np.einsum('aub,aA,AuB->bB', psi[c], L, Xh[c], optimize=True)

    def theta(L, c, R):               # Theta[a, u, b, v] = L X^_c X^_{c+1} R
        return np.einsum('aA,AuM,MvB,bB->aubv', L, Xh[c], Xh[c + 1], R, optimize=True)

    for _ in range(sweeps):
        R = [None] * (Lx + 1)
        R[Lx] = one
        for c in range(Lx - 1, 1, -1):
            R[c] = right_env(c, R[c + 1])
        L = one
        for c in range(Lx - 1):       # left to right
            Th = theta(L, c, R[c + 2])
            a, u, b, v = Th.shape
            M = Th.transpose(0, 1, 3, 2).reshape(a * u, v * b)
            U, S, Vt = np.linalg.svd(M, full_matrices=False)
            chi = min(D, S.shape[0])
            if degen is not None and degenerate_cut(S, chi):
                degen.append(c)
            k = resolved(S, chi, a * u, np.linalg.norm(M))
            psi[c] = (U[:, :chi] * k).reshape(a, u, chi)
            psi[c + 1] = ((S[:chi] * k)[:, None] * Vt[:chi]).reshape(chi, v, b)
            L = left_env(c, L)
        Ls = [None] * Lx
        Ls[0] = one
        for c in range(Lx - 2):
            Ls[c + 1] = left_env(c, Ls[c])
        R = one
        for c in range(Lx - 2, -1, -1):   # right to left
            Th = theta(Ls[c], c, R)
            a, u, b, v = Th.shape
            M = Th.transpose(0, 1, 3, 2).reshape(a * u, v * b)
            U, S, Vt = np.linalg.svd(M, full_matrices=False)
            chi = min(D, S.shape[0])
            if degen is not None and degenerate_cut(S, chi):
                degen.append(c)
            k = resolved(S, chi, v * b, np.linalg.norm(M))
            psi[c + 1] = (Vt[:chi] * k[:, None]).reshape(chi, v, b)
            psi[c] = (U[:, :chi] * (S[:chi] * k)).reshape(a, u, chi)
            R = right_env(c + 1, R)
    return psi


def compress_variational(X, D, sweeps, degen=None):
    """Successive SVD followed by `sweeps` two-site variational sweeps (reading
    above).  Returns (tensors, ln of the removed norm, truncated bonds of the
    successive-SVD start).  degen as in compress, for every cut taken."""
    Xh, lognorm = qr_sweep(X)
    psi, lm, truncated = compress(Xh, D, degen)
    psi[0] = psi[0] * np.exp(lm)      # Xh ~ psi with the norm in the centre
    psi = fit_two_site(Xh, psi, D, sweeps, degen)
    m = np.linalg.norm(psi[0])
    psi[0] = psi[0] / m
    return psi, lognorm + np.log(m), truncated


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


def build_envs(model, D, fit_sweeps=0):
    """Bottom-up boundary-MPS environments and ln Z~ (fit_sweeps > 0: each
    compression is refined by that many two-site variational sweeps).

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
    degen = [[] for _ in range(Ly + 1)]
    env[Ly] = trivial_env(Lx)
    for k in range(Ly - 1, 0, -1):
        X = apply_row(model, k, env[k + 1])
        if fit_sweeps > 0:
            env[k], ell[k], trunc[k] = compress_variational(X, D, fit_sweeps, degen[k])
        else:
            env[k], ell[k], trunc[k] = compress(X, D, degen[k])
    lo, sign = row_overlap(model, 0, env[1])
    return dict(env=env, ell=ell, trunc=trunc, logZ=ell.sum() + lo, sign=sign,
                D=D, degenerate=[len(d) for d in degen])
