"""Derivative of ln Z~ with the truncation isometries frozen (oracle, FP64).

The paper mentions derivatives of the logarithm of the approximate
contraction (Sec. 4, caption of the TRG comparison figure) but does not
define them.  The reading adopted here:

  * Each compression step of the environment build (App. A, successive SVD)
    maps the MPO-MPS product psi to an approximation of it.  On the states the
    build actually meets, that map equals the orthogonal projector P_k onto
    span{|sites 0..c*-1> x |right block of env k from column c*>}, where c* is
    the leftmost column whose left bond was truncated; the QR sweep and the
    SVDs that cut nothing change only the gauge.  Freezing the truncation
    means: keep P_k fixed (the identity if env k truncated nothing).
  * Then Z~_frozen(K) = <top| P_1 TM_1 P_2 TM_2 ... P_{Ly-1} TM_{Ly-1} |.> is
    multilinear in the site tensors and equals Z~ at the build point, and the
    derivative is exact wherever nothing was truncated.
  * d ln Z~ / d A_site is the environment of the site divided by Z~.  For the
    rows above the untruncated bottom region the environment comes from the
    upper state U_k = <top| P_1 TM_1 ... TM_{k-1} P_k (an MPS, compressed
    without loss) and the stored env k+1; the bottom region (rows whose envs
    below are all exact) is contracted exactly column by column with U on top.
  * Chain rule: A depends on K = beta J through the bond split of App. A and on
    beta h through exp(beta h s); d/dJ = beta d/dK, d/d beta = sum_b J_b d/dK_b
    + sum_i h_i d/d(beta h_i).  K = 0 (where the split is not differentiable)
    is rejected.

Test infrastructure only (see the package docstring).  Pinned by
tests/test_oracle_grad.py against brute force (untruncated), central finite
differences of frozen_logZ (truncated), and the identity
beta d_beta ln Z~ = sum_b J_b d_J ln Z~ (h = 0).
"""
import numpy as np

from . import bmps
from .ising import SPIN, Model


# ---------------------------------------------------------------------------
# frozen projectors and the forward frozen contraction

def cstar(envs):
    """Leftmost truncated column of every env (None where nothing was cut)."""
    return [min(t) if t else None for t in envs['trunc']]


def project(X, E, c0):
    """P_{c0} applied to the MPS X (list of [a,u,b]): overlap of columns
    c0.. with the right-isometric env tensors E[c0..], absorbed into column
    c0-1.  c0 = None is the identity.  Returns (tensors, ln scale): the
    overlap is kept at unit largest entry while it is carried and the removed
    scale is returned in logs (it can pass the fp64 range)."""
    if c0 is None:
        return [x.copy() for x in X], 0.0
    Lx = len(X)
    O = np.ones((1, 1))
    logscale = 0.0
    for c in range(Lx - 1, c0 - 1, -1):
        O = np.einsum('aub,eud,bd->ae', X[c], E[c], O)
        m = np.abs(O).max()
        if m > 0.0:
            O = O / m
            logscale += np.log(m)
    out = [X[c].copy() for c in range(c0 - 1)]
    out.append(np.einsum('aub,be->aue', X[c0 - 1], O))
    out.extend(E[c].copy() for c in range(c0, Lx))
    return out, logscale


def exact_compress(X):
    """The same MPS with bonds reduced to their exact ranks (no truncation).
    Returns (tensors, ln of the removed scale)."""
    Y, lognorm, _ = bmps.compress(X, 10 ** 9)
    return Y, lognorm


def frozen_logZ(model, envs, cs=None):
    """ln Z~_frozen for the couplings of `model`, with the projectors of the
    build `envs` (computed at other couplings) held fixed."""
    cs = cstar(envs) if cs is None else cs
    Ly, Lx = model.Ly, model.Lx
    phi = bmps.trivial_env(Lx)
    logs = 0.0
    for k in range(Ly - 1, 0, -1):
        X = bmps.apply_row(model, k, phi)
        X, lp = project(X, envs['env'][k], cs[k])
        phi, ln = exact_compress(X)
        logs += ln + lp
    lo, sign = bmps.row_overlap(model, 0, phi)
    return logs + lo


# ---------------------------------------------------------------------------
# derivatives of the leg factors (App. A split)

def dleg(K):
    """dP/dK [s, mu] and dQ/dK [mu, s] of the closed-form bond split."""
    K = float(K)
    if K == 0.0:
        raise ValueError("the bond split is not differentiable at K = 0")
    ch, sh = np.cosh(K), np.sinh(K)
    sg = 1.0 if K > 0 else -1.0
    d0 = sh / (2.0 * np.sqrt(ch))
    d1 = ch / (2.0 * np.sqrt(abs(sh)))
    dP = np.empty((2, 2))
    dQ = np.empty((2, 2))
    dP[:, 0] = d0
    dP[:, 1] = sg * d1 * SPIN
    dQ[0, :] = d0
    dQ[1, :] = d1 * SPIN
    return dP, dQ


def site_derivatives(model, r, c, g):
    """Contract the site environment g[l,u,d,x] (already divided by Z~) with
    the derivative of the MPO tensor wrt each of its bonds and its field.
    Returns dict {('h'|'v'|'f', index): value} of d ln Z~ / dK or / d(beta h)."""
    m = model
    beta = m.beta
    f = np.exp(beta * m.field(r, c) * SPIN)
    legs = dict(L=m.left_leg(r, c), R=m.right_leg(r, c), U=m.up_leg(r, c), D=m.down_leg(r, c))

    def contract(f_, L, R, U, D):
        A = np.einsum('s,ls,sx,us,sd->ludx', f_, L, R, U, D)
        return float((A * g).sum())

    out = {}
    if c > 0:
        _, dQ = dleg(beta * m.Jh[r, c - 1])
        out[('h', (r, c - 1))] = contract(f, dQ, legs['R'], legs['U'], legs['D'])
    if c < m.Lx - 1:
        dP, _ = dleg(beta * m.Jh[r, c])
        out[('h', (r, c))] = contract(f, legs['L'], dP, legs['U'], legs['D'])
    if r > 0:
        _, dQ = dleg(beta * m.Jv[r - 1, c])
        out[('v', (r - 1, c))] = contract(f, legs['L'], legs['R'], dQ, legs['D'])
    if r < m.Ly - 1:
        dP, _ = dleg(beta * m.Jv[r, c])
        out[('v', (r, c))] = contract(f, legs['L'], legs['R'], legs['U'], dP)
    out[('f', (r, c))] = contract(f * SPIN, legs['L'], legs['R'], legs['U'], legs['D'])
    return out


# ---------------------------------------------------------------------------
# site environments

def row_site_envs(model, r, U, E):
    """Environments g[l,u,d,x] / Z of every site of row r in <U|TM_r|E>."""
    Lx = model.Lx
    M = [model.site_tensor(r, c).sum(0) for c in range(Lx)]      # [l,u,d,x]
    # left envs L[c][y, l, a]: columns < c
    Lf = [np.ones((1, 1, 1))]
    for c in range(Lx):
        t = np.einsum('yla,yuz,ludx,adb->zxb', Lf[-1], U[c], M[c], E[c])
        Lf.append(t / np.abs(t).max())
    Rf = [None] * (Lx + 1)
    Rf[Lx] = np.ones((1, 1, 1))
    for c in range(Lx - 1, -1, -1):
        t = np.einsum('yuz,ludx,adb,zxb->yla', U[c], M[c], E[c], Rf[c + 1])
        Rf[c] = t / np.abs(t).max()
    out = []
    for c in range(Lx):
        g = np.einsum('yla,yuz,adb,zxb->ludx', Lf[c], U[c], E[c], Rf[c + 1])
        Z = float((g * M[c]).sum())
        out.append(g / Z)
    return out


_LET = 'abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWX'


def _column_subscripts(h):
    """Index letters of one strip column: U bonds (left/right), horizontal legs
    (left/right) and vertical legs v_0 (above the strip) .. v_h (below)."""
    assert 3 * h + 3 <= len(_LET)
    xl = _LET[0:h]
    xr = _LET[h:2 * h]
    v = _LET[2 * h:3 * h + 1]
    y, yp = _LET[3 * h + 1], _LET[3 * h + 2]
    return y, yp, xl, xr, v


def strip_site_envs(model, r0, U):
    """Environments g / Z of every site of rows r0..Ly-1, contracted exactly
    column by column with the bra U on top (legs of the bonds above row r0)
    and nothing below.  Column vectors are indexed [y, x_r0, ..., x_{Ly-1}]
    (U bond, then the horizontal leg of every strip row)."""
    Ly, Lx = model.Ly, model.Lx
    rows = list(range(r0, Ly))
    h = len(rows)
    M = [[model.site_tensor(r, c).sum(0) for c in range(Lx)] for r in rows]   # [l,u,d,x]
    y, yp, xl, xr, v = _column_subscripts(h)
    site_subs = [xl[i] + v[i] + v[i + 1] + xr[i] for i in range(h)]

    def left_step(Lc, c):
        expr = ','.join([y + xl, y + v[0] + yp] + site_subs) + '->' + yp + xr
        return np.einsum(expr, Lc, U[c], *[M[i][c] for i in range(h)], optimize=True)

    def right_step(Rc, c):
        expr = ','.join([yp + xr, y + v[0] + yp] + site_subs) + '->' + y + xl
        return np.einsum(expr, Rc, U[c], *[M[i][c] for i in range(h)], optimize=True)

    shape0 = (1,) * (h + 1)
    Lv = [np.ones(shape0)]
    for c in range(Lx):
        t = left_step(Lv[-1], c)
        Lv.append(t / np.abs(t).max())
    Rv = [None] * (Lx + 1)
    Rv[Lx] = np.ones(shape0)
    for c in range(Lx - 1, -1, -1):
        t = right_step(Rv[c + 1], c)
        Rv[c] = t / np.abs(t).max()

    out = {}
    for c in range(Lx):
        for j in range(h):
            ops = [Lv[c], Rv[c + 1], U[c], np.ones(1)]
            subs = [y + xl, yp + xr, y + v[0] + yp, v[h]]   # v_h: the absent leg below
            for i in range(h):
                if i != j:
                    ops.append(M[i][c])
                    subs.append(site_subs[i])
            g = np.einsum(','.join(subs) + '->' + site_subs[j], *ops, optimize=True)
            Z = float((g * M[j][c]).sum())
            out[(rows[j], c)] = g / Z
    return out


# ---------------------------------------------------------------------------
# the derivative

def bottom_region_start(envs):
    """kb: smallest k >= 1 with envs k..Ly-1 all untruncated (Ly if env Ly-1
    itself was truncated).  Rows kb-1..Ly-1 form the exact bottom strip."""
    Ly = len(envs['env']) - 1
    kb = Ly
    for k in range(Ly - 1, 0, -1):
        if envs['trunc'][k]:
            break
        kb = k
    return kb


def grad_frozen(model, envs):
    """d ln Z~ / dJh [Ly][Lx-1], d ln Z~ / dJv [Ly-1][Lx], d ln Z~ / d beta,
    and d ln Z~ / d(beta h) [Ly][Lx], all with the truncations frozen."""
    Ly, Lx, beta = model.Ly, model.Lx, model.beta
    cs = cstar(envs)
    kb = bottom_region_start(envs)
    dK = {}

    def add(dct):
        for key, val in dct.items():
            dK[key] = dK.get(key, 0.0) + val

    # upper states for rows 0 .. kb-1 (bra on the legs above row k)
    U = [np.ones((1, 1, 1)) for _ in range(Lx)]     # row 0: no legs above
    for k in range(0, kb - 1):
        g = row_site_envs(model, k, U, envs['env'][k + 1])
        for c in range(Lx):
            add(site_derivatives(model, k, c, g[c]))
        # U_{k+1} = P_{k+1} (U_k TM_k), compressed without loss
        Y = []
        for c in range(Lx):
            M = model.site_tensor(k, c).sum(0)               # [l,u,d,x]
            t = np.einsum('yuz,ludx->yldzx', U[c], M)
            y_, l_, d_, z_, x_ = t.shape
            Y.append(t.reshape(y_ * l_, d_, z_ * x_))
        Y, _ = project(Y, envs['env'][k + 1], cs[k + 1])
        U, _ = exact_compress(Y)
    r0 = max(kb - 1, 0)
    g = strip_site_envs(model, r0, U)
    for (r, c), gg in g.items():
        add(site_derivatives(model, r, c, gg))

    out = _assemble(model, dK)
    out.update(kb=kb, cstar=cs)
    return out


def _assemble(model, dK):
    """d/dK and d/d(beta h) per bond and site -> dJh, dJv, d beta, dH."""
    Ly, Lx, beta = model.Ly, model.Lx, model.beta
    dJh = np.zeros((Ly, Lx - 1))
    dJv = np.zeros((Ly - 1, Lx))
    dH = np.zeros((Ly, Lx))
    for (kind, idx), val in dK.items():
        if kind == 'h':
            dJh[idx] += beta * val
        elif kind == 'v':
            dJv[idx] += beta * val
        else:
            dH[idx] += val
    dbeta = ((dJh * model.Jh).sum() + (dJv * model.Jv).sum()) / beta if beta != 0 else 0.0
    if model.h is not None:
        dbeta += (dH * model.h).sum()
    return dict(dJh=dJh, dJv=dJv, dbeta=dbeta, dH=dH)


# ---------------------------------------------------------------------------
# two-sided estimate: upper boundary built top-down, lower boundary bottom-up

def upper_envs(model, D):
    """Top-down boundary MPS: U[r] approximates rows 0..r-1 with their down
    legs open (U[0] is the trivial boundary), built by the same
    apply-and-compress step as the bottom-up environments (App. A), with the
    row MPO applied from above."""
    Ly, Lx = model.Ly, model.Lx
    U = [None] * Ly
    U[0] = bmps.trivial_env(Lx)
    for r in range(1, Ly):
        X = []
        for c in range(Lx):
            M = model.site_tensor(r - 1, c).sum(axis=0)    # [l,u,d,x]
            t = np.einsum('aub,ludx->aldbx', U[r - 1][c], M)
            a, l, d, b, x = t.shape
            X.append(t.reshape(a * l, d, b * x))
        U[r], _, _ = bmps.compress(X, D)
    return U


def grad_two_sided(model, envs, D=None):
    """Estimate of d ln Z / dJh, dJv, d beta and d(beta h) from two
    boundaries: every site's environment is the exact contraction of its row
    between the top-down boundary of the rows above and the stored bottom-up
    env of the rows below, divided by that row's value.  Exact when nothing
    is truncated; it is not the derivative of ln Z~ (the frozen form is)."""
    D = envs['D'] if D is None else D
    Ly, Lx = model.Ly, model.Lx
    U = upper_envs(model, D)
    dK = {}
    for r in range(Ly):
        g = row_site_envs(model, r, U[r], envs['env'][r + 1])
        for c in range(Lx):
            for key, val in site_derivatives(model, r, c, g[c]).items():
                dK[key] = dK.get(key, 0.0) + val
    return _assemble(model, dK)
