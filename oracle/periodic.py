"""Periodic boundaries through alternately frozen lines (oracle, FP64).

Section "Arbitrary boundary conditions" (the cylinder figure and the table of
TNMH iterations for periodic Gaussian spin glasses): a lattice whose boundary
identifies opposite edges is sampled with the open-boundary machinery by
keeping one line of spins unchanged during a TNMH step.  The frozen spins act
on their free neighbours as local fields, the rest is an open lattice sampled
and accepted as before, and the frozen line moves from step to step so that
every spin gets refreshed.

Readings adopted:
  * Geometry.  The lattice is Ly x Lx and wraps along x (wrap_x), along y
    (wrap_y) or both (torus).  Jh[r][c] couples (r,c)-(r,(c+1) mod Lx), shape
    [Ly][Lx] when wrapped along x and [Ly][Lx-1] otherwise; Jv[r][c] couples
    (r,c)-((r+1) mod Ly,c), shape [Ly][Lx] when wrapped along y and [Ly-1][Lx]
    otherwise.  A wrapped direction has at least three sites, so no two sites
    share two bonds.
  * Cut.  A step freezes column cut_col of every chain if the lattice wraps
    along x, and row cut_row if it wraps along y (on the torus a cross, the
    smallest set whose removal leaves a rectangle).  The free spins form an
    open lattice of (Ly - wrap_y) x (Lx - wrap_x) sites whose site (r', c') is
    ((cut_row + 1 + r') mod Ly, (cut_col + 1 + c') mod Lx) in a wrapped
    direction and (r', c') otherwise: the open lattice starts just after the
    frozen line.  Its couplings are those between free sites; a free site next
    to the frozen line gets the field J s_frozen of that bond, added to its own
    field in the order left, right, up, down (one double-precision sum each;
    J s is exact for s = +-1).
  * Acceptance.  The open model's energy differs from the periodic one by a sum
    over the frozen spins alone, the same for the current state and the
    proposal, so Eq. (mh-acc) with the prior of Eq. (tns-prior) is evaluated
    with the open model's energies and ln q (the current state's ln q by the
    eval mode of the sampler under the new cut).  The step is a Metropolis-
    Hastings update of the free spins given the frozen ones, hence leaves the
    periodic Boltzmann distribution invariant for any sequence of cuts chosen
    independently of the state.
  * Random numbers.  Chain j of instance m draws its proposal with id j and
    inst m at step t, and its acceptance from counter (0, j, t, m << 2 | 1),
    the counters of chain j of instance m of a batch of open instances.
  * The cut schedule is an input of every step (the paper alternates two
    opposite lines, or picks lines at random); on the torus no two fixed
    crosses refresh every site, since the two sites where the row of one meets
    the column of the other stay frozen.

Chains of one instance whose frozen lines agree share one environment build
(the open model depends on the frozen spins only).

Single-spin-flip Metropolis sweeps (Sec. 3) on the identified lattice follow
oracle.metropolis with the wrapping neighbours: checkerboard order (r + c
even first), which needs an even length along a wrapped direction so that
same-colour sites share no bond; local field h + left + right + up + down in
that order; flip iff u < exp(-(beta 2 s F)); u from Philox stream 2 at counter
(sweep * 2^14 + i // 4, chain j, step, m << 2 | 2), word i % 4.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .ising import Model
from .bmps import build_envs
from .sampler import sample, eval_logq
from .mh import accept_uniforms, mh_decide
from .metropolis import sweep_uniforms


def check_shapes(Lx, Ly, Jh, Jv, h, wrap_x, wrap_y):
    assert not wrap_x or Lx >= 3, "a wrapped direction needs at least 3 sites"
    assert not wrap_y or Ly >= 3, "a wrapped direction needs at least 3 sites"
    assert np.shape(Jh) == (Ly, Lx if wrap_x else Lx - 1)
    assert np.shape(Jv) == (Ly if wrap_y else Ly - 1, Lx)
    assert h is None or np.shape(h) == (Ly, Lx)


def energy(spins, Jh, Jv, h, wrap_x, wrap_y):
    """Eq. (ising) on the identified lattice: -sum h s - sum over every bond
    (including the wrapping ones) of J s_i s_j, per configuration."""
    s = np.asarray(spins, dtype=np.float64)
    Ly, Lx = s.shape[-2:]
    check_shapes(Lx, Ly, Jh, Jv, h, wrap_x, wrap_y)
    right = np.roll(s, -1, axis=-1) if wrap_x else s[..., :, 1:]
    left = s if wrap_x else s[..., :, :-1]
    down = np.roll(s, -1, axis=-2) if wrap_y else s[..., 1:, :]
    up = s if wrap_y else s[..., :-1, :]
    e = -(np.asarray(Jh) * left * right).sum(axis=(-1, -2))
    e = e - (np.asarray(Jv) * up * down).sum(axis=(-1, -2))
    if h is not None:
        e = e - (np.asarray(h) * s).sum(axis=(-1, -2))
    return e


def n_bonds(Lx, Ly, wrap_x, wrap_y):
    return Ly * (Lx if wrap_x else Lx - 1) + (Ly if wrap_y else Ly - 1) * Lx


def link_overlap(a, b, wrap_x, wrap_y):
    """sum over every bond <ij> of the identified lattice of a_i a_j b_i b_j."""
    ab = np.asarray(a, dtype=np.int64) * np.asarray(b, dtype=np.int64)
    right = np.roll(ab, -1, axis=-1) if wrap_x else ab[..., :, 1:]
    left = ab if wrap_x else ab[..., :, :-1]
    down = np.roll(ab, -1, axis=-2) if wrap_y else ab[..., 1:, :]
    up = ab if wrap_y else ab[..., :-1, :]
    return (left * right).sum(axis=(-1, -2)) + (up * down).sum(axis=(-1, -2))


def open_sites(Lx, Ly, cut_row, cut_col, wrap_x, wrap_y):
    """Rows and columns of the periodic lattice that the open lattice's rows
    r' and columns c' stand for."""
    rows = (cut_row + 1 + np.arange(Ly - 1)) % Ly if wrap_y else np.arange(Ly)
    cols = (cut_col + 1 + np.arange(Lx - 1)) % Lx if wrap_x else np.arange(Lx)
    return rows, cols


def cut_model(Jh, Jv, h, beta, spins, cut_row, cut_col, wrap_x, wrap_y):
    """The open model of the free spins given one configuration's frozen line(s)."""
    Jh = np.asarray(Jh, dtype=np.float64)
    Jv = np.asarray(Jv, dtype=np.float64)
    s = np.asarray(spins, dtype=np.float64)
    Ly, Lx = s.shape
    check_shapes(Lx, Ly, Jh, Jv, h, wrap_x, wrap_y)
    rows, cols = open_sites(Lx, Ly, cut_row, cut_col, wrap_x, wrap_y)
    R, C = np.meshgrid(rows, cols, indexing="ij")
    Lyo, Lxo = len(rows), len(cols)
    Jho = Jh[R[:, :-1], C[:, :-1]]        # bond from column cols[c'] to cols[c' + 1]
    Jvo = Jv[R[:-1, :], C[:-1, :]]        # bond from row rows[r'] to rows[r' + 1]
    left = np.zeros((Lyo, Lxo))
    right = np.zeros((Lyo, Lxo))
    up = np.zeros((Lyo, Lxo))
    down = np.zeros((Lyo, Lxo))
    if wrap_x:
        left[:, 0] = Jh[rows, cut_col] * s[rows, cut_col]
        right[:, -1] = Jh[rows, (cut_col - 1) % Lx] * s[rows, cut_col]
    if wrap_y:
        up[0, :] = Jv[cut_row, cols] * s[cut_row, cols]
        down[-1, :] = Jv[(cut_row - 1) % Ly, cols] * s[cut_row, cols]
    base = np.zeros((Lyo, Lxo)) if h is None else np.asarray(h, dtype=np.float64)[R, C]
    ho = (((base + left) + right) + up) + down
    return Model(Jho, Jvo, ho, beta), rows, cols


def frozen_key(spins, cut_row, cut_col, wrap_x, wrap_y):
    s = np.asarray(spins, dtype=np.int8)
    parts = []
    if wrap_x:
        parts.append(s[:, cut_col])
    if wrap_y:
        parts.append(s[cut_row, :])
    return b"".join(p.tobytes() for p in parts)


def step(instances, spins, seed, t, cut_row, cut_col, D, wrap_x, wrap_y, fit_sweeps=0):
    """One TNMH step with the given cut for every chain.

    instances: list of dicts (Jh, Jv, h or None, beta, chains); spins
    [sum chains][Ly][Lx] int8, chains of instance 0 first.  Returns the new
    spins, their periodic energies and the accept flags.  fit_sweeps: the
    compression of the environment builds (oracle.bmps.build_envs).
    """
    spins = np.array(spins, dtype=np.int8)
    out = spins.copy()
    acc = np.zeros(spins.shape[0], dtype=bool)
    Ly, Lx = spins.shape[1:]
    g0 = 0
    for m, it in enumerate(instances):
        C = it["chains"]
        u = accept_uniforms(C, seed, t, inst=m)
        groups = {}
        for j in range(C):
            groups.setdefault(frozen_key(spins[g0 + j], cut_row, cut_col, wrap_x, wrap_y), []).append(j)
        for js in groups.values():
            model, rows, cols = cut_model(it["Jh"], it["Jv"], it.get("h"), it["beta"], spins[g0 + js[0]],
                                          cut_row, cut_col, wrap_x, wrap_y)
            envs = build_envs(model, D, fit_sweeps)
            cur = spins[g0 + np.array(js)][:, rows][:, :, cols]
            ev = eval_logq(model, envs, cur)
            prop = sample(model, envs, len(js), seed, step=t, inst=m, ids=np.array(js))
            ok, _ = mh_decide(ev["logq"], ev["energy"], prop["logq"], prop["energy"], model.beta,
                              u[np.array(js)])
            for k, j in enumerate(js):
                if ok[k]:
                    out[g0 + j][np.ix_(rows, cols)] = prop["spins"][k]
                acc[g0 + j] = ok[k]
        g0 += C
    E = np.zeros(spins.shape[0])
    g0 = 0
    for it in instances:
        C = it["chains"]
        E[g0:g0 + C] = energy(out[g0:g0 + C], it["Jh"], it["Jv"], it.get("h"), wrap_x, wrap_y)
        g0 += C
    return out, E, acc


def local_field(s, Jh, Jv, h, wrap_x, wrap_y):
    """F[..., r, c] = h + J_left s_left + J_right s_right + J_up s_up + J_down s_down
    on the identified lattice, added in this order (0 for a missing neighbour)."""
    s = np.asarray(s, dtype=np.float64)
    Ly, Lx = s.shape[-2:]
    Jh = np.asarray(Jh, dtype=np.float64)
    Jv = np.asarray(Jv, dtype=np.float64)
    left = np.zeros(s.shape)
    right = np.zeros(s.shape)
    up = np.zeros(s.shape)
    down = np.zeros(s.shape)
    for c in range(Lx):
        if c > 0 or wrap_x:
            left[..., :, c] = Jh[:, (c - 1) % Lx] * s[..., :, (c - 1) % Lx]
        if c < Lx - 1 or wrap_x:
            right[..., :, c] = Jh[:, c] * s[..., :, (c + 1) % Lx]
    for r in range(Ly):
        if r > 0 or wrap_y:
            up[..., r, :] = Jv[(r - 1) % Ly, :] * s[..., (r - 1) % Ly, :]
        if r < Ly - 1 or wrap_y:
            down[..., r, :] = Jv[r, :] * s[..., (r + 1) % Ly, :]
    F = np.zeros(s.shape) if h is None else np.broadcast_to(np.asarray(h, dtype=np.float64), s.shape).copy()
    return (((F + left) + right) + up) + down


def sweeps(instances, spins, seed, step, nsweeps, wrap_x, wrap_y):
    """nsweeps checkerboard Metropolis sweeps of every chain on the identified
    lattice (new array) and the accepted flips per chain."""
    s = np.array(spins, dtype=np.float64)
    T, Ly, Lx = s.shape
    assert not (wrap_x and Lx % 2) and not (wrap_y and Ly % 2), "checkerboard needs even wrapped lengths"
    rr, cc = np.meshgrid(np.arange(Ly), np.arange(Lx), indexing="ij")
    colour = (rr + cc) & 1
    flips = np.zeros(T, dtype=np.int64)
    g0 = 0
    for m, it in enumerate(instances):
        C = it["chains"]
        x = s[g0:g0 + C]
        for k in range(nsweeps):
            u = sweep_uniforms(C, Ly * Lx, seed, step, k, inst=m).reshape(C, Ly, Lx)
            for col in (0, 1):
                F = local_field(x, it["Jh"], it["Jv"], it.get("h"), wrap_x, wrap_y)
                flip = (u < np.exp(-(it["beta"] * ((2.0 * x) * F)))) & (colour == col)[None]
                x = np.where(flip, -x, x)
                flips[g0:g0 + C] += flip.sum(axis=(1, 2))
        s[g0:g0 + C] = x
        g0 += C
    return s.astype(np.int8), flips
