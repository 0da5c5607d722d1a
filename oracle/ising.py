"""Ising instance, energy and local tensors (oracle, FP64).

Conventions
    Lattice Ly x Lx with open boundaries, row r = 0..Ly-1, column c = 0..Lx-1,
    site i = r*Lx + c.
    Jh[r][c] couples (r,c)-(r,c+1)  shape [Ly][Lx-1]
    Jv[r][c] couples (r,c)-(r+1,c)  shape [Ly-1][Lx]
    h[r][c]  field on (r,c)         shape [Ly][Lx] (None means 0)
    A spin value s in {+1,-1} has index (1-s)/2, so index 0 is +1.

Test infrastructure only (see the package docstring).
"""
import numpy as np

SPIN = np.array([1.0, -1.0])  # spin value of index 0 and index 1


def energy(spins, Jh, Jv, h=None):
    """Eq. (ising): H = -sum_i h_i s_i - sum_<ij> J_ij s_i s_j, per configuration.

    spins: int array [..., Ly, Lx] of +-1.  Returns float64 [...].
    """
    s = np.asarray(spins, dtype=np.float64)
    e = -(np.asarray(Jh) * s[..., :, :-1] * s[..., :, 1:]).sum(axis=(-1, -2))
    e = e - (np.asarray(Jv) * s[..., :-1, :] * s[..., 1:, :]).sum(axis=(-1, -2))
    if h is not None:
        e = e - (np.asarray(h) * s).sum(axis=(-1, -2))
    return e


def bond_weight(K):
    """App. A Eq. (transfMatrixFerro): W(s,s') = exp(K s s') with K = beta*J."""
    K = np.asarray(K, dtype=np.float64)
    return np.exp(K[..., None, None] * SPIN[:, None] * SPIN[None, :])


def bond_factors(K):
    """App. A: split W = P Q through the SVD of the symmetric 2x2 bond matrix.

    W = cosh K * (1,1)(1,1)^T + sinh K * (1,-1)(1,-1)^T, so with the singular
    vectors (1,+-1)/sqrt(2) and singular values 2cosh K, 2|sinh K| the square-root
    split (L = U sqrt(S), R = sqrt(S) V^T) reads, up to a +-1 gauge per column,
        P(s, 0) = sqrt(cosh K),  P(s, 1) = s * sqrt(|sinh K|)
        Q(0, s) = sqrt(cosh K),  Q(1, s) = sign(K) * s * sqrt(|sinh K|)
    P belongs to the left/top site of the bond and Q to the right/bottom site.
    Returns P [..., 2(s), 2(mu)] and Q [..., 2(mu), 2(s)].
    """
    K = np.asarray(K, dtype=np.float64)
    ch = np.sqrt(np.cosh(K))
    sh = np.sqrt(np.abs(np.sinh(K)))
    sg = np.where(K >= 0.0, 1.0, -1.0)
    P = np.empty(K.shape + (2, 2))
    Q = np.empty(K.shape + (2, 2))
    P[..., :, 0] = ch[..., None]
    P[..., :, 1] = sh[..., None] * SPIN
    Q[..., 0, :] = ch[..., None]
    Q[..., 1, :] = (sg * sh)[..., None] * SPIN
    return P, Q


class Model:
    """A 2D Ising instance with open boundaries and its bond factors."""

    def __init__(self, Jh, Jv, h, beta):
        self.Jh = np.asarray(Jh, dtype=np.float64)
        self.Jv = np.asarray(Jv, dtype=np.float64)
        self.Ly = self.Jv.shape[0] + 1
        self.Lx = self.Jh.shape[1] + 1
        assert self.Jh.shape == (self.Ly, self.Lx - 1)
        assert self.Jv.shape == (self.Ly - 1, self.Lx)
        self.h = None if h is None else np.asarray(h, dtype=np.float64)
        self.beta = float(beta)
        self.Ph, self.Qh = bond_factors(self.beta * self.Jh)
        self.Pv, self.Qv = bond_factors(self.beta * self.Jv)
        self.gauge_h = None
        self.gauge_v = None

    @property
    def n_sites(self):
        return self.Lx * self.Ly

    def field(self, r, c):
        return 0.0 if self.h is None else self.h[r, c]

    def set_gauge(self, Oh=None, Ov=None):
        """Insert an orthogonal 2x2 matrix O on the bond leg: P -> P O, Q -> O^T Q.

        W = P Q is unchanged, so every gauge-invariant output must be unchanged
        (the SVD split of App. A is only defined up to such a gauge).
        Oh: [Ly][Lx-1][2][2], Ov: [Ly-1][Lx][2][2].
        """
        Ph, Qh = bond_factors(self.beta * self.Jh)
        Pv, Qv = bond_factors(self.beta * self.Jv)
        if Oh is not None:
            Ph = np.einsum('...sm,...mn->...sn', Ph, Oh)
            Qh = np.einsum('...mn,...ms->...ns', Oh, Qh)
        if Ov is not None:
            Pv = np.einsum('...sm,...mn->...sn', Pv, Ov)
            Qv = np.einsum('...mn,...ms->...ns', Ov, Qv)
        self.Ph, self.Qh, self.Pv, self.Qv = Ph, Qh, Pv, Qv

    # Leg factors of site (r,c); a leg absent at the open boundary is a
    # dimension-1 leg carrying the value 1.
    def left_leg(self, r, c):   # [l, s]  (Q side of bond (r,c-1)-(r,c))
        return self.Qh[r, c - 1] if c > 0 else np.ones((1, 2))

    def right_leg(self, r, c):  # [s, x]  (P side of bond (r,c)-(r,c+1))
        return self.Ph[r, c] if c < self.Lx - 1 else np.ones((2, 1))

    def up_leg(self, r, c):     # [u, s]  (Q side of bond (r-1,c)-(r,c))
        return self.Qv[r - 1, c] if r > 0 else np.ones((1, 2))

    def down_leg(self, r, c):   # [s, d]  (P side of bond (r,c)-(r+1,c))
        return self.Pv[r, c] if r < self.Ly - 1 else np.ones((2, 1))

    def site_tensor(self, r, c):
        """App. A Eq. (tensor-general), one slice per spin value.

        T[s, l, u, d, x] = exp(beta h s) L(l,s) R(s,x) U(u,s) D(s,d); the MPO
        tensor is the sum over s, a fixed spin keeps one slice (App. A, the
        fixed-spin tensor).  The field factor is the site part of Eq. (ising).
        """
        f = np.exp(self.beta * self.field(r, c) * SPIN)
        return np.einsum('s,ls,sx,us,sd->sludx', f, self.left_leg(r, c),
                         self.right_leg(r, c), self.up_leg(r, c),
                         self.down_leg(r, c))
