"""Exact references, independent of the tensor-network code (oracle, FP64).

    brute_force      enumeration of all 2^N configurations, N <= 20:
                     Eqs. (boltzmann), (pf-ising)
    transfer_logZ    exact row-by-row transfer matrix over 2^Lx states, updated
                     one column at a time, with log-scaling (Lx <= ~18)
    log_boltzmann    ln pi(s) = -beta H(s) - ln Z, Eq. (boltzmann)
    onsager_minus_beta_f   bulk -beta f of the square-lattice ferromagnet
                     (Onsager 1944), the L -> infinity limit of ln Z / N

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .ising import energy


def all_configs(Ly, Lx):
    """All 2^(Ly*Lx) configurations; bit i of the index n is site i (1 -> -1)."""
    N = Ly * Lx
    n = np.arange(2 ** N, dtype=np.int64)
    bits = (n[:, None] >> np.arange(N)[None, :]) & 1
    return (1 - 2 * bits).reshape(-1, Ly, Lx).astype(np.int8)


def brute_force(Jh, Jv, h, beta):
    """Returns (configs, energies, ln Z, ln pi) by full enumeration."""
    Ly, Lx = np.asarray(Jv).shape[0] + 1, np.asarray(Jh).shape[1] + 1
    cfg = all_configs(Ly, Lx)
    E = energy(cfg, Jh, Jv, h)
    a = -beta * E
    amax = a.max()
    logZ = amax + np.log(np.exp(a - amax).sum())
    return cfg, E, logZ, a - logZ


def transfer_logZ(Jh, Jv, h, beta):
    """Exact ln Z by the row transfer matrix, one column update at a time.

    The state vector is indexed by the spins of the current row (bit c of the
    index is column c, 1 -> -1).  Moving from row r-1 to row r replaces one
    column's spin at a time, multiplying by exp(beta Jv s_old s_new) and summing
    over s_old; the horizontal bonds and fields of row r are diagonal.
    """
    Jh = np.asarray(Jh, dtype=np.float64)
    Jv = np.asarray(Jv, dtype=np.float64)
    Ly, Lx = Jv.shape[0] + 1, Jh.shape[1] + 1
    n = np.arange(2 ** Lx)
    s = (1 - 2 * ((n[:, None] >> np.arange(Lx)[None, :]) & 1)).astype(np.float64)

    def diag(r):
        e = (Jh[r][None, :] * s[:, :-1] * s[:, 1:]).sum(1)
        if h is not None:
            e = e + (np.asarray(h)[r][None, :] * s).sum(1)
        return beta * e   # -beta H restricted to row r

    logscale = 0.0
    a = diag(0)
    m = a.max()
    vec = np.exp(a - m)
    logscale += m
    for r in range(1, Ly):
        for c in range(Lx):
            K = beta * Jv[r - 1, c]
            flip = n ^ (1 << c)
            same, other = np.exp(K), np.exp(-K)
            vec = same * vec + other * vec[flip]
        a = diag(r)
        m = a.max()
        vec = vec * np.exp(a - m)
        logscale += m
        tot = vec.sum()
        vec /= tot
        logscale += np.log(tot)
    return logscale + np.log(vec.sum())


def log_boltzmann(spins, Jh, Jv, h, beta, logZ):
    """Eq. (boltzmann) in logs: ln pi(s) = -beta H(s) - ln Z."""
    return -beta * energy(spins, Jh, Jv, h) - logZ


def onsager_minus_beta_f(K):
    """Bulk -beta f(K) of the isotropic square-lattice Ising ferromagnet.

    -beta f = ln 2 + (1 / 8 pi^2) * int_0^{2pi} int_0^{2pi}
              ln[cosh^2(2K) - sinh(2K) (cos t1 + cos t2)] dt1 dt2
    evaluated with scipy's adaptive quadrature (the inner integral has a
    closed form in t2, used to keep the integrand smooth at K_c).
    """
    from scipy.integrate import quad
    c2 = np.cosh(2 * K) ** 2
    s2 = np.sinh(2 * K)

    def inner(t1):
        # int_0^{2pi} ln(a - b cos t2) dt2 = 2 pi ln((a + sqrt(a^2 - b^2)) / 2)
        a = c2 - s2 * np.cos(t1)
        b = s2
        return 2 * np.pi * np.log((a + np.sqrt(max(a * a - b * b, 0.0))) / 2.0)

    val, _ = quad(inner, 0.0, 2 * np.pi, limit=400, epsabs=1e-13, epsrel=1e-13,
                  points=[np.pi])
    return np.log(2.0) + val / (8 * np.pi ** 2)
