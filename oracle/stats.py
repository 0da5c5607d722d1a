"""Chain statistics (oracle, FP64): Eqs. (cauto) and (c-auto-int).

C_X(t) = (<X(t0) X(t0+t)> - <X(t0)><X(t0+t)>) / (<X^2> - <X>^2), averaged over
chains and over t0 after equilibration, and tau_int(t) = 1 + 2 sum_{t'<=t} C(t').

Readings adopted (the paper gives neither): the first 10% of the steps are
discarded as burn-in, and the sum is cut at Sokal's automatic window, the
smallest W with W >= 6 tau_int(W).

Test infrastructure only (see the package docstring).
"""
import numpy as np


def autocorr(series):
    """C(t) for series [steps, chains], t = 0..steps-1 (Eq. cauto)."""
    x = np.asarray(series, dtype=np.float64)
    n = x.shape[0]
    x = x - x.mean()
    var = (x * x).mean()
    if var == 0.0:
        return np.concatenate([[1.0], np.zeros(n - 1)])
    c = np.array([(x[:n - t] * x[t:]).mean() for t in range(n)])
    return c / var


def tau_int(series, burn=0.1, c_window=6.0):
    """Integrated autocorrelation time with Sokal's window (Eq. c-auto-int)."""
    x = np.asarray(series, dtype=np.float64)
    x = x[int(burn * x.shape[0]):]
    C = autocorr(x)
    tau = 1.0
    for W in range(1, len(C)):
        tau = tau + 2.0 * C[W]
        if W >= c_window * tau:
            return tau, W
    return tau, len(C) - 1


# ---------------------------------------------------------------------------
# Equilibration test of Sec. 3, Eq. (Delta), for spin glasses with Gaussian
# couplings of unit variance and no field.  Integrating by parts over one
# Gaussian coupling gives E_J[J <s_i s_j>] = beta E_J[1 - <s_i s_j>^2], so at
# equilibrium the disorder-averaged energy per site and the link overlap
# satisfy
#     Delta = [<H>]_av / |V| + beta (|E| - sum_<ij> [<s_i s_j>^2]_av) / |V| = 0,
# |V| sites, |E| bonds.  <s_i s_j>^2 is estimated from two independent
# replicas a, b of the same instance: s_i^a s_j^a s_i^b s_j^b.

def link_overlap(a, b):
    """sum over the bonds <ij> of a_i a_j b_i b_j, per configuration pair
    (a, b: int arrays [..., Ly, Lx] of +-1)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    ab = a * b
    return ((ab[..., :, :-1] * ab[..., :, 1:]).sum(axis=(-1, -2))
            + (ab[..., :-1, :] * ab[..., 1:, :]).sum(axis=(-1, -2)))


def delta(mean_energy, mean_link_overlap, beta, n_sites, n_bonds):
    """Eq. (Delta) from the disorder averages of <H> and of sum_<ij> <s_i s_j>^2."""
    return mean_energy / n_sites + beta * (n_bonds - mean_link_overlap) / n_sites
