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
