"""Exponential integral E1 in FP64 (oracle; test infrastructure only).

The real-space Stokeslet of the Hasimoto split (Section 3.2, eq. 3.15) needs
E1(z) = int_z^inf e^-t / t dt for z = xi^2 r^2 > 0 (eq. 3.16).  Written from
two textbook representations (Abramowitz & Stegun 5.1.11 and 5.1.22):

  z <= 1 :  E1(z) = -gamma - ln z - sum_{k>=1} (-z)^k / (k k!)
  z >  1 :  E1(z) = e^-z / (z + 1 - 1^2/(z + 3 - 2^2/(z + 5 - ...)))

Pinned against mpmath / scipy in the tests.
"""
import numpy as np

EULER_GAMMA = 0.57721566490153286060651209008240243


def e1(z):
    z = np.asarray(z, dtype=np.float64)
    out = np.empty_like(z)
    small = z <= 1.0
    zs = z[small]
    if zs.size:
        # series: terms t_k = (-z)^k / (k k!)
        acc = np.zeros_like(zs)
        p = np.ones_like(zs)  # (-z)^k / k!
        for k in range(1, 40):
            p = p * (-zs) / k
            acc += p / k
        out[small] = -EULER_GAMMA - np.log(zs) - acc
    zl = z[~small]
    if zl.size:
        # continued fraction evaluated bottom-up at fixed depth
        depth = 120
        t = zl + 2.0 * depth + 1.0
        for k in range(depth, 0, -1):
            t = zl + 2.0 * k - 1.0 - (k * k) / t
        out[~small] = np.exp(-zl) / t
    return out
