"""Exact results for the 2D square-lattice Ising model (J = 1, k_B = 1), used
to pin the oracle's Markov chain to the physics it must sample.

- brute_force(L, T): direct enumeration of all 2^(L*L) states of the L x L
  torus (L = 4: 65536 states); exact <e> and <|m|> per spin.
- kaufman_energy(L, T): exact energy per spin of the finite L x L torus from
  Kaufman's partition function (Phys. Rev. 76, 1232 (1949)), in the form
  given by Ferdinand and Fisher (Phys. Rev. 185, 832 (1969)):
      Z = 1/2 (2 sinh 2K)^(L^2/2) (Z1 + Z2 + Z3 + Z4),
      Z1,2 = prod_{r=0}^{L-1} 2 cosh / sinh (L g_{2r+1} / 2),
      Z3,4 = prod_{r=0}^{L-1} 2 cosh / sinh (L g_{2r} / 2),
      cosh g_k = cosh 2K coth 2K - cos(pi k / L) (k >= 1),
      g_0 = 2K + ln tanh K,
  and e = -(1/L^2) d ln Z / dK.
- brute_force_moments(L, T): exact canonical averages <E>, <E^2>, <|M|>,
  <M^2>, <M^4> (whole-lattice E, M) by the same enumeration.
- kaufman_specific_heat(L, T): exact specific heat per spin of the finite
  torus, c = K^2 d^2 ln Z / dK^2 / L^2 (K = 1/T), from the same Z.
- onsager_energy(T): Onsager's infinite-lattice energy per spin,
      u = -coth 2K [1 + (2/pi)(2 tanh^2 2K - 1) K1(kappa)],
      kappa = 2 sinh 2K / cosh^2 2K.
- yang_magnetisation(T): (1 - sinh^-4 2K)^(1/8) below T_c, 0 above.
"""
import math

import mpmath
import numpy as np

TC = 2.0 / math.log(1.0 + math.sqrt(2.0))


def brute_force(L, T):
    n = L * L
    idx = np.arange(1 << n, dtype=np.uint32)
    spins = ((idx[:, None] >> np.arange(n, dtype=np.uint32)[None, :]) & 1).astype(np.int8) * 2 - 1
    s = spins.reshape(-1, L, L).astype(np.int32)
    E = -(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))
    M = s.sum(axis=(1, 2))
    E = E.astype(np.float64)
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()
    e = (w * E).sum() / Z / n
    am = (w * np.abs(M)).sum() / Z / n
    return float(e), float(am)


def brute_force_moments(L, T):
    n = L * L
    idx = np.arange(1 << n, dtype=np.uint32)
    spins = ((idx[:, None] >> np.arange(n, dtype=np.uint32)[None, :]) & 1).astype(np.int8) * 2 - 1
    s = spins.reshape(-1, L, L).astype(np.int32)
    E = (-(s * np.roll(s, -1, axis=2)).sum(axis=(1, 2)) - (s * np.roll(s, -1, axis=1)).sum(axis=(1, 2))).astype(
        np.float64)
    M = s.sum(axis=(1, 2)).astype(np.float64)
    w = np.exp(-(E - E.min()) / T)
    Z = w.sum()

    def avg(x):
        return float((w * x).sum() / Z)

    return {"E": avg(E), "E2": avg(E * E), "absM": avg(np.abs(M)), "M2": avg(M * M), "M4": avg(M ** 4)}


def kaufman_specific_heat(L, T, dps=60):
    with mpmath.workdps(dps):
        K = 1 / mpmath.mpf(T)
        d2 = mpmath.diff(lambda k: _lnZ(L, k), K, 2)
        return float(K * K * d2 / (L * L))


def _lnZ(L, K):
    K = mpmath.mpf(K)
    c2, s2 = mpmath.cosh(2 * K), mpmath.sinh(2 * K)
    base = c2 * c2 / s2  # cosh 2K coth 2K

    def gamma(k):
        if k == 0:
            return 2 * K + mpmath.log(mpmath.tanh(K))
        return mpmath.acosh(base - mpmath.cos(mpmath.pi * k / L))

    z1 = z2 = z3 = z4 = mpmath.mpf(1)
    for r in range(L):
        go = gamma(2 * r + 1) * L / 2
        ge = gamma(2 * r) * L / 2
        z1 *= 2 * mpmath.cosh(go)
        z2 *= 2 * mpmath.sinh(go)
        z3 *= 2 * mpmath.cosh(ge)
        z4 *= 2 * mpmath.sinh(ge)
    return mpmath.log(mpmath.mpf(1) / 2) + (L * L / mpmath.mpf(2)) * mpmath.log(2 * s2) + mpmath.log(z1 + z2 + z3 + z4)


def kaufman_energy(L, T, dps=60):
    with mpmath.workdps(dps):
        K = 1 / mpmath.mpf(T)
        d = mpmath.diff(lambda k: _lnZ(L, k), K)
        return float(-d / (L * L))


def onsager_energy(T):
    from scipy.special import ellipk

    K = 1.0 / T
    s2, c2, t2 = math.sinh(2 * K), math.cosh(2 * K), math.tanh(2 * K)
    kappa = 2 * s2 / (c2 * c2)
    return -(1.0 / t2) * (1.0 + (2.0 / math.pi) * (2 * t2 * t2 - 1.0) * ellipk(kappa * kappa))


def yang_magnetisation(T):
    if T >= TC:
        return 0.0
    return (1.0 - math.sinh(2.0 / T) ** -4) ** 0.125


def binned_mean(x, nbins=20):
    """Mean and its standard error from nbins contiguous bins (absorbs the
    chain's autocorrelation when a bin is much longer than it)."""
    x = np.asarray(x, dtype=np.float64)
    nb = len(x) // nbins
    b = x[: nb * nbins].reshape(nbins, nb).mean(axis=1)
    return float(b.mean()), float(b.std(ddof=1) / math.sqrt(nbins))
