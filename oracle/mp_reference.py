"""High-precision reference reflectivity (test infrastructure only).

The Parratt recursion (an algorithm independent of the Abeles matrix product
that the FP64 oracle evaluates; identical in exact arithmetic) carried out in
mpmath at a chosen number of decimal digits, in the physical frame
(Im kz >= 0, e^{+2 i kz d}), with the same media, Nevot-Croce roughness and
row conventions as the oracle (Sec. 2.1 forward model; roughness per
interface, sigma of row j+1 for the interface above medium j+1):

    X_{N+1} = 0,
    X_j = (r'_j + X_{j+1} e^{2 i kz_{j+1} d_{j+1}}) / (1 + r'_j X_{j+1} e^{2 i kz_{j+1} d_{j+1}}),
    r'_j = (kz_j - kz_{j+1}) / (kz_j + kz_{j+1}) exp(-2 kz_j kz_{j+1} sigma_{j+1}^2),
    R = |X_0|^2.

Pinned by tests/test_oracle_pins.py: at one interface it equals the
Fresnel / Nevot-Croce closed form evaluated at the same precision, and on
shallow stacks the FP64 Abeles oracle agrees with it to rounding.
"""
from __future__ import annotations

import mpmath


def parratt_R(rows, q, dps=50):
    """R(q) of the stack `rows` ((L+2) x 4: d, rho_re, rho_im, sigma) at
    `dps` decimal digits, returned as an mpmath number."""
    with mpmath.workdps(dps):
        N = len(rows) - 2
        q = mpmath.mpf(q)
        rho0 = mpmath.mpf(rows[0][1])
        k = [q / 2]
        for j in range(1, N + 2):
            w = q * q / 4 - 4 * mpmath.pi * (mpmath.mpf(rows[j][1]) - rho0) \
                + 1j * 4 * mpmath.pi * abs(mpmath.mpf(rows[j][2]))
            k.append(mpmath.sqrt(w))

        def rp(j):
            if k[j] == k[j + 1]:
                return mpmath.mpc(0)
            r = (k[j] - k[j + 1]) / (k[j] + k[j + 1])
            return r * mpmath.exp(-2 * k[j] * k[j + 1] * mpmath.mpf(rows[j + 1][3]) ** 2)

        X = rp(N)
        for j in range(N - 1, -1, -1):
            Y = X * mpmath.exp(2j * k[j + 1] * mpmath.mpf(rows[j + 1][0]))
            r = rp(j)
            X = (r + Y) / (1 + r * Y)
        return abs(X) ** 2
