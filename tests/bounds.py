"""Error bounds of results that are fixed linear maps of the current series J.

delta mu (Eq. (4): Omega times the time integral of J_ind) and J_ind = J - J(0)
are linear in J, so a J within eps max|J| of the oracle bounds their errors by
the map's norm times eps max|J|.  Their own relative errors are inflated by
cancellation (J_ind is a small difference of large currents), so the parity
tests check them against these bounds."""

import numpy as np

J_TOL = 1e-10


def dmu_bound(j_ref, dt, omega, eps=J_TOL):
    """|d dmu_n| <= Omega t_n (max_m |dJ_m| + |dJ_0|) <= 2 Omega T eps max|J| (trapezoid weights sum to t_n)."""
    n = len(j_ref) - 1
    return 2.0 * abs(omega) * n * dt * eps * float(np.abs(j_ref).max())


def jind_bound(j_ref, eps=J_TOL):
    """|d(J_n - J_0)| <= 2 eps max|J|."""
    return 2.0 * eps * float(np.abs(j_ref).max())
