"""Fixtures under tests/golden/: values that the paper's printed formulas fix
exactly, checked against the code that uses them."""
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return [ln.split() for ln in fh if ln.strip() and not ln.startswith("#")]


def test_inlet_rows_follow_eq7():
    """The seeded input generator's nozzle profiles (both the parabolic
    velocity and the cubic temperature of eq. 7) at r_j = j + 1/2, R = 4,
    with U_max = 0.08, T_min = 0.2, T_max = 1.0."""
    from paper_1002_3028_amd import inputs
    rows = _rows("eq7_inlet_R4.txt")
    nr = len(rows)
    u_max, t_min, t_max = 0.08, 0.2, 1.0
    ux, ur, T = inputs.inlet_rows(nr, 4.0, u_max, T_in=t_max, T_amb=t_min, n_t=2,
                                  t_profile="cubic")
    for j, rr, uu, tt in rows:
        j = int(j)
        assert abs(float(Fraction(rr)) * 4.0 - (j + 0.5)) == 0.0
        for q in range(2):
            assert abs(ux[q, j] - u_max * float(Fraction(uu))) <= 1e-16
            assert abs(T[q, j] - (t_min + (t_max - t_min) * float(Fraction(tt)))) <= 1e-15
            assert ur[q, j] == 0.0
    # the flat profile keeps the velocity and sets T_max on the nozzle
    ux2, _, T2 = inputs.inlet_rows(nr, 4.0, u_max, T_in=t_max, T_amb=t_min)
    assert np.array_equal(ux2[0], ux[0])
    assert np.array_equal(T2[0], np.where(np.arange(nr) + 0.5 < 4.0, t_max, t_min))
