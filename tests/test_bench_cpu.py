"""Host-side accounting of bench.py: the algorithmic arithmetic per node update
that the roofline and ALU fractions divide by, counted by hand for known
equilibrium structures."""
import numpy as np

import bench


def test_dense_and_odd_polynomial_flops():
    q, D = 5, 5
    G = np.ones((q, D + 1))
    # phi sum (4 adds) + per population 5 FMAs of Horner and the BGK FMA, 2 flops each
    assert bench.algorithmic_flops_per_nu(G) == 4 + 5 * (2 * 5 + 2)
    G = np.zeros((q, 10))
    G[:, 1::2] = 1.0   # odd in phi, degree 9: Horner in phi^2 over 5 terms
    assert bench.algorithmic_flops_per_nu(G) == 4 + 1 + 5 * (2 * 4 + 1 + 2)


def test_power_sum_flops_follow_the_strided_layout():
    q = 5
    G = np.zeros((2, q, 4))
    G[0, :, 1:4] = 1.0      # integer class: degrees 1, 2, 3 -> phi * (3 terms in phi)
    G[1, :, 1:3] = 1.0      # half class: degrees 1, 2 -> phi^(3/2) * (2 terms in phi)
    # phi sum 4; class 0: 5 x (2 FMAs + 1 multiply by phi^d0); class 1: one product for
    # the class factor, 5 x (1 FMA + 1 FMA); BGK 5 FMAs
    assert bench.algorithmic_flops_power_sum(np.array([0.0, 0.5]), G) == 4 + 5 * 6 + 1 + 5 * 4 + 10
    H = np.zeros((2, q, 8))
    H[0, :, [1, 4, 7]] = 1.0    # degrees 1, 4, 7: phi * (3 terms in phi^3): 2 products for phi^3
    H[1, :, [2, 5]] = 1.0       # degrees 2, 5: phi^2 (1 product) * (2 terms in phi^3)
    assert bench.algorithmic_flops_power_sum(np.array([0.0, 0.5]), H) == \
        4 + 2 + 5 * 6 + (2 + 1 + 1) + 5 * 4 + 10
