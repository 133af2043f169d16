"""The sign-folded form of the scaled Legendre recurrence run by the analysis
kernels and the split-bf16 synthesis tiles (the three-term recurrence in degree of
Section 3, with the scaling c_l folded into a'_l): with sigma_l = -1 for
l = 2, 3 (mod 4) and +1 otherwise, P_l = sigma_l Q_l obeys
P_l = P_{l-2} + a'_l s_l z P_{l-1}, s_l = +1 for odd l and -1 for even l, whenever
Q_l = a'_l z Q_{l-1} - Q_{l-2}.  Checked here in binary64 on random data, from start
degrees of every residue mod 4 (negative ones included: the seed start sits at
l = m - 1, m - 2)."""
import numpy as np
import pytest


def sigma(l):
    return -1.0 if (l & 2) else 1.0  # two's complement: also right for l < 0


@pytest.mark.parametrize("l0", [-2, -1, 0, 1, 2, 3, 5, 18, 33])
def test_sign_folded_recurrence_matches(l0):
    rng = np.random.default_rng(100 + l0 + 2)
    n = 40
    a = rng.uniform(0.5, 2.0, n)        # a'_{l0+2+k}
    z = rng.uniform(-1.0, 1.0)
    q = [rng.normal(), rng.normal()]     # Q_{l0}, Q_{l0+1}
    p = [sigma(l0) * q[0], sigma(l0 + 1) * q[1]]
    for k in range(n):
        l = l0 + 2 + k
        q.append(a[k] * z * q[-1] - q[-2])
        sl = 1.0 if (l & 1) else -1.0
        p.append(p[-2] + a[k] * (sl * z) * p[-1])
    for k, (qq, pp) in enumerate(zip(q, p)):
        l = l0 + k
        assert sigma(l) * pp == pytest.approx(qq, rel=1e-12, abs=1e-12 * (1 + abs(qq)))


def test_block_factor_choice():
    """The kernels pick the factor of the even steps of a block from the parity of
    its first degree: -z when it is even, +z when odd."""
    for lp0 in range(-3, 40):
        for s in range(16):
            l = lp0 + s
            z_even = (-1.0 if (lp0 & 1) == 0 else 1.0)  # factor of z at the even steps
            factor = z_even if (s % 2 == 0) else -z_even
            assert factor == (1.0 if (l & 1) else -1.0)
