"""Theorems 1 and 2 of the paper as a route independent of the spin-frame
formulation: the vector transforms expressed through scalar transforms of the
Cartesian components, recombined with Clebsch-Gordan weights (Section 4.1,
Theorem 1, eq. (xi_klm) and (mu_klm); Section 4.2, Theorem 2, eq. (nulm1),
(nulm2) and (etalm)).  The scalar transforms are supplied by the caller (scipy
sums on the CPU, or the library's scalar transforms on the GPU).  Test
infrastructure only."""
import functools
import math


@functools.lru_cache(maxsize=None)
def cg(j1, m1, j2, m2, J, M):
    """Standard <j1 m1 j2 m2 | J M> (sympy, exact), zero outside its range."""
    from sympy.physics.wigner import clebsch_gordan
    if j1 < 0 or J < 0 or abs(m1) > j1 or abs(m2) > j2 or abs(M) > J or m1 + m2 != M:
        return 0.0
    if not (abs(j1 - j2) <= J <= j1 + j2):
        return 0.0
    return float(clebsch_gordan(j1, j2, J, m1, m2, M))


def c_l(l):
    return math.sqrt((l + 1) / (2 * l + 1)) if l >= 0 else 0.0


def d_l(l):
    return math.sqrt(l / (2 * l + 1)) if l >= 0 else 0.0


def theorem1_combine(L, g1, g2, g3):
    """(a, b) lists of length L(L+2) from the scalar forward coefficients
    g_k(l, m) of the three Cartesian components (degree <= L+1; g_k returns 0
    outside 0 <= l, |m| <= l)."""
    xi1 = lambda l, m: c_l(l + 1) * cg(l, m, 1, 1, l + 1, m + 1)
    xi2 = lambda l, m: d_l(l - 1) * cg(l, m, 1, 1, l - 1, m + 1)
    xi3 = lambda l, m: c_l(l + 1) * cg(l, m, 1, -1, l + 1, m - 1)
    xi4 = lambda l, m: d_l(l - 1) * cg(l, m, 1, -1, l - 1, m - 1)
    xi5 = lambda l, m: c_l(l + 1) * cg(l, m, 1, 0, l + 1, m)
    xi6 = lambda l, m: d_l(l - 1) * cg(l, m, 1, 0, l - 1, m)
    mu1 = lambda l, m: cg(l, m, 1, 1, l, m + 1)
    mu2 = lambda l, m: cg(l, m, 1, 0, l, m)
    mu3 = lambda l, m: cg(l, m, 1, -1, l, m - 1)
    r2 = math.sqrt(2.0)
    a, b = [], []
    for l in range(1, L + 1):
        for m in range(-l, l + 1):
            a.append((1 / r2) * (
                xi1(l - 1, m - 1) * (-g1(l - 1, m - 1) + 1j * g2(l - 1, m - 1))
                + xi2(l + 1, m - 1) * (-g1(l + 1, m - 1) + 1j * g2(l + 1, m - 1))
                + xi3(l - 1, m + 1) * (g1(l - 1, m + 1) + 1j * g2(l - 1, m + 1))
                + xi4(l + 1, m + 1) * (g1(l + 1, m + 1) + 1j * g2(l + 1, m + 1)))
                + xi5(l - 1, m) * g3(l - 1, m) + xi6(l + 1, m) * g3(l + 1, m))
            b.append(-(1j / r2) * (
                mu1(l, m - 1) * (-g1(l, m - 1) + 1j * g2(l, m - 1))
                + mu3(l, m + 1) * (g1(l, m + 1) + 1j * g2(l, m + 1)))
                - 1j * mu2(l, m) * g3(l, m))
    return a, b


def theorem2_coeffs(L, a, b, literal_zero_cases=False):
    """Scalar coefficients of the three Cartesian components of the adjoint
    transform: {(l, m): (x, y, z)} for 0 <= l <= L+1.  Each component is the
    sum of three of the theorem's nine scalar syntheses, so by linearity their
    coefficients add before the synthesis.  With literal_zero_cases the printed
    zero cases of nu^(2) and nu^(4) are applied as written."""
    A = lambda l, m: a[l * l + l + m - 1] if 1 <= l <= L and abs(m) <= l else 0.0
    B = lambda l, m: b[l * l + l + m - 1] if 1 <= l <= L and abs(m) <= l else 0.0
    r2 = math.sqrt(2.0)
    out = {}
    for l in range(0, L + 2):
        for m in range(-l, l + 1):
            nu = [0.0] * 7
            if l <= L - 1:
                p = A(l + 1, m + 1) * cg(l, m, 1, 1, l + 1, m + 1)
                q = A(l + 1, m - 1) * cg(l, m, 1, -1, l + 1, m - 1)
                nu[1] = c_l(l + 1) * (p - q)
                nu[3] = 1j * c_l(l + 1) * (p + q)
                nu[5] = A(l + 1, m) * c_l(l + 1) * cg(l, m, 1, 0, l + 1, m)
            if 2 <= l <= L + 1:
                p = A(l - 1, m + 1) * cg(l, m, 1, 1, l - 1, m + 1)
                q = A(l - 1, m - 1) * cg(l, m, 1, -1, l - 1, m - 1)
                nu[2] = d_l(l - 1) * (p - q)
                nu[4] = 1j * d_l(l - 1) * (p + q)
                nu[6] = A(l - 1, m) * d_l(l - 1) * cg(l, m, 1, 0, l - 1, m)
                if literal_zero_cases:
                    if abs(m) in (l - 1, l):
                        nu[2] = 0.0
                    if abs(m) in (l - 2, l - 1):
                        nu[4] = 0.0
            eta1 = eta2 = eta3 = 0.0
            if 1 <= l <= L:
                p = B(l, m + 1) * cg(l, m, 1, 1, l, m + 1)
                q = B(l, m - 1) * cg(l, m, 1, -1, l, m - 1)
                eta1 = 1j * (p - q)
                eta2 = p + q
                eta3 = 1j * B(l, m) * cg(l, m, 1, 0, l, m)
            out[(l, m)] = (-(1 / r2) * (nu[1] + nu[2] + eta1),
                           -(1 / r2) * (nu[3] + nu[4] - eta2),
                           nu[5] + nu[6] + eta3)
    return out
