"""Seeded synthetic inputs for the VSHT library, its tests and its benchmark.

This module holds no arithmetic of the transforms themselves: it only builds
quadrature grids, point sets and random coefficients/fields.  Both the HIP
path and the CPU oracle consume what it returns.

Recipes (every generator is seeded and deterministic):

* Gauss-Legendre product grid (Section 5.1, item 1): ``n_theta`` GL nodes in
  z = cos(theta) times ``n_phi`` equispaced longitudes phi_j = 2 pi j / n_phi.
  The default for bandlimit L is (L+1) x (2L+2), which integrates spherical
  polynomials of degree 2L+1 exactly, so the forward transform inverts the
  adjoint on band-limited coefficients.  The southern nodes are the exact
  negatives of the northern ones (and the weights are mirrored) so that rings
  pair bitwise; weights are the GL weights times 2 pi / n_phi and sum to 4 pi.
  Points are ring-major, north to south, and within a ring ordered by j.
* Scattered points: z ~ U[-1, 1], phi ~ U[0, 2 pi), i.e. uniform on S^2; equal
  weights 4 pi / M.  They stand in for the paper's symmetric spherical designs,
  whose point files are not available here.
* Coefficients a_{l,m}, b_{l,m} (1 <= l <= L, |m| <= l, index l*l+l+m-1): real
  and imaginary parts iid N(0, 1) from ``numpy.random.default_rng(seed)``
  (all real parts of a, all imaginary parts of a, then the same for b),
  scaled per degree by l^-1 or (l(l+1))^-1/2.  This stands in for the smooth
  spectra of the paper's test fields.
* Batched bandlimits: ``default_rng(seed).integers(32, 512, count, endpoint=True)``.
"""
import numpy as np


def num_coeffs(L):
    """Number of (l, m) pairs with 1 <= l <= L, |m| <= l."""
    return L * (L + 2)


def degree_of_index(L):
    """Array l(j) for j in [0, L(L+2))."""
    return np.concatenate([np.full(2 * l + 1, l, dtype=np.int64) for l in range(1, L + 1)])


def order_of_index(L):
    """Array m(j) for j in [0, L(L+2))."""
    return np.concatenate([np.arange(-l, l + 1, dtype=np.int64) for l in range(1, L + 1)])


def gl_nodes(n):
    """GL nodes (descending, north first) and weights on [-1, 1], mirrored exactly.

    numpy's nodes are refined by Newton steps on P_n and the weights
    w = 2 / ((1 - x^2) P_n'(x)^2) are evaluated in 80-bit extended precision
    (numpy.longdouble), then rounded to binary64; the library routine alone
    leaves weight errors near 1e-8 relative at n ~ 1000."""
    x0, _ = np.polynomial.legendre.leggauss(n)
    x = x0[::-1].astype(np.longdouble)
    one = np.longdouble(1)

    def pn_and_deriv(x):
        p0 = np.ones_like(x)
        p1 = x.copy()
        if n == 0:
            return p0, np.zeros_like(x)
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * x * p1 - k * p0) / (k + 1)
        dp = n * (x * p1 - p0) / (x * x - one)
        return p1, dp

    for _ in range(3):
        p, dp = pn_and_deriv(x)
        x = x - p / dp
    _, dp = pn_and_deriv(x)
    w = 2 / ((one - x * x) * dp * dp)
    x = x.astype(np.float64)
    w = w.astype(np.float64)
    h = n // 2
    # mirror the northern half onto the southern half bitwise
    x[n - h:] = -x[:h][::-1]
    w[n - h:] = w[:h][::-1]
    if n % 2 == 1:
        x[h] = 0.0
    return x, w


def gl_grid(L, n_theta=None, n_phi=None):
    """Gauss-Legendre product grid.  Returns (xyz (N,3), w (N,)) as float64."""
    n_theta = L + 1 if n_theta is None else n_theta
    n_phi = 2 * L + 2 if n_phi is None else n_phi
    z, wz = gl_nodes(n_theta)
    s = np.sqrt((1.0 - z) * (1.0 + z))
    j = np.arange(n_phi)
    phi = 2.0 * np.pi * j / n_phi
    c, sn = np.cos(phi), np.sin(phi)
    xyz = np.empty((n_theta, n_phi, 3))
    xyz[:, :, 0] = s[:, None] * c[None, :]
    xyz[:, :, 1] = s[:, None] * sn[None, :]
    xyz[:, :, 2] = z[:, None]
    w = np.repeat(wz * (2.0 * np.pi / n_phi), n_phi)
    return xyz.reshape(-1, 3), w


def reduced_gl_grid(L, min_phi=4):
    """Reduced Gauss-Legendre iso-latitude grid: L + 1 GL rings, ring r with
    n_r = max(min_phi, ceil((2L + 2) sin(theta_r))) equispaced longitudes and a
    first longitude pi / n_r on every other ring (rings of unequal length and
    phase, as in reduced and HEALPix-like grids).  Weights are the GL weight of
    the ring times 2 pi / n_r.  Returns (xyz (N,3), w (N,)) as float64."""
    z, wz = gl_nodes(L + 1)
    s = np.sqrt((1.0 - z) * (1.0 + z))
    pts, wts = [], []
    for r in range(L + 1):
        n = max(min_phi, int(np.ceil((2 * L + 2) * s[r])))
        phi = 2.0 * np.pi * np.arange(n) / n + (np.pi / n if r % 2 else 0.0)
        pts.append(np.stack([s[r] * np.cos(phi), s[r] * np.sin(phi), np.full(n, z[r])], axis=-1))
        wts.append(np.full(n, wz[r] * 2.0 * np.pi / n))
    return np.concatenate(pts), np.concatenate(wts)


def healpix_grid(nside):
    """HEALPix layout (the equal-area iso-latitude rings of Gorski et al.) with
    N_side = nside: 4 nside - 1 rings.  Polar-cap ring i < nside has z = 1 - i^2 /
    (3 nside^2) and 4 i points at phi = (pi / (2 i)) (j + 1/2); belt ring
    nside <= i <= 2 nside has z = 4/3 - 2 i / (3 nside) and 4 nside points at
    phi = (pi / (2 nside)) (j + (1 - (i - nside + 1) % 2) / 2).  Southern rings
    mirror the northern ones (z negated bitwise, same longitudes).  Equal
    weights 4 pi / (12 nside^2).  Returns (xyz (N,3), w (N,)) as float64,
    rings from north to south."""
    N = nside
    north = []
    for i in range(1, 2 * N + 1):
        if i < N:
            z = 1.0 - i * i / (3.0 * N * N)
            n = 4 * i
            phi = (np.pi / (2 * i)) * (np.arange(n) + 0.5)
        else:
            z = 4.0 / 3.0 - 2.0 * i / (3.0 * N)
            n = 4 * N
            shift = 0.5 * (1 - (i - N + 1) % 2)
            phi = (np.pi / (2 * N)) * (np.arange(n) + shift)
        north.append((z, phi))
    rings = north + [(-z, phi) for z, phi in reversed(north[:-1])]  # ring 2N is the equator
    pts = []
    for z, phi in rings:
        s = np.sqrt((1.0 - z) * (1.0 + z))
        pts.append(np.stack([s * np.cos(phi), s * np.sin(phi), np.full(len(phi), z)], axis=-1))
    xyz = np.concatenate(pts)
    return xyz, np.full(len(xyz), 4.0 * np.pi / (12 * N * N))


def uniform_points(M, seed):
    """M points uniform on S^2 and equal weights 4 pi / M."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, M)
    phi = rng.uniform(0.0, 2.0 * np.pi, M)
    s = np.sqrt((1.0 - z) * (1.0 + z))
    xyz = np.stack([s * np.cos(phi), s * np.sin(phi), z], axis=1)
    return xyz, np.full(M, 4.0 * np.pi / M)


def random_coeffs(L, seed, scale="inv_l"):
    """(a, b) complex128 of length L(L+2); scale 'inv_l', 'inv_sqrt_ll1' or 'none'."""
    K = num_coeffs(L)
    rng = np.random.default_rng(seed)
    ar = rng.standard_normal(K)
    ai = rng.standard_normal(K)
    br = rng.standard_normal(K)
    bi = rng.standard_normal(K)
    l = degree_of_index(L).astype(np.float64)
    if scale == "inv_l":
        f = 1.0 / l
    elif scale == "inv_sqrt_ll1":
        f = 1.0 / np.sqrt(l * (l + 1.0))
    elif scale == "none":
        f = np.ones_like(l)
    else:
        raise ValueError(scale)
    return (ar + 1j * ai) * f, (br + 1j * bi) * f


def random_field(n, seed, sigma=1.0):
    """(n, 3) complex128 with Re, Im iid N(0, sigma^2) (not tangent in general)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))) * sigma


def batch_bandlimits(count=256, seed=1, lo=32, hi=512):
    """Bandlimits of the batched workload: uniform integers in [lo, hi]."""
    return np.random.default_rng(seed).integers(lo, hi, count, endpoint=True)


def sample_indices(total, count, seed):
    """count distinct indices in [0, total), sorted, drawn without replacement."""
    rng = np.random.default_rng(seed)
    count = min(count, total)
    return np.sort(rng.choice(total, size=count, replace=False))
