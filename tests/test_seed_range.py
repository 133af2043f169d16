"""Why the Legendre stages carry an exponent past the seeds.  The normalised
associated Legendre functions (Section 3) are run here by their three-term
recurrence in degree with a separate decimal exponent, for every order m and
every northern Gauss-Legendre ring.  Up to L = 1664 every function whose seed
Lambda_{m,m} = O(s^m) falls below the smallest normal binary64 number stays
below 1e-16 at all degrees m <= l <= L+1, so flushing such seeds would lose
nothing; above it (Table 3 reaches L = 2250) flushed seeds start functions of
order one, which is why each (order, ring) starts from a state computed with a
carried exponent at its first significant degree."""
import numpy as np
import pytest

import vsht_inputs as vi

NORMAL_MIN_LOG10 = np.log10(np.finfo(np.float64).tiny)


def peaks(L):
    """(log10 |Lambda_{m,m}(z_r)|, max over m <= l <= L+1 of log10 |Lambda_{l,m}(z_r)|,
    theta_r) for every order m and northern ring r."""
    z, _ = vi.gl_nodes(L + 1)
    z = np.asarray(z, np.float64)[: (L + 2) // 2]
    s = np.sqrt((1 - z) * (1 + z))
    M = np.arange(L + 1)
    k = np.arange(1, L + 1)
    cum = np.concatenate([[0.0], np.cumsum(np.log10((2 * k - 1) / (2 * k)))])
    lseed = 0.5 * (np.log10((2 * M + 1) / (4 * np.pi)) + cum)[:, None] + M[:, None] * np.log10(s)[None, :]
    e = lseed.copy()
    q2 = np.ones_like(e)
    q1 = np.sqrt(2 * M + 3.0)[:, None] * z[None, :] * q2
    best = np.maximum(lseed, e + np.log10(np.abs(q1) + 1e-300))
    for d in range(2, L + 2):
        l = (M + d).astype(np.float64)
        ok = (M + d) <= L + 1
        a = np.sqrt((4 * l * l - 1) / np.maximum(l * l - M * M, 1))
        b = np.sqrt(np.maximum((l - 1) ** 2 - M * M, 0) / (4 * (l - 1) ** 2 - 1))
        q0 = a[:, None] * (z[None, :] * q1 - b[:, None] * q2)
        q0 = np.where(ok[:, None], q0, q1)
        big = np.abs(q0) > 1e100
        sc = np.where(big, 1e-100, 1.0)
        q0 = q0 * sc
        q1 = q1 * sc
        e = e + np.where(big, 100.0, 0.0)
        q2, q1 = q1, q0
        best = np.where(ok[:, None], np.maximum(best, e + np.log10(np.abs(q1) + 1e-300)), best)
    return lseed, best, np.arccos(z)


def flushed_peak(L):
    """Largest log10 |Lambda_{l,m}| among the (m, ring) whose seed is below the
    normal range, and how many such (m, ring) there are."""
    lseed, best, _ = peaks(L)
    flushed = lseed < NORMAL_MIN_LOG10
    return (float(best[flushed].max()) if flushed.any() else -np.inf), int(flushed.sum())


def test_recurrence_matches_library_values():
    """The log-scaled recurrence against scipy's Y_{l,m} (|Y_{l,m}(theta, 0)| =
    |Lambda_{l,m}(cos theta)|) at a size where every value is representable:
    catches a wrong recurrence coefficient or seed."""
    from scipy.special import sph_harm_y
    L = 40
    lseed, best, theta = peaks(L)
    ls = np.arange(L + 2)
    for m in (0, 1, 3, 17, 40):
        vals = np.abs(np.array([sph_harm_y(l, m, theta, 0.0) for l in ls[m:]]))
        assert np.allclose(lseed[m], np.log10(vals[0]), atol=1e-10)
        assert np.allclose(best[m], np.log10(vals.max(axis=0)), atol=1e-10)
    assert flushed_peak(L)[1] == 0


@pytest.mark.timeout(300)
def test_nothing_significant_flushed_at_the_served_limit():
    peak, n = flushed_peak(1664)
    assert n > 0             # seeds do leave the normal range at this size
    assert peak < -16.0, peak
