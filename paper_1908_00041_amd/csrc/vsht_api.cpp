// vsht_api.cpp -- host side of the library: argument checking, analysis of
// the point set (rings, north/south pairs), binary64 tables, workspace, and
// the extern "C" entry points declared in include/vsht.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

#include "vsht_internal.h"

using namespace vsht;

namespace {

thread_local std::string g_last_error;

vsht_status fail(vsht_status s, const std::string &msg) {
    g_last_error = msg;
    return s;
}

vsht_status hip_fail(hipError_t e, const char *what) {
    g_last_error = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? VSHT_ENOMEM : VSHT_EDEVICE;
}

// Longest ring: the ring stages' DFT core holds up to 4096 points per sequence
// (each length's stages are checked against its per-thread limits by fft_fits;
// lengths above kMaxBluesteinN never take Bluestein's longer convolution, so a
// ring's two sequences stay within the LDS of a workgroup).
constexpr int64_t kMaxNphi = 4096;
// Largest bandlimit served (parity-tested at L = 2250, Table 3's largest, and at
// this limit).  The Legendre stages start every (order, ring pair) from a state
// computed with a carried exponent, so seeds Lambda_{m,m} = O(s^m) below
// binary64's range are no limit.
constexpr int kMaxL = 4096;

struct DeviceGuard {
    int old = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&old) == hipSuccess && old != dev) {
            if (hipSetDevice(dev) == hipSuccess) changed = true;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(old);
    }
};

template <typename T>
hipError_t upload(T **dst, const std::vector<T> &src, size_t *bytes) {
    *dst = nullptr;
    if (src.empty()) return hipSuccess;
    hipError_t e = hipMalloc((void **)dst, sizeof(T) * src.size());
    if (e != hipSuccess) return e;
    *bytes += sizeof(T) * src.size();
    return hipMemcpy(*dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice);
}

void free_plan_memory(Plan *p) {
    const NfftPlan &nf = p->nfft;
    void *ptrs[] = {p->d_rings, p->d_pairs, p->d_ffts, p->d_tw,  p->d_pair_z, p->d_aprime,
                    p->d_cscale, p->d_etab, p->d_rsq,  p->d_seeds, p->d_start, p->d_sblk, p->d_weights, p->d_xyz,
                    p->d_pb, p->d_fg, p->d_fg64, p->d_fpart, p->d_many, p->d_state, nf.d_ffts, nf.d_tw, nf.d_vpairs, nf.d_vz,
                    nf.d_vs, nf.d_vseeds, nf.d_vstart, nf.d_vsblk, nf.d_psihat, nf.d_pts, nf.d_tiles, nf.d_vpb, nf.d_g1,
                    nf.d_g};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
}

// Factor n for the Stockham stages: the largest prime above 5 (if any) first,
// where the stage needs no twiddles, then radix 4, 2 and the odd primes ascending.
std::vector<int> factorize(int n) {
    std::vector<int> f;
    while (n % 4 == 0) { f.push_back(4); n /= 4; }
    while (n % 2 == 0) { f.push_back(2); n /= 2; }
    for (int p = 3; (long)p * p <= n; p += 2)
        while (n % p == 0) { f.push_back(p); n /= p; }
    if (n > 1) f.push_back(n);
    auto big = std::max_element(f.begin(), f.end());
    if (big != f.end() && *big > 5) std::rotate(f.begin(), big, big + 1);
    return f;
}

// Largest prime the odd-radix Stockham stage handles; longer prime factors go
// through Bluestein's convolution (for n <= kMaxBluesteinN).
constexpr int kMaxGenericRadix = 64;
constexpr int kMaxBluesteinN = 2048;

// In-place DFT (sign -1) of a power-of-two length, extended precision.
void host_fft_pow2(std::vector<std::complex<long double>> &x) {
    const size_t M = x.size();
    for (size_t i = 1, j = 0; i < M; ++i) {
        size_t bit = M >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(x[i], x[j]);
    }
    const long double pi = 3.141592653589793238462643383279502884L;
    for (size_t len = 2; len <= M; len <<= 1) {
        for (size_t i = 0; i < M; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const long double ang = -2.0L * pi * (long double)k / (long double)len;
                const std::complex<long double> w(cosl(ang), sinl(ang));
                const auto u = x[i + k], v = x[i + k + len / 2] * w;
                x[i + k] = u + v;
                x[i + k + len / 2] = u - v;
            }
    }
}

void push_twiddles(int n, std::vector<double> &tw) {
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int k = 0; k < n; ++k) {
        const long double a = -two_pi * (long double)k / (long double)n;
        tw.push_back((double)cosl(a));
        tw.push_back((double)sinl(a));
    }
}

// Index of the descriptor for DFT length n (created, with its tables, on first use).
int fft_descriptor(int n, std::map<int, int> &index, std::vector<FftDesc> &ffts, std::vector<double> &tw) {
    auto it = index.find(n);
    if (it != index.end()) return it->second;
    FftDesc fd{};
    fd.n = n;
    std::vector<int> f = factorize(n);
    const int pmax = f.empty() ? 1 : *std::max_element(f.begin(), f.end());
    if (pmax > kMaxGenericRadix && n <= kMaxBluesteinN) {
        int M = 1;
        while (M < 2 * n - 1) M <<= 1;
        fd.blue = 1;
        fd.M = M;
        fd.mdesc = fft_descriptor(M, index, ffts, tw);  // may reallocate ffts
        fd.lds_shift = ffts[fd.mdesc].lds_shift;          // the ring buffer holds the length-M sequences
        // the ring stages take e^{i phi_j} from the length-n table as well
        fd.tw_offset = (int64_t)(tw.size() / 2);
        push_twiddles(n, tw);
        const long double pi = 3.141592653589793238462643383279502884L;
        std::vector<std::complex<long double>> w(n);
        for (int k = 0; k < n; ++k) {
            const long long k2 = ((long long)k * k) % (2LL * n);  // exact angle reduction
            const long double a = -pi * (long double)k2 / (long double)n;
            w[k] = std::complex<long double>(cosl(a), sinl(a));
        }
        fd.chirp_offset = (int64_t)(tw.size() / 2);
        for (int k = 0; k < n; ++k) {
            tw.push_back((double)w[k].real());
            tw.push_back((double)w[k].imag());
        }
        fd.bhat_offset = (int64_t)(tw.size() / 2);
        for (int dir = 0; dir < 2; ++dir) {  // kernel conj(w) (forward), then w (inverse)
            std::vector<std::complex<long double>> b(M, 0.0L);
            for (int k = 0; k < n; ++k) {
                const auto v = dir == 0 ? std::conj(w[k]) : w[k];
                b[k] = v;
                if (k > 0) b[M - k] = v;
            }
            host_fft_pow2(b);
            for (int k = 0; k < M; ++k) {
                tw.push_back((double)(b[k].real() / M));
                tw.push_back((double)(b[k].imag() / M));
            }
        }
    } else {
        fd.nfac = (int)f.size();
        for (size_t q = 0; q < f.size(); ++q) fd.fac[q] = f[q];
        fd.tw_offset = (int64_t)(tw.size() / 2);
        push_twiddles(n, tw);
        const int R = fd.nfac > 0 ? fd.fac[0] : 1;
        // an odd first radix leaves unit and odd strides only: no LDS padding
        fd.lds_shift = (R % 2 == 1) ? 30 : 4;
        if (R > 5 && R <= kSmallTab) {
            fd.rtab_offset = (int64_t)(tw.size() / 2);
            const long double pi = 3.141592653589793238462643383279502884L;
            std::vector<float> tf(2 * R);
            for (int q = 0; q < R; ++q) {
                const long double a = -2.0L * pi * (long double)q / (long double)R;
                tw.push_back((double)cosl(a));
                tw.push_back((double)sinl(a));
                tf[2 * q] = (float)cosl(a);
                tf[2 * q + 1] = (float)sinl(a);
            }
            std::vector<double> packed(2 * R, 0.0);  // R complex slots hold the 2R binary32 values
            std::memcpy(packed.data(), tf.data(), tf.size() * sizeof(float));
            tw.insert(tw.end(), packed.begin(), packed.end());
        }
    }
    const int id = (int)ffts.size();
    ffts.push_back(fd);
    index.emplace(n, id);
    return id;
}

// Whether every stage of the DFT `fd` fits a workgroup of nt threads under the
// kernels' per-thread work limits (the same dispatch rules as fft_core).
bool fft_fits(const FftDesc &fd, const std::vector<FftDesc> &ffts, int nt) {
    if (fd.blue) return fft_fits(ffts[fd.mdesc], ffts, nt);
    const int n = fd.n;
    for (int f = 0; f < fd.nfac; ++f) {
        const int R = fd.fac[f];
        const int nb = n / R, half = (R - 1) / 2;
        if (f == 0 && R > 5 && R <= kSmallTab && first_stage_waves(n, R) <= kMaxRoundsFirst * (nt / 64)) continue;
        if (R <= 5) {
            if ((nb + nt - 1) / nt > kMaxItemsSmall) return false;
        } else if (nb * ((half + kKP - 1) / kKP) > kMaxItemsOdd * nt) {
            return false;
        }
    }
    return true;
}

// Smallest multiple of `mult` that is >= n and has no prime factor above 5.
int smooth_at_least(int n, int mult) {
    for (int m = (n + mult - 1) / mult * mult;; m += mult) {
        int r = m;
        for (int p : {2, 3, 5})
            while (r % p == 0) r /= p;
        if (r == 1) return m;
    }
}

// Start blocks and states of the Legendre stages for NP ring pairs (z, s on the
// device), allocated into *start and *sblk.
hipError_t build_start_tables(int L, int NP, const double *d_z, const double *d_s, const double *d_aprime,
                              const double *d_cscale, LegStart **start, int **sblk, size_t *bytes) {
    const size_t cnt = (size_t)(L + 1) * NP;
    hipError_t e = hipMalloc((void **)start, sizeof(LegStart) * cnt);
    if (e != hipSuccess) return e;
    if ((e = hipMalloc((void **)sblk, sizeof(int) * cnt)) != hipSuccess) return e;
    *bytes += (sizeof(LegStart) + sizeof(int)) * cnt;
    int *d_bad = nullptr;
    if ((e = hipMalloc((void **)&d_bad, sizeof(int))) != hipSuccess) return e;
    int bad = 0;
    e = hipMemcpy(d_bad, &bad, sizeof(int), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = launch_start_kernel(d_z, d_s, NP, L, d_aprime, d_cscale, *start, *sblk, d_bad, nullptr);
    if (e == hipSuccess) e = hipMemcpy(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost);
    (void)hipFree(d_bad);
    if (e == hipSuccess && bad) e = hipErrorNotSupported;  // a start state outside the normal range
    return e;
}

// Largest bandlimit the double-Fourier-sphere path serves: its column kernels keep
// the 2L+1 orders of a row in registers, five per thread of 512 (2L+1 <= 2560).  The
// DFT lengths must also fit the LDS DFT kernels (checked when the sizes are chosen).
constexpr int kMaxNfftL = 1279;

// Tables of the double-Fourier-sphere evaluation of a scattered plan.
// Window width of the grid path for a target accuracy eps (0: the default of the
// precision): the exponential-of-semicircle window with beta = 2.3 w on a twice
// oversampled grid loses about one digit per grid point of width, so
// w = ceil(-log10 eps) + 1, even, within [4, kNfftMaxW].
int nfft_width(int precision, double eps) {
    if (!(eps > 0.0)) return precision == VSHT_FP64 ? 14 : 8;
    int w = (int)std::ceil(-std::log10(eps)) + 1;
    w += w & 1;
    return std::min(16, std::max(4, w));
}

hipError_t build_nfft(Plan &P, int64_t n, const double *xyz, double nfft_eps) {
    NfftPlan &nf = P.nfft;
    const int L = P.L;
    const size_t rsz = P.precision == VSHT_FP64 ? 8 : 4;
    nf.w = nfft_width(P.precision, nfft_eps);
    nf.beta = 2.30 * nf.w;
    // the smallest 5-smooth lengths (nt a multiple of 4, ng even) whose DFT stages fit
    // a 512-thread workgroup and whose two sequences fit its LDS
    auto fits = [&](int n) {
        std::map<int, int> fi;
        std::vector<FftDesc> fd;
        std::vector<double> t;
        const int id = fft_descriptor(n, fi, fd, t);
        const int64_t len = fd[id].blue ? fd[id].M : fd[id].n;
        return fft_fits(fd[id], fd, 512) && ring_lds_bytes_for(len, rsz) <= kLdsPerWorkgroup;
    };
    nf.nt = smooth_at_least(2 * L + 2, 4);
    for (int k = 0; k < 64 && !fits(nf.nt); ++k) nf.nt = smooth_at_least(nf.nt + 4, 4);
    nf.npv = nf.nt / 4;
    nf.ng = smooth_at_least(std::max(2 * (2 * L + 1), 2 * nf.w), 2);
    for (int k = 0; k < 64 && !fits(nf.ng); ++k) nf.ng = smooth_at_least(nf.ng + 2, 2);
    std::map<int, int> fidx;
    std::vector<FftDesc> ffts;
    std::vector<double> tw;
    nf.fft_nt = fft_descriptor(nf.nt, fidx, ffts, tw);
    nf.fft_ng = fft_descriptor(nf.ng, fidx, ffts, tw);
    auto stored = [&](int id) -> int64_t { return ffts[id].blue ? ffts[id].M : ffts[id].n; };
    nf.lds_stride = std::max(stored(nf.fft_nt), stored(nf.fft_ng));
    if (!fft_fits(ffts[nf.fft_nt], ffts, 512) || !fft_fits(ffts[nf.fft_ng], ffts, 512) ||
        ring_lds_bytes_for(nf.lds_stride, rsz) > kLdsPerWorkgroup)
        return hipErrorInvalidValue;
    size_t bytes = 0;
    hipError_t e;
    if ((e = upload(&nf.d_ffts, ffts, &bytes)) != hipSuccess) return e;
    if ((e = upload(&nf.d_tw, tw, &bytes)) != hipSuccess) return e;
    // virtual ring pairs: northern colatitude theta_p = 2 pi (p + 1/2) / nt, p < nt/4
    const long double pi = 3.141592653589793238462643383279502884L;
    std::vector<double> vz(nf.npv), vs(nf.npv);
    for (int q = 0; q < nf.npv; ++q) {
        const long double th = 2.0L * pi * (q + 0.5L) / nf.nt;
        vz[q] = (double)cosl(th);
        vs[q] = (double)sinl(th);
    }
    if ((e = upload(&nf.d_vz, vz, &bytes)) != hipSuccess) return e;
    {
        std::vector<PairDesc> vp(nf.npv);
        for (int q = 0; q < nf.npv; ++q) vp[q] = PairDesc{q, nf.nt / 2 - 1 - q};
        if ((e = upload(&nf.d_vpairs, vp, &bytes)) != hipSuccess) return e;
    }
    if ((e = upload(&nf.d_vs, vs, &bytes)) != hipSuccess) return e;
    e = hipMalloc((void **)&nf.d_vseeds, sizeof(double) * (size_t)(L + 1) * nf.npv);
    if (e != hipSuccess) return e;
    if ((e = launch_seed_kernel(nf.d_vs, nf.npv, L, nf.d_vseeds, nullptr)) != hipSuccess) return e;
    if ((e = build_start_tables(L, nf.npv, nf.d_vz, nf.d_vs, P.d_aprime, P.d_cscale, &nf.d_vstart, &nf.d_vsblk,
                                &bytes)) != hipSuccess)
        return e;
    // window transform psih(k) = alpha int_{-1}^{1} exp(beta (sqrt(1 - t^2) - 1)) cos(k alpha t) dt,
    // alpha = w h / 2, with t = sin(u) (a smooth integrand) and composite Simpson
    {
        const long double alpha = (long double)nf.w * pi / nf.ng;
        const int nq = 4000;
        std::vector<double> ph(2 * L + 1);
        for (int k = -L; k <= L; ++k) {
            long double acc = 0.0L;
            for (int i = 0; i <= nq; ++i) {
                const long double u = -pi / 2 + pi * i / nq;
                const long double f = expl(nf.beta * (cosl(u) - 1.0L)) * cosl(k * alpha * sinl(u)) * cosl(u);
                acc += f * (i == 0 || i == nq ? 1.0L : (i % 2 ? 4.0L : 2.0L));
            }
            ph[k + L] = (double)(alpha * acc * (pi / nq) / 3.0L);
        }
        if ((e = upload(&nf.d_psihat, ph, &bytes)) != hipSuccess) return e;
    }
    // points in grid-cell order
    {
        const double h = 2.0 * M_PI / nf.ng;
        std::vector<NfftPoint> pts(n);
        std::vector<int64_t> key(n);
        for (int64_t k = 0; k < n; ++k) {
            const double x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
            const double sn = std::sqrt(x * x + y * y);
            NfftPoint &q = pts[k];
            q.z = z;
            q.s = sn;
            q.theta = std::atan2(sn, z);
            if (sn > 0.0) {
                q.c = x / sn;
                q.sn = y / sn;
                q.phi = std::atan2(y, x);
                if (q.phi < 0.0) q.phi += 2.0 * M_PI;
                if (q.phi >= 2.0 * M_PI) q.phi = 0.0;
            } else {
                q.c = 1.0;
                q.sn = 0.0;
                q.phi = 0.0;
            }
            q.idx = k;
            // the window's first row and column, as the gather computes them
            const double hw = 0.5 * nf.w;
            const int j0 = (int)std::ceil(q.theta / h - hw), i0 = (int)std::ceil(q.phi / h - hw);
            const int64_t tj = (j0 + nf.w / 2) / kGatherTile, ti = (i0 + nf.w / 2) / kGatherTile;
            key[k] = ((tj * (nf.ng / kGatherTile + 2) + ti) * nf.ng + j0) * (int64_t)(nf.ng + nf.w) + i0;
        }
        std::vector<int64_t> order(n);
        for (int64_t k = 0; k < n; ++k) order[k] = k;
        std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        std::vector<NfftPoint> sorted(n);
        for (int64_t k = 0; k < n; ++k) sorted[k] = pts[order[k]];
        if ((e = upload(&nf.d_pts, sorted, &bytes)) != hipSuccess) return e;
        // runs of points in one tile
        std::vector<NfftTile> tiles;
        const double hw = 0.5 * nf.w;
        for (int64_t k = 0; k < n; ++k) {
            const NfftPoint &q = sorted[k];
            const int j0 = (int)std::ceil(q.theta / h - hw), i0 = (int)std::ceil(q.phi / h - hw);
            const int tj = (j0 + nf.w / 2) / kGatherTile, ti = (i0 + nf.w / 2) / kGatherTile;
            if (tiles.empty() || tiles.back().tj != tj || tiles.back().ti != ti)
                tiles.push_back(NfftTile{tj, ti, 0, 0, k});
            ++tiles.back().count;
        }
        nf.ntiles = (int)tiles.size();
        if ((e = upload(&nf.d_tiles, tiles, &bytes)) != hipSuccess) return e;
    }
    const size_t vpb = (size_t)(L + 1) * nf.npv * 16 * rsz;
    const size_t g1 = (size_t)2 * nf.ng * (2 * L + 1) * 2 * rsz;
    const size_t g = (size_t)2 * nf.ng * nf.ng * 2 * rsz;
    if ((e = hipMalloc(&nf.d_vpb, vpb)) != hipSuccess) return e;
    if ((e = hipMalloc(&nf.d_g1, g1)) != hipSuccess) return e;
    if ((e = hipMalloc(&nf.d_g, g)) != hipSuccess) return e;
    if ((e = hipDeviceSynchronize()) != hipSuccess) return e;
    P.table_bytes += bytes + sizeof(double) * (size_t)(L + 1) * nf.npv;
    P.workspace_bytes += vpb + g1 + g;
    nf.on = 1;
    return hipSuccess;
}

struct RingScan {
    bool ok = true;
    std::string why;
    std::vector<RingDesc> rings;
};

// Group consecutive points with bitwise-equal z into rings and check each is
// an equispaced circle not at a pole.
RingScan scan_rings(int64_t n, const double *xyz, const double *w) {
    RingScan rs;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    // (cos, sin)(2 pi t / len) per ring length, in extended precision once per length
    std::map<int64_t, std::vector<std::pair<double, double>>> unit;
    auto roots = [&](int64_t len) -> const std::vector<std::pair<double, double>> & {
        auto it = unit.find(len);
        if (it != unit.end()) return it->second;
        std::vector<std::pair<double, double>> v(len);
        for (int64_t t = 0; t < len; ++t) {
            const long double a = two_pi * (long double)t / (long double)len;
            v[t] = {(double)cosl(a), (double)sinl(a)};
        }
        return unit.emplace(len, std::move(v)).first->second;
    };
    int64_t i = 0;
    while (i < n) {
        int64_t j = i + 1;
        const double z = xyz[3 * i + 2];
        while (j < n && xyz[3 * j + 2] == z) ++j;
        const int64_t cnt = j - i;
        RingDesc r{};
        r.z = z;
        r.s = std::sqrt((1.0 - z) * (1.0 + z));
        r.offset = i;
        r.nphi = (int32_t)cnt;
        if (!(r.s > 0.0)) {
            rs.ok = false;
            rs.why = "point at a pole";
            return rs;
        }
        if (cnt > kMaxNphi) {
            rs.ok = false;
            rs.why = "ring longer than supported";
            return rs;
        }
        r.phi0 = std::atan2(xyz[3 * i + 1], xyz[3 * i]);
        r.c0 = std::cos(r.phi0);
        r.s0 = std::sin(r.phi0);
        // expected point t: s e^{i (phi0 + 2 pi t / cnt)}, rounding error a few ulp,
        // far below the 1e-12 tolerance
        const std::vector<std::pair<double, double>> &u = roots(cnt);
        for (int64_t t = 0; t < cnt; ++t) {
            const double ex = r.s * (r.c0 * u[t].first - r.s0 * u[t].second);
            const double ey = r.s * (r.s0 * u[t].first + r.c0 * u[t].second);
            if (std::fabs(xyz[3 * (i + t)] - ex) > 1e-12 || std::fabs(xyz[3 * (i + t) + 1] - ey) > 1e-12) {
                rs.ok = false;
                rs.why = "ring points not equispaced in longitude";
                return rs;
            }
        }
        r.uniform_w = 1;
        r.w = w ? w[i] : 1.0;
        if (w)
            for (int64_t t = 1; t < cnt; ++t)
                if (w[i + t] != w[i]) r.uniform_w = 0;
        rs.rings.push_back(r);
        i = j;
    }
    return rs;
}

// Validate the arguments of one plan (Section 4.1: a quadrature rule has N >= 2
// nodes; every point a unit vector).
vsht_status check_plan_args(int L, int64_t n, const double *xyz, const double *w, int precision) {
    if (L < 1) return fail(VSHT_EINVAL, "L must be >= 1");
    if (L > 65535) return fail(VSHT_EINVAL, "L too large");
    if (L > kMaxL) return fail(VSHT_EUNSUPPORTED, "L > " + std::to_string(kMaxL) + " is not served");
    if (n < 1) return fail(VSHT_EINVAL, "n must be >= 1");
    if (w && n < 2) return fail(VSHT_EINVAL, "a quadrature rule needs n >= 2 points");
    if (!xyz) return fail(VSHT_EINVAL, "xyz is NULL");
    if (precision != VSHT_FP64 && precision != VSHT_FP32 && precision != VSHT_BF16X3 &&
        precision != VSHT_BF16X6)
        return fail(VSHT_EINVAL, "unknown precision");
    for (int64_t k = 0; k < n; ++k) {
        const double x = xyz[3 * k], y = xyz[3 * k + 1], z = xyz[3 * k + 2];
        if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
            return fail(VSHT_EINVAL, "non-finite point at index " + std::to_string(k));
        const double r = std::sqrt(x * x + y * y + z * z);
        if (std::fabs(r - 1.0) > 1e-12)
            return fail(VSHT_EINVAL, "point " + std::to_string(k) + " is not a unit vector");
        if (w && !std::isfinite(w[k]))
            return fail(VSHT_EINVAL, "non-finite weight at index " + std::to_string(k));
    }

    return VSHT_OK;
}

vsht_status resolve_device(const vsht_opts *opts, int *dev) {
    *dev = 0;
    if (opts && opts->device >= 0) {
        *dev = opts->device;
    } else {
        hipError_t e = hipGetDevice(dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    }
    DeviceGuard guard(*dev);
    static std::once_flag attr_once;
    static hipError_t attr_err = hipSuccess;
    std::call_once(attr_once, [] { attr_err = set_kernel_attributes(); });
    if (attr_err != hipSuccess) return hip_fail(attr_err, "hipFuncSetAttribute");
    return VSHT_OK;
}

// Build the tables and workspace of one plan on the current device.
vsht_status build_plan(Plan &P, int L, int64_t n, const double *xyz, const double *w, int precision,
                       int dev, int flags, double nfft_eps) {
    P.L = L;
    P.precision = precision;
    P.device = dev;
    P.n = n;
    P.has_weights = w ? 1 : 0;
    P.tri_size = tri_size(L);
    const size_t rsz = precision == VSHT_FP64 ? 8 : 4;  // bytes per real

    RingScan scan = scan_rings(n, xyz, w);
    if (scan.ok && (int64_t)scan.rings.size() * 2 > n && n > 8) {
        scan.ok = false;
        scan.why = "too many rings";
    }
    if (scan.ok) {
        // every ring length must fit the ring DFT stages of a 512-thread workgroup;
        // a point set with one that does not is planned as scattered points
        std::map<int, int> fi;
        std::vector<FftDesc> fd;
        std::vector<double> t;
        for (const RingDesc &r : scan.rings) {
            const int id = fft_descriptor(r.nphi, fi, fd, t);
            if (!fft_fits(fd[id], fd, 512)) {
                scan.ok = false;
                scan.why = "ring length " + std::to_string(r.nphi) + " does not fit the ring DFT stages";
                break;
            }
        }
    }
    std::vector<double> tmp;
    hipError_t e = hipSuccess;

    // scaled recurrence tables, binary64 (computed in extended precision):
    // Lambda_{l,m} = c_{l,m} Q_{l,m},  Q_l = a'_l z Q_{l-1} - Q_{l-2},
    // c_m = c_{m+1} = 1, c_l = (alpha_l / alpha_{l-1}) c_{l-2}, a'_l = alpha_l c_{l-1} / c_l,
    // alpha_l = sqrt((4 l^2 - 1) / (l^2 - m^2)); a'_{m+1} = sqrt(2m+3); a'_m is unused (0).
    std::vector<double> aprime(P.tri_size, 0.0), cscale(P.tri_size, 1.0);
    for (int m = 0; m <= L; ++m) {
        const int64_t t0 = tri_offset(L, m);
        const long double mm = m;
        auto alpha = [&](int l) {
            const long double ll = l;
            return sqrtl((4.0L * ll * ll - 1.0L) / (ll * ll - mm * mm));
        };
        long double cprev2 = 1.0L, cprev1 = 1.0L;  // c_{l-2}, c_{l-1}
        aprime[t0] = 0.0;
        cscale[t0] = 1.0;
        if (m + 1 <= L + 1) {
            aprime[t0 + 1] = (double)sqrtl(2.0L * mm + 3.0L);
            cscale[t0 + 1] = 1.0;
        }
        for (int l = m + 2; l <= L + 1; ++l) {
            const long double al = alpha(l), alm1 = alpha(l - 1);
            const long double cl = (al / alm1) * cprev2;
            aprime[t0 + l - m] = (double)(al * cprev1 / cl);
            cscale[t0 + l - m] = (double)cl;
            cprev2 = cprev1;
            cprev1 = cl;
        }
    }
    // the kernels read a' in whole blocks of up to 32 degrees and mask the
    // entries beyond L+1, so the table carries 32 zeros of padding
    aprime.resize(aprime.size() + 32, 0.0);
    if ((e = upload(&P.d_aprime, aprime, &P.table_bytes)) != hipSuccess) goto hip_error;
    if ((e = upload(&P.d_cscale, cscale, &P.table_bytes)) != hipSuccess) goto hip_error;
    {
        // e_{l,m} = sqrt((l^2 - m^2) / (4 l^2 - 1)) and 1 / sqrt(l (l+1))
        std::vector<double> etab(P.tri_size, 0.0), rsq(L + 2, 0.0);
        for (int m = 0; m <= L; ++m) {
            const int64_t t0 = tri_offset(L, m);
            for (int l = m; l <= L + 1; ++l) {
                const long double ll = l, mm = m;
                etab[t0 + l - m] = l == 0 ? 0.0 : (double)sqrtl((ll * ll - mm * mm) / (4.0L * ll * ll - 1.0L));
            }
        }
        for (int l = 1; l <= L + 1; ++l) rsq[l] = (double)(1.0L / sqrtl((long double)l * (l + 1)));
        if ((e = upload(&P.d_etab, etab, &P.table_bytes)) != hipSuccess) goto hip_error;
        if ((e = upload(&P.d_rsq, rsq, &P.table_bytes)) != hipSuccess) goto hip_error;
    }

    if (scan.ok) {
        P.kind = VSHT_PLAN_RINGS;
        std::vector<RingDesc> &rings = scan.rings;
        // FFT descriptors per distinct length
        std::map<int, int> fft_index;
        std::vector<FftDesc> ffts;
        std::vector<double> tw;
        for (auto &r : rings) {
            r.fft = fft_descriptor(r.nphi, fft_index, ffts, tw);
            const FftDesc &fd = ffts[r.fft];
            P.max_nphi = std::max<int64_t>(P.max_nphi, r.nphi);
            P.max_fft_len = std::max<int64_t>(P.max_fft_len, fd.blue ? fd.M : fd.n);
        }
        P.ring_nt_min = 256;
        for (auto &r : rings) {
            if (fft_fits(ffts[r.fft], ffts, 256)) continue;
            if (!fft_fits(ffts[r.fft], ffts, 512)) {
                free_plan_memory(&P);
                P = Plan();
                return fail(VSHT_EUNSUPPORTED, "ring length " + std::to_string(r.nphi) +
                                                   " has prime factors the ring DFT kernels cannot take");
            }
            P.ring_nt_min = 512;
        }
        // pair rings with z_S == -z_N bitwise
        std::unordered_map<uint64_t, std::vector<int>> byz;
        auto key = [](double z) {
            if (z == 0.0) z = 0.0;
            uint64_t u;
            std::memcpy(&u, &z, 8);
            return u;
        };
        for (int r = 0; r < (int)rings.size(); ++r) byz[key(rings[r].z)].push_back(r);
        std::vector<int> used(rings.size(), 0);
        std::vector<PairDesc> pairs;
        for (int r = 0; r < (int)rings.size(); ++r) {
            if (used[r]) continue;
            used[r] = 1;
            PairDesc pd{r, -1};
            if (rings[r].z != 0.0 && !(flags & VSHT_OPT_NO_FOLD)) {
                auto it = byz.find(key(-rings[r].z));
                if (it != byz.end())
                    for (int c : it->second)
                        if (!used[c]) {
                            used[c] = 1;
                            pd.rs = c;
                            break;
                        }
            }
            pairs.push_back(pd);
        }
        // pairs in order of increasing sin(theta): the first tile of 64 pairs is
        // the one nearest the poles, which the reduced-precision syntheses
        // compute one precision wider
        std::stable_sort(pairs.begin(), pairs.end(), [&](const PairDesc &x, const PairDesc &y) {
            return rings[x.rn].s < rings[y.rn].s;
        });
        // the ring at z = 0 (if any) goes last: its Legendre values are known in
        // closed form and the kernels treat it separately
        for (size_t q = 0; q < pairs.size(); ++q)
            if (pairs[q].rs < 0 && rings[pairs[q].rn].z == 0.0) {
                PairDesc eq = pairs[q];
                pairs.erase(pairs.begin() + q);
                pairs.push_back(eq);
                P.eq_ring = eq.rn;
                break;
            }
        for (size_t q = 0; q < pairs.size(); ++q) {
            rings[pairs[q].rn].pair = (int32_t)q;
            rings[pairs[q].rn].south = 0;
            if (pairs[q].rs >= 0) {
                rings[pairs[q].rs].pair = (int32_t)q;
                rings[pairs[q].rs].south = 1;
            }
        }
        P.n_rings = (int64_t)rings.size();
        P.n_pairs = (int64_t)pairs.size();
        P.n_ffts = (int)ffts.size();
        std::vector<double> pz(pairs.size()), ps(pairs.size());
        for (size_t q = 0; q < pairs.size(); ++q) {
            pz[q] = rings[pairs[q].rn].z;
            ps[q] = rings[pairs[q].rn].s;
        }
        bool any_nonuniform = false;
        for (auto &r : rings) any_nonuniform |= !r.uniform_w;
        if ((e = upload(&P.d_rings, rings, &P.table_bytes)) != hipSuccess) goto hip_error;
        if ((e = upload(&P.d_pairs, pairs, &P.table_bytes)) != hipSuccess) goto hip_error;
        if ((e = upload(&P.d_ffts, ffts, &P.table_bytes)) != hipSuccess) goto hip_error;
        if ((e = upload(&P.d_tw, tw, &P.table_bytes)) != hipSuccess) goto hip_error;
        if ((e = upload(&P.d_pair_z, pz, &P.table_bytes)) != hipSuccess) goto hip_error;
        if (w && any_nonuniform) {
            std::vector<double> wv(w, w + n);
            if ((e = upload(&P.d_weights, wv, &P.table_bytes)) != hipSuccess) goto hip_error;
        }
        // seeds Lambda_{m,m}(z_p) on the device, binary64
        {
            double *d_ps = nullptr;
            size_t dummy = 0;
            if ((e = upload(&d_ps, ps, &dummy)) != hipSuccess) goto hip_error;
            e = hipMalloc((void **)&P.d_seeds, sizeof(double) * (size_t)(L + 1) * P.n_pairs);
            if (e == hipSuccess) {
                P.table_bytes += sizeof(double) * (size_t)(L + 1) * P.n_pairs;
                e = launch_seed_kernel(d_ps, (int)P.n_pairs, L, P.d_seeds, nullptr);
            }
            if (e == hipSuccess)
                e = build_start_tables(L, (int)P.n_pairs, P.d_pair_z, d_ps, P.d_aprime, P.d_cscale, &P.d_start,
                                       &P.d_sblk, &P.table_bytes);
            if (e == hipSuccess) e = hipDeviceSynchronize();
            (void)hipFree(d_ps);
            if (e != hipSuccess) goto hip_error;
        }
        // workspace
        {
            // ring buffer [(L+1)][NR][4] (forward) and pair buffer [(L+1)][NP][8] (adjoint)
            const size_t per_m = std::max((size_t)P.n_rings * 4, (size_t)P.n_pairs * 8);
            const size_t pb = (size_t)(L + 1) * per_m * 2 * rsz;
            const size_t fg = (size_t)(P.tri_size + kFgPadRows) * 4 * 2 * rsz;
            if ((e = hipMalloc(&P.d_pb, pb)) != hipSuccess) goto hip_error;
            if ((e = hipMalloc(&P.d_fg, fg)) != hipSuccess) goto hip_error;
            P.workspace_bytes = pb + fg;
            if (rsz == 4) {  // the adjoint's g in binary64 as well
                const size_t fg64 = (size_t)(P.tri_size + kFgPadRows) * 4 * 2 * 8;
                if ((e = hipMalloc(&P.d_fg64, fg64)) != hipSuccess) goto hip_error;
                P.workspace_bytes += fg64;
            }
            const int groups = analysis_groups(P.n_pairs, P.eq_ring);
            if (groups > 1) {
                const size_t part = (size_t)groups * P.tri_size * 8 * rsz;
                if ((e = hipMalloc(&P.d_fpart, part)) != hipSuccess) goto hip_error;
                P.workspace_bytes += part;
            }
        }
    } else {
        P.kind = VSHT_PLAN_SCATTERED;
        std::vector<double> xv(xyz, xyz + 3 * n);
        if ((e = upload(&P.d_xyz, xv, &P.table_bytes)) != hipSuccess) goto hip_error;
        if (w) {
            std::vector<double> wv(w, w + n);
            if ((e = upload(&P.d_weights, wv, &P.table_bytes)) != hipSuccess) goto hip_error;
        }
        const size_t fg = (size_t)(P.tri_size + kFgPadRows) * 4 * 2 * rsz;
        if ((e = hipMalloc(&P.d_fg, fg)) != hipSuccess) goto hip_error;
        P.workspace_bytes = fg;
        if (rsz == 4) {
            const size_t fg64 = (size_t)(P.tri_size + kFgPadRows) * 4 * 2 * 8;
            if ((e = hipMalloc(&P.d_fg64, fg64)) != hipSuccess) goto hip_error;
            P.workspace_bytes += fg64;
        }
        if (!(flags & VSHT_OPT_SCATTERED_DIRECT) && L <= kMaxNfftL) {
            e = build_nfft(P, n, xyz, nfft_eps);
            if (e == hipErrorInvalidValue) {
                e = hipSuccess;  // grid sizes the DFT kernels cannot take: direct evaluation
                NfftPlan &nf = P.nfft;
                void *q[] = {nf.d_ffts, nf.d_tw,     nf.d_vpairs, nf.d_vz,     nf.d_vs, nf.d_vseeds, nf.d_vstart,
                             nf.d_vsblk, nf.d_psihat, nf.d_pts,    nf.d_tiles, nf.d_vpb, nf.d_g1, nf.d_g};
                for (void *x : q)
                    if (x) (void)hipFree(x);
                nf = NfftPlan();
            }
            if (e != hipSuccess) goto hip_error;
        }
    }
    return VSHT_OK;

hip_error:
    free_plan_memory(&P);
    P = Plan();
    return hip_fail(e, "plan setup");
}

}  // namespace

// A batch: one plan per field plus the batched launch state and its graphs.
struct BatchPlan {
    std::vector<Plan> fields;
    BatchState *st = nullptr;
    hipStream_t cap = nullptr;          // capture stream (default priority)
    hipGraphExec_t exec[4] = {};        // by direction set: 1 adjoint, 2 forward, 3 both
    std::vector<const void *> bound_adj, bound_fwd;
    int last_dirs = 0;
    std::string tune_cache;             // autotune results file ("" = none)

    void drop_graphs() {
        for (auto &x : exec)
            if (x) {
                (void)hipGraphExecDestroy(x);
                x = nullptr;
            }
    }
    ~BatchPlan() {
        drop_graphs();
        if (st) batch_destroy(st);
        if (cap) (void)hipStreamDestroy(cap);
        for (auto &f : fields) free_plan_memory(&f);
    }
};

struct vsht_plan_s {
    Plan p;                       // the plan, or the summary of a batch
    BatchPlan *batch = nullptr;   // non-null for a batch plan
    ~vsht_plan_s() { delete batch; }
};

extern "C" {

int64_t vsht_num_coeffs(int L) { return L >= 1 ? (int64_t)L * (L + 2) : 0; }

const char *vsht_status_string(vsht_status s) {
    switch (s) {
        case VSHT_OK: return "VSHT_OK";
        case VSHT_EINVAL: return "VSHT_EINVAL: invalid argument";
        case VSHT_ENOWEIGHTS: return "VSHT_ENOWEIGHTS: plan has no quadrature weights";
        case VSHT_ENOMEM: return "VSHT_ENOMEM: out of memory";
        case VSHT_EDEVICE: return "VSHT_EDEVICE: HIP error";
        case VSHT_EUNSUPPORTED: return "VSHT_EUNSUPPORTED: not supported for this plan";
    }
    return "unknown vsht_status";
}

const char *vsht_last_error(void) { return g_last_error.c_str(); }

// Fields of vsht_opts beyond the precision and device.
static vsht_status check_opts(const vsht_opts *opts) {
    if (!opts) return VSHT_OK;
    if (opts->flags & ~(VSHT_OPT_SCATTERED_DIRECT | VSHT_OPT_NO_FOLD)) return fail(VSHT_EINVAL, "unknown flag in opts");
    if (!(opts->nfft_eps >= 0.0 && opts->nfft_eps < 1.0)) return fail(VSHT_EINVAL, "nfft_eps must lie in [0, 1)");
    return VSHT_OK;
}

vsht_status vsht_plan(int L, int64_t n, const double *xyz, const double *w, const vsht_opts *opts,
                      vsht_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(VSHT_EINVAL, "out is NULL");
    *out = nullptr;
    const int precision = opts ? opts->precision : VSHT_FP64;
    vsht_status s = check_plan_args(L, n, xyz, w, precision);
    if (s != VSHT_OK) return s;
    if ((s = check_opts(opts)) != VSHT_OK) return s;
    int dev = 0;
    if ((s = resolve_device(opts, &dev)) != VSHT_OK) return s;
    DeviceGuard guard(dev);
    auto *h = new (std::nothrow) vsht_plan_s();
    if (!h) return fail(VSHT_ENOMEM, "host allocation");
    if ((s = build_plan(h->p, L, n, xyz, w, precision, dev, opts ? opts->flags : 0, opts ? opts->nfft_eps : 0.0)) !=
        VSHT_OK) {
        delete h;
        return s;
    }
    *out = h;
    return VSHT_OK;
}

static size_t complex_bytes(const Plan &P) { return P.precision == VSHT_FP64 ? 16 : 8; }

// A caller's buffer must start on a whole complex element of the plan's type.
static bool misaligned(const void *x, size_t cb) { return ((uintptr_t)x % cb) != 0; }

static vsht_status check_call(vsht_plan_t plan, const void *x, const void *y, const void *z) {
    g_last_error.clear();
    if (!plan) return fail(VSHT_EINVAL, "plan is NULL");
    if (plan->batch) return fail(VSHT_EINVAL, "batch plan: use the vsht_batch_* calls");
    if (!x || !y || !z) return fail(VSHT_EINVAL, "NULL buffer");
    const size_t cb = complex_bytes(plan->p);
    if (misaligned(x, cb) || misaligned(y, cb) || misaligned(z, cb))
        return fail(VSHT_EINVAL, "buffer not aligned to its " + std::to_string(cb) + "-byte complex elements");
    return VSHT_OK;
}

vsht_status vsht_forward(vsht_plan_t plan, const void *T, void *a, void *b, void *stream) {
    vsht_status s = check_call(plan, T, a, b);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (!P.has_weights) return fail(VSHT_ENOWEIGHTS, "forward needs a plan created with weights");
    if (P.kind != VSHT_PLAN_RINGS && !P.nfft.on)
        return fail(VSHT_EUNSUPPORTED, "forward transform on scattered points needs the grid path");
    DeviceGuard guard(P.device);
    hipError_t e = launch_forward(P, T, a, b, true, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "forward launch");
}

vsht_status vsht_forward_unweighted(vsht_plan_t plan, const void *T, void *a, void *b,
                                    void *stream) {
    vsht_status s = check_call(plan, T, a, b);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (P.kind != VSHT_PLAN_RINGS && !P.nfft.on)
        return fail(VSHT_EUNSUPPORTED, "forward transform on scattered points needs the grid path");
    DeviceGuard guard(P.device);
    hipError_t e = launch_forward(P, T, a, b, false, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "forward launch");
}

vsht_status vsht_forward_static(vsht_plan_t plan, const void *T, void *a, void *b, void *stream) {
    static_assert(VSHT_STATIC_SCRATCH_BYTES == kStaticScratchBytes, "one scratch size");
    vsht_status s = check_call(plan, T, a, b);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (!P.has_weights) return fail(VSHT_ENOWEIGHTS, "forward needs a plan created with weights");
    if (P.kind != VSHT_PLAN_RINGS) return fail(VSHT_EUNSUPPORTED, "the static-scratch forward needs a ring plan");
    const size_t need = static_forward_bytes(P);
    if (need > kStaticScratchBytes)
        return fail(VSHT_EUNSUPPORTED, "the plan needs " + std::to_string(need) +
                                           " bytes of scratch; the static array holds " +
                                           std::to_string(kStaticScratchBytes));
    DeviceGuard guard(P.device);
    hipError_t e = launch_forward_static(P, T, a, b, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "static-scratch forward launch");
}

vsht_status vsht_adjoint(vsht_plan_t plan, const void *a, const void *b, void *T, void *stream) {
    vsht_status s = check_call(plan, a, b, T);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    DeviceGuard guard(P.device);
    hipError_t e = launch_adjoint(P, a, b, T, false, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "adjoint launch");
}

int64_t vsht_num_sht_coeffs(int L) { return L >= 0 ? (int64_t)(L + 1) * (L + 1) : 0; }

vsht_status vsht_sht_forward(vsht_plan_t plan, const void *f, void *flm, void *stream) {
    vsht_status s = check_call(plan, f, flm, flm);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (P.kind != VSHT_PLAN_RINGS) return fail(VSHT_EUNSUPPORTED, "scalar transforms need a ring plan");
    if (!P.has_weights) return fail(VSHT_ENOWEIGHTS, "forward needs a plan created with weights");
    DeviceGuard guard(P.device);
    hipError_t e = launch_sht_forward(P, f, flm, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "scalar forward launch");
}

vsht_status vsht_sht_adjoint(vsht_plan_t plan, const void *flm, void *f, void *stream) {
    vsht_status s = check_call(plan, flm, flm, f);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (P.kind != VSHT_PLAN_RINGS) return fail(VSHT_EUNSUPPORTED, "scalar transforms need a ring plan");
    DeviceGuard guard(P.device);
    hipError_t e = launch_sht_adjoint(P, flm, f, (hipStream_t)stream);
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "scalar adjoint launch");
}


// Fields per launch of the *_many calls on a ring plan: up to 64, and no more than
// fit 4 GiB of workspace (at least one).
static int many_chunk(const Plan &P, int64_t count) {
    const size_t per = field_ws(P).total();
    const int64_t fit = std::max<int64_t>(1, (int64_t)(((size_t)4 << 30) / std::max<size_t>(per, 1)));
    return (int)std::min<int64_t>({count, (int64_t)64, fit});
}

// The many-field workspace for nf fields (grown on demand; waits for the device
// before replacing a smaller one, which earlier calls may still use).
static hipError_t ensure_many(Plan &P, int nf) {
    const size_t need = field_ws(P).total() * (size_t)nf;
    if (P.d_many && P.many_bytes >= need) return hipSuccess;
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return e;
    if (P.d_many) (void)hipFree(P.d_many);
    P.d_many = nullptr;
    P.many_bytes = 0;
    if ((e = hipMalloc(&P.d_many, need)) != hipSuccess) return e;
    P.many_bytes = need;
    return hipSuccess;
}

vsht_status vsht_forward_many(vsht_plan_t plan, int64_t count, const void *T, void *a, void *b,
                              int flags, void *stream) {
    vsht_status s = check_call(plan, T, a, b);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (count < 0) return fail(VSHT_EINVAL, "count < 0");
    if (flags & ~VSHT_UNIT_WEIGHTS) return fail(VSHT_EINVAL, "unknown flag for the forward transform");
    const bool weighted = !(flags & VSHT_UNIT_WEIGHTS);
    if (weighted && !P.has_weights) return fail(VSHT_ENOWEIGHTS, "forward needs a plan created with weights");
    if (P.kind != VSHT_PLAN_RINGS && !P.nfft.on)
        return fail(VSHT_EUNSUPPORTED, "forward transform on scattered points needs the grid path");
    DeviceGuard guard(P.device);
    const size_t cb = complex_bytes(P);
    const size_t t_stride = (size_t)P.n * 3 * cb, c_stride = (size_t)vsht_num_coeffs(P.L) * cb;
    const int chunk = P.kind == VSHT_PLAN_RINGS ? many_chunk(P, count) : 1;
    for (int64_t f = 0; f < count; f += chunk) {
        const int nf = (int)std::min<int64_t>(chunk, count - f);
        const char *Tf = static_cast<const char *>(T) + f * t_stride;
        char *af = static_cast<char *>(a) + f * c_stride, *bf = static_cast<char *>(b) + f * c_stride;
        hipError_t e;
        if (nf > 1) {
            if ((e = ensure_many(plan->p, nf)) != hipSuccess) return hip_fail(e, "many-field workspace");
            e = launch_forward_many(P, nf, P.d_many, Tf, af, bf, weighted, (hipStream_t)stream);
        } else {
            e = launch_forward(P, Tf, af, bf, weighted, (hipStream_t)stream);
        }
        if (e != hipSuccess) return hip_fail(e, "forward launch");
    }
    return VSHT_OK;
}

vsht_status vsht_adjoint_many(vsht_plan_t plan, int64_t count, const void *a, const void *b, void *T,
                              int flags, void *stream) {
    vsht_status s = check_call(plan, a, b, T);
    if (s != VSHT_OK) return s;
    const Plan &P = plan->p;
    if (count < 0) return fail(VSHT_EINVAL, "count < 0");
    if (flags & ~VSHT_TIMES_WEIGHTS) return fail(VSHT_EINVAL, "unknown flag for the adjoint transform");
    const bool weighted = (flags & VSHT_TIMES_WEIGHTS) != 0;
    if (weighted && !P.has_weights) return fail(VSHT_ENOWEIGHTS, "VSHT_TIMES_WEIGHTS needs a plan created with weights");
    DeviceGuard guard(P.device);
    const size_t cb = complex_bytes(P);
    const size_t t_stride = (size_t)P.n * 3 * cb, c_stride = (size_t)vsht_num_coeffs(P.L) * cb;
    const int chunk = P.kind == VSHT_PLAN_RINGS ? many_chunk(P, count) : 1;
    for (int64_t f = 0; f < count; f += chunk) {
        const int nf = (int)std::min<int64_t>(chunk, count - f);
        const char *af = static_cast<const char *>(a) + f * c_stride, *bf = static_cast<const char *>(b) + f * c_stride;
        char *Tf = static_cast<char *>(T) + f * t_stride;
        hipError_t e;
        if (nf > 1) {
            if ((e = ensure_many(plan->p, nf)) != hipSuccess) return hip_fail(e, "many-field workspace");
            e = launch_adjoint_many(P, nf, P.d_many, af, bf, Tf, weighted, (hipStream_t)stream);
        } else {
            e = launch_adjoint(P, af, bf, Tf, weighted, (hipStream_t)stream);
        }
        if (e != hipSuccess) return hip_fail(e, "adjoint launch");
    }
    return VSHT_OK;
}

size_t vsht_workspace_bytes(vsht_plan_t plan) {
    if (!plan) return 0;
    if (plan->batch) {
        size_t t = 0;
        for (const Plan &f : plan->batch->fields) t += f.workspace_bytes;
        return t;
    }
    return plan->p.workspace_bytes + plan->p.many_bytes;
}

vsht_status vsht_plan_info(vsht_plan_t plan, vsht_plan_info_t *info) {
    g_last_error.clear();
    if (!plan || !info) return fail(VSHT_EINVAL, "NULL argument");
    const Plan &P = plan->p;
    info->L = P.L;
    info->precision = P.precision;
    info->kind = P.kind;
    info->n_points = P.n;
    info->n_rings = P.n_rings;
    info->n_pairs = P.n_pairs;
    info->max_nphi = P.max_nphi;
    info->has_weights = P.has_weights;
    info->workspace_bytes = P.workspace_bytes;
    info->table_bytes = P.table_bytes;
    info->nfft_grid = P.nfft.on ? P.nfft.ng : 0;
    return VSHT_OK;
}

static void drop_records(Plan &P) {
    for (auto &r : P.records) {
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    P.records.clear();
}

vsht_status vsht_set_stage_timing(vsht_plan_t plan, int enable) {
    g_last_error.clear();
    if (!plan) return fail(VSHT_EINVAL, "plan is NULL");
    DeviceGuard guard(plan->p.device);
    if (!enable) {
        (void)hipDeviceSynchronize();
        drop_records(plan->p);
    }
    plan->p.timing = enable ? 1 : 0;
    return VSHT_OK;
}

vsht_status vsht_get_stage_times(vsht_plan_t plan, double *ms, int64_t *count, int nstages) {
    g_last_error.clear();
    if (!plan || !ms || !count || nstages < 0) return fail(VSHT_EINVAL, "NULL argument");
    if (nstages > VSHT_NUM_STAGES) nstages = VSHT_NUM_STAGES;
    for (int s = 0; s < nstages; ++s) {
        ms[s] = 0.0;
        count[s] = 0;
    }
    Plan &P = plan->p;
    DeviceGuard guard(P.device);
    hipError_t err = hipSuccess;
    for (auto &r : P.records) {
        hipError_t e = hipEventSynchronize(r.stop);
        float t = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&t, r.start, r.stop);
        if (e != hipSuccess) err = e;
        else if (r.stage < nstages) {
            ms[r.stage] += t;
            count[r.stage] += 1;
        }
    }
    drop_records(P);
    return err == hipSuccess ? VSHT_OK : hip_fail(err, "stage timing");
}

vsht_status vsht_plan_destroy(vsht_plan_t plan) {
    g_last_error.clear();
    if (!plan) return VSHT_OK;
    {
        DeviceGuard guard(plan->p.device);
        (void)hipDeviceSynchronize();
        drop_records(plan->p);
        if (!plan->batch) free_plan_memory(&plan->p);
        delete plan;
    }
    return VSHT_OK;
}

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
vsht_status vsht_plan_batch(int nfields, const int *L, const int64_t *n, const double *const *xyz,
                            const double *const *w, const vsht_opts *opts, vsht_plan_t *out) {
    g_last_error.clear();
    if (!out) return fail(VSHT_EINVAL, "out is NULL");
    *out = nullptr;
    if (nfields < 1) return fail(VSHT_EINVAL, "nfields must be >= 1");
    if (!L || !n || !xyz || !w) return fail(VSHT_EINVAL, "NULL argument");
    if (vsht_status so = check_opts(opts); so != VSHT_OK) return so;
    const int precision = opts ? opts->precision : VSHT_FP64;
    for (int f = 0; f < nfields; ++f) {
        if (!w[f]) return fail(VSHT_EINVAL, "field " + std::to_string(f) + ": weights are required");
        vsht_status s = check_plan_args(L[f], n[f], xyz[f], w[f], precision);
        if (s != VSHT_OK) {
            g_last_error = "field " + std::to_string(f) + ": " + g_last_error;
            return s;
        }
    }
    int dev = 0;
    vsht_status s = resolve_device(opts, &dev);
    if (s != VSHT_OK) return s;
    DeviceGuard guard(dev);
    auto *h = new (std::nothrow) vsht_plan_s();
    if (!h) return fail(VSHT_ENOMEM, "host allocation");
    h->batch = new (std::nothrow) BatchPlan();
    if (!h->batch) {
        delete h;
        return fail(VSHT_ENOMEM, "host allocation");
    }
    BatchPlan &B = *h->batch;
    if (opts && opts->tune_cache) B.tune_cache = opts->tune_cache;
    B.fields.resize(nfields);
    Plan &S = h->p;  // summary
    S.precision = precision;
    S.device = dev;
    S.kind = VSHT_PLAN_BATCH;
    S.has_weights = 1;
    for (int f = 0; f < nfields; ++f) {
        s = build_plan(B.fields[f], L[f], n[f], xyz[f], w[f], precision, dev, opts ? opts->flags : 0,
                       opts ? opts->nfft_eps : 0.0);
        if (s == VSHT_OK && B.fields[f].kind != VSHT_PLAN_RINGS)
            s = fail(VSHT_EUNSUPPORTED, "a batch needs iso-latitude ring grids");
        // the batched analysis holds all of a field's ring-pair tiles in one workgroup
        if (s == VSHT_OK && analysis_groups(B.fields[f].n_pairs, B.fields[f].eq_ring) > 1)
            s = fail(VSHT_EUNSUPPORTED, "a batch field may have at most 1024 ring pairs (" +
                                            std::to_string(B.fields[f].n_pairs) + " given)");
        if (s != VSHT_OK) {
            g_last_error = "field " + std::to_string(f) + ": " + g_last_error;
            delete h;
            return s;
        }
        const Plan &F = B.fields[f];
        S.L = std::max(S.L, F.L);
        S.n += F.n;
        S.n_rings += F.n_rings;
        S.n_pairs += F.n_pairs;
        S.max_nphi = std::max(S.max_nphi, F.max_nphi);
        S.workspace_bytes += F.workspace_bytes;
        S.table_bytes += F.table_bytes;
    }
    std::vector<const Plan *> ptrs;
    for (auto &f : B.fields) ptrs.push_back(&f);
    hipError_t e = batch_create(ptrs, &B.st);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&B.cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        delete h;
        return hip_fail(e, "batch setup");
    }
    *out = h;
    return VSHT_OK;
}

static vsht_status check_batch(vsht_plan_t plan) {
    g_last_error.clear();
    if (!plan) return fail(VSHT_EINVAL, "plan is NULL");
    if (!plan->batch) return fail(VSHT_EINVAL, "not a batch plan");
    return VSHT_OK;
}

static bool same_pointers(const std::vector<const void *> &v, std::initializer_list<const void *const *> arrs,
                          size_t F) {
    if (v.size() != arrs.size() * F) return false;
    size_t k = 0;
    for (auto a : arrs)
        for (size_t i = 0; i < F; ++i)
            if (v[k++] != a[i]) return false;
    return true;
}

static void remember(std::vector<const void *> &v, std::initializer_list<const void *const *> arrs, size_t F) {
    v.clear();
    for (auto a : arrs)
        for (size_t i = 0; i < F; ++i) v.push_back(a[i]);
}

static vsht_status check_ptr_arrays(std::initializer_list<const void *const *> arrs, size_t F, size_t cb) {
    for (auto a : arrs) {
        if (!a) return fail(VSHT_EINVAL, "NULL pointer array");
        for (size_t i = 0; i < F; ++i) {
            if (!a[i]) return fail(VSHT_EINVAL, "NULL buffer for field " + std::to_string(i));
            if (misaligned(a[i], cb))
                return fail(VSHT_EINVAL, "buffer of field " + std::to_string(i) + " not aligned to its " +
                                             std::to_string(cb) + "-byte complex elements");
        }
    }
    return VSHT_OK;
}

// Replay (capturing on first use) the graph of the stages of `dirs`.
static vsht_status batch_run(BatchPlan &B, int dirs, hipStream_t stream) {
    hipError_t e = hipSuccess;
    if (!B.exec[dirs]) {
        hipGraph_t g = nullptr;
        e = hipStreamBeginCapture(B.cap, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
        hipError_t el = batch_launch(B.st, dirs, B.cap);
        e = hipStreamEndCapture(B.cap, &g);
        if (el != hipSuccess || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return hip_fail(el != hipSuccess ? el : e, "batch capture");
        }
        e = hipGraphInstantiate(&B.exec[dirs], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            B.exec[dirs] = nullptr;
            return hip_fail(e, "hipGraphInstantiate");
        }
    }
    e = hipGraphLaunch(B.exec[dirs], stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    B.last_dirs = dirs;
    return VSHT_OK;
}

static vsht_status batch_bind(BatchPlan &B, int dirs, const void *const *a, const void *const *b,
                              void *const *T, void *const *a2, void *const *b2, hipStream_t stream) {
    const size_t F = B.fields.size();
    hipError_t e = hipSuccess;
    if ((dirs & 1) && !same_pointers(B.bound_adj, {a, b, (const void *const *)T}, F)) {
        e = batch_bind_adjoint(B.st, a, b, T, stream);
        if (e != hipSuccess) return hip_fail(e, "batch bind");
        remember(B.bound_adj, {a, b, (const void *const *)T}, F);
    }
    if ((dirs & 2) && !same_pointers(B.bound_fwd, {(const void *const *)T, (const void *const *)a2,
                                                   (const void *const *)b2}, F)) {
        e = batch_bind_forward(B.st, T, a2, b2, stream);
        if (e != hipSuccess) return hip_fail(e, "batch bind");
        remember(B.bound_fwd, {(const void *const *)T, (const void *const *)a2, (const void *const *)b2}, F);
    }
    return VSHT_OK;
}

vsht_status vsht_batch_adjoint(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                               void *stream) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    BatchPlan &B = *plan->batch;
    if ((s = check_ptr_arrays({a, b, (const void *const *)T}, B.fields.size(), complex_bytes(B.fields[0]))) != VSHT_OK) return s;
    DeviceGuard guard(plan->p.device);
    if ((s = batch_bind(B, 1, a, b, T, nullptr, nullptr, (hipStream_t)stream)) != VSHT_OK) return s;
    return batch_run(B, 1, (hipStream_t)stream);
}

vsht_status vsht_batch_forward(vsht_plan_t plan, const void *const *T, void *const *a, void *const *b,
                               void *stream) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    BatchPlan &B = *plan->batch;
    if ((s = check_ptr_arrays({T, (const void *const *)a, (const void *const *)b}, B.fields.size(), complex_bytes(B.fields[0]))) != VSHT_OK)
        return s;
    DeviceGuard guard(plan->p.device);
    if ((s = batch_bind(B, 2, nullptr, nullptr, const_cast<void *const *>(T), a, b, (hipStream_t)stream)) != VSHT_OK)
        return s;
    return batch_run(B, 2, (hipStream_t)stream);
}

vsht_status vsht_batch_roundtrip(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                                 void *const *a2, void *const *b2, void *stream) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    BatchPlan &B = *plan->batch;
    if ((s = check_ptr_arrays({a, b, (const void *const *)T, (const void *const *)a2, (const void *const *)b2},
                              B.fields.size(), complex_bytes(B.fields[0]))) != VSHT_OK)
        return s;
    DeviceGuard guard(plan->p.device);
    if ((s = batch_bind(B, 3, a, b, T, a2, b2, (hipStream_t)stream)) != VSHT_OK) return s;
    return batch_run(B, 3, (hipStream_t)stream);
}

vsht_status vsht_batch_set_config(vsht_plan_t plan, int adj_nw, int fwd_merge, int lpt, int ring_nt,
                                  int chains) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    if (adj_nw != 1 && adj_nw != 2 && adj_nw != 4) return fail(VSHT_EINVAL, "adj_nw must be 1, 2 or 4");
    if (ring_nt != 256 && ring_nt != 512) return fail(VSHT_EINVAL, "ring_nt must be 256 or 512");
    if (chains && !kBatchChainsEnabled)
        return fail(VSHT_EUNSUPPORTED, "parallel size-class chains are switched off in this build");
    BatchPlan &B = *plan->batch;
    DeviceGuard guard(plan->p.device);
    hipError_t e = hipDeviceSynchronize();  // no replay may still read the work lists
    if (e == hipSuccess) {
        B.drop_graphs();
        BatchConfig c;
        c.adj_nw = adj_nw;
        c.fwd_merge = fwd_merge ? 1 : 0;
        c.lpt = lpt ? 1 : 0;
        c.ring_nt = ring_nt;
        c.chains = chains ? 1 : 0;
        e = batch_configure(B.st, c);
    }
    return e == hipSuccess ? VSHT_OK : hip_fail(e, "batch configure");
}

vsht_status vsht_batch_get_config(vsht_plan_t plan, int *adj_nw, int *fwd_merge, int *lpt, int *ring_nt,
                                  int *chains) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    if (!adj_nw || !fwd_merge || !lpt || !ring_nt || !chains) return fail(VSHT_EINVAL, "NULL argument");
    const BatchConfig c = batch_config(plan->batch->st);
    *adj_nw = c.adj_nw;
    *fwd_merge = c.fwd_merge;
    *lpt = c.lpt;
    *ring_nt = c.ring_nt;
    *chains = c.chains;
    return VSHT_OK;
}

// Autotune cache: one line per batch, "<key> adj_nw fwd_merge lpt ring_nt chains ms".
// The key names the line format ("b2"), the device architecture, the precision, the
// field count and an FNV-1a digest of every field's (L, points, rings, longest stored
// DFT length); lines of another format never match it.
static std::string tune_key(const BatchPlan &B, int dev) {
    hipDeviceProp_t prop{};
    std::string arch = hipGetDeviceProperties(&prop, dev) == hipSuccess ? prop.gcnArchName : "unknown";
    arch = arch.substr(0, arch.find(':'));  // "gfx950" of "gfx950:sramecc+:xnack-"
    for (char &c : arch)
        if (c == ' ') c = '_';
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](int64_t v) {
        for (int i = 0; i < 8; ++i) {
            h ^= (uint64_t)((v >> (8 * i)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const Plan &f : B.fields) {
        mix(f.L);
        mix(f.n);
        mix(f.n_rings);
        mix(f.max_fft_len);
    }
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)h);
    return "b2:" + arch + ":p" + std::to_string(B.fields.empty() ? 0 : B.fields[0].precision) + ":f" +
           std::to_string(B.fields.size()) + ":" + buf;
}

static bool tune_lookup(const std::string &path, const std::string &key, int c[5], double *ms) {
    std::FILE *fp = std::fopen(path.c_str(), "r");
    if (!fp) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof line, fp)) {
        char k[256];
        int v[5];
        double t;
        if (std::sscanf(line, "%255s %d %d %d %d %d %lf", k, &v[0], &v[1], &v[2], &v[3], &v[4], &t) == 7 &&
            key == k) {
            for (int i = 0; i < 5; ++i) c[i] = v[i];
            *ms = t;
            found = true;  // the last entry for a key wins
        }
    }
    std::fclose(fp);
    return found;
}

static void tune_store(const std::string &path, const std::string &key, int nw, int fm, int lpt, int rnt,
                       int ch, double ms) {
    std::FILE *fp = std::fopen(path.c_str(), "a");
    if (!fp) return;  // the cache is an optimisation: a file that cannot be written is skipped
    std::fprintf(fp, "%s %d %d %d %d %d %.9g\n", key.c_str(), nw, fm, lpt, rnt, ch, ms);
    std::fclose(fp);
}

vsht_status vsht_batch_autotune(vsht_plan_t plan, const void *const *a, const void *const *b, void *const *T,
                                void *const *a2, void *const *b2, int reps, double *best_ms, void *stream) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    if (reps < 1) return fail(VSHT_EINVAL, "reps must be >= 1");
    BatchPlan &B = *plan->batch;
    if ((s = check_ptr_arrays({a, b, (const void *const *)T, (const void *const *)a2, (const void *const *)b2},
                              B.fields.size(), complex_bytes(B.fields[0]))) != VSHT_OK)
        return s;
    DeviceGuard guard(plan->p.device);
    const std::string key = tune_key(B, plan->p.device);
    if (!B.tune_cache.empty()) {
        int c[5];
        double ms = 0.0;
        if (tune_lookup(B.tune_cache, key, c, &ms)) {
            if (best_ms) *best_ms = ms;
            return vsht_batch_set_config(plan, c[0], c[1], c[2], c[3], c[4]);
        }
    }
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    float best = -1.f;
    int bn = 4, bm = 0, bl = 1, br = 256, bc = 0;
    const int nws[1] = {4};  // the synthesis shape is fixed (four waves); adj_nw has no effect
    for (int i = 0; i < 1 && s == VSHT_OK; ++i)
        for (int fm = 0; fm < 2 && s == VSHT_OK; ++fm)
            for (int lpt = 0; lpt < 2 && s == VSHT_OK; ++lpt)
            for (int rnt : {256, 512})
            for (int ch = 0; ch < (kBatchChainsEnabled ? 2 : 1); ++ch) {
                if (s != VSHT_OK) break;
                s = vsht_batch_set_config(plan, nws[i], fm, lpt, rnt, ch);
                if (s == VSHT_OK) s = vsht_batch_roundtrip(plan, a, b, T, a2, b2, stream);  // capture + warm
                if (s != VSHT_OK) break;
                e = hipEventRecord(e0, st);
                for (int r = 0; r < reps && e == hipSuccess; ++r)
                    if (batch_run(B, 3, st) != VSHT_OK) e = hipErrorUnknown;
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    s = hip_fail(e, "autotune timing");
                    break;
                }
                ms /= reps;
                if (best < 0.f || ms < best) {
                    best = ms;
                    bn = nws[i];
                    bm = fm;
                    bl = lpt;
                    br = rnt;
                    bc = ch;
                }
            }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (s != VSHT_OK) return s;
    if (best_ms) *best_ms = best;
    if (!B.tune_cache.empty()) tune_store(B.tune_cache, key, bn, bm, bl, br, bc, best);
    return vsht_batch_set_config(plan, bn, bm, bl, br, bc);
}

vsht_status vsht_batch_field_times(vsht_plan_t plan, double *start_us, double *end_us) {
    vsht_status s = check_batch(plan);
    if (s != VSHT_OK) return s;
    if (!start_us || !end_us) return fail(VSHT_EINVAL, "NULL argument");
    BatchPlan &B = *plan->batch;
    if (!B.last_dirs) return fail(VSHT_EINVAL, "the batch has not run yet");
    DeviceGuard guard(plan->p.device);
    std::vector<double> t0, t1;
    hipError_t e = batch_field_times(B.st, B.last_dirs, t0, t1);
    if (e != hipSuccess) return hip_fail(e, "batch field times");
    for (size_t i = 0; i < t0.size(); ++i) {
        start_us[i] = t0[i];
        end_us[i] = t1[i];
    }
    return VSHT_OK;
}

}  // extern "C"
