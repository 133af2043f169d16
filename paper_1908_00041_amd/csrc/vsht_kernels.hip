// vsht_kernels.hip -- gfx950 kernels of the forward and adjoint VSHT.
//
// Pipeline on an iso-latitude ring grid (the formulation is stated at the top
// of vsht_internal.h):
//
//  forward  T --(k_ring_fwd)--> PB --(k_leg_fwd)--> FG --(k_recombine)--> a, b
//  adjoint  a, b --(k_prep)--> FG --(k_leg_adj)--> PB --(k_ring_adj)--> T
//
//  k_ring_*    one workgroup per north/south ring pair: rotate between
//              Cartesian and (theta, phi) components, mixed-radix Stockham DFT
//              over longitude in LDS, fold (N+S, N-S) / unfold (E+O, E-O).
//  k_leg_fwd   one workgroup per order m: the Legendre recurrence runs with
//              one lane per ring pair and writes Lambda tiles to LDS; the
//              contraction reads them back with one lane per degree l' and
//              takes the ring-pair data from scalar registers.
//  k_leg_adj   one wave per (m, 64 ring pairs): recurrence and contraction in
//              the same lane, coefficients from scalar registers.
//
// Legendre values are always produced in binary64 (seeds and recurrence);
// the contraction runs in the plan's arithmetic type.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include "vsht_internal.h"

namespace vsht {

template <typename real>
struct C2 {
    real x, y;
};

template <typename real>
__device__ __forceinline__ C2<real> cmul(C2<real> a, C2<real> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

__device__ __forceinline__ int uniform_int(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Value of a binary64 register in lane `lane` (wave-uniform result).
__device__ __forceinline__ double readlane_f64(double v, int lane) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)b, lane);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// ---------------------------------------------------------------------------
// Seeds Lambda_{m,m}(z_p) = (-1)^m sqrt((2m+1)/(4pi) prod_{k<=m} (2k-1)/(2k)) s^m,
// built as a running product whose binary exponent is carried separately, so
// no intermediate underflows; the final value is rounded once (to zero or a
// subnormal when it is below the binary64 range).
// ---------------------------------------------------------------------------
__global__ void k_seeds(const double *__restrict__ pair_s, int NP, int L,
                        double *__restrict__ seeds) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    const double s = pair_s[p];
    double mant = 0.28209479177387814347403972578;  // 1/sqrt(4 pi)
    int e2 = 0;
    seeds[p] = mant;
    for (int m = 1; m <= L; ++m) {
        mant *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
        int ex;
        mant = frexp(mant, &ex);
        e2 += ex;
        seeds[(size_t)m * NP + p] = ldexp(mant, e2);
    }
}

// ---------------------------------------------------------------------------
// LDS mixed-radix Stockham DFT of `nseq` sequences of length n stored
// back-to-back in `buf`.  Stage with radix R and span Ns maps input index
// j + t n/R (t < R) to output (j / Ns) Ns R + (j mod Ns) + k Ns with
//     X = sum_t x[j + t n/R] * w^(t q),  w = e^{-+2 pi i / (Ns R)},  q = (j mod Ns) + k Ns,
// which leaves the result in natural order after the last stage.  Every
// thread computes up to MAXO outputs per stage into registers, the block
// synchronises, then the outputs overwrite the inputs.  Twiddles are read
// from the plan's binary64 table e^{-2 pi i k / n}.
// ---------------------------------------------------------------------------
template <typename real, int NT, int MAXO>
__device__ void fft_lds(C2<real> *buf, int nseq, const FftDesc &fd, const double *__restrict__ tw,
                        bool inverse) {
    const int n = fd.n;
    const int total = nseq * n;
    const double *twn = tw + 2 * fd.tw_offset;
    int Ns = 1;
    for (int f = 0; f < fd.nfac; ++f) {
        const int R = fd.fac[f];
        const int nR = n / R;
        const int step = n / (Ns * R);
        C2<real> out[MAXO];
#pragma unroll
        for (int i = 0; i < MAXO; ++i) {
            const int o = threadIdx.x + i * NT;
            if (o < total) {
                const int sq = o / n;
                const int oo = o - sq * n;
                const int jr = oo % Ns;
                const int k = (oo / Ns) % R;
                const int jq = oo / (Ns * R);
                const int j = jq * Ns + jr;
                const int dq = (jr + k * Ns) * step;  // < n
                const C2<real> *x = buf + sq * n + j;
                real ar = 0, ai = 0;
                int ti = 0;
                for (int t = 0; t < R; ++t) {
                    const C2<real> v = x[t * nR];
                    const real wr = (real)twn[2 * ti];
                    const real wi = inverse ? -(real)twn[2 * ti + 1] : (real)twn[2 * ti + 1];
                    ar += v.x * wr - v.y * wi;
                    ai += v.x * wi + v.y * wr;
                    ti += dq;
                    if (ti >= n) ti -= n;
                }
                out[i] = {ar, ai};
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < MAXO; ++i) {
            const int o = threadIdx.x + i * NT;
            if (o < total) buf[o] = out[i];
        }
        __syncthreads();
        Ns *= R;
    }
}

// ---------------------------------------------------------------------------
// Forward ring stage: per pair, per ring: T_theta = e_theta . (w T),
// T_phi = e_phi . (w T), DFT over longitude, scale by e^{-+ i m phi_0} / s,
// then fold N/S.  Output PB[m][p][0] = N + S, PB[m][p][1] = N - S.
// ---------------------------------------------------------------------------
constexpr int kRingNT = 512;
constexpr int kRingMaxO = 12;  // 2 sequences: 2 * nphi <= kRingNT * kRingMaxO
constexpr int kRingMaxM = 4;   // L + 1 <= kRingNT * kRingMaxM
constexpr int kRingMaxB = 6;   // nphi <= kRingNT * kRingMaxB

template <typename real>
struct RingArgs {
    const C2<real> *Tin;
    C2<real> *Tout;
    const double *weights;
    C2<real> *PB;
    const RingDesc *rings;
    const PairDesc *pairs;
    const FftDesc *ffts;
    const double *tw;
    int L;
    int NP;
    int weighted;
};

template <typename real>
__global__ __launch_bounds__(kRingNT) void k_ring_fwd(RingArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    C2<real> *buf = reinterpret_cast<C2<real> *>(smem_raw);
    const int p = blockIdx.x;
    const PairDesc pd = A.pairs[p];
    const int L = A.L;
    C2<real> st[kRingMaxM][4];
#pragma unroll
    for (int i = 0; i < kRingMaxM; ++i)
#pragma unroll
        for (int c = 0; c < 4; ++c) st[i][c] = {0, 0};

    for (int side = 0; side < 2; ++side) {
        const int r = side == 0 ? pd.rn : pd.rs;
        if (r < 0) break;
        const RingDesc rd = A.rings[r];
        const FftDesc fd = A.ffts[rd.fft];
        const int n = rd.nphi;
        const double *twn = A.tw + 2 * fd.tw_offset;
        for (int j = threadIdx.x; j < n; j += kRingNT) {
            // e^{i phi_j} = e^{i phi_0} conj(e^{-2 pi i j / n})
            const double er = twn[2 * j], ei = -twn[2 * j + 1];
            const real c = (real)(rd.c0 * er - rd.s0 * ei);
            const real sn = (real)(rd.s0 * er + rd.c0 * ei);
            const int64_t k = rd.offset + j;
            real w = 1;
            if (A.weighted) w = (real)(rd.uniform_w ? rd.w : A.weights[k]);
            const C2<real> t1 = A.Tin[3 * k], t2 = A.Tin[3 * k + 1], t3 = A.Tin[3 * k + 2];
            const real z = (real)rd.z, s = (real)rd.s;
            C2<real> th, ph;
            th.x = w * (z * (c * t1.x + sn * t2.x) - s * t3.x);
            th.y = w * (z * (c * t1.y + sn * t2.y) - s * t3.y);
            ph.x = w * (c * t2.x - sn * t1.x);
            ph.y = w * (c * t2.y - sn * t1.y);
            buf[j] = th;
            buf[n + j] = ph;
        }
        __syncthreads();
        fft_lds<real, kRingNT, kRingMaxO>(buf, 2, fd, A.tw, false);
        const double inv_s = 1.0 / rd.s;
#pragma unroll
        for (int i = 0; i < kRingMaxM; ++i) {
            const int m = threadIdx.x + i * kRingNT;
            if (m <= L) {
                const int bp = m % n;
                const int bm = bp == 0 ? 0 : n - bp;
                double cph = 1.0, sph = 0.0;
                if (rd.phi0 != 0.0) sincos(m * rd.phi0, &sph, &cph);
                // +m: times e^{-i m phi0} / s ; -m: times e^{+i m phi0} / s
                const C2<real> fp = {(real)(cph * inv_s), (real)(-sph * inv_s)};
                const C2<real> fm = {(real)(cph * inv_s), (real)(sph * inv_s)};
                C2<real> v[4];
                v[0] = cmul(buf[bp], fp);
                v[1] = cmul(buf[n + bp], fp);
                v[2] = cmul(buf[bm], fm);
                v[3] = cmul(buf[n + bm], fm);
                if (side == 0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) st[i][c] = v[c];
                } else {
                    C2<real> *o = A.PB + ((size_t)m * A.NP + p) * 8;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        o[c] = {st[i][c].x + v[c].x, st[i][c].y + v[c].y};
                        o[4 + c] = {st[i][c].x - v[c].x, st[i][c].y - v[c].y};
                    }
                }
            }
        }
        __syncthreads();
    }
    if (pd.rs < 0) {
#pragma unroll
        for (int i = 0; i < kRingMaxM; ++i) {
            const int m = threadIdx.x + i * kRingNT;
            if (m <= L) {
                C2<real> *o = A.PB + ((size_t)m * A.NP + p) * 8;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    o[c] = st[i][c];
                    o[4 + c] = st[i][c];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint ring stage: per pair, per ring: H_m = (E_m +- O_m) e^{i m phi_0} / s
// placed in longitude bin m mod n (all aliases summed), inverse DFT, then
// T = T_theta e_theta + T_phi e_phi.
// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(kRingNT) void k_ring_adj(RingArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    C2<real> *buf = reinterpret_cast<C2<real> *>(smem_raw);
    const int p = blockIdx.x;
    const PairDesc pd = A.pairs[p];
    const int L = A.L;
    for (int side = 0; side < 2; ++side) {
        const int r = side == 0 ? pd.rn : pd.rs;
        if (r < 0) break;
        const real sgn = side == 0 ? (real)1 : (real)-1;
        const RingDesc rd = A.rings[r];
        const FftDesc fd = A.ffts[rd.fft];
        const int n = rd.nphi;
        const double inv_s = 1.0 / rd.s;
        for (int b = threadIdx.x; b < n; b += kRingNT) {
            C2<real> hth = {0, 0}, hph = {0, 0};
            // orders m = b + k n (k >= 0) and m = b - k n (k >= 1) with |m| <= L
            for (int pass = 0; pass < 2; ++pass) {
                int m = pass == 0 ? b : b - n;
                while (pass == 0 ? (m <= L) : (m >= -L)) {
                    const int am = m < 0 ? -m : m;
                    const int slot = m < 0 ? 2 : 0;
                    const C2<real> *e = A.PB + ((size_t)am * A.NP + p) * 8;
                    const C2<real> eth = e[slot], eph = e[slot + 1];
                    const C2<real> oth = e[4 + slot], oph = e[4 + slot + 1];
                    double cph = 1.0, sph = 0.0;
                    if (rd.phi0 != 0.0) sincos(m * rd.phi0, &sph, &cph);
                    const C2<real> f = {(real)(cph * inv_s), (real)(sph * inv_s)};
                    const C2<real> th = {eth.x + sgn * oth.x, eth.y + sgn * oth.y};
                    const C2<real> ph = {eph.x + sgn * oph.x, eph.y + sgn * oph.y};
                    const C2<real> a = cmul(th, f), c = cmul(ph, f);
                    hth.x += a.x; hth.y += a.y;
                    hph.x += c.x; hph.y += c.y;
                    m = pass == 0 ? m + n : m - n;
                }
            }
            buf[b] = hth;
            buf[n + b] = hph;
        }
        __syncthreads();
        fft_lds<real, kRingNT, kRingMaxO>(buf, 2, fd, A.tw, true);
        const double *twn = A.tw + 2 * fd.tw_offset;
        for (int j = threadIdx.x; j < n; j += kRingNT) {
            const double er = twn[2 * j], ei = -twn[2 * j + 1];
            const real c = (real)(rd.c0 * er - rd.s0 * ei);
            const real sn = (real)(rd.s0 * er + rd.c0 * ei);
            const real z = (real)rd.z, s = (real)rd.s;
            const C2<real> th = buf[j], ph = buf[n + j];
            const int64_t k = rd.offset + j;
            A.Tout[3 * k] = {z * c * th.x - sn * ph.x, z * c * th.y - sn * ph.y};
            A.Tout[3 * k + 1] = {z * sn * th.x + c * ph.x, z * sn * th.y + c * ph.y};
            A.Tout[3 * k + 2] = {-s * th.x, -s * th.y};
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Scaled Legendre recurrence.  With Lambda_{l,m} = c_{l,m} Q_{l,m} and
// c_{m,m} = c_{m+1,m} = 1, c_{l,m} = (alpha_l / alpha_{l-1}) c_{l-2,m}, the
// three-term recurrence becomes
//     Q_l = a'_l z Q_{l-1} - Q_{l-2},   a'_l = alpha_l c_{l-1} / c_l,
// two binary64 operations per step.  Starting from the state
// (Q_{m-1}, Q_{m-2}) = (0, -Lambda_{m,m}) the first step yields Q_m itself.
// c_{l,m} stays in [0.24, 1.13] for L <= 1024, so nothing is lost; it is
// applied to the outputs (analysis) or folded into the coefficients (synthesis).
// ---------------------------------------------------------------------------

// ---------------------------------------------------------------------------
// Forward Legendre contraction on MFMA:
//   FG[tri(m, l')][c] = c_{l'} sum_p Q_{l',m}(z_p) PB[m][p][(l'+m)&1][c].
// Workgroup = 5 waves for one order m.  Wave 4 (the producer, lane = ring
// pair) advances the recurrence 64 degrees for 64 pairs and stores Q into a
// double-buffered LDS tile, and copies the tile's 64 x 16 pair data next to
// it.  Waves 0..3 (consumers) each own 16 consecutive degrees and multiply
// Q[16 x 4 pairs] by PB[4 pairs x 16 columns] with v_mfma_f64_16x16x4; the 16
// columns are 8 of the even-parity sum S and 8 of the odd-parity difference D,
// and each output row keeps the half that matches its parity.
// ---------------------------------------------------------------------------
constexpr int kFwRows = 64;          // degrees per chunk (4 consumer waves x 16)
constexpr int kFwTile = 64;          // ring pairs per tile (producer lanes)
constexpr int kFwPitch = kFwTile + 1;
constexpr int kFwThreads = 320;

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct LegFwdArgs64 {
    const double *PB;      // [(L+1)][NP][16]
    double *F;             // [tri][8]
    const double *seeds;   // [(L+1)][NP]
    const double *pz;
    const double *aprime;  // [tri]
    const double *cscale;  // [tri]
    double *state;         // [(L+1)][NP][2]
    int L;
    int NP;
};

__global__ __launch_bounds__(kFwThreads) void k_leg_fwd_mfma64(LegFwdArgs64 A) {
    extern __shared__ unsigned char smem_raw[];
    double *qbuf = reinterpret_cast<double *>(smem_raw);                 // [2][kFwRows][kFwPitch]
    double *gbuf = qbuf + 2 * kFwRows * kFwPitch;                        // [2][kFwTile][16]
    const int L = A.L, NP = A.NP;
    const int m = blockIdx.x;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t t0 = tri_offset(L, m);
    const int nl = L + 2 - m;
    const int nchunk = (nl + kFwRows - 1) / kFwRows;
    const int ntile = (NP + kFwTile - 1) / kFwTile;
    const int total = nchunk * ntile;
    double *state = A.state + (size_t)m * NP * 2;

    f64x4 acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
    for (int it = 0; it <= total; ++it) {
        if (wave == 4 && it < total) {
            const int ch = it / ntile, t = it - ch * ntile;
            const int base = m + ch * kFwRows;
            const int p = t * kFwTile + lane;
            const bool valid = p < NP;
            double *qb = qbuf + (it & 1) * kFwRows * kFwPitch;
            double *gb = gbuf + (it & 1) * kFwTile * 16;
            // pair data for this tile (zero beyond the last pair)
            {
                const double *src = A.PB + ((size_t)m * NP + p) * 16;
#pragma unroll
                for (int c = 0; c < 16; ++c) gb[lane * 16 + c] = valid ? src[c] : 0.0;
            }
            const double z = valid ? A.pz[p] : 0.0;
            double q1, q2;
            if (ch == 0) {
                q1 = 0.0;
                q2 = valid ? -A.seeds[(size_t)m * NP + p] : 0.0;
            } else {
                q1 = valid ? state[2 * p] : 0.0;
                q2 = valid ? state[2 * p + 1] : 0.0;
            }
            // this chunk's a' values, one per lane, broadcast step by step
            const int lpl = base + lane;
            const double areg = lpl <= L + 1 ? A.aprime[t0 + lpl - m] : 0.0;
#pragma unroll
            for (int s = 0; s < kFwRows; ++s) {
                const double as = readlane_f64(areg, s);
                const double v = fma(as, z * q1, -q2);
                qb[s * kFwPitch + lane] = v;
                q2 = q1;
                q1 = v;
            }
            if (valid) {
                state[2 * p] = q1;
                state[2 * p + 1] = q2;
            }
        }
        if (wave < 4 && it >= 1) {
            const int jt = it - 1;
            const int ch = jt / ntile, t = jt - ch * ntile;
            const double *qb = qbuf + (jt & 1) * kFwRows * kFwPitch;
            const double *gb = gbuf + (jt & 1) * kFwTile * 16;
            if (t == 0) {
                acc0 = f64x4{0, 0, 0, 0};
                acc1 = f64x4{0, 0, 0, 0};
            }
            const int i = lane & 15, k = lane >> 4;
            const double *arow = qb + (wave * 16 + i) * kFwPitch + k;
            const double *bcol = gb + k * 16 + i;
            double av[16], bv[16];
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                av[g] = arow[4 * g];
                bv[g] = bcol[4 * g * 16];
            }
#pragma unroll
            for (int g = 0; g < 16; g += 2) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g], bv[g], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av[g + 1], bv[g + 1], acc1, 0, 0, 0);
            }
            if (t == ntile - 1) {
                const int base = m + ch * kFwRows + wave * 16;
                const int j = lane & 15;
                // v_mfma_f64_16x16x4 result: lane l, register r holds row 4r + l/16,
                // column l%16 (measured on gfx950).  Row parity (lp + m) & 1 equals
                // (l/16) & 1 and selects S (column < 8) or D (column >= 8).
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int lp = base + 4 * r + (lane >> 4);
                    if (lp <= L + 1 && ((j >> 3) == ((lane >> 4) & 1))) {
                        const int64_t ti = t0 + lp - m;
                        A.F[ti * 8 + (j & 7)] = A.cscale[ti] * (acc0[r] + acc1[r]);
                    }
                }
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Adjoint Legendre synthesis (VALU): for pair p and order m,
//   PB[m][p][0][c] = sum_{l'+m even} Q_{l',m}(z_p) FG[tri(m,l')][c]
//   PB[m][p][1][c] = sum_{l'+m odd}  Q_{l',m}(z_p) FG[tri(m,l')][c]
// (FG already carries c_{l'}).  One wave per (64 pairs, m); the coefficients
// and a' are wave-uniform and live in scalar registers.
// ---------------------------------------------------------------------------
template <typename real>
struct LegArgs {
    const C2<real> *FGin;
    C2<real> *PBout;
    const double *seeds;
    const double *pz;
    const double *aprime;
    int L;
    int NP;
};

template <typename real>
__global__ __launch_bounds__(64) void k_leg_adj(LegArgs<real> A) {
    const int L = A.L, NP = A.NP;
    const int m = blockIdx.y;
    const int p = blockIdx.x * 64 + threadIdx.x;
    const bool valid = p < NP;
    const int64_t t0 = tri_offset(L, m);
    const double *ap = A.aprime + t0 - m;       // indexed by l'
    const C2<real> *g = A.FGin + (t0 - m) * 4;  // indexed by l'
    const double z = valid ? A.pz[p] : 0.0;
    double q1 = 0.0;
    double q2 = valid ? -A.seeds[(size_t)m * NP + p] : 0.0;
    C2<real> E[4], O[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) E[c] = O[c] = {0, 0};
    int lp = m;
    for (; lp + 1 <= L + 1; lp += 2) {
        const double v1 = fma(ap[lp], z * q1, -q2);       // parity even (lp - m even)
        const double v2 = fma(ap[lp + 1], z * v1, -q1);   // parity odd
        const real a1 = (real)v1, a2 = (real)v2;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            E[c].x += a1 * g[lp * 4 + c].x;
            E[c].y += a1 * g[lp * 4 + c].y;
            O[c].x += a2 * g[(lp + 1) * 4 + c].x;
            O[c].y += a2 * g[(lp + 1) * 4 + c].y;
        }
        q2 = v1;
        q1 = v2;
    }
    if (lp <= L + 1) {
        const double v1 = fma(ap[lp], z * q1, -q2);
        const real a1 = (real)v1;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            E[c].x += a1 * g[lp * 4 + c].x;
            E[c].y += a1 * g[lp * 4 + c].y;
        }
    }
    if (valid) {
        C2<real> *o = A.PBout + ((size_t)m * NP + p) * 8;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            o[c] = E[c];
            o[4 + c] = O[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Forward Legendre contraction (VALU, any arithmetic type): one lane per
// degree, recurrence by a producer wave through LDS as in the MFMA kernel,
// ring-pair data in scalar registers.  Used for binary32.
// ---------------------------------------------------------------------------
constexpr int kLfChunk = 128;
constexpr int kLfTile = 64;
constexpr int kLfPitch = kLfTile + 1;

template <typename real>
struct LegFwdArgs {
    const C2<real> *PBin;
    C2<real> *FGout;
    const double *seeds;
    const double *pz;
    const double *aprime;
    const double *cscale;
    double *state;
    int L;
    int NP;
};

template <typename real>
__global__ __launch_bounds__(192) void k_leg_fwd(LegFwdArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    real *tile = reinterpret_cast<real *>(smem_raw);  // [2][64][kLfPitch]
    const int L = A.L, NP = A.NP;
    const int m = blockIdx.x;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int64_t t0 = tri_offset(L, m);
    const int nl = L + 2 - m;
    const int nchunk = (nl + kLfChunk - 1) / kLfChunk;
    const int ntile = (NP + kLfTile - 1) / kLfTile;
    double *state = A.state + (size_t)m * NP * 2;
    const double *ap = A.aprime + t0 - m;

    for (int ch = 0; ch < nchunk; ++ch) {
        const int base = m + ch * kLfChunk;
        C2<real> acc[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] = {0, 0};
        for (int t = 0; t < ntile; ++t) {
            if (wave == 0) {
                const int p = t * kLfTile + lane;
                const bool valid = p < NP;
                const double z = valid ? A.pz[p] : 0.0;
                double q1 = 0.0, q2 = 0.0;
                if (ch == 0) {
                    q2 = valid ? -A.seeds[(size_t)m * NP + p] : 0.0;
                } else if (valid) {
                    q1 = state[2 * p];
                    q2 = state[2 * p + 1];
                }
                for (int s = 0; s < kLfChunk; ++s) {
                    const int lp = base + s;
                    const double v = lp <= L + 1 ? fma(ap[lp], z * q1, -q2) : 0.0;
                    tile[((s & 1) * 64 + (s >> 1)) * kLfPitch + lane] = (real)v;
                    q2 = q1;
                    q1 = v;
                }
                if (valid) {
                    state[2 * p] = q1;
                    state[2 * p + 1] = q2;
                }
            }
            __syncthreads();
            if (wave >= 1) {
                const int q = wave - 1;
                const int npt = min(kLfTile, NP - t * kLfTile);
                const C2<real> *g = A.PBin + ((size_t)m * NP + (size_t)t * kLfTile) * 8 + q * 4;
                const real *trow = tile + (q * 64 + lane) * kLfPitch;
                for (int pp = 0; pp < npt; ++pp) {
                    const real lam = trow[pp];
                    const C2<real> *gp = g + pp * 8;
#pragma unroll
                    for (int c = 0; c < 4; ++c) {
                        acc[c].x += lam * gp[c].x;
                        acc[c].y += lam * gp[c].y;
                    }
                }
            }
            __syncthreads();
        }
        if (wave >= 1) {
            const int lp = base + 2 * lane + (wave - 1);
            if (lp <= L + 1) {
                const real cs = (real)A.cscale[t0 + lp - m];
                C2<real> *o = A.FGout + (t0 + lp - m) * 4;
#pragma unroll
                for (int c = 0; c < 4; ++c) o[c] = {cs * acc[c].x, cs * acc[c].y};
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Three-term recombination (forward):
//   a_{l,mu} = [l e_{l+1} F^th_{l+1} - (l+1) e_l F^th_{l-1} - i mu F^ph_l] / sqrt(l(l+1))
//   b_{l,mu} = [l e_{l+1} F^ph_{l+1} - (l+1) e_l F^ph_{l-1} + i mu F^th_l] / sqrt(l(l+1))
// with e_l = sqrt((l^2-m^2)/(4l^2-1)) and F_{.,-m} = (-1)^m FG[.][2..3].
// ---------------------------------------------------------------------------
template <typename real>
struct CoefArgs {
    const C2<real> *FG;
    C2<real> *FGout;
    const C2<real> *ain, *bin;
    C2<real> *aout, *bout;
    const double *cscale;
    int L;
};

__device__ __forceinline__ double e_lm(int l, int m) {
    const double L = l, M = m;
    return sqrt((L * L - M * M) / (4.0 * L * L - 1.0));
}

template <typename real>
__global__ void k_recombine(CoefArgs<real> A) {
    const int L = A.L;
    const int m = blockIdx.y;
    const int l = (m > 1 ? m : 1) + blockIdx.x * blockDim.x + threadIdx.x;
    if (l > L) return;
    const int64_t t0 = tri_offset(L, m);
    const C2<real> *F = A.FG + (t0 - m) * 4;  // indexed by l'
    const double ep = e_lm(l + 1, m), em = (l - 1 >= m) ? e_lm(l, m) : 0.0;
    const double inv = 1.0 / sqrt((double)l * (l + 1));
    const real cp = (real)(l * ep * inv), cm = (real)((l + 1) * em * inv);
    for (int sgn = 0; sgn < (m == 0 ? 1 : 2); ++sgn) {
        const int mu = sgn == 0 ? m : -m;
        const int off = sgn == 0 ? 0 : 2;
        const real parity = (sgn == 1 && (m & 1)) ? (real)-1 : (real)1;
        const real fmu = (real)(mu * inv);
        const C2<real> th1 = F[(l + 1) * 4 + off], ph1 = F[(l + 1) * 4 + off + 1];
        const C2<real> th0 = F[l * 4 + off], ph0 = F[l * 4 + off + 1];
        C2<real> thm = {0, 0}, phm = {0, 0};
        if (l - 1 >= m) {
            thm = F[(l - 1) * 4 + off];
            phm = F[(l - 1) * 4 + off + 1];
        }
        C2<real> av, bv;
        // -i mu F^ph  = (mu F^ph.y, -mu F^ph.x);  +i mu F^th = (-mu F^th.y, mu F^th.x)
        av.x = parity * (cp * th1.x - cm * thm.x + fmu * ph0.y);
        av.y = parity * (cp * th1.y - cm * thm.y - fmu * ph0.x);
        bv.x = parity * (cp * ph1.x - cm * phm.x - fmu * th0.y);
        bv.y = parity * (cp * ph1.y - cm * phm.y + fmu * th0.x);
        const int64_t j = (int64_t)l * l + l + mu - 1;
        A.aout[j] = av;
        A.bout[j] = bv;
    }
}

// ---------------------------------------------------------------------------
// Adjoint prep: FG[tri(m, l')] = c_{l'} (g^th_{+m}, g^ph_{+m}, (-1)^m g^th_{-m}, (-1)^m g^ph_{-m}),
//   g^th_{l',mu} = (l'-1) e_{l'} at_{l'-1} - (l'+2) e_{l'+1} at_{l'+1} - i mu bt_{l'}
//   g^ph_{l',mu} = (l'-1) e_{l'} bt_{l'-1} - (l'+2) e_{l'+1} bt_{l'+1} + i mu at_{l'}
// with at = a / sqrt(l(l+1)) (zero outside 1 <= l <= L, |mu| <= l).
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ C2<real> coef_scaled(const C2<real> *c, int L, int l, int mu) {
    if (l < 1 || l > L || mu > l || -mu > l) return {0, 0};
    const C2<real> v = c[(int64_t)l * l + l + mu - 1];
    const real f = (real)(1.0 / sqrt((double)l * (l + 1)));
    return {v.x * f, v.y * f};
}

template <typename real>
__global__ void k_prep(CoefArgs<real> A) {
    const int L = A.L;
    const int m = blockIdx.y;
    const int lp = m + blockIdx.x * blockDim.x + threadIdx.x;
    if (lp > L + 1) return;
    const int64_t t0 = tri_offset(L, m);
    const double cs = A.cscale[t0 + lp - m];  // Lambda = c Q: fold c_{l'} in
    const real c1 = (real)(cs * (lp - 1) * (lp >= 1 ? e_lm(lp, m) : 0.0));
    const real c2 = (real)(cs * (lp + 2) * e_lm(lp + 1, m));
    const real csr = (real)cs;
    C2<real> *o = A.FGout + (t0 + lp - m) * 4;
    for (int sgn = 0; sgn < 2; ++sgn) {
        const int mu = sgn == 0 ? m : -m;
        const real parity = (sgn == 1 && (m & 1)) ? (real)-1 : (real)1;
        const real fmu = (real)mu;
        const C2<real> am1 = coef_scaled(A.ain, L, lp - 1, mu), ap1 = coef_scaled(A.ain, L, lp + 1, mu);
        const C2<real> bm1 = coef_scaled(A.bin, L, lp - 1, mu), bp1 = coef_scaled(A.bin, L, lp + 1, mu);
        const C2<real> a0 = coef_scaled(A.ain, L, lp, mu), b0 = coef_scaled(A.bin, L, lp, mu);
        C2<real> gth, gph;
        // -i mu b = (mu b.y, -mu b.x); +i mu a = (-mu a.y, mu a.x)
        gth.x = parity * (c1 * am1.x - c2 * ap1.x + csr * fmu * b0.y);
        gth.y = parity * (c1 * am1.y - c2 * ap1.y - csr * fmu * b0.x);
        gph.x = parity * (c1 * bm1.x - c2 * bp1.x - csr * fmu * a0.y);
        gph.y = parity * (c1 * bm1.y - c2 * bp1.y + csr * fmu * a0.x);
        o[2 * sgn] = gth;
        o[2 * sgn + 1] = gph;
    }
}

// ---------------------------------------------------------------------------
// Adjoint at scattered points, evaluated directly: one lane per point,
//   s T_theta = sum_{m>=0} sum_{l'} Lambda_{l',m}(z) (g^th_{l',+m} e^{i m phi} + [m>0] g'^th e^{-i m phi})
// and likewise for phi; then T = T_theta e_theta + T_phi e_phi.  At an exact
// pole only |m| = 1 survives and Lambda_{l',1}/s is replaced by its limit
// -sqrt((2l'+1)/(4 pi l'(l'+1))) l'(l'+1)/2 z^{l'+1}.
// ---------------------------------------------------------------------------
template <typename real>
struct ScatArgs {
    const C2<real> *FG;
    const double *xyz;
    const double *aprime;
    const double *cscale;
    C2<real> *Tout;
    int64_t n;
    int L;
};

template <typename real>
__global__ __launch_bounds__(64) void k_adj_scattered(ScatArgs<real> A) {
    const int64_t k = (int64_t)blockIdx.x * 64 + threadIdx.x;
    const bool valid = k < A.n;
    const int L = A.L;
    double x = 0, y = 0, z = 1;
    if (valid) {
        x = A.xyz[3 * k];
        y = A.xyz[3 * k + 1];
        z = A.xyz[3 * k + 2];
    }
    const double s = sqrt(x * x + y * y);
    const bool pole = !(s > 0.0);
    const double c = pole ? 1.0 : x / s, sn = pole ? 0.0 : y / s;
    double thr = 0, thi = 0, phr = 0, phi_ = 0;  // s T_theta, s T_phi (or limits at poles)
    double er = 1.0, ei = 0.0;                     // e^{i m phi}
    double mant = 0.28209479177387814347403972578;
    int e2 = 0;
    for (int m = 0; m <= L; ++m) {
        if (m > 0) {
            mant *= -sqrt((2.0 * m + 1.0) / (2.0 * m)) * s;
            int ex;
            mant = frexp(mant, &ex);
            e2 += ex;
            const double ner = er * c - ei * sn;
            ei = er * sn + ei * c;
            er = ner;
        }
        const int64_t t0 = tri_offset(L, m);
        const C2<real> *g = A.FG + (t0 - m) * 4;
        const double *ap = A.aprime + t0 - m;
        double h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
        if (!pole) {
            double q1 = 0.0, q2 = -ldexp(mant, e2);
            for (int lp = m; lp <= L + 1; ++lp) {
                const double v = fma(ap[lp], z * q1, -q2);
                q2 = q1;
                q1 = v;
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    h[2 * cc] += v * (double)g[lp * 4 + cc].x;
                    h[2 * cc + 1] += v * (double)g[lp * 4 + cc].y;
                }
            }
        } else if (m == 1) {
            // the coefficients carry c_{l'}: divide it out of the limit of Lambda/s
            const double *cs = A.cscale + t0 - m;
            for (int lp = 1; lp <= L + 1; ++lp) {
                const double ll = (double)lp * (lp + 1);
                double v = -sqrt((2.0 * lp + 1.0) / (4.0 * M_PI * ll)) * ll * 0.5 / cs[lp];
                if (z < 0 && ((lp + 1) & 1)) v = -v;
#pragma unroll
                for (int cc = 0; cc < 4; ++cc) {
                    h[2 * cc] += v * (double)g[lp * 4 + cc].x;
                    h[2 * cc + 1] += v * (double)g[lp * 4 + cc].y;
                }
            }
        }
        // +m with e^{i m phi}
        thr += h[0] * er - h[1] * ei;
        thi += h[0] * ei + h[1] * er;
        phr += h[2] * er - h[3] * ei;
        phi_ += h[2] * ei + h[3] * er;
        if (m > 0) {  // -m with e^{-i m phi}
            thr += h[4] * er + h[5] * ei;
            thi += -h[4] * ei + h[5] * er;
            phr += h[6] * er + h[7] * ei;
            phi_ += -h[6] * ei + h[7] * er;
        }
    }
    if (!valid) return;
    const double inv_s = pole ? 1.0 : 1.0 / s;
    thr *= inv_s; thi *= inv_s; phr *= inv_s; phi_ *= inv_s;
    // e_theta = (z c, z sn, -s), e_phi = (-sn, c, 0)
    A.Tout[3 * k] = {(real)(z * c * thr - sn * phr), (real)(z * c * thi - sn * phi_)};
    A.Tout[3 * k + 1] = {(real)(z * sn * thr + c * phr), (real)(z * sn * thi + c * phi_)};
    A.Tout[3 * k + 2] = {(real)(-s * thr), (real)(-s * thi)};
}

// ===========================================================================
// launchers
// ===========================================================================
static size_t ring_lds_bytes(const Plan &p, size_t real_size) {
    return (size_t)2 * p.max_nphi * 2 * real_size;
}

template <typename real>
static hipError_t forward_impl(const Plan &p, const void *T, void *a, void *b, bool weighted,
                               hipStream_t st) {
    RingArgs<real> R{};
    R.Tin = static_cast<const C2<real> *>(T);
    R.weights = p.d_weights;
    R.PB = static_cast<C2<real> *>(p.d_pb);
    R.rings = p.d_rings;
    R.pairs = p.d_pairs;
    R.ffts = p.d_ffts;
    R.tw = p.d_tw;
    R.L = p.L;
    R.NP = (int)p.n_pairs;
    R.weighted = weighted ? 1 : 0;
    const size_t lds = ring_lds_bytes(p, sizeof(real));
    {
        StageScope sc(p, VSHT_STAGE_RING_FWD, st);
        hipLaunchKernelGGL(k_ring_fwd<real>, dim3((unsigned)p.n_pairs), dim3(kRingNT), lds, st, R);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    if constexpr (sizeof(real) == 8) {
        LegFwdArgs64 G{};
        G.PB = static_cast<const double *>(p.d_pb);
        G.F = static_cast<double *>(p.d_fg);
        G.seeds = p.d_seeds;
        G.pz = p.d_pair_z;
        G.aprime = p.d_aprime;
        G.cscale = p.d_cscale;
        G.state = static_cast<double *>(p.d_state);
        G.L = p.L;
        G.NP = (int)p.n_pairs;
        const size_t lds2 = (size_t)(2 * kFwRows * kFwPitch + 2 * kFwTile * 16) * sizeof(double);
        StageScope sc(p, VSHT_STAGE_LEG_FWD, st);
        hipLaunchKernelGGL(k_leg_fwd_mfma64, dim3(p.L + 1), dim3(kFwThreads), lds2, st, G);
    } else {
        LegFwdArgs<real> G{};
        G.PBin = static_cast<const C2<real> *>(p.d_pb);
        G.FGout = static_cast<C2<real> *>(p.d_fg);
        G.seeds = p.d_seeds;
        G.pz = p.d_pair_z;
        G.aprime = p.d_aprime;
        G.cscale = p.d_cscale;
        G.state = static_cast<double *>(p.d_state);
        G.L = p.L;
        G.NP = (int)p.n_pairs;
        const size_t lds2 = (size_t)2 * 64 * kLfPitch * sizeof(real);
        StageScope sc(p, VSHT_STAGE_LEG_FWD, st);
        hipLaunchKernelGGL(k_leg_fwd<real>, dim3(p.L + 1), dim3(192), lds2, st, G);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    CoefArgs<real> C{};
    C.FG = static_cast<const C2<real> *>(p.d_fg);
    C.aout = static_cast<C2<real> *>(a);
    C.bout = static_cast<C2<real> *>(b);
    C.L = p.L;
    {
        StageScope sc(p, VSHT_STAGE_RECOMBINE, st);
        hipLaunchKernelGGL(k_recombine<real>, dim3((p.L + 255) / 256, p.L + 1), dim3(256), 0, st, C);
    }
    return hipGetLastError();
}

template <typename real>
static hipError_t adjoint_impl(const Plan &p, const void *a, const void *b, void *T,
                               hipStream_t st) {
    CoefArgs<real> C{};
    C.ain = static_cast<const C2<real> *>(a);
    C.bin = static_cast<const C2<real> *>(b);
    C.FGout = static_cast<C2<real> *>(p.d_fg);
    C.cscale = p.d_cscale;
    C.L = p.L;
    {
        StageScope sc(p, VSHT_STAGE_PREP, st);
        hipLaunchKernelGGL(k_prep<real>, dim3((p.L + 2 + 255) / 256, p.L + 1), dim3(256), 0, st, C);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    if (p.kind == VSHT_PLAN_SCATTERED) {
        ScatArgs<real> S{};
        S.FG = static_cast<const C2<real> *>(p.d_fg);
        S.xyz = p.d_xyz;
        S.aprime = p.d_aprime;
        S.cscale = p.d_cscale;
        S.Tout = static_cast<C2<real> *>(T);
        S.n = p.n;
        S.L = p.L;
        StageScope sc(p, VSHT_STAGE_SCATTERED, st);
        hipLaunchKernelGGL(k_adj_scattered<real>, dim3((unsigned)((p.n + 63) / 64)), dim3(64), 0,
                           st, S);
        return hipGetLastError();
    }

    LegArgs<real> G{};
    G.FGin = static_cast<const C2<real> *>(p.d_fg);
    G.PBout = static_cast<C2<real> *>(p.d_pb);
    G.seeds = p.d_seeds;
    G.pz = p.d_pair_z;
    G.aprime = p.d_aprime;
    G.L = p.L;
    G.NP = (int)p.n_pairs;
    {
        StageScope sc(p, VSHT_STAGE_LEG_ADJ, st);
        hipLaunchKernelGGL(k_leg_adj<real>, dim3((unsigned)((p.n_pairs + 63) / 64), p.L + 1),
                           dim3(64), 0, st, G);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    RingArgs<real> R{};
    R.Tout = static_cast<C2<real> *>(T);
    R.PB = static_cast<C2<real> *>(p.d_pb);
    R.rings = p.d_rings;
    R.pairs = p.d_pairs;
    R.ffts = p.d_ffts;
    R.tw = p.d_tw;
    R.L = p.L;
    R.NP = (int)p.n_pairs;
    const size_t lds = ring_lds_bytes(p, sizeof(real));
    {
        StageScope sc(p, VSHT_STAGE_RING_ADJ, st);
        hipLaunchKernelGGL(k_ring_adj<real>, dim3((unsigned)p.n_pairs), dim3(kRingNT), lds, st, R);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const Plan &p, const void *T, void *a, void *b, bool weighted,
                          hipStream_t st) {
    if (p.precision == VSHT_FP64) return forward_impl<double>(p, T, a, b, weighted, st);
    return forward_impl<float>(p, T, a, b, weighted, st);
}

hipError_t launch_adjoint(const Plan &p, const void *a, const void *b, void *T, hipStream_t st) {
    if (p.precision == VSHT_FP64) return adjoint_impl<double>(p, a, b, T, st);
    return adjoint_impl<float>(p, a, b, T, st);
}

hipError_t launch_seed_kernel(const double *pair_s, int NP, int L, double *seeds, hipStream_t st) {
    hipLaunchKernelGGL(k_seeds, dim3((NP + 127) / 128), dim3(128), 0, st, pair_s, NP, L, seeds);
    return hipGetLastError();
}

hipError_t set_kernel_attributes() {
    hipError_t e;
    const int big = 160 * 1024;
    e = hipFuncSetAttribute((const void *)k_ring_fwd<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_ring_fwd<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_ring_adj<double>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_ring_adj<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    e = hipFuncSetAttribute((const void *)k_leg_fwd_mfma64, hipFuncAttributeMaxDynamicSharedMemorySize, big);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_leg_fwd<float>, hipFuncAttributeMaxDynamicSharedMemorySize, big);
}

}  // namespace vsht
