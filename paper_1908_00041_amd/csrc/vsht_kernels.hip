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

#include <mutex>

#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <new>
#include <vector>

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

// Load of a value that is the same for the whole workgroup from memory that no
// kernel writes while it runs (plan tables, argument blocks, work lists):
// through the constant address space, so that it becomes a scalar load.
template <typename T>
__device__ __forceinline__ T ld_const(const T *p) {
#if defined(__HIP_DEVICE_COMPILE__)
    return *(const __attribute__((address_space(4))) T *)p;
#else
    return *p;  // host pass of the kernel templates: never executed
#endif
}

// Accesses of device memory through a pointer the compiler cannot trace to a
// kernel argument (one that passed through integers, readfirstlane, or was
// loaded from a table) become flat instructions, and flat instructions count
// against the LDS wait counter too: every wait for an LDS access then also
// waits for the global loads in flight.  gld / gst access such a pointer as
// global memory (all of the library's buffers are).
#if defined(__HIP_DEVICE_COMPILE__)
#define VSHT_GLOBAL_AS __attribute__((address_space(1)))
#else
#define VSHT_GLOBAL_AS
#endif
// (Scalars only: a structure copy becomes a memcpy whose source loses the cast;
// complex values go through a two-element vector.)
template <typename T>
__device__ __forceinline__ T gld(const T *p) {
    return *(const VSHT_GLOBAL_AS T *)p;
}
template <typename T>
__device__ __forceinline__ void gst(T *p, T v) {
    *(VSHT_GLOBAL_AS T *)p = v;
}
template <typename real>
__device__ __forceinline__ C2<real> gld(const C2<real> *p) {
    typedef real V __attribute__((ext_vector_type(2)));
    const V v = *(const VSHT_GLOBAL_AS V *)p;
    return {v.x, v.y};
}
template <typename real>
__device__ __forceinline__ void gst(C2<real> *p, C2<real> c) {
    typedef real V __attribute__((ext_vector_type(2)));
    V v;
    v.x = c.x;
    v.y = c.y;
    *(VSHT_GLOBAL_AS V *)p = v;
}

// The same for a structure read through a pointer taken from another table,
// made wave-uniform dword by dword (keeps its fields in scalar registers).
template <typename T>
__device__ __forceinline__ T ld_uniform(const T *p) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized structure");
    struct Words {
        uint32_t d[sizeof(T) / 4];
    };
    Words w;
    const uint32_t *q = reinterpret_cast<const uint32_t *>(p);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w.d[i] = gld(q + i);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w.d[i] = __builtin_amdgcn_readfirstlane(w.d[i]);
    return __builtin_bit_cast(T, w);
}

// The argument block of field f of a launch over fields (blockIdx.z), kept in
// scalar registers: the offsets depend only on the workgroup, and without the
// per-dword readfirstlane the compiler may keep the copy in private memory.
template <typename T>
__device__ __forceinline__ T field_args(const T &A, int f) {
    static_assert(sizeof(T) % 4 == 0, "dword-sized structure");
    struct Words {
        uint32_t d[sizeof(T) / 4];
    };
    Words w = __builtin_bit_cast(Words, A.at_field(f));
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) w.d[i] = __builtin_amdgcn_readfirstlane(w.d[i]);
    return __builtin_bit_cast(T, w);
}

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
// Start blocks and states (plan time).  One thread per (p, m): the seed as in
// k_seeds (same operations, so a start at block 0 is (0, -seeds[m][p]) bit for
// bit), then the recurrence Q_l = a'_l z Q_{l-1} - Q_{l-2} exactly as the
// Legendre stages evaluate it, on a state (q1, q2) scaled by 2^E: scaling by a
// power of two commutes with every rounding in the normal range, so the state
// saved at each block boundary is the unscaled recurrence's state.  The first
// degree with |c_l Q_l| >= 2^kSignificantExp2 (Lambda = c Q) fixes the block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_leg_start(const double *__restrict__ pair_z,
                                                 const double *__restrict__ pair_s, int NP, int L,
                                                 const double *__restrict__ aprime,
                                                 const double *__restrict__ cscale,
                                                 LegStart *__restrict__ start, int *__restrict__ sblk,
                                                 int *__restrict__ bad) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    const int m = blockIdx.y;
    if (p >= NP) return;
    const double s = pair_s[p], z = pair_z[p];
    double mant = 0.28209479177387814347403972578;  // 1/sqrt(4 pi)
    int e2 = 0;
    for (int k = 1; k <= m; ++k) {
        mant *= -sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
        int ex;
        mant = frexp(mant, &ex);
        e2 += ex;
    }
    const int64_t t0 = tri_offset(L, m);
    const double *ap = aprime + t0 - m, *cs = cscale + t0 - m;  // indexed by l'
    double q1 = 0.0, q2 = -mant;  // true state = (q1, q2) 2^E
    int E = e2;
    double bq1 = q1, bq2 = q2;
    int bE = E, bl = m;
    int blk = kStartNever;
    for (int l = m; l <= L + 1; ++l) {
        if (((l - m) & (kStartBlock - 1)) == 0) {
            bq1 = q1;
            bq2 = q2;
            bE = E;
            bl = l;
        }
        const double v = fma(ap[l] * z, q1, -q2);
        int ev;
        (void)frexp(v * cs[l], &ev);  // |c_l v| in [2^(ev-1), 2^ev)
        if (v != 0.0 && ev - 1 + E >= kSignificantExp2) {
            blk = (bl - m) / kStartBlock;
            break;
        }
        q2 = q1;
        q1 = v;
        int eq;
        (void)frexp(q1, &eq);
        if (q1 != 0.0 && (eq > 64 || eq < -64)) {
            q1 = ldexp(q1, -eq);
            q2 = ldexp(q2, -eq);
            E += eq;
        }
    }
    LegStart st{0.0, 0.0};
    if (blk != kStartNever) {
        st.q1 = ldexp(bq1, bE);
        st.q2 = ldexp(bq2, bE);
        const double lo = 2.2250738585072014e-308;  // smallest normal binary64
        if (blk > 0 && !(fabs(st.q1) >= lo && fabs(st.q2) >= lo)) *bad = 1;
    }
    start[(size_t)m * NP + p] = st;
    sblk[(size_t)m * NP + p] = blk;
}

// A lane's start in a Legendre stage: block (kStartNever for lanes without a
// ring pair) and state.  The lane's recurrence holds (0, 0) until its block
// boundary, where it takes the state.
__device__ __forceinline__ PairDesc ld_pair(const PairDesc *p) { return {gld(&p->rn), gld(&p->rs)}; }

struct LaneStart {
    double q1, q2;
    int blk;
};
__device__ __forceinline__ LaneStart lane_start(const LegStart *__restrict__ start, const int *__restrict__ sblk,
                                                size_t idx, bool valid) {
    LaneStart r{0.0, 0.0, kStartNever};
    if (valid) {
        r.q1 = gld(&start[idx].q1);
        r.q2 = gld(&start[idx].q2);
        r.blk = gld(sblk + idx);
    }
    return r;
}
// first start block of the wave (wave-uniform)
__device__ __forceinline__ int wave_min_blk(int b) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) b = min(b, __shfl_xor(b, o));
    return uniform_int(b);
}
// entering the degree block that begins d = l' - m degrees after m
__device__ __forceinline__ void take_start(const LaneStart &S, int d, double &q1, double &q2) {
    if (d == kStartBlock * S.blk) {
        q1 = S.q1;
        q2 = S.q2;
    }
}

// ---------------------------------------------------------------------------
// LDS mixed-radix Stockham DFT of two sequences of length n stored
// back-to-back in `buf`.  A stage with radix R and span Ns reads x[j + t n/R]
// (t < R) for butterfly j, multiplies input t by W^t with
// W = e^{-+2 pi i (j mod Ns) / (Ns R)}, applies an R-point DFT and writes
// output k to (j / Ns) Ns R + (j mod Ns) + k Ns, which leaves natural order
// after the last stage.  Each thread keeps its outputs in registers across
// one barrier and then overwrites the inputs in place.
//   R = 2, 3, 4, 5   whole butterflies with fixed constants;
//   other odd R      u_t = y_t + y_{R-t}, v_t = y_t - y_{R-t} and
//                    X_k, X_{R-k} = x_0 + sum_t u_t cos(2pi tk/R) +- i v_t sin(2pi tk/R),
//                    one work item per (butterfly, group of kKP output pairs).
// Twiddles: one entry of the binary64 table e^{-2 pi i k/n} per butterfly,
// powers by repeated binary64 multiplication.
// ---------------------------------------------------------------------------
struct CD {
    double x, y;
};
// Complex sequences in LDS.  Element i sits at p[i + (i >> ps)]: ps = 4 puts one
// pad element after every 16, which spreads the stride-4 and stride-2 writes of
// a first radix-4 or radix-2 stage over the banks; lengths whose first stage
// has an odd radix keep unit- and odd-stride accesses only, which are free of
// bank conflicts unpadded (ps = 30).  The choice is the DFT descriptor's.
template <typename real>
struct Seq {
    C2<real> *p;
    int ps;
    __device__ __forceinline__ C2<real> &operator[](int i) const { return p[i + (i >> ps)]; }
};
__device__ __forceinline__ CD cd_mul(CD a, CD b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename real>
__device__ __forceinline__ C2<real> cmul_d(C2<real> v, CD w) {
    const double vx = v.x, vy = v.y;
    return {(real)(vx * w.x - vy * w.y), (real)(vx * w.y + vy * w.x)};
}
template <typename real>
__device__ __forceinline__ C2<real> cadd(C2<real> a, C2<real> b) { return {a.x + b.x, a.y + b.y}; }
template <typename real>
__device__ __forceinline__ C2<real> csub(C2<real> a, C2<real> b) { return {a.x - b.x, a.y - b.y}; }
// a + i s b (s = +-1)
template <typename real>
__device__ __forceinline__ C2<real> cadd_i(C2<real> a, C2<real> b, real s) {
    return {a.x - s * b.y, a.y + s * b.x};
}
__device__ __forceinline__ CD tw_at(const double *twn, int k, bool inv) {
    const double re = gld(twn + 2 * k), im = gld(twn + 2 * k + 1);
    return {re, inv ? -im : im};
}

// Thread index hidden from loop-invariant code motion: every FFT stage is
// inlined into one kernel, and hoisting each stage's index arithmetic out of
// the stage loop would keep all of it live at once.
__device__ __forceinline__ int opaque_tid() {
    int t = threadIdx.x;
    asm volatile("" : "+v"(t));
    return t;
}

// R-point DFT of x into y; sg = -1 forward (e^{-i}), +1 inverse.
template <typename real, int R>
__device__ __forceinline__ void dft_small(const C2<real> *x, C2<real> *y, real sg) {
    if constexpr (R == 2) {
        y[0] = cadd(x[0], x[1]);
        y[1] = csub(x[0], x[1]);
    } else if constexpr (R == 3) {
        const real h = (real)0.5, s3 = (real)0.86602540378443864676372317075294;
        const C2<real> sum = cadd(x[1], x[2]), dif = csub(x[1], x[2]);
        y[0] = cadd(x[0], sum);
        const C2<real> t1 = {x[0].x - h * sum.x, x[0].y - h * sum.y};
        const C2<real> t2 = {s3 * dif.x, s3 * dif.y};
        y[1] = cadd_i(t1, t2, sg);
        y[2] = cadd_i(t1, t2, -sg);
    } else if constexpr (R == 4) {
        const C2<real> a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
        const C2<real> c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
        y[0] = cadd(a, c);
        y[2] = csub(a, c);
        y[1] = cadd_i(b, d, sg);
        y[3] = cadd_i(b, d, -sg);
    } else if constexpr (R == 5) {
        const real c1 = (real)0.30901699437494742410229341718282;   // cos(2pi/5)
        const real c2 = (real)-0.80901699437494742410229341718282;  // cos(4pi/5)
        const real s1 = (real)0.95105651629515357211643933337938;   // sin(2pi/5)
        const real s2 = (real)0.58778525229247312916870595463907;   // sin(4pi/5)
        const C2<real> u1 = cadd(x[1], x[4]), u2 = cadd(x[2], x[3]);
        const C2<real> v1 = csub(x[1], x[4]), v2 = csub(x[2], x[3]);
        y[0] = cadd(x[0], cadd(u1, u2));
        const C2<real> a1 = {x[0].x + c1 * u1.x + c2 * u2.x, x[0].y + c1 * u1.y + c2 * u2.y};
        const C2<real> a2 = {x[0].x + c2 * u1.x + c1 * u2.x, x[0].y + c2 * u1.y + c1 * u2.y};
        const C2<real> b1 = {s1 * v1.x + s2 * v2.x, s1 * v1.y + s2 * v2.y};
        const C2<real> b2 = {s2 * v1.x - s1 * v2.x, s2 * v1.y - s1 * v2.y};
        y[1] = cadd_i(a1, b1, sg);
        y[4] = cadd_i(a1, b1, -sg);
        y[2] = cadd_i(a2, b2, sg);
        y[3] = cadd_i(a2, b2, -sg);
    }
}

template <typename real, int NT, int R, int MAXI>
__device__ __forceinline__ void fft_stage_small(Seq<real> buf, int buf_off, int n, int Ns,
                                                const double *__restrict__ twn, bool inv) {
    const int nb = n / R;
    const int items = nb;
    const int step = n / (Ns * R);
    const real sg = inv ? (real)1 : (real)-1;
    const int tid = opaque_tid();
    const int off = buf_off;
    C2<real> out[MAXI][R];
    int dst[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int it = tid + i * NT;
        dst[i] = -1;
        if (it < items) {
            const int j = it;
            const int jr = j % Ns;
            C2<real> x[R];
            x[0] = buf[off + j];
            if (jr == 0) {
#pragma unroll
                for (int t = 1; t < R; ++t) x[t] = buf[off + j + t * nb];
            } else {
                const CD W = tw_at(twn, jr * step, inv);
                CD Wt = W;
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    x[t] = cmul_d(buf[off + j + t * nb], Wt);
                    if (t + 1 < R) Wt = cd_mul(Wt, W);
                }
            }
            dft_small<real, R>(x, out[i], sg);
            dst[i] = off + (j / Ns) * Ns * R + jr;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
        if (dst[i] >= 0) {
#pragma unroll
            for (int r = 0; r < R; ++r) buf[dst[i] + r * Ns] = out[i][r];
        }
    __syncthreads();
}


// The same radix-R stage applied to both sequences of a ring in one pass
// (sequence q at buf offset q * stride): a work item is one butterfly position
// of both sequences, which share its twiddle, so the stage costs one barrier
// pair instead of two.
template <typename real, int NT, int R, int MAXI>
__device__ __forceinline__ void fft_stage_small2(Seq<real> buf, int stride, int n, int Ns,
                                                 const double *__restrict__ twn, bool inv) {
    const int nb = n / R;
    const int step = n / (Ns * R);
    const real sg = inv ? (real)1 : (real)-1;
    const int tid = opaque_tid();
    C2<real> out[MAXI][2][R];
    int dst[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int j = tid + i * NT;
        dst[i] = -1;
        if (j < nb) {
            const int jr = j % Ns;
            CD Wp[R];
#pragma unroll
            for (int t = 0; t < R; ++t) Wp[t] = {1.0, 0.0};
            if (jr != 0) {
                const CD W = tw_at(twn, jr * step, inv);
                Wp[1] = W;
#pragma unroll
                for (int t = 2; t < R; ++t) Wp[t] = cd_mul(Wp[t - 1], W);
            }
#pragma unroll
            for (int sq = 0; sq < 2; ++sq) {
                C2<real> x[R];
                const int base = sq * stride + j;
                x[0] = buf[base];
#pragma unroll
                for (int t = 1; t < R; ++t) {
                    const C2<real> v = buf[base + t * nb];
                    x[t] = jr == 0 ? v : cmul_d(v, Wp[t]);
                }
                dft_small<real, R>(x, out[i][sq], sg);
            }
            dst[i] = (j / Ns) * Ns * R + jr;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
        if (dst[i] >= 0) {
#pragma unroll
            for (int sq = 0; sq < 2; ++sq)
#pragma unroll
                for (int r = 0; r < R; ++r) buf[sq * stride + dst[i] + r * Ns] = out[i][sq][r];
        }
    __syncthreads();
}

template <typename real, int NT, int MAXI>
__device__ __forceinline__ void fft_stage_odd(Seq<real> buf, int buf_off, int n, int R, int Ns,
                                              const double *__restrict__ twn, const CD *wR, bool inv) {
    const int nb = n / R;
    const int half = (R - 1) / 2;
    const int G = (half + kKP - 1) / kKP;
    const int items = nb * G;
    const int step = n / (Ns * R);
    const int stepR = n / R;  // table stride of omega_R
    const int tid = opaque_tid();
    const int off = buf_off;
    C2<real> out[MAXI][2 * kKP + 1];
    int dst[MAXI], grp[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int it = tid + i * NT;
        dst[i] = -1;
        grp[i] = 0;
        if (it < items) {
            const int g = it % G;
            const int j = it / G;
            const int jr = j % Ns;
            const int sb = off + j;
            const C2<real> x0 = buf[sb];
            const CD W = tw_at(twn, jr * step, inv);
            const CD WR = tw_at(twn, (int)(((int64_t)jr * R * step) % n), inv);  // W^R
            C2<real> A[kKP], B[kKP], S = {0, 0};
            int q[kKP], kq[kKP];
#pragma unroll
            for (int kk = 0; kk < kKP; ++kk) {
                A[kk] = B[kk] = {0, 0};
                kq[kk] = g * kKP + kk + 1;
                q[kk] = 0;
            }
            CD Wt = {1.0, 0.0};
#pragma unroll 1
            for (int t = 1; t <= half; ++t) {
                Wt = cd_mul(Wt, W);
                const CD Wm = cd_mul(WR, CD{Wt.x, -Wt.y});  // W^{R-t}
                const C2<real> yt = cmul_d(buf[sb + t * nb], Wt);
                const C2<real> ym = cmul_d(buf[sb + (R - t) * nb], Wm);
                const C2<real> u = cadd(yt, ym), v = csub(yt, ym);
                S = cadd(S, u);
#pragma unroll
                for (int kk = 0; kk < kKP; ++kk) {
                    q[kk] += kq[kk];
                    if (q[kk] >= R) q[kk] -= R;
                    const CD w = R <= kSmallTab ? wR[q[kk]] : tw_at(twn, q[kk] * stepR, inv);
                    const real wc = (real)w.x, ws = (real)w.y;
                    A[kk].x += u.x * wc;
                    A[kk].y += u.y * wc;
                    B[kk].x += v.x * ws;
                    B[kk].y += v.y * ws;
                }
            }
            // X_k = x0 + A + i B,  X_{R-k} = x0 + A - i B  (w carries the direction's sign)
#pragma unroll
            for (int kk = 0; kk < kKP; ++kk) {
                const C2<real> a = cadd(x0, A[kk]);
                out[i][2 * kk] = cadd_i(a, B[kk], (real)1);
                out[i][2 * kk + 1] = cadd_i(a, B[kk], (real)-1);
            }
            out[i][2 * kKP] = cadd(x0, S);
            dst[i] = off + (j / Ns) * Ns * R + jr;
            grp[i] = g;
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
        if (dst[i] >= 0) {
#pragma unroll
            for (int kk = 0; kk < kKP; ++kk) {
                const int k = grp[i] * kKP + kk + 1;
                if (k <= half) {
                    buf[dst[i] + k * Ns] = out[i][2 * kk];
                    buf[dst[i] + (R - k) * Ns] = out[i][2 * kk + 1];
                }
            }
            if (grp[i] == 0) buf[dst[i]] = out[i][2 * kKP];
        }
    __syncthreads();
}

// Entry q of the first-radix table e^{-2 pi i q / R} in the working precision,
// read with a scalar load (q is wave-uniform).
#if defined(__HIP_DEVICE_COMPILE__)
#define VSHT_CONST_AS __attribute__((address_space(4)))
#else
#define VSHT_CONST_AS
#endif
template <typename real>
__device__ __forceinline__ const VSHT_CONST_AS C2<real> *rtab_base(const double *rtab, int R);
template <>
__device__ __forceinline__ const VSHT_CONST_AS C2<double> *rtab_base<double>(const double *rtab, int) {
    return (const VSHT_CONST_AS C2<double> *)rtab;
}
template <>
__device__ __forceinline__ const VSHT_CONST_AS C2<float> *rtab_base<float>(const double *rtab, int R) {
    return (const VSHT_CONST_AS C2<float> *)(rtab + 2 * R);
}

// First stage (Ns = 1, so no twiddles) of an odd prime radix R > 5 on both
// sequences in one pass.  Each wave owns one group g of kKU output pairs
// k = kKU g + 1 .. kKU g + kKU (and R - k) and its lanes run over the 2 n / R
// columns of the two sequences, so every cos/sin factor is the same across the
// wave and comes from the scalar unit:
//     u_t = x_t + x_{R-t},  v_t = x_t - x_{R-t},
//     X_k = x_0 + sum_t u_t cos(2 pi k t / R) + i sum_t v_t (-+ sin(2 pi k t / R)),
//     X_{R-k} = the same with the second sum negated.
template <typename real, int NT, int MAXI>
__device__ __forceinline__ void fft_stage_odd_first(Seq<real> buf, int stride, int n, int R,
                                                    const double *rtab, bool inv) {
    const int nb = n / R;
    const int half = (R - 1) / 2;
    const int cols = 2 * nb;
    const int wpg = (cols + 63) >> 6;  // waves per group
    const int nw = first_stage_waves(n, R);
    const int wave0 = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const real bs = inv ? (real)-1 : (real)1;
    const VSHT_CONST_AS C2<real> *tab = rtab_base<real>(rtab, R);
    C2<real> out[MAXI][2 * kKU + 1];
    int dst[MAXI], grp[MAXI];
#pragma unroll
    for (int i = 0; i < MAXI; ++i) {
        const int wv = wave0 + i * (NT / 64);
        dst[i] = -1;
        grp[i] = 0;
        if (wv < nw) {
            const int g = wv / wpg;
            const int cs0 = (wv - g * wpg) * 64 + lane;
            // lanes past the last column compute on column 0 and store nothing, so the
            // loop stays in uniform control flow and the table reads stay scalar
            const bool valid = cs0 < cols;
            {
                const int cs = valid ? cs0 : 0;
                const int sq = cs >= nb ? 1 : 0;
                const int j = cs - sq * nb;
                const int sb = sq * stride + j;
                const C2<real> x0 = buf[sb];
                C2<real> A[kKU], B[kKU], S = {0, 0};
                int q[kKU], kq[kKU];
#pragma unroll
                for (int kk = 0; kk < kKU; ++kk) {
                    A[kk] = B[kk] = {0, 0};
                    kq[kk] = g * kKU + kk + 1;
                    if (kq[kk] > half) kq[kk] = 0;  // beyond the last pair: contributes nothing used
                    q[kk] = 0;
                }
#pragma unroll 2
                for (int t = 1; t <= half; ++t) {
                    const C2<real> xt = buf[sb + t * nb];
                    const C2<real> xm = buf[sb + (R - t) * nb];
                    const C2<real> u = cadd(xt, xm), v = csub(xt, xm);
                    S = cadd(S, u);
#pragma unroll
                    for (int kk = 0; kk < kKU; ++kk) {
                        q[kk] += kq[kk];
                        if (q[kk] >= R) q[kk] -= R;
                        const C2<real> w = tab[q[kk]];
                        A[kk].x += u.x * w.x;
                        A[kk].y += u.y * w.x;
                        B[kk].x += v.x * w.y;
                        B[kk].y += v.y * w.y;
                    }
                }
#pragma unroll
                for (int kk = 0; kk < kKU; ++kk) {
                    const C2<real> a = cadd(x0, A[kk]);
                    out[i][2 * kk] = cadd_i(a, B[kk], bs);
                    out[i][2 * kk + 1] = cadd_i(a, B[kk], -bs);
                }
                out[i][2 * kKU] = cadd(x0, S);
                dst[i] = valid ? sq * stride + j * R : -1;
                grp[i] = g;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < MAXI; ++i)
        if (dst[i] >= 0) {
#pragma unroll
            for (int kk = 0; kk < kKU; ++kk) {
                const int k = grp[i] * kKU + kk + 1;
                if (k <= half) {
                    buf[dst[i] + k] = out[i][2 * kk];
                    buf[dst[i] + R - k] = out[i][2 * kk + 1];
                }
            }
            if (grp[i] == 0) buf[dst[i]] = out[i][2 * kKU];
        }
    __syncthreads();
}

// Two sequences of length fdp->n in buf; wR is an LDS
// scratch of kSmallTab entries.
// The number of work items per thread (MAXI) is chosen per stage so that the
// outputs kept across the barrier fit in registers.
template <typename real, int NT, int R>
__device__ __forceinline__ void fft_small_dispatch(Seq<real> buf, int off, int n, int Ns,
                                                   const double *twn, bool inv) {
    static_assert(kMaxItemsSmall == 4, "dispatch below instantiates up to 4 items per thread");
    const int per = (n / R + NT - 1) / NT;
    if (per <= 1) fft_stage_small<real, NT, R, 1>(buf, off, n, Ns, twn, inv);
    else if (per <= 2) fft_stage_small<real, NT, R, 2>(buf, off, n, Ns, twn, inv);
    else fft_stage_small<real, NT, R, 4>(buf, off, n, Ns, twn, inv);
}

// Both sequences in one pass when a thread's outputs across the barrier stay
// within kMaxJointOut complex values; returns false (nothing done) otherwise.
constexpr int kMaxJointOut = 16;
template <typename real, int NT, int R>
__device__ __forceinline__ bool fft_small_joint(Seq<real> buf, int stride, int n, int Ns,
                                                const double *twn, bool inv) {
    const int per = (n / R + NT - 1) / NT;
    if (per <= 1 && 2 * R <= kMaxJointOut) {
        fft_stage_small2<real, NT, R, 1>(buf, stride, n, Ns, twn, inv);
        return true;
    }
    if constexpr (4 * R <= kMaxJointOut) {
        if (per <= 2) {
            fft_stage_small2<real, NT, R, 2>(buf, stride, n, Ns, twn, inv);
            return true;
        }
    }
    if constexpr (8 * R <= kMaxJointOut) {
        if (per <= 4) {
            fft_stage_small2<real, NT, R, 4>(buf, stride, n, Ns, twn, inv);
            return true;
        }
    }
    return false;
}

// Mixed-radix Stockham DFT of the two sequences at buf offsets 0 and `stride`.
// Stages are applied to one sequence at a time (the two sequences of a ring
// share each stage's twiddle set), so a thread holds at most 4 small
// butterflies or 2 odd-radix work items across a barrier (n <= 4096).
template <typename real, int NT>
__device__ __forceinline__ void fft_core(Seq<real> buf, int stride, const FftDesc *fdp,
                                         const double *__restrict__ tw, CD *wR, bool inv) {
    const int n = ld_const(&fdp->n);
    const int nfac = ld_const(&fdp->nfac);
    const double *twn = tw + 2 * ld_const(&fdp->tw_offset);
    int Ns = 1;
    for (int f = 0; f < nfac; ++f) {
        const int R = ld_const(&fdp->fac[f]);
        if (f == 0 && R > 5 && R <= kSmallTab) {
            // twiddle-free first stage (longer stages take the general path below)
            static_assert(kMaxRoundsFirst == 2, "dispatch below instantiates up to 2 waves per slot");
            const int rounds = (first_stage_waves(n, R) + NT / 64 - 1) / (NT / 64);
            const double *rtab = tw + 2 * ld_const(&fdp->rtab_offset);
            if (rounds <= 1) {
                fft_stage_odd_first<real, NT, 1>(buf, stride, n, R, rtab, inv);
                Ns *= R;
                continue;
            }
            if (rounds <= 2) {
                fft_stage_odd_first<real, NT, 2>(buf, stride, n, R, rtab, inv);
                Ns *= R;
                continue;
            }
        }
        if (R > 5 && R <= kSmallTab) {
            for (int qq = threadIdx.x; qq < R; qq += NT) wR[qq] = tw_at(twn, qq * (n / R), inv);
            __syncthreads();
        }
        bool joint = false;
        switch (R) {
            case 2: joint = fft_small_joint<real, NT, 2>(buf, stride, n, Ns, twn, inv); break;
            case 3: joint = fft_small_joint<real, NT, 3>(buf, stride, n, Ns, twn, inv); break;
            case 4: joint = fft_small_joint<real, NT, 4>(buf, stride, n, Ns, twn, inv); break;
            case 5: joint = fft_small_joint<real, NT, 5>(buf, stride, n, Ns, twn, inv); break;
            default: break;
        }
        for (int sq = 0; sq < (joint ? 0 : 2); ++sq) {
            const int off = sq * stride;
            switch (R) {
                case 2: fft_small_dispatch<real, NT, 2>(buf, off, n, Ns, twn, inv); break;
                case 3: fft_small_dispatch<real, NT, 3>(buf, off, n, Ns, twn, inv); break;
                case 4: fft_small_dispatch<real, NT, 4>(buf, off, n, Ns, twn, inv); break;
                case 5: fft_small_dispatch<real, NT, 5>(buf, off, n, Ns, twn, inv); break;
                default: {
                    const int items = (n / R) * (((R - 1) / 2 + kKP - 1) / kKP);
                    static_assert(kMaxItemsOdd == 2, "dispatch below instantiates up to 2 items per thread");
                    if (items <= NT) fft_stage_odd<real, NT, 1>(buf, off, n, R, Ns, twn, wR, inv);
                    else fft_stage_odd<real, NT, 2>(buf, off, n, R, Ns, twn, wR, inv);
                    break;
                }
            }
        }
        Ns *= R;
    }
}

// Storage stride of the second sequence of a ring whose DFT is described by fdp.
__device__ __forceinline__ int seq_stride(const FftDesc *fdp) {
    return ld_const(&fdp->blue) ? ld_const(&fdp->M) : ld_const(&fdp->n);
}

// DFT of length n of the two sequences of a ring (element i of sequence q at
// buf[q * stride + i], stride >= seq_stride), forward (e^{-2 pi i j m / n}) or inverse.
// Lengths with a prime factor above the generic-radix limit use Bluestein's
// identity j m = (j^2 + m^2 - (m - j)^2) / 2: with w_k = e^{-i pi k^2 / n},
//     X_m = w_m sum_j (x_j w_j) conj(w_{m-j}),
// a cyclic convolution of length M >= 2n - 1 (a power of two) evaluated with
// two mixed-radix DFTs of length M and the tabulated transform of the kernel
// (already divided by M); the inverse uses conj(w).
template <typename real, int NT>
__device__ __forceinline__ void fft_lds(Seq<real> buf, int stride, const FftDesc *ffts, const FftDesc *fdp,
                                        const double *__restrict__ tw, CD *wR, bool inv) {
    if (!ld_const(&fdp->blue)) {
        fft_core<real, NT>(buf, stride, fdp, tw, wR, inv);
        return;
    }
    const int n = ld_const(&fdp->n), M = ld_const(&fdp->M);
    const double *ch = tw + 2 * ld_const(&fdp->chirp_offset);
    const double *bh = tw + 2 * (ld_const(&fdp->bhat_offset) + (inv ? M : 0));
    for (int i = threadIdx.x; i < M; i += NT) {
        const CD w = tw_at(ch, i < n ? i : 0, inv);
#pragma unroll
        for (int sq = 0; sq < 2; ++sq) {
            C2<real> &v = buf[sq * stride + i];
            v = i < n ? cmul_d(v, w) : C2<real>{0, 0};
        }
    }
    __syncthreads();
    const FftDesc *md = ffts + ld_const(&fdp->mdesc);
    fft_core<real, NT>(buf, stride, md, tw, wR, false);
    for (int i = threadIdx.x; i < M; i += NT) {
        const CD w = tw_at(bh, i, false);
#pragma unroll
        for (int sq = 0; sq < 2; ++sq) {
            C2<real> &v = buf[sq * stride + i];
            v = cmul_d(v, w);
        }
    }
    __syncthreads();
    fft_core<real, NT>(buf, stride, md, tw, wR, true);
    for (int i = threadIdx.x; i < n; i += NT) {
        const CD w = tw_at(ch, i, inv);
#pragma unroll
        for (int sq = 0; sq < 2; ++sq) {
            C2<real> &v = buf[sq * stride + i];
            v = cmul_d(v, w);
        }
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Ring stages: one workgroup per ring.
//   forward: T_theta = e_theta . (w T), T_phi = e_phi . (w T), DFT over
//            longitude, scale by e^{-+ i m phi_0} / s, store
//            RB[m][r] = (G^th_{+m}, G^ph_{+m}, G^th_{-m}, G^ph_{-m}) for 0 <= m <= L.
//   adjoint: H_m = (E_m +- O_m) e^{i m phi_0} / s (sign + for the northern
//            ring of a pair, - for the southern) placed in bin m mod n with all
//            aliases summed, inverse DFT, T = T_theta e_theta + T_phi e_phi.
// The north/south fold of the forward transform happens when the Legendre
// stage loads RB.
// ---------------------------------------------------------------------------
constexpr int kRingNT = 512;  // threads per ring workgroup (256 serves rings whose DFT length is <= 2048)
constexpr int kRingNTSmall = 256;
constexpr int kMaxLenSmallRing = 2048;

template <typename real>
struct RingArgs {
    const C2<real> *Tin;
    C2<real> *Tout;
    const double *weights;
    C2<real> *buf;  // RB (forward) or PB (adjoint)
    const RingDesc *rings;
    const PairDesc *pairs;
    const FftDesc *ffts;
    const double *tw;
    int L;
    int NP;
    int NR;
    int weighted;
    int scalar;  // scalar transforms: one complex value f per point, T_theta = s f, T_phi = 0
    // launches over several fields (blockIdx.z = field): per-field strides of the
    // caller's field and of the ring/pair buffer, in complex elements (0 otherwise)
    int64_t zs_T, zs_buf;
    __device__ RingArgs at_field(int f) const {
        RingArgs r = *this;
        if (f) {
            if (Tin) r.Tin = Tin + f * zs_T;
            if (Tout) r.Tout = Tout + f * zs_T;
            r.buf = buf + f * zs_buf;
        }
        return r;
    }
};

// Workgroup -> ring of the single-field adjoint ring stage.  Workgroups are
// dealt to the 8 XCDs round robin (b mod 8); with b = 16 (q / 8) + 8 s + q mod 8
// the northern (s = 0) and southern (s = 1) rings of pair q run on one XCD, 8
// workgroups apart, so the southern ring finds the pair's Fourier records in
// that XCD's L2.  Returns -1 for the southern slot of an unpaired ring.
template <typename real>
__device__ __forceinline__ int ring_of_block(const RingArgs<real> &A, int b) {
    const int q = 8 * (b >> 4) + (b & 7), south = (b >> 3) & 1;
    if (q >= A.NP) return -1;
    const PairDesc pd = ld_const(A.pairs + q);
    return south ? pd.rs : pd.rn;
}

template <typename real, int NT>
__device__ __forceinline__ void ring_fwd_body(const RingArgs<real> &A, int r, unsigned char *smem_raw) {
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    const int NR = A.NR;
    const int L = A.L;
    const RingDesc rd = ld_uniform(A.rings + r);
    const FftDesc *fdp = A.ffts + rd.fft;
    const Seq<real> buf = {lds, ld_const(&fdp->lds_shift)};
    const int n = rd.nphi;
    const int n2 = seq_stride(fdp);
    const double *twn = A.tw + 2 * ld_const(&fdp->tw_offset);
    for (int j = threadIdx.x; j < n; j += NT) {
        // e^{i phi_j} = e^{i phi_0} conj(e^{-2 pi i j / n})
        const double er = gld(twn + 2 * j), ei = -gld(twn + 2 * j + 1);
        const real c = (real)(rd.c0 * er - rd.s0 * ei);
        const real sn = (real)(rd.s0 * er + rd.c0 * ei);
        const int64_t k = rd.offset + j;
        real w = 1;
        if (A.weighted) w = (real)(rd.uniform_w ? rd.w : gld(A.weights + k));
        const real z = (real)rd.z, s = (real)rd.s;
        C2<real> th, ph;
        if (A.scalar) {
            // the scalar analysis of f is the theta analysis of T_theta = s f (the
            // output stage divides by s again)
            const C2<real> f = gld(A.Tin + k);
            th = {w * s * f.x, w * s * f.y};
            ph = {0, 0};
        } else {
            const C2<real> t1 = gld(A.Tin + 3 * k), t2 = gld(A.Tin + 3 * k + 1), t3 = gld(A.Tin + 3 * k + 2);
            th.x = w * (z * (c * t1.x + sn * t2.x) - s * t3.x);
            th.y = w * (z * (c * t1.y + sn * t2.y) - s * t3.y);
            ph.x = w * (c * t2.x - sn * t1.x);
            ph.y = w * (c * t2.y - sn * t1.y);
        }
        buf[j] = th;
        buf[n2 + j] = ph;
    }
    __syncthreads();
    fft_lds<real, NT>(buf, n2, A.ffts, fdp, A.tw, wR, false);
    const double inv_s = 1.0 / rd.s;
    for (int m = threadIdx.x; m <= L; m += NT) {
        const int bp = m % n;
        const int bm = bp == 0 ? 0 : n - bp;
        double cph = 1.0, sph = 0.0;
        if (rd.phi0 != 0.0) sincos(m * rd.phi0, &sph, &cph);
        // +m: times e^{-i m phi0} / s ; -m: times e^{+i m phi0} / s
        const C2<real> fp = {(real)(cph * inv_s), (real)(-sph * inv_s)};
        const C2<real> fm = {(real)(cph * inv_s), (real)(sph * inv_s)};
        C2<real> *o = A.buf + ((size_t)m * NR + r) * 4;
        gst(o, cmul(buf[bp], fp));
        gst(o + 1, cmul(buf[n2 + bp], fp));
        gst(o + 2, cmul(buf[bm], fm));
        gst(o + 3, cmul(buf[n2 + bm], fm));
    }
}

template <typename real, int NT>
__device__ __forceinline__ void ring_adj_body(const RingArgs<real> &A, int r, unsigned char *smem_raw) {
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    const int L = A.L;
    const RingDesc rd = ld_uniform(A.rings + r);
    const FftDesc *fdp = A.ffts + rd.fft;
    const Seq<real> buf = {lds, ld_const(&fdp->lds_shift)};
    const int n = rd.nphi;
    const int n2 = seq_stride(fdp);
    const int p = rd.pair;
    const real sgn = rd.south ? (real)-1 : (real)1;
    const double inv_s = 1.0 / rd.s;
    for (int b = threadIdx.x; b < n; b += NT) {
        C2<real> hth = {0, 0}, hph = {0, 0};
        // orders m = b + k n (k >= 0) and m = b - k n (k >= 1) with |m| <= L
        for (int pass = 0; pass < 2; ++pass) {
            int m = pass == 0 ? b : b - n;
            while (pass == 0 ? (m <= L) : (m >= -L)) {
                const int am = m < 0 ? -m : m;
                const int slot = m < 0 ? 2 : 0;
                const C2<real> *e = A.buf + ((size_t)am * A.NP + p) * 8;
                const C2<real> eth = gld(e + slot), eph = gld(e + slot + 1);
                const C2<real> oth = gld(e + 4 + slot), oph = gld(e + 4 + slot + 1);
                double cph = 1.0, sph = 0.0;
                if (rd.phi0 != 0.0) sincos(m * rd.phi0, &sph, &cph);
                const C2<real> f = {(real)(cph * inv_s), (real)(sph * inv_s)};
                const C2<real> th = {eth.x + sgn * oth.x, eth.y + sgn * oth.y};
                const C2<real> ph = {eph.x + sgn * oph.x, eph.y + sgn * oph.y};
                const C2<real> a = cmul(th, f), c = cmul(ph, f);
                hth.x += a.x;
                hth.y += a.y;
                hph.x += c.x;
                hph.y += c.y;
                m = pass == 0 ? m + n : m - n;
            }
        }
        buf[b] = hth;
        buf[n2 + b] = hph;
    }
    __syncthreads();
    fft_lds<real, NT>(buf, n2, A.ffts, fdp, A.tw, wR, true);
    const double *twn = A.tw + 2 * ld_const(&fdp->tw_offset);
    for (int j = threadIdx.x; j < n; j += NT) {
        const double er = gld(twn + 2 * j), ei = -gld(twn + 2 * j + 1);
        const real c = (real)(rd.c0 * er - rd.s0 * ei);
        const real sn = (real)(rd.s0 * er + rd.c0 * ei);
        const real z = (real)rd.z, s = (real)rd.s;
        C2<real> th = buf[j], ph = buf[n2 + j];
        const int64_t k = rd.offset + j;
        if (A.weighted) {  // W S: the Hermitian transpose of the weighted analysis
            const real w = (real)(rd.uniform_w ? rd.w : gld(A.weights + k));
            th.x *= w; th.y *= w; ph.x *= w; ph.y *= w;
        }
        if (A.scalar) {  // f = s T_theta: the synthesised sum before the division by s
            gst(A.Tout + k, C2<real>{s * th.x, s * th.y});
            continue;
        }
        gst(A.Tout + 3 * k, C2<real>{z * c * th.x - sn * ph.x, z * c * th.y - sn * ph.y});
        gst(A.Tout + 3 * k + 1, C2<real>{z * sn * th.x + c * ph.x, z * sn * th.y + c * ph.y});
        gst(A.Tout + 3 * k + 2, C2<real>{-s * th.x, -s * th.y});
    }
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, 2) void k_ring_fwd(RingArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    ring_fwd_body<real, NT>(field_args(A, blockIdx.z), blockIdx.x, smem_raw);
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, 2) void k_ring_adj(RingArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    const int r = ring_of_block(A, blockIdx.x);
    if (r < 0) return;
    ring_adj_body<real, NT>(field_args(A, blockIdx.z), r, smem_raw);
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
// Legendre stages on MFMA.  Every wave owns a tile of 64 ring pairs (lane =
// pair) and advances the scaled recurrence itself, 16 degrees at a time; the
// 16 x 64 block of Q goes through a wave-private LDS tile (pair index
// XOR-swizzled with the row, conflict-free both ways) into the layout of a
// 16x16x4 MFMA (binary64 or binary32).
//
// forward  F[tri(m,l')][c] = c_{l'} sum_p Q_{l',m}(z_p) X_p[(l'+m)&1][c],
//          X_p[0] = RB[m][rN] + RB[m][rS], X_p[1] = RB[m][rN] - RB[m][rS]:
//          rows = 16 degrees, K = 4 pairs, columns = 8 of X[0] then 8 of X[1]
//          (each row keeps the half matching its parity).  The wave's X block
//          stays in the MFMA B registers for all degrees; the partial sums of
//          the waves of a workgroup (one per tile) are added through LDS.
// adjoint  PB[m][p][q][c] = sum_{l'+m = q mod 2} Q_{l',m}(z_p) FG[tri(m,l')][c]:
//          rows = 16 pairs, K = 4 degrees, columns = 8 for even l'+m then 8
//          for odd (B is zero in the other half).  No barriers: each wave
//          accumulates its 64 pairs over all degrees.
// ---------------------------------------------------------------------------
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <typename real>
struct Mfma;
template <>
struct Mfma<double> {
    typedef f64x4 acc_t;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    // lane l, register r holds row 4r + l/16, column l%16 (measured on gfx950)
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * r + (lane >> 4); }
};
template <>
struct Mfma<float> {
    typedef f32x4 acc_t;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    // lane l, register r holds row 4(l/16) + r, column l%16 (measured on gfx950)
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int kTileP = 64;   // ring pairs per wave
constexpr int kRowsB = 16;   // degrees per block
// Tile swizzles (64 banks of 4 bytes): the recurrence writes one row for 64
// consecutive pairs; the analysis MFMA reads, per 32 lanes, 16 rows x 2
// pairs; the synthesis MFMA reads 2 rows x 16 pairs.  XOR-ing the pair with
// 2 (row & 15) resp. 16 (row & 3) makes each of these access groups hit
// distinct banks.
struct SwzFwd {
    static __device__ __forceinline__ int at(int row, int pair) {
        return row * kTileP + (pair ^ ((row & 15) << 1));
    }
};
struct SwzAdj {
    static __device__ __forceinline__ int at(int row, int pair) {
        return row * kTileP + (pair ^ ((row & 3) << 4));
    }
};

// Advance the recurrence 16 degrees (lp0 .. lp0+15) for the wave's pairs and
// store Q into the wave's tile.  areg holds a'_{lp0 + lane} in lanes 0..15.
template <typename real, typename Swz>
__device__ __forceinline__ void recur16(real *qt, double areg, double z, double &q1, double &q2,
                                        int lane) {
#pragma unroll
    for (int s = 0; s < kRowsB; ++s) {
        const double az = readlane_f64(areg, s) * z;
        const double v = fma(az, q1, -q2);
        qt[Swz::at(s, lane)] = (real)v;
        q2 = q1;
        q1 = v;
    }
}

template <typename real>
struct LegFwdArgs {
    const real *RB;        // [(L+1)][NR][8]
    real *F;               // [tri][8]
    const PairDesc *pairs;
    const double *seeds;   // [(L+1)][NP] (the equator pair's seed)
    const LegStart *start; // [(L+1)][NP]
    const int *sblk;       // [(L+1)][NP]
    const double *pz;
    const double *aprime;  // [tri]
    const double *cscale;  // [tri]
    int L;
    int NP;                // all pairs (seed / pair table stride)
    int NPT;               // pairs handled by the tiles (the equator, if any, is pair NPT)
    int NR;
    int eq_ring;           // ring at z = 0 handled in closed form, or -1
    int64_t gstride;       // several workgroups per order m: group g writes its partial
                           // triangle at F + g gstride (summed afterwards); 0 otherwise
    int64_t zs_RB, zs_F;   // per-field strides (reals) of a launch over fields (blockIdx.z)
    __device__ LegFwdArgs at_field(int f) const {
        LegFwdArgs r = *this;
        if (f) {
            r.RB = RB + f * zs_RB;
            r.F = F + f * zs_F;
        }
        return r;
    }
};

// Valid half of a 16x16 analysis block in compact form: 128 values per wave.
template <typename real>
struct FwdCompact;
template <>
struct FwdCompact<double> {
    // lane l holds rows 4r + l/16; row parity (l/16)&1 must equal column half j/8
    static __device__ __forceinline__ bool lane_valid(int lane) {
        return ((lane & 15) >> 3) == ((lane >> 4) & 1);
    }
    static __device__ __forceinline__ bool valid(int lane, int r) { return lane_valid(lane); }
    static __device__ __forceinline__ int slot(int lane, int r) {
        return ((lane >> 4) * 8 + (lane & 7)) * 4 + r;
    }
    // inverse: compact slot -> (row, column)
    static __device__ __forceinline__ void rc(int o, int &row, int &col) {
        const int r = o & 3, c = o >> 2, k4 = c >> 3;
        row = 4 * r + k4;
        col = (k4 & 1) * 8 + (c & 7);
    }
};
template <>
struct FwdCompact<float> {
    // lane l holds rows 4(l/16) + r; row parity r&1 must equal column half j/8
    static __device__ __forceinline__ bool valid(int lane, int r) { return (r & 1) == ((lane & 15) >> 3); }
    static __device__ __forceinline__ int slot(int lane, int r) { return lane * 2 + (r >> 1); }
    static __device__ __forceinline__ void rc(int o, int &row, int &col) {
        const int lane = o >> 1, h = o & 1;
        const int j = lane & 15;
        const int r = 2 * h + (j >> 3);
        row = 4 * (lane >> 4) + r;
        col = j;
    }
};

// acc += bcast_k(g) * r, where bcast_k(g) is g of lane k of the lane's row of 16
// (binary64 DPP row broadcast).  The assembler form is the only one that puts
// the broadcast on the FMA itself.  A DPP read needs two wait states after a
// vector ALU write of its source, which the compiler does not see inside the
// assembler text: the first FMA of each group of eight waits them out.
template <int K, bool kWait>
__device__ __forceinline__ void fmac_row_bcast(double &acc, double g, double r) {
    if constexpr (kWait)
        asm("s_nop 1\n\tv_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "+v"(acc)
            : "v"(g), "v"(r), "n"(K));
    else
        asm("v_fmac_f64_dpp %0, %1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf"
            : "+v"(acc)
            : "v"(g), "v"(r), "n"(K));
}
// ---------------------------------------------------------------------------
// Binary64 Legendre stages on the four-block 4x4x4 MFMA (v_mfma_f64_4x4x4f64).
// On gfx950 lane l holds A[block (l>>2)&3][row l&3][k l>>4],
// B[block (l>>2)&3][k l>>4][column l&3] and D[block (l>>2)&3][row l>>4][column l&3]
// (measured).  Each block is a 4 x 4 product of one parity class, so no
// product is spent on the degrees of the other parity; per 16 degrees x 64
// ring pairs a wave issues 32 of them (the 16x16x4 form needs 16 of four
// times the cost, half of it on zeros).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double mma44(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// Analysis tile of 16 degrees x 64 pairs as [64 pairs][8 slots] of 16 bytes:
// slot q = 2i + pi of a pair holds its rows 4i + pi and 4i + pi + 2 (the two A
// operands one lane needs for the same parity block), so a lane reads both with
// one 16-byte access.  The slot is XOR-ed with (pair >> 1) & 7: the 16 lanes
// of a write (one slot of 16 consecutive pairs) then cover all 16 bank groups.
struct SwzQ2Fwd {
    static __device__ __forceinline__ int slot(int pair, int q) { return pair * 8 + (q ^ ((pair >> 1) & 7)); }
};

// First 16-degree block that the wave (wfirst) and the workgroup (gfirst) of an
// analysis must contract: earlier blocks hold zeros only.  A wave skips its
// blocks before wfirst; blocks before gfirst skip the reduction as well.  The
// waves exchange wfirst through xch (nw ints of the reduction buffer, free again
// after the second barrier).
__device__ __forceinline__ void first_blocks(int sblk, int nblk, int wave, int nw, int *xch, int &wfirst,
                                             int &gfirst) {
    wfirst = min(wave_min_blk(sblk) * (kStartBlock / kRowsB), nblk);
    if ((threadIdx.x & 63) == 0) xch[wave] = wfirst;
    __syncthreads();
    gfirst = nblk;
    for (int w = 0; w < nw; ++w) gfirst = min(gfirst, xch[w]);
    __syncthreads();
}

// The analyses run the recurrence on P_l = sigma_l Q_l, sigma_l = -1 for l = 2, 3
// (mod 4) and +1 otherwise: then P_l = P_{l-2} + a'_l (+-z) P_{l-1} (+z for odd l, -z
// for even l), one product and one FMA that accumulates into P_{l-2}'s register, and
// sigma_l is applied to the reduced sums.  a'_{l'} comes lane-wise (lane j holds
// a'_{lp0 + (j & 15)}, every row of 16 lanes alike) from a vector load issued one block
// ahead, and reaches the FMA by row broadcast (a scalar load would be waited for with
// the LDS traffic).
__device__ __forceinline__ double sigma_state(int l, double q) { return (l & 2) ? -q : q; }

// Sixteen steps from degree lp0: step s: P <- P_{l-2} + a'_{lp0+s} (z_s P_{l-1}), with
// z_s = z_even for even s and -z_even for odd s (the sign is a source modifier of the
// product); put(s, P_{lp0+s}) stores the value.
template <int S, typename Put>
__device__ __forceinline__ void fwd_steps(double acur, double z_even, double &p1, double &p2, Put &&put) {
    if constexpr (S < kRowsB) {
        const double t = ((S & 1) ? -z_even : z_even) * p1;
        fmac_row_bcast<S, S == 0>(p2, acur, t);  // p2 is now P_{lp0+S}
        put(S, p2);
        fwd_steps<S + 1>(acur, z_even, p2, p1, put);
    }
}

// Analysis, binary64: workgroup = order m, waves = tiles of 64 ring pairs.
// Instruction (row group r, pair step g): block b = (parity pi = b>>1, column
// half h = b&1), rows = degrees lp0 + 4i + 2r + pi, K = pairs 4g + k,
// columns 4h + j of X[pi] (X[0] = N + S, X[1] = N - S).
__device__ __forceinline__ void leg_fwd_f64q_body(const LegFwdArgs<double> &A, int m, int group,
                                                  unsigned char *smem_raw) {
    const int L = A.L, NP = A.NP, NPT = A.NPT, NR = A.NR;
    const int nw = blockDim.x >> 6;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tile = group * nw + wave;
    double2 *qt = reinterpret_cast<double2 *>(smem_raw) + wave * (kRowsB / 2) * kTileP;
    double *red = reinterpret_cast<double *>(smem_raw) + nw * kRowsB * kTileP;  // [2][nw][128]
    const int64_t t0 = tri_offset(L, m);
    const double *RBm = A.RB + (size_t)m * NR * 8;
    const int b = (lane >> 2) & 3, pi = b >> 1, h = b & 1, j = lane & 3, k = lane >> 4, i = lane & 3;
    const int col = 4 * h + j;
    double bv[16];
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        const int pp = tile * kTileP + 4 * g + k;
        double v = 0.0;
        if (pp < NPT) {
            const PairDesc pd = ld_pair(A.pairs + pp);
            const double xn = gld(RBm + ((size_t)pd.rn * 8 + col));
            const double xs = pd.rs >= 0 ? gld(RBm + ((size_t)pd.rs * 8 + col)) : 0.0;
            v = pi == 0 ? xn + xs : xn - xs;
        }
        bv[g] = v;
    }
    const int p = tile * kTileP + lane;
    const bool valid = p < NPT;
    const double z = valid ? gld(A.pz + (p)) : 0.0;
    const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * NP + p, valid);
    double q1 = 0.0, q2 = 0.0;
    const double seq = A.eq_ring >= 0 ? gld(A.seeds + ((size_t)m * NP + NPT)) : 0.0;
    const double *xeq = A.eq_ring >= 0 ? RBm + (size_t)A.eq_ring * 8 : nullptr;
    const double *ap = A.aprime + t0 - m;  // indexed by l'
    const int nl = L + 2 - m;
    const int nblk = (nl + kRowsB - 1) / kRowsB;
    int wfirst, gfirst;
    first_blocks(S.blk, nblk, wave, nw, reinterpret_cast<int *>(red), wfirst, gfirst);
    // recurrence on P (fwd_steps)
    const double z_even = (m & 1) ? z : -z;  // factor of the even steps s (degree m + 16 blk + s)
    // a' of block b, lane-wise, loaded without a branch (the index is clamped into the
    // order's row, and entries past L+1 are zeroed where they are used)
    auto load_a = [&](int b) -> double { return gld(ap + min(m + b * kRowsB + (lane & 15), L + 1)); };
    // output slots o = threadIdx.x + 64 u (u < 2) of the reduction
    auto out_slot = [&](int o, int &lp_off, int &c) {
        const int r = o >> 6, ln = o & 63;
        const int bb = (ln >> 2) & 3;
        lp_off = 4 * (ln >> 4) + 2 * r + (bb >> 1);
        c = 4 * (bb & 1) + (ln & 3);
    };
    const int nout = blockDim.x == 64 ? 2 : 1;  // slots per thread (threads >= 128 have none)
    double xq[2] = {0.0, 0.0};                   // the equator ring's value of each slot's column
    if (xeq)
        for (int u = 0; u < nout; ++u) {
            int so, c;
            out_slot((threadIdx.x + u * 64) & 127, so, c);
            xq[u] = gld(xeq + c);
        }
    // One 16-degree block; araw holds its a' (loaded one block earlier), anext receives
    // the next block's.
    auto block = [&](int blk, double araw, double &anext) {
        const int lp0 = m + blk * kRowsB;
        // c_{l'} of the thread's slots, loaded here and used after the reduction
        double csc[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int so, c;
            out_slot((threadIdx.x + u * 64) & 127, so, c);
            csc[u] = gld(A.cscale + (t0 + min(lp0 + so, L + 1) - m));
        }
        anext = load_a(max(blk + 1, wfirst));
        double acc0 = 0.0, acc1 = 0.0;
        if (blk >= wfirst) {
            if (blk * kRowsB == kStartBlock * S.blk) {  // the lane's start state, as P
                q1 = sigma_state(lp0 - 1, S.q1);
                q2 = sigma_state(lp0 - 2, S.q2);
            }
            const double acur = lp0 + (lane & 15) <= L + 1 ? araw : 0.0;
            // row 4i + pi + 2r goes to half r of the lane's LDS slot 2i + pi (eight-byte
            // writes: packing two rows for one sixteen-byte write cost register moves)
            double *qd = reinterpret_cast<double *>(qt);
            fwd_steps<0>(acur, z_even, q1, q2, [&](int st, double v) {
                qd[2 * SwzQ2Fwd::slot(lane, 2 * (st >> 2) + (st & 1)) + ((st >> 1) & 1)] = v;
            });
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int g = 0; g < 16; ++g) {
                const double2 av = qt[SwzQ2Fwd::slot(4 * g + k, 2 * i + pi)];
                const double a0 = av.x, a1 = av.y;
                acc0 = mma44(a0, bv[g], acc0);
                acc1 = mma44(a1, bv[g], acc1);
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (blk >= gfirst) {
            // D lane l: row (l >> 4) of block b -> degree offset 4(l>>4) + 2r + pi, column col
            double *rw = red + ((blk & 1) * nw + wave) * 128;
            rw[lane] = acc0;
            rw[64 + lane] = acc1;
            __syncthreads();
        }
        // the next block's a' counts as defined here, after this block's products: the
        // copy that passes it to the next block cannot be moved up to wait for the load
        // just issued, and the wait here does not include the stores below
        asm volatile("" : "+v"(anext)::"memory");
        // sum over waves and store; the buffer of block blk is rewritten at blk + 2,
        // after the next barrier, so one barrier per block suffices
        if (threadIdx.x >= 128) return;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u >= nout) break;
            const int o = threadIdx.x + u * 64;
            int so, c;
            out_slot(o, so, c);
            const int lp = lp0 + so;
            if (lp <= L + 1) {
                double sum = 0.0;
                if (blk >= gfirst) {
                    const double *rb = red + (blk & 1) * nw * 128;
                    for (int w = 0; w < nw; ++w) sum += rb[w * 128 + o];
                    if (lp & 2) sum = -sum;  // sigma_{l'}
                }
                const int64_t ti = t0 + lp - m;
                if (xeq && (so & 1) == 0 && group == 0) {
                    const int kk = (lp - m) >> 1;
                    sum += ((kk & 1) ? -seq : seq) * xq[u];
                }
                gst(A.F + (group * A.gstride + ti * 8 + c), csc[u] * sum);
            }
        }
    };
    double an = load_a(wfirst);
    asm volatile("" : "+v"(an)::"memory");  // waited for here, once, not in the loop
    for (int blk = 0; blk < nblk; ++blk) {
        const double araw = an;
        block(blk, araw, an);
    }
}

// One workgroup: order m, tiles [group nw, group nw + nw) of ring pairs.
template <typename real>
__device__ __forceinline__ void leg_fwd_body(const LegFwdArgs<real> &A, int m, int group,
                                             unsigned char *smem_raw) {
    typedef typename Mfma<real>::acc_t acc_t;
    const int L = A.L, NP = A.NP, NPT = A.NPT, NR = A.NR;
    const int nw = blockDim.x >> 6;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tile = group * nw + wave;
    real *qt = reinterpret_cast<real *>(smem_raw) + wave * kRowsB * kTileP;     // private tile
    real *red = reinterpret_cast<real *>(smem_raw) + nw * kRowsB * kTileP;      // [2][nw][128]
    const int64_t t0 = tri_offset(L, m);
    const real *RBm = A.RB + (size_t)m * NR * 8;

    // the tile's folded ring data in MFMA B layout: lane (j + 16k) holds
    // X[pair 4g + k][column j] for g = 0..15
    const int j = lane & 15, k = lane >> 4;
    real bv[16];
#pragma unroll
    for (int g = 0; g < 16; ++g) {
        const int pp = tile * kTileP + 4 * g + k;
        real v = 0;
        if (pp < NPT) {
            const PairDesc pd = ld_pair(A.pairs + pp);
            const real xn = gld(RBm + ((size_t)pd.rn * 8 + (j & 7)));
            const real xs = pd.rs >= 0 ? gld(RBm + ((size_t)pd.rs * 8 + (j & 7))) : (real)0;
            v = j < 8 ? xn + xs : xn - xs;
        }
        bv[g] = v;
    }
    const int p = tile * kTileP + lane;
    const bool valid = p < NPT;
    const double z = valid ? gld(A.pz + (p)) : 0.0;
    const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * NP + p, valid);
    double q1 = 0.0, q2 = 0.0;
    // equator ring (z = 0): Q_{m+2k} = (-1)^k Lambda_{m,m}(0), odd degrees vanish
    const double seq = A.eq_ring >= 0 ? gld(A.seeds + ((size_t)m * NP + NPT)) : 0.0;
    const real *xeq = A.eq_ring >= 0 ? RBm + (size_t)A.eq_ring * 8 : nullptr;
    const int nl = L + 2 - m;
    const int nblk = (nl + kRowsB - 1) / kRowsB;
    int wfirst, gfirst;
    first_blocks(S.blk, nblk, wave, nw, reinterpret_cast<int *>(red), wfirst, gfirst);
    // recurrence on P (fwd_steps); a' of block b, lane-wise, loaded one block ahead
    // without a branch (index clamped into the order's row, zeroed where used)
    const double z_even = (m & 1) ? z : -z;
    const double *ap = A.aprime + t0 - m;  // indexed by l'
    auto load_a = [&](int b) -> double { return gld(ap + min(m + b * kRowsB + (lane & 15), L + 1)); };
    const int nout = blockDim.x == 64 ? 2 : 1;  // output slots per thread (threads >= 128 have none)
    real xq[2] = {0, 0};                         // the equator ring's value of each slot's column
    if (xeq)
        for (int u = 0; u < nout; ++u) {
            int row, col;
            FwdCompact<real>::rc((threadIdx.x + u * 64) & 127, row, col);
            xq[u] = gld(xeq + (col & 7));
        }
    // One 16-degree block; araw holds its a' (loaded one block earlier), anext receives
    // the next block's.
    auto block = [&](int blk, double araw, double &anext) {
        const int lp0 = m + blk * kRowsB;
        double csc[2];  // c_{l'} of the thread's slots, used after the reduction
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int row, col;
            FwdCompact<real>::rc((threadIdx.x + u * 64) & 127, row, col);
            csc[u] = gld(A.cscale + (t0 + min(lp0 + row, L + 1) - m));
        }
        anext = load_a(max(blk + 1, wfirst));
        acc_t acc0 = {0, 0, 0, 0}, acc1 = {0, 0, 0, 0};
        if (blk >= wfirst) {
            if (blk * kRowsB == kStartBlock * S.blk) {  // the lane's start state, as P
                q1 = sigma_state(lp0 - 1, S.q1);
                q2 = sigma_state(lp0 - 2, S.q2);
            }
            const double acur = lp0 + (lane & 15) <= L + 1 ? araw : 0.0;
            fwd_steps<0>(acur, z_even, q1, q2, [&](int st, double v) { qt[SwzFwd::at(st, lane)] = (real)v; });
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int g = 0; g < 16; g += 2) {
                const real a0 = qt[SwzFwd::at(j, 4 * g + k)];
                const real a1 = qt[SwzFwd::at(j, 4 * (g + 1) + k)];
                acc0 = Mfma<real>::mma(a0, bv[g], acc0);
                acc1 = Mfma<real>::mma(a1, bv[g + 1], acc1);
            }
        }
        if (blk >= gfirst) {
            // valid half of this wave's partial block -> red[blk & 1][wave]
            real *rw = red + ((blk & 1) * nw + wave) * 128;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (FwdCompact<real>::valid(lane, r)) rw[FwdCompact<real>::slot(lane, r)] = acc0[r] + acc1[r];
            __syncthreads();
        }
        asm volatile("" : "+v"(anext)::"memory");  // as in leg_fwd_f64q_body
        // sum over waves and store; the buffer of block blk is rewritten at
        // blk + 2, after the next barrier, so one barrier per block suffices
        if (threadIdx.x >= 128) return;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u >= nout) break;
            const int o = threadIdx.x + u * 64;
            int row, col;
            FwdCompact<real>::rc(o, row, col);
            const int lp = lp0 + row;
            if (lp <= L + 1) {
                real sum = 0;
                if (blk >= gfirst) {
                    const real *rb = red + (blk & 1) * nw * 128;
                    for (int w = 0; w < nw; ++w) sum += rb[w * 128 + o];
                    if (lp & 2) sum = -sum;  // sigma_{l'}
                }
                const int64_t ti = t0 + lp - m;
                if (xeq && col < 8 && group == 0) {
                    // even-parity row: the equator adds Q_{lp}(0) X_eq
                    const int kk = (lp - m) >> 1;
                    const double qe = (kk & 1) ? -seq : seq;
                    sum += (real)qe * xq[u];
                }
                gst(A.F + (group * A.gstride + ti * 8 + (col & 7)), (real)csc[u] * sum);
            }
        }
    };
    double an = load_a(wfirst);
    asm volatile("" : "+v"(an)::"memory");  // waited for here, once, not in the loop
    for (int blk = 0; blk < nblk; ++blk) {
        const double araw = an;
        block(blk, araw, an);
    }
}

// F[i] = sum_g part[g n + i], g in increasing order (analysis split over several
// workgroups per order; deterministic, no atomics)
template <typename real>
__global__ __launch_bounds__(256) void k_sum_groups(const real *__restrict__ part, real *__restrict__ F,
                                                    int64_t n, int groups, int64_t zs_part, int64_t zs_F) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    part += blockIdx.z * zs_part;  // field of a launch over fields
    F += blockIdx.z * zs_F;
    real acc = part[i];
    for (int g = 1; g < groups; ++g) acc += part[(int64_t)g * n + i];
    F[i] = acc;
}

template <typename real>
__global__ __launch_bounds__(1024) void k_leg_fwd_mfma(LegFwdArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    if constexpr (sizeof(real) == 8)
        leg_fwd_f64q_body(field_args(A, blockIdx.z), blockIdx.x, blockIdx.y, smem_raw);
    else
        leg_fwd_body(field_args(A, blockIdx.z), blockIdx.x, blockIdx.y, smem_raw);
}

template <typename real>
struct LegArgs {
    const real *FG;       // [tri][8]
    const double *FG64;   // g as binary64 rows, [tri][8]: FG itself on the binary64 path, the
                          // plan's binary64 triangle (written by the prep) on the binary32 paths
    real *PB;             // [(L+1)][NP][16]
    const double *seeds;  // the equator pair's seed
    const LegStart *start;
    const int *sblk;
    const double *pz;
    const double *aprime;
    int L;
    int NP;
    int NPT;              // pairs handled by the tiles (the equator, if any, is pair NPT)
    int64_t zs_FG, zs_FG64, zs_PB;  // per-field strides (elements) of a launch over fields
    __device__ LegArgs at_field(int f) const {
        LegArgs r = *this;
        if (f) {
            r.FG = FG + f * zs_FG;
            r.FG64 = FG64 + f * zs_FG64;
            r.PB = PB + f * zs_PB;
        }
        return r;
    }
};

// Ring pairs of the split-bf16 syntheses that run in binary64 (the polar unit).
// The spin-frame synthesis divides by sin(theta) a sum whose terms near the
// poles are up to ~1/sin(theta) larger than the sum, so a rounding of the
// Legendre values or of g becomes eps / sin(theta) at that ring; over the L + 1
// rings of a Gauss-Legendre grid the squared error of ring r falls off as 1/r^2,
// and the 32 pairs nearest the poles carry all but a few percent of it.
constexpr int kPolarPairs = 32;

// Synthesis on the vector unit, binary64.  Each lane carries PPL ring pairs
// through a range of degrees, and each degree costs, per pair, the recurrence
// step and eight FMAs (the four complex columns of g, into the even or the odd
// sum).  a'_{l'} and g[l'] are the same for the whole wave: kAdjChunk degrees at a
// time are staged in the wave's LDS buffer with coalesced loads issued one chunk
// ahead, and every FMA takes its g value by DPP row broadcast.  On gfx950 the
// binary64 vector FMA rate equals the binary64 matrix-core rate and the
// binary32 vector rate (without packed binary32), so this form serves the
// binary32 path too (g then comes from the plan's binary64 triangle FG64 and only
// the sums are stored in binary32), and it needs neither the LDS staging of the
// Legendre values nor products on zero parity blocks.
constexpr int kAdjChunk = 32;  // degrees per LDS buffer (two buffers)
static_assert(kAdjChunk == kStartBlock, "a chunk is one start block");
static_assert(kStartBlock % kRowsB == 0, "start blocks are whole 16-degree blocks");
struct alignas(16) AdjRow {
    double g[8];  // g[l'] (theta, phi) x (+m, -m), complex
    double a;     // a'_{l'}
};

template <int K0, int C = 0>
__device__ __forceinline__ void fmac_row_bcast8(double (&S)[8], double g, double r) {
    fmac_row_bcast<K0 + C, C == 0>(S[C], g, r);
    if constexpr (C + 1 < 8) fmac_row_bcast8<K0, C + 1>(S, g, r);
}

template <int K0, int N, int C = 0>
__device__ __forceinline__ void fmac_row_bcastn(double (&S)[N], double g, double r) {
    fmac_row_bcast<K0 + C, C == 0>(S[C], g, r);
    if constexpr (C + 1 < N) fmac_row_bcastn<K0, N, C + 1>(S, g, r);
}

// One workgroup of order m, all its waves staging g and a' together (kAdjChunk
// rows at a time, two buffers, coalesced loads one chunk ahead); the calling
// wave carries PPL pairs per lane, pw + PPL lane + u (u < PPL, pair < pend), and
// the g columns [C0, C0 + NC) through the degrees l' = m .. L+1, into even (E)
// and odd (O) sums.  FG: binary64 rows of the triangle (row l' of order m at
// FG + 8 (tri(m) - m + l')).  eqw: the wave also forms the equator pair (index
// NPT): at z = 0 the scaled recurrence gives Q_{m+2k} = (-1)^k Q_m and
// Q_{m+2k+1} = 0, so its even sum is Lambda_{m,m}(0) sum_k (-1)^k g[m + 2k] and
// its odd sum 0 (lanes = column (lane & 7) x row group (lane >> 3)).
template <typename out, int PPL, int C0, int NC>
__device__ __forceinline__ void adj_valu_block(const LegArgs<out> &A, const double *__restrict__ FG, int m, int pw,
                                               int pend, bool eqw, AdjRow *buf) {
    const int nt = blockDim.x, lane = threadIdx.x & 63;
    const int L = A.L, NP = A.NP, NPT = A.NPT, Lp1 = L + 1;
    const int64_t t0 = tri_offset(L, m);
    const double *g = FG + (t0 - m) * 8;  // row l' at g + 8 l'
    const double *ap = A.aprime + t0 - m;
    static_assert(PPL == 1 || PPL == 2, "one or two pairs per lane");
    // start chunks and states wait in LDS (registers are the limit of the degree loop)
    __shared__ double2 s_state[4][PPL][kTileP];
    __shared__ int s_blk[4][PPL][kTileP];
    const int wave = threadIdx.x >> 6;
    double z[PPL], q1[PPL], q2[PPL];
    double E[PPL][NC], O[PPL][NC];
    int first = kStartNever;  // first chunk in which the wave's pairs are not all zero
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        // the lane's pairs are adjacent, so that both start near the same chunk
        const int p = pw + PPL * lane + u;
        const bool valid = p < pend;
        z[u] = valid ? gld(A.pz + (p)) : 0.0;
        q1[u] = q2[u] = 0.0;
        const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * NP + p, valid);
        s_state[wave][u][lane] = double2{S.q1, S.q2};
        s_blk[wave][u][lane] = S.blk;
        first = min(first, S.blk);
        // re-define the loaded values here, so that the degree loop below does not
        // read registers filled by loads (the wait inserted for those would also
        // wait for the staging loads of the next chunk)
        asm volatile("" : "+v"(z[u]));
#pragma unroll
        for (int c = 0; c < NC; ++c) E[u][c] = O[u][c] = 0.0;
    }
    first = wave_min_blk(first);
    const int nl = Lp1 - m + 1;
    const int nchunk = (nl + kAdjChunk - 1) / kAdjChunk;
    // staging: item i < 8 kAdjChunk is g value (i & 7) of row i >> 3; thread t < kAdjChunk
    // also takes a' of row t (workgroups of 64 threads take four g items each)
    constexpr int kG = 8 * kAdjChunk / 64;
    double sg[kG];
    double sa = 0.0;
    auto stage_load = [&](int k) {
        const int lp0 = m + k * kAdjChunk;
#pragma unroll
        for (int r = 0; r < kG; ++r) {
            const int i = threadIdx.x + r * nt;
            const int lp = lp0 + (i >> 3);
            sg[r] = (i < 8 * kAdjChunk && lp <= Lp1) ? gld(g + ((int64_t)lp * 8 + (i & 7))) : 0.0;
        }
        const int la = lp0 + (int)threadIdx.x;
        sa = ((int)threadIdx.x < kAdjChunk && la <= Lp1) ? gld(ap + (la)) : 0.0;
    };
    auto stage_store = [&](int k) {
        AdjRow *b = buf + (k & 1) * kAdjChunk;
#pragma unroll
        for (int r = 0; r < kG; ++r) {
            const int i = threadIdx.x + r * nt;
            if (i < 8 * kAdjChunk) b[i >> 3].g[i & 7] = sg[r];
        }
        if ((int)threadIdx.x < kAdjChunk) b[threadIdx.x].a = sa;
    };
    double eacc = 0;
    stage_load(0);
    stage_store(0);
    __syncthreads();
    for (int k = 0; k < nchunk; ++k) {
        if (k + 1 < nchunk) stage_load(k + 1);  // in flight while chunk k is used
        const AdjRow *rows = buf + (k & 1) * kAdjChunk;
        const int nd = min(kAdjChunk, nl - k * kAdjChunk);
        if (eqw) {
#pragma unroll
            for (int e = 0; e < kAdjChunk / 16; ++e) {
                const int d = 2 * ((lane >> 3) + 8 * e);  // even row of the chunk
                if (d < nd) {
                    const double v = rows[d].g[lane & 7];
                    eacc += (((k * kAdjChunk + d) >> 1) & 1) ? -v : v;
                }
            }
        }
        // the chunk starts an even number of degrees after m: row d has the parity of d;
        // lanes 0-7 of every row of 16 hold g of degree d, lanes 8-15 that of d + 1, and
        // each FMA takes its value by row broadcast.  Chunks before the wave's first
        // start hold zeros only.
        if (k >= first) {
#pragma unroll
            for (int u = 0; u < PPL; ++u)
                if (s_blk[wave][u][lane] == k) {
                    const double2 v = s_state[wave][u][lane];
                    q1[u] = v.x;
                    q2[u] = v.y;
                }
            const int sel = (lane >> 3) & 1, col = lane & 7;
            double Gn = rows[sel].g[col], a0n = rows[0].a, a1n = rows[1].a;
            for (int d = 0; d < nd; d += 2) {
                const double G = Gn, a0 = a0n, a1 = a1n;
                // the next step's operands, read while this step computes
                const int dn = d + 2 < kAdjChunk ? d + 2 : d;
                Gn = rows[dn + sel].g[col];
                a0n = rows[dn].a;
                a1n = rows[dn + 1].a;
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const double v = fma(a0 * z[u], q1[u], -q2[u]);
                    fmac_row_bcastn<C0, NC>(E[u], G, v);
                    q2[u] = q1[u];
                    q1[u] = v;
                }
                // the odd step runs also past the last degree (nd odd): that row was
                // staged with g = 0 and a' = 0, so it adds zeros, and without the branch
                // the two steps need no register moves
#pragma unroll
                for (int u = 0; u < PPL; ++u) {
                    const double v = fma(a1 * z[u], q1[u], -q2[u]);
                    fmac_row_bcastn<8 + C0, NC>(O[u], G, v);
                    q2[u] = q1[u];
                    q1[u] = v;
                }
            }
        }
        if (k + 1 < nchunk) stage_store(k + 1);
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < PPL; ++u) {
        const int p = pw + PPL * lane + u;
        if (p < pend) {
            out *o = A.PB + ((size_t)m * NP + p) * 16;
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                gst(o + (C0 + c), (out)E[u][c]);
                gst(o + (8 + C0 + c), (out)O[u][c]);
            }
        }
    }
    if (eqw) {
        // the eight row groups of each column (lanes c, c + 8, ..., c + 56)
        eacc += __shfl_xor(eacc, 8);
        eacc += __shfl_xor(eacc, 16);
        eacc += __shfl_xor(eacc, 32);
        if (lane < 8) {
            out *o = A.PB + ((size_t)m * NP + NPT) * 16;
            gst(o + (lane), (out)(gld(A.seeds + ((size_t)m * NP + NPT)) * eacc));
            gst(o + (8 + lane), (out)0);
        }
    }
}

// One wave of the split-bf16 paths' binary32 tile: pairs [p0, p0 + 64) of order
// m over the degrees below lB, each lane's pair from its start S, on the
// binary32 16x16x4 MFMA through the wave's Q tile qt.  Each 16-degree block is summed apart and added to the
// totals (two-level summation).  acc[b]: lane l, register r -> pair
// p0 + 16 b + Mfma<float>::row(l, r), column l % 16 (8 even-sum columns, then 8 odd).
__device__ __forceinline__ void adj_tile_f32(const LegArgs<float> &A, int m, int p0, int lB, double z,
                                             const LaneStart &S, f32x4 (&acc)[4], float *qt) {
    const int lane = threadIdx.x & 63;
    const int L = A.L;
    const int64_t t0 = tri_offset(L, m);
    const float *g = A.FG + (t0 - m) * 8;  // indexed by l'
    const int j = lane & 15, k = lane >> 4;
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = f32x4{0, 0, 0, 0};
    // degrees before the wave's first start block hold zeros only
    const int lA = min(m + kStartBlock * wave_min_blk(S.blk), lB);
    double q1 = 0.0, q2 = 0.0;
    const int nblk = (lB - lA + kRowsB - 1) / kRowsB;
    for (int blk = 0; blk < nblk; ++blk) {
        const int lp0 = lA + blk * kRowsB;
        take_start(S, lp0 - m, q1, q2);
        const int la = lp0 + (lane & 15);
        const double areg = la < lB ? gld(A.aprime + (t0 + la - m)) : 0.0;
        // B operands: lane (j + 16k) holds g[row 4gg + k][j & 7] if the row's
        // parity matches the column half (row parity == (lp - m) & 1 == k & 1)
        float bv[4];
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            const int lp = lp0 + 4 * gg + k;
            bv[gg] = (lp < lB && (j >> 3) == (k & 1)) ? gld(g + ((int64_t)lp * 8 + (j & 7))) : 0.f;
        }
        recur16<float, SwzAdj>(qt, areg, z, q1, q2, lane);
        f32x4 ab[4];
#pragma unroll
        for (int b = 0; b < 4; ++b) ab[b] = f32x4{0, 0, 0, 0};
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                // A: lane (i + 16k) holds Q[row 4gg + k][pair 16b + i]
                const float a = qt[SwzAdj::at(4 * gg + k, 16 * b + j)];
                ab[b] = Mfma<float>::mma(a, bv[gg], ab[b]);
            }
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[b] += ab[b];
    }
}

// ---------------------------------------------------------------------------
// Equator ring (z = 0) of the synthesis: Q_{m+2k}(0) = (-1)^k Lambda_{m,m}(0)
// and odd degrees vanish, so PB[m][eq][0][c] = Lambda_{m,m}(0) sum_k (-1)^k
// FG[tri(m, m+2k)][c] and PB[m][eq][1] = 0.  One wave per order m.
// ---------------------------------------------------------------------------
template <typename real>
__device__ __forceinline__ void equator_adj_body(const LegArgs<real> &A, int m) {
    // 256 threads: column c = t & 7 of row groups t >> 3 (32 of them), four rows in
    // flight per thread; the 32 partial sums of a column meet in the wave (shuffles)
    // and across the four waves (LDS)
    __shared__ real part[4][8];
    const int L = A.L, NP = A.NP;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t t0 = tri_offset(L, m);
    const real *g = A.FG + t0 * 8;  // row l' = m + i
    const int c = t & 7, rg = t >> 3;
    const int nk = (L + 1 - m) / 2 + 1;  // even rows 2 kk <= L + 1 - m
    real acc = 0;
#pragma unroll 4
    for (int kk = rg; kk < nk; kk += 32) {
        const real v = gld(g + ((int64_t)(2 * kk) * 8 + c));
        acc += (kk & 1) ? -v : v;
    }
    acc += __shfl_xor(acc, 8);
    acc += __shfl_xor(acc, 16);
    acc += __shfl_xor(acc, 32);
    if (lane < 8) part[wave][lane] = acc;
    __syncthreads();
    if (t < 8) {
        const real sum = (part[0][t] + part[1][t]) + (part[2][t] + part[3][t]);
        real *o = A.PB + ((size_t)m * NP + A.NPT) * 16;
        gst(o + (t), (real)gld(A.seeds + ((size_t)m * NP + A.NPT)) * sum);
        gst(o + (8 + t), (real)0);
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_equator_adj(LegArgs<real> A) {
    equator_adj_body(field_args(A, blockIdx.z), blockIdx.x);
}

// ---------------------------------------------------------------------------
// BF16x3 and BF16x6 Legendre stages.  A binary32 operand x is split into bf16
// parts by repeated rounding, x = p0 + p1 (+ p2) + r with p0 = bf16(x),
// p1 = bf16(x - p0), p2 = bf16(x - p0 - p1) (each difference exact in binary32).
// BF16x3 keeps two parts (|r| <= 2^-17 |x|) and forms a product as
// p0 p0' + p0 p1' + p1 p0'; the dropped terms are below 2^-16 relative.
// BF16x6 keeps three parts (|r| <= 2^-26 |x|) and adds p0 p2' + p1 p1' + p2 p0';
// the dropped terms are below 2^-24 relative, binary32's own rounding.  All
// products run on the 16x16x32 bf16 MFMA with binary32 accumulation.  The
// Legendre recurrence, its seeds and its scaling stay binary64.
// Operand layouts of v_mfma_f32_16x16x32_bf16 (measured on gfx950): lane l
// holds A[row l%16][k 8(l/16)+t] and B[k 8(l/16)+t][col l%16], t = 0..7, and
// D register r of lane l is [row 4(l/16)+r][col l%16].
// ---------------------------------------------------------------------------
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

// NP = products per product: 3 (BF16x3, two parts) or 6 (BF16x6, three parts)
template <int NP>
struct Bf16 {
    static_assert(NP == 3 || NP == 6, "BF16x3 or BF16x6");
    static constexpr int kParts = NP == 6 ? 3 : 2;
    static constexpr int kAdjLdsPerWave = kParts * kTileP * 32 * 2;  // split Q tiles of the synthesis
};
template <int NP>
struct Split8 {
    bf16x8_t p[Bf16<NP>::kParts];
};

// split of two values into NS parts, each part packed as two bf16 in 32 bits
template <int NS>
__device__ __forceinline__ void split2(float a, float b, uint32_t (&o)[NS]) {
    float ra = a, rb = b;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const f32x2_t v = {ra, rb};
        const uint32_t h = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2_t));
        o[k] = h;
        ra -= __builtin_bit_cast(float, h << 16);
        rb -= __builtin_bit_cast(float, h & 0xffff0000u);
    }
}

template <int NP>
__device__ __forceinline__ Split8<NP> split8(const float (&v)[8]) {
    constexpr int NS = Bf16<NP>::kParts;
    u32x4_t w[NS];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        uint32_t o[NS];
        split2<NS>(v[2 * i], v[2 * i + 1], o);
#pragma unroll
        for (int k = 0; k < NS; ++k) w[k][i] = o[k];
    }
    Split8<NP> r;
#pragma unroll
    for (int k = 0; k < NS; ++k) r.p[k] = __builtin_bit_cast(bf16x8_t, w[k]);
    return r;
}

// the leading part product into hi and the correction products into lo: lo stays
// ~2^-8 of hi, so its rounding is negligible and hi sees one rounding per call
template <int NP>
__device__ __forceinline__ void mma_split2(const Split8<NP> &a, const Split8<NP> &b, f32x4 &hi, f32x4 &lo) {
    hi = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[0], hi, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[1], lo, 0, 0, 0);
    lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[0], lo, 0, 0, 0);
    if constexpr (NP == 6) {
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[2], lo, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[1], lo, 0, 0, 0);
        lo = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[2], b.p[0], lo, 0, 0, 0);
    }
}

// the part products p_i p_j' with i + j < parts, largest first
template <int NP>
__device__ __forceinline__ f32x4 mma_split(const Split8<NP> &a, const Split8<NP> &b, f32x4 acc) {
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[0], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[1], acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[0], acc, 0, 0, 0);
    if constexpr (NP == 6) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[0], b.p[2], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[1], b.p[1], acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.p[2], b.p[0], acc, 0, 0, 0);
    }
    return acc;
}


// Q tile of the analysis: [16 degrees][64 pairs] binary32 whose groups of 8
// pairs are XOR-ed with the row, so that the 8 consecutive pairs one lane
// reads stay contiguous and the 16 rows read together start in different banks.
struct SwzFwd8 {
    static __device__ __forceinline__ int at(int row, int pair) {
        return row * kTileP + ((((pair >> 3) ^ (row & 7)) << 3) | (pair & 7));
    }
};

// Analysis, BF16x3/BF16x6: as k_leg_fwd_mfma<float> (same grid, reduction and
// epilogue) with the wave's 64-pair block contracted as two K = 32 chunks.
template <int NPROD>
__device__ __forceinline__ void leg_fwd_bf16_body(const LegFwdArgs<float> &A, int m, int group,
                                                  unsigned char *smem_raw) {
    const int L = A.L, NP = A.NP, NPT = A.NPT, NR = A.NR;
    const int nw = blockDim.x >> 6;
    const int wave = uniform_int(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int tile = group * nw + wave;
    float *qt = reinterpret_cast<float *>(smem_raw) + wave * kRowsB * kTileP;
    float *red = reinterpret_cast<float *>(smem_raw) + nw * kRowsB * kTileP;  // [2][nw][128]
    const int64_t t0 = tri_offset(L, m);
    const float *RBm = A.RB + (size_t)m * NR * 8;

    // B: lane (j + 16kg) holds X[pair 32c + 8kg + t][column j] of chunk c
    const int j = lane & 15, kg = lane >> 4;
    Split8<NPROD> bx[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        float v[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int pp = tile * kTileP + 32 * c + 8 * kg + t;
            float x = 0.f;
            if (pp < NPT) {
                const PairDesc pd = ld_pair(A.pairs + pp);
                const float xn = gld(RBm + ((size_t)pd.rn * 8 + (j & 7)));
                const float xs = pd.rs >= 0 ? gld(RBm + ((size_t)pd.rs * 8 + (j & 7))) : 0.f;
                x = j < 8 ? xn + xs : xn - xs;
            }
            v[t] = x;
        }
        bx[c] = split8<NPROD>(v);
    }
    const int p = tile * kTileP + lane;
    const bool valid = p < NPT;
    const double z = valid ? gld(A.pz + (p)) : 0.0;
    const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * NP + p, valid);
    double q1 = 0.0, q2 = 0.0;
    const double seq = A.eq_ring >= 0 ? gld(A.seeds + ((size_t)m * NP + NPT)) : 0.0;
    const float *xeq = A.eq_ring >= 0 ? RBm + (size_t)A.eq_ring * 8 : nullptr;
    const double *ap = A.aprime + t0 - m;  // indexed by l'
    const int nl = L + 2 - m;
    const int nblk = (nl + kRowsB - 1) / kRowsB;
    int wfirst, gfirst;
    first_blocks(S.blk, nblk, wave, nw, reinterpret_cast<int *>(red), wfirst, gfirst);
    // recurrence on P (fwd_steps); a' of block b, lane-wise, loaded one block ahead
    // without a branch (index clamped into the order's row, zeroed where used)
    const double z_even = (m & 1) ? z : -z;
    auto load_a = [&](int b) -> double { return gld(ap + min(m + b * kRowsB + (lane & 15), L + 1)); };
    const int nout = blockDim.x == 64 ? 2 : 1;  // output slots per thread (threads >= 128 have none)
    float xq[2] = {0.f, 0.f};                    // the equator ring's value of each slot's column
    if (xeq)
        for (int u = 0; u < nout; ++u) {
            int row, col;
            FwdCompact<float>::rc((threadIdx.x + u * 64) & 127, row, col);
            xq[u] = gld(xeq + (col & 7));
        }
    // One 16-degree block; araw holds its a' (loaded one block earlier), anext receives
    // the next block's.
    auto block = [&](int blk, double araw, double &anext) {
        const int lp0 = m + blk * kRowsB;
        float csc[2];  // c_{l'} of the thread's slots, used after the reduction
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            int row, col;
            FwdCompact<float>::rc((threadIdx.x + u * 64) & 127, row, col);
            csc[u] = (float)gld(A.cscale + (t0 + min(lp0 + row, L + 1) - m));
        }
        anext = load_a(max(blk + 1, wfirst));
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        if (blk >= wfirst) {
            if (blk * kRowsB == kStartBlock * S.blk) {  // the lane's start state, as P
                q1 = sigma_state(lp0 - 1, S.q1);
                q2 = sigma_state(lp0 - 2, S.q2);
            }
            const double acur = lp0 + (lane & 15) <= L + 1 ? araw : 0.0;
            fwd_steps<0>(acur, z_even, q1, q2, [&](int st, double v) { qt[SwzFwd8::at(st, lane)] = (float)v; });
            __builtin_amdgcn_wave_barrier();
#pragma unroll
            for (int c = 0; c < 2; ++c) {
                const float4 *src = reinterpret_cast<const float4 *>(qt + SwzFwd8::at(j, 32 * c + 8 * kg));
                const float4 u0 = src[0], u1 = src[1];
                const float v[8] = {u0.x, u0.y, u0.z, u0.w, u1.x, u1.y, u1.z, u1.w};
                acc = mma_split<NPROD>(split8<NPROD>(v), bx[c], acc);
            }
            __builtin_amdgcn_wave_barrier();
        }
        if (blk >= gfirst) {
            float *rw = red + ((blk & 1) * nw + wave) * 128;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (FwdCompact<float>::valid(lane, r)) rw[FwdCompact<float>::slot(lane, r)] = acc[r];
            __syncthreads();
        }
        asm volatile("" : "+v"(anext)::"memory");  // as in leg_fwd_f64q_body
        if (threadIdx.x >= 128) return;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            if (u >= nout) break;
            const int o = threadIdx.x + u * 64;
            int row, col;
            FwdCompact<float>::rc(o, row, col);
            const int lp = lp0 + row;
            if (lp <= L + 1) {
                float sum = 0.f;
                if (blk >= gfirst) {
                    const float *rb = red + (blk & 1) * nw * 128;
                    for (int w = 0; w < nw; ++w) sum += rb[w * 128 + o];
                    if (lp & 2) sum = -sum;  // sigma_{l'}
                }
                const int64_t ti = t0 + lp - m;
                if (xeq && col < 8 && group == 0) {
                    const int kk = (lp - m) >> 1;
                    const double qe = (kk & 1) ? -seq : seq;
                    sum += (float)qe * xq[u];
                }
                gst(A.F + (group * A.gstride + ti * 8 + (col & 7)), csc[u] * sum);
            }
        }
    };
    double an = load_a(wfirst);
    asm volatile("" : "+v"(an)::"memory");  // waited for here, once, not in the loop
    for (int blk = 0; blk < nblk; ++blk) {
        const double araw = an;
        block(blk, araw, an);
    }
}

template <int NP>
__global__ __launch_bounds__(1024) void k_leg_fwd_bf16(LegFwdArgs<float> A) {
    extern __shared__ unsigned char smem_raw[];
    leg_fwd_bf16_body<NP>(field_args(A, blockIdx.z), blockIdx.x, blockIdx.y, smem_raw);
}

// Synthesis, BF16x3/BF16x6: one wave per 64 ring pairs, degrees in
// blocks of 32 (one K = 32 chunk).  Each lane advances the recurrence of its
// own pair and writes that pair's 32 values, already split, as one row of each
// of the wave's part tiles ([64 pairs][32 degrees] bf16, 16-byte slot q of pair
// p stored at slot q ^ ((p >> 2) & 3) so that 16 lanes of a row group hit
// distinct banks).
constexpr int kRowsA = 32;
static_assert(kRowsA == kStartBlock, "a split-bf16 synthesis block is one start block");

// The split-bf16 paths' polar tile: pairs [p0, p0 + 16 NB) of order m (the pairs
// next to the poles) over all degrees in binary64 on the 16x16x4 binary64 MFMA,
// with g from the plan's binary64 triangle, through the wave's Q tile qt (lane =
// pair for the recurrence; lanes beyond the tile's pairs run it unused).  The
// sums are stored in binary32.
template <int NB>
__device__ __forceinline__ void adj_tile_f64_polar(const LegArgs<float> &A, int m, int p0, int pend, double *qt) {
    typedef Mfma<double>::acc_t acc_t;
    const int lane = threadIdx.x & 63;
    const int L = A.L, NP = A.NP;
    const int64_t t0 = tri_offset(L, m);
    const double *g = A.FG64 + (t0 - m) * 8;  // indexed by l'
    const int p = p0 + lane;
    const bool valid = lane < 16 * NB && p < pend;
    const double z = valid ? gld(A.pz + (p)) : 0.0;
    const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * NP + p, valid);
    double q1 = 0.0, q2 = 0.0;
    const int j = lane & 15, k = lane >> 4;
    acc_t acc[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[b] = acc_t{0, 0, 0, 0};
    const int nblk = (L + 2 - m + kRowsB - 1) / kRowsB;
    const int first = min(wave_min_blk(S.blk) * (kStartBlock / kRowsB), nblk);
    for (int blk = first; blk < nblk; ++blk) {
        const int lp0 = m + blk * kRowsB;
        take_start(S, lp0 - m, q1, q2);
        const int la = lp0 + (lane & 15);
        const double areg = la <= L + 1 ? gld(A.aprime + (t0 + la - m)) : 0.0;
        // B operands: lane (j + 16k) holds g[row 4gg + k][j & 7] if the row's
        // parity matches the column half (row parity == (lp - m) & 1 == k & 1)
        double bv[4];
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
            const int lp = lp0 + 4 * gg + k;
            bv[gg] = (lp <= L + 1 && (j >> 3) == (k & 1)) ? gld(g + ((int64_t)lp * 8 + (j & 7))) : 0.0;
        }
        recur16<double, SwzAdj>(qt, areg, z, q1, q2, lane);
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                // A: lane (i + 16k) holds Q[row 4gg + k][pair 16b + i]
                const double a = qt[SwzAdj::at(4 * gg + k, 16 * b + j)];
                acc[b] = Mfma<double>::mma(a, bv[gg], acc[b]);
            }
        }
    }
    // accumulator b: lane l, register r -> pair p0 + 16b + row, column l % 16
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int pp = p0 + 16 * b + Mfma<double>::row(lane, r);
            if (pp < pend) gst(A.PB + (((size_t)m * NP + pp) * 16 + j), (float)acc[b][r]);
        }
}

template <int NPROD>
__device__ __forceinline__ void adj_tile_bf16(const LegArgs<float> &A, int m, int p0, int lB, double z,
                                              const LaneStart &S, f32x4 (&acc)[4], u32x4_t *th) {
    // pairs [p0, p0 + 64) over the degrees below lB, each from its start S; acc as
    // in adj_tile_f32 (register r of acc[b]: pair 16 b + 4 (l/16) + r)
    constexpr int NS = Bf16<NPROD>::kParts;
    const int lane = threadIdx.x & 63;
    const int L = A.L;
    const int64_t t0 = tri_offset(L, m);
    const float *g = A.FG + (t0 - m) * 8;    // indexed by l'
    const double *ap = A.aprime + t0 - m;    // indexed by l'
    const int j = lane & 15, kg = lane >> 4;
    f32x4 acl[4];  // leading products in acc, correction products in acl
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] = acl[b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int lA = min(m + kStartBlock * wave_min_blk(S.blk), lB);
    double q1 = 0.0, q2 = 0.0;
    const int nblk = (lB - lA + kRowsA - 1) / kRowsA;
    // The recurrence runs on P = sigma Q (fwd_steps) and sigma_{l'} goes into g: the
    // products sum sigma_{l'} P_{l'} g_{l'} = Q_{l'} g_{l'}.  a' comes lane-wise for the two
    // 16-degree halves of a block, loaded one block ahead without a branch.
    const double z_even = (lA & 1) ? z : -z;  // factor of the even steps (degree parity of lA)
    auto load_a = [&](int b, int half) -> double {
        return gld(ap + min(lA + b * kRowsA + 16 * half + (lane & 15), lB - 1));
    };
    double an0 = load_a(0, 0), an1 = load_a(0, 1);
    asm volatile("" : "+v"(an0), "+v"(an1)::"memory");  // waited for here, once
    for (int blk = 0; blk < nblk; ++blk) {
        const int lp0 = lA + blk * kRowsA;
        if (lp0 - m == kStartBlock * S.blk) {  // the lane's start state, as P
            q1 = sigma_state(lp0 - 1, S.q1);
            q2 = sigma_state(lp0 - 2, S.q2);
        }
        // B: lane (j + 16kg) holds sigma_{l'} g[l' = lp0 + 8kg + t][j & 7] when the parity
        // of l' - m (= t & 1) matches the column half j / 8, else 0
        float bv[8];
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int lp = lp0 + 8 * kg + t;
            const float x = (lp < lB && (t & 1) == (j >> 3)) ? gld(g + ((int64_t)lp * 8 + (j & 7))) : 0.f;
            bv[t] = (lp & 2) ? -x : x;
        }
        const Split8<NPROD> bs = split8<NPROD>(bv);
        // a' past lB - 1 is zeroed (P then repeats and stays bounded; its g is zero)
        const double a0 = lp0 + (lane & 15) <= lB - 1 ? an0 : 0.0;
        const double a1 = lp0 + 16 + (lane & 15) <= lB - 1 ? an1 : 0.0;
        an0 = load_a(blk + 1, 0);
        an1 = load_a(blk + 1, 1);
        uint32_t hq[NS][16];
        double held = 0.0;  // the even step's value, split together with the odd one's
        auto put = [&](int st, double v) {
            if ((st & 1) == 0) {
                held = v;
            } else {
                uint32_t o[NS];
                split2<NS>((float)held, (float)v, o);
#pragma unroll
                for (int k = 0; k < NS; ++k) hq[k][st >> 1] = o[k];
            }
        };
        fwd_steps<0>(a0, z_even, q1, q2, put);
        fwd_steps<0>(a1, z_even, q1, q2, [&](int st, double v) { put(st + 16, v); });
        const int sw = (lane >> 2) & 3;
#pragma unroll
        for (int k = 0; k < NS; ++k)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                th[k * kTileP * 4 + lane * 4 + (q ^ sw)] =
                    u32x4_t{hq[k][4 * q], hq[k][4 * q + 1], hq[k][4 * q + 2], hq[k][4 * q + 3]};
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            // A: lane (j + 16kg) holds Q[pair 16b + j][degrees lp0 + 8kg .. + 7]
            const int P = 16 * b + j;
            const int slot = P * 4 + (kg ^ ((P >> 2) & 3));
            Split8<NPROD> qa;
#pragma unroll
            for (int k = 0; k < NS; ++k) qa.p[k] = __builtin_bit_cast(bf16x8_t, th[k * kTileP * 4 + slot]);
            mma_split2<NPROD>(qa, bs, acc[b], acl[b]);
        }
        __builtin_amdgcn_wave_barrier();
        asm volatile("" : "+v"(an0), "+v"(an1)::"memory");  // as in leg_fwd_f64q_body
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[b] += acl[b];
}

// ---------------------------------------------------------------------------
// The synthesis launch: workgroups of four waves over (column x, order y).
//   NPROD = 0 (binary64 and binary32 plans): workgroup x takes pairs
//     [512 x, 512 x + 512), 128 per wave, on the binary64 vector unit; x = 0 also
//     forms the equator pair.
//   NPROD = 3, 6 (split-bf16): 64-pair tiles, one per wave, the first (the pairs
//     next to the poles after the polar ones) on the binary32 MFMA tile, the
//     others on the split-bf16 tiles; the equator comes from k_equator_adj.
//     BF16x6 (bar 1e-6) puts the P pairs nearest the poles on a binary64 MFMA
//     tile in the first wave slot (binary64 vector work would wait behind the
//     bf16 MFMA stream of the other waves); the tiles then start at P.
//     BF16x3's bound leaves those pairs on the binary32 tile.
// The order of m is reversed in every other round of 256 workgroups (the rounds
// in which workgroups reach the compute units), so that each unit gets long and
// short orders alike.
// ---------------------------------------------------------------------------
__host__ __device__ inline int adj_polar_pairs(int NPT, int nprod) {
    return nprod == 6 ? (NPT < kPolarPairs ? NPT : kPolarPairs) : 0;
}
// wave slots of a split-bf16 launch: [polar tile,] binary32 tile, split-bf16 tiles
__host__ __device__ inline int adj_slots(int NPT, int nprod) {
    const int P = adj_polar_pairs(NPT, nprod);
    return (P > 0 ? 1 : 0) + (NPT - P + kTileP - 1) / kTileP;
}
template <int NPROD>
__host__ __device__ constexpr size_t adj_lds_block() {
    if constexpr (NPROD == 0)
        return 2 * kAdjChunk * sizeof(AdjRow);
    else
        return 4 * (size_t)Bf16<NPROD>::kAdjLdsPerWave > 2 * kAdjChunk * sizeof(AdjRow)
                   ? 4 * (size_t)Bf16<NPROD>::kAdjLdsPerWave
                   : 2 * kAdjChunk * sizeof(AdjRow);
}
// waves per synthesis workgroup: the vector-unit form takes 128 pairs per wave and
// as many waves (up to four) as the pairs fill; the split-bf16 forms take four
__host__ __device__ inline int adj_waves(int NPT, int nprod) {
    if (nprod != 0) return 4;
    const int w = (NPT + 2 * kTileP - 1) / (2 * kTileP);
    return w < 1 ? 1 : (w > 4 ? 4 : w);
}
// workgroup columns of a synthesis launch over NPT tile pairs
__host__ __device__ inline int adj_columns(int NPT, int nprod) {
    if (nprod == 0) {
        const int per = 2 * kTileP * adj_waves(NPT, nprod);
        return NPT > 0 ? (NPT + per - 1) / per : 1;
    }
    return (adj_slots(NPT, nprod) + 3) / 4;
}

template <typename real, int NPROD>
__device__ __forceinline__ void leg_adj_group(const LegArgs<real> &A, int m, int x, unsigned char *smem) {
    const int wave = uniform_int(threadIdx.x >> 6);
    if constexpr (NPROD == 0) {
        const int nw = blockDim.x >> 6;  // adj_waves(NPT, 0)
        adj_valu_block<real, 2, 0, 8>(A, A.FG64, m, (x * nw + wave) * 2 * kTileP, A.NPT,
                                      x == 0 && wave == 0 && A.NP > A.NPT, reinterpret_cast<AdjRow *>(smem));
    } else {
        const int P = adj_polar_pairs(A.NPT, NPROD);
        const int slot = x * 4 + wave;
        unsigned char *wl = smem + wave * Bf16<NPROD>::kAdjLdsPerWave;
        if (P > 0 && slot == 0) {
            adj_tile_f64_polar<kPolarPairs / 16>(A, m, 0, P, reinterpret_cast<double *>(wl));
            return;
        }
        const int tile = slot - (P > 0 ? 1 : 0);
        const int p0 = P + tile * kTileP;
        if (p0 >= A.NPT) return;
        const int lane = threadIdx.x & 63;
        const int p = p0 + lane;
        const bool valid = p < A.NPT;
        const double z = valid ? gld(A.pz + (p)) : 0.0;
        const LaneStart S = lane_start(A.start, A.sblk, (size_t)m * A.NP + p, valid);
        f32x4 acc[4];
        if (tile == 0)
            adj_tile_f32(A, m, p0, A.L + 2, z, S, acc, reinterpret_cast<float *>(wl));
        else
            adj_tile_bf16<NPROD>(A, m, p0, A.L + 2, z, S, acc, reinterpret_cast<u32x4_t *>(wl));
        const int j = lane & 15;
#pragma unroll
        for (int b = 0; b < 4; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int pp = p0 + 16 * b + Mfma<float>::row(lane, r);
                if (pp < A.NPT) gst(A.PB + (((size_t)m * A.NP + pp) * 16 + j), acc[b][r]);
            }
    }
}

template <typename real, int NPROD>
__global__ __launch_bounds__(256, NPROD == 0 ? 4 : 1) void k_leg_adj(LegArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    const int y = blockIdx.y, base = y & ~255, r = y & 255;
    const int cnt = min(256, A.L + 1 - base);
    const int m = (y >> 8) & 1 ? base + cnt - 1 - r : y;
    leg_adj_group<real, NPROD>(field_args(A, blockIdx.z), m, blockIdx.x, smem_raw);
}

// ---------------------------------------------------------------------------
// Three-term recombination (forward):
//   a_{l,mu} = [l e_{l+1} F^th_{l+1} - (l+1) e_l F^th_{l-1} - i mu F^ph_l] / sqrt(l(l+1))
//   b_{l,mu} = [l e_{l+1} F^ph_{l+1} - (l+1) e_l F^ph_{l-1} + i mu F^th_l] / sqrt(l(l+1))
// with e_l = e_{l,m} = sqrt((l^2-m^2)/(4l^2-1)) (plan table) and
// F_{.,-m} = (-1)^m FG[.][2..3].  One thread per (l, m >= 0); threads of a
// block share l and run over m, so the coefficient writes are contiguous.
// ---------------------------------------------------------------------------
template <typename real>
struct CoefArgs {
    const C2<real> *FG;
    C2<real> *FGout;
    const C2<real> *ain, *bin;
    C2<real> *aout, *bout;
    const double *cscale;   // [tri] c_{l',m}
    const double *etab;     // [tri] e_{l',m}
    const double *rsq;      // [L+2] 1 / sqrt(l (l+1)), 0 for l = 0
    double *FG64;           // binary32 paths: g in binary64, [tri][8] (prep output)
    int L;
    int fg32;               // binary32 paths: also write g in binary32 to FGout (the split-bf16
                            // tiles and the direct scattered evaluation read it)
    // per-field strides of a launch over fields (blockIdx.z): triangle (complex
    // elements, FG and FGout), coefficients (complex elements), FG64 (doubles)
    int64_t zs_FG, zs_coef, zs_FG64;
    __device__ CoefArgs at_field(int f) const {
        CoefArgs r = *this;
        if (f) {
            r.FG = FG + f * zs_FG;
            r.FGout = FGout + f * zs_FG;
            if (ain) r.ain = ain + f * zs_coef;
            if (bin) r.bin = bin + f * zs_coef;
            if (aout) r.aout = aout + f * zs_coef;
            if (bout) r.bout = bout + f * zs_coef;
            if (FG64) r.FG64 = FG64 + f * zs_FG64;
        }
        return r;
    }
};

// Both coefficient kernels work on tiles of kTM orders x kTL degrees staged in
// LDS, so that the coefficient side (contiguous in m for fixed l) and the
// triangle side (contiguous in l' for fixed m) are both read and written in
// contiguous runs.
constexpr int kTM = 16, kTL = 32;

// Both run with 256 threads; every thread issues all of its loads of a phase
// before the first use, so a phase costs one memory latency.
constexpr int kCoefNT = 256;

template <typename real>
__device__ __forceinline__ void recombine_body(const CoefArgs<real> &A, int bx, int by) {
    // F rows l0-1 .. l0+kTL of each order: (th,+m) (ph,+m) (th,-m) (ph,-m); an odd
    // stride between orders keeps the 16-byte reads of consecutive orders conflict free
    constexpr int kRowR = (kTL + 2) * 4 + 1;
    __shared__ C2<real> fs[kTM * kRowR];
    const int L = A.L;
    const int l0 = 1 + bx * kTL, m0 = by * kTM;
    if (m0 > L || m0 > l0 + kTL - 1) return;
    constexpr int kItems = kTM * (kTL + 2) * 4, kPer = (kItems + kCoefNT - 1) / kCoefNT;
    C2<real> v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int c = idx & 3, i = (idx >> 2) % (kTL + 2), mi = (idx >> 2) / (kTL + 2);
        const int m = m0 + mi, lp = l0 - 1 + i;
        v[q] = {0, 0};
        if (idx < kItems && m <= L && lp >= m && lp <= L + 1) v[q] = gld(A.FG + ((tri_offset(L, m) + lp - m) * 4 + c));
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        if (idx < kItems) fs[(idx / (4 * (kTL + 2))) * kRowR + idx % (4 * (kTL + 2))] = v[q];
    }
    __syncthreads();
    constexpr int kOut = (kTM * kTL) / kCoefNT;
    static_assert(kOut * kCoefNT == kTM * kTL, "whole outputs per thread");
    double cpv[kOut], cmv[kOut], inv[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int mi = idx % kTM, li = idx / kTM;
        const int l = l0 + li, m = m0 + mi;
        cpv[q] = cmv[q] = inv[q] = 0.0;
        if (l <= L && m <= l) {
            const double *et = A.etab + tri_offset(L, m) - m;  // indexed by l'
            inv[q] = gld(A.rsq + (l));
            cpv[q] = gld(et + l + 1);
            cmv[q] = l - 1 >= m ? gld(et + l) : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int mi = idx % kTM, li = idx / kTM;
        const int l = l0 + li, m = m0 + mi;
        if (l > L || m > l) continue;
        const real cp = (real)(l * cpv[q] * inv[q]);
        const real cm = (real)((l + 1) * cmv[q] * inv[q]);
        const int64_t base = (int64_t)l * l + l - 1;
#pragma unroll
        for (int sgn = 0; sgn < 2; ++sgn) {
            if (sgn == 1 && m == 0) break;
            const int mu = sgn == 0 ? m : -m;
            const real parity = (sgn == 1 && (m & 1)) ? (real)-1 : (real)1;
            const real fmu = (real)(mu * inv[q]);
            const C2<real> *fm = fs + mi * kRowR + 4 * li, *f0 = fm + 4, *fp = fm + 8;
            const C2<real> th1 = fp[2 * sgn], ph1 = fp[2 * sgn + 1];
            const C2<real> th0 = f0[2 * sgn], ph0 = f0[2 * sgn + 1];
            const C2<real> thm = fm[2 * sgn], phm = fm[2 * sgn + 1];
            C2<real> av, bv;
            // -i mu F^ph = (mu F^ph.y, -mu F^ph.x);  +i mu F^th = (-mu F^th.y, mu F^th.x)
            av.x = parity * (cp * th1.x - cm * thm.x + fmu * ph0.y);
            av.y = parity * (cp * th1.y - cm * thm.y - fmu * ph0.x);
            bv.x = parity * (cp * ph1.x - cm * phm.x - fmu * th0.y);
            bv.y = parity * (cp * ph1.y - cm * phm.y + fmu * th0.x);
            gst(A.aout + (base + mu), av);
            gst(A.bout + (base + mu), bv);
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint prep: FG[tri(m, l')] = c_{l'} (g^th_{+m}, g^ph_{+m}, (-1)^m g^th_{-m}, (-1)^m g^ph_{-m}),
//   g^th_{l',mu} = (l'-1) e_{l'} at_{l'-1} - (l'+2) e_{l'+1} at_{l'+1} - i mu bt_{l'}
//   g^ph_{l',mu} = (l'-1) e_{l'} bt_{l'-1} - (l'+2) e_{l'+1} bt_{l'+1} + i mu at_{l'}
// with at = a / sqrt(l(l+1)) (zero outside 1 <= l <= L, |mu| <= l).
// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_recombine(CoefArgs<real> A) {
    recombine_body(field_args(A, blockIdx.z), blockIdx.x, blockIdx.y);
}

template <typename real>
__device__ __forceinline__ void prep_body(const CoefArgs<real> &A, int bx, int by) {
    // coefficients of degrees l0-1 .. l0+kTL for the tile's orders, [l][sign][a,b][m]; an
    // odd stride between degrees keeps the 16-byte reads of consecutive degrees conflict free.
    // The map is evaluated in binary64 for every precision: the binary32 paths store g
    // both in binary32 (FG, for the split-bf16 tiles) and in binary64 (FG64, for the
    // binary64 vector-unit synthesis and the polar wave).
    constexpr int kRowP = 4 * kTM + 1;
    __shared__ C2<double> cs[(kTL + 2) * kRowP];
    const int L = A.L;
    const int l0 = bx * kTL, m0 = by * kTM;  // l' in [l0, l0+kTL)
    if (m0 > L || m0 > l0 + kTL - 1) return;
    constexpr int kItems = (kTL + 2) * 2 * 2 * kTM, kPer = (kItems + kCoefNT - 1) / kCoefNT;
    C2<real> v[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int mi = idx % kTM, r = idx / kTM;
        const int ab = r & 1, sg = (r >> 1) & 1, i = r >> 2;
        const int l = l0 - 1 + i, m = m0 + mi;
        v[q] = {0, 0};
        if (idx < kItems && l >= 1 && l <= L && m <= l) {
            const int mu = sg ? -m : m;
            v[q] = gld((ab ? A.bin : A.ain) + ((int64_t)l * l + l + mu - 1));
        }
    }
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        if (idx < kItems) {
            const int mi = idx % kTM, r = idx / kTM;
            const int l = l0 - 1 + (r >> 2);
            const double rs = (l >= 1 && l <= L) ? gld(A.rsq + (l)) : 0.0;
            cs[(r >> 2) * kRowP + (r & 3) * kTM + mi] = {(double)v[q].x * rs, (double)v[q].y * rs};
        }
    }
    __syncthreads();
    constexpr int kOut = (kTM * kTL) / kCoefNT;
    static_assert(kOut * kCoefNT == kTM * kTL, "whole outputs per thread");
    double cscv[kOut], e0v[kOut], e1v[kOut];
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int li = idx % kTL, mi = idx / kTL;
        const int lp = l0 + li, m = m0 + mi;
        cscv[q] = e0v[q] = e1v[q] = 0.0;
        if (m <= L && lp >= m && lp <= L + 1) {
            const int64_t ti = tri_offset(L, m) + lp - m;
            cscv[q] = gld(A.cscale + (ti));  // Lambda = c Q: fold c_{l'} in
            e0v[q] = gld(A.etab + (ti));
            e1v[q] = lp + 1 <= L + 1 ? gld(A.etab + (ti + 1)) : 0.0;
        }
    }
#pragma unroll
    for (int q = 0; q < kOut; ++q) {
        const int idx = threadIdx.x + q * kCoefNT;
        const int li = idx % kTL, mi = idx / kTL;
        const int lp = l0 + li, m = m0 + mi;
        if (m > L || lp < m || lp > L + 1) continue;
        const int64_t ti = tri_offset(L, m) + lp - m;
        const double csc = cscv[q];
        const double c1 = csc * (lp - 1) * e0v[q];
        const double c2 = csc * (lp + 2) * e1v[q];
        const double csr = csc;
        C2<real> *o = A.FGout + ti * 4;
#pragma unroll
        for (int sgn = 0; sgn < 2; ++sgn) {
            const int mu = sgn == 0 ? m : -m;
            const double parity = (sgn == 1 && (m & 1)) ? -1.0 : 1.0;
            const double fmu = (double)mu;
            const C2<double> *cm1 = cs + li * kRowP + 2 * sgn * kTM + mi, *c0 = cm1 + kRowP, *cp1 = c0 + kRowP;
            const C2<double> am1 = cm1[0], bm1 = cm1[kTM];
            const C2<double> a0 = c0[0], b0 = c0[kTM];
            const C2<double> ap1 = cp1[0], bp1 = cp1[kTM];
            C2<double> gth, gph;
            // -i mu b = (mu b.y, -mu b.x); +i mu a = (-mu a.y, mu a.x)
            gth.x = parity * (c1 * am1.x - c2 * ap1.x + csr * fmu * b0.y);
            gth.y = parity * (c1 * am1.y - c2 * ap1.y - csr * fmu * b0.x);
            gph.x = parity * (c1 * bm1.x - c2 * bp1.x - csr * fmu * a0.y);
            gph.y = parity * (c1 * bm1.y - c2 * bp1.y + csr * fmu * a0.x);
            if constexpr (sizeof(real) == 8) {
                gst(o + (2 * sgn), {gth.x, gth.y});
                gst(o + (2 * sgn + 1), {gph.x, gph.y});
            } else {
                if (A.fg32) {
                    gst(o + (2 * sgn), {(float)gth.x, (float)gth.y});
                    gst(o + (2 * sgn + 1), {(float)gph.x, (float)gph.y});
                }
                C2<double> *o64 = reinterpret_cast<C2<double> *>(A.FG64) + ti * 4;
                gst(o64 + 2 * sgn, gth);
                gst(o64 + 2 * sgn + 1, gph);
            }
        }
    }
}

template <typename real>
__global__ __launch_bounds__(256) void k_prep(CoefArgs<real> A) {
    prep_body(field_args(A, blockIdx.z), blockIdx.x, blockIdx.y);
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
    const double *weights;  // per point; used when weighted != 0
    int64_t n;
    int L;
    int weighted;
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
            // a seed below 2^-960 runs scaled by 2^-E until its values reach 2^-960
            // (the smaller ones add nothing at binary64's precision); the state is
            // then scaled back, exactly
            double q1 = 0.0, q2;
            int E = 0, lp = m;
            if (e2 < -960) {
                q2 = -mant;
                E = e2;
            } else {
                q2 = -ldexp(mant, e2);
            }
            for (; E < 0 && lp <= L + 1; ++lp) {
                const double v = fma(ap[lp], z * q1, -q2);
                int ev;
                (void)frexp(v, &ev);
                if (v != 0.0 && ev + E > -960) {
                    q1 = ldexp(q1, E);
                    q2 = ldexp(q2, E);
                    E = 0;
                    break;  // degree lp again, unscaled
                }
                q2 = q1;
                q1 = v;
                (void)frexp(q1, &ev);
                if (q1 != 0.0 && (ev > 64 || ev < -64)) {
                    q1 = ldexp(q1, -ev);
                    q2 = ldexp(q2, -ev);
                    E += ev;
                }
            }
            if (E < 0) lp = L + 2;  // never significant
            for (; lp <= L + 1; ++lp) {
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
    double inv_s = pole ? 1.0 : 1.0 / s;
    if (A.weighted) inv_s *= A.weights[k];
    thr *= inv_s; thi *= inv_s; phr *= inv_s; phi_ *= inv_s;
    // e_theta = (z c, z sn, -s), e_phi = (-sn, c, 0)
    A.Tout[3 * k] = {(real)(z * c * thr - sn * phr), (real)(z * c * thi - sn * phi_)};
    A.Tout[3 * k + 1] = {(real)(z * sn * thr + c * phr), (real)(z * sn * thi + c * phi_)};
    A.Tout[3 * k + 2] = {(real)(-s * thr), (real)(-s * thi)};
}

// ===========================================================================
// Scattered points through the double Fourier sphere (adjoint).
// The spin-frame components T_theta,m(theta), T_phi,m(theta) of the synthesised
// field are, continued to theta in [0, 2 pi) with signed sin(theta),
// trigonometric polynomials of degree <= L (derivatives of sin^m(theta) times
// polynomials in cos(theta), and those over sin(theta)) that satisfy
// T_m(2 pi - theta) = (-1)^{|m|+1} T_m(theta).  The synthesis runs on nt > 2L
// equispaced colatitudes theta_t = 2 pi (t + 1/2) / nt, t < nt/2 (nt/4 virtual
// north/south ring pairs, never at a pole), the other half follows from the
// symmetry, and a DFT over t gives their exact Fourier coefficients
// c_{k,m}, |k| <= L.  With the window transform
// psih(k) = int psi(u) e^{-i k u} du, the grid values
//     g(theta_j, phi_i) = sum_{k,m} c_{k,m} h^2 / (psih(k) psih(m)) e^{i (k theta_j + m phi_i)}
// (two inverse DFTs of length ng) reproduce T at any point as the windowed sum
// sum_{j,i} g(theta_j, phi_i) psi(theta - theta_j) psi(phi - phi_i), up to the
// kernel's aliasing error.
// ===========================================================================
template <typename real>
struct NfftArgs {
    const real *PB;            // virtual pair buffer [(L+1)][npv][16]
    C2<real> *g1;              // [2][ng][2L+1]
    C2<real> *g;               // [2][ng][ng]
    const double *vs;          // sin theta of each virtual pair
    const double *psihat;      // [2L+1]
    const FftDesc *ffts;
    const double *tw;
    const NfftPoint *pts;
    const NfftTile *tiles;     // gather tiles (point ranges of pts)
    const double *weights;
    C2<real> *Tout;
    const C2<real> *Tin;       // forward: the field at the points
    real *RB;                  // forward: ring buffer of the virtual rings [(L+1)][nt/2][8]
    int64_t n;
    double beta, h;
    int fft_nt, fft_ng;
    int L, nt, npv, ng, w;
    int stride;                // LDS sequence stride
    int weighted;
};

constexpr int kNfftNT = 512;
constexpr int kNfftMaxK = 5;   // (2L+1) / kNfftNT, rounded up, for L <= 1279
constexpr int kNfftMaxW = 16;

// One workgroup per order m in [-L, L]: theta samples of T_theta,m and T_phi,m,
// DFT of length nt, deconvolution, zero padding, inverse DFT of length ng,
// column m of g1.
template <typename real>
__global__ __launch_bounds__(kNfftNT, 1) void k_nfft_cols(NfftArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    Seq<real> buf = {lds, ld_const(&A.ffts[A.fft_nt].lds_shift)};
    const int L = A.L, nt = A.nt, npv = A.npv, ng = A.ng, S = A.stride;
    const int b = blockIdx.x;  // m + L
    const int m = b - L;
    const int am = m < 0 ? -m : m;
    const int slot = m < 0 ? 2 : 0;  // complex column (theta) of +-m; phi is slot + 1
    const real ext = (am & 1) ? (real)1 : (real)-1;
    for (int t = threadIdx.x; t < nt; t += kNfftNT) {
        const bool upper = t < nt / 2;
        const int tt = upper ? t : nt - 1 - t;  // sample in (0, pi)
        const bool north = tt < nt / 4;
        const int p = north ? tt : nt / 2 - 1 - tt;
        const C2<real> *e = reinterpret_cast<const C2<real> *>(A.PB + ((size_t)am * npv + p) * 16);
        const C2<real> Et = e[slot], Ep = e[slot + 1], Ot = e[4 + slot], Op = e[4 + slot + 1];
        const real f = (upper ? (real)1 : ext) / (real)A.vs[p];
        const real so = north ? (real)1 : (real)-1;
        buf[t] = {(Et.x + so * Ot.x) * f, (Et.y + so * Ot.y) * f};
        buf[S + t] = {(Ep.x + so * Op.x) * f, (Ep.y + so * Op.y) * f};
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_nt, A.tw, wR, false);
    // d_k = DFT[k mod nt] e^{-i pi k / nt} / nt * h^2 / (psih(k) psih(m)), |k| <= L
    C2<real> dk[kNfftMaxK][2];
#pragma unroll
    for (int q = 0; q < kNfftMaxK; ++q) {
        const int k = threadIdx.x + q * kNfftNT - L;
        if (k <= L) {
            const int src = k >= 0 ? k : nt + k;
            double sp, cp;
            sincos(-M_PI * (double)k / (double)nt, &sp, &cp);
            const double sc = A.h * A.h / ((double)nt * A.psihat[k + L] * A.psihat[m + L]);
            const CD ph = {cp * sc, sp * sc};
            dk[q][0] = cmul_d(buf[src], ph);
            dk[q][1] = cmul_d(buf[S + src], ph);
        }
    }
    __syncthreads();
    buf.ps = ld_const(&A.ffts[A.fft_ng].lds_shift);  // layout of the second DFT
    for (int i = threadIdx.x; i < ng; i += kNfftNT) {
        buf[i] = {0, 0};
        buf[S + i] = {0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kNfftMaxK; ++q) {
        const int k = threadIdx.x + q * kNfftNT - L;
        if (k <= L) {
            const int dst = k >= 0 ? k : ng + k;
            buf[dst] = dk[q][0];
            buf[S + dst] = dk[q][1];
        }
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_ng, A.tw, wR, true);
    const int nm = 2 * L + 1;
    for (int j = threadIdx.x; j < ng; j += kNfftNT) {
        A.g1[(size_t)j * nm + b] = buf[j];
        A.g1[((size_t)ng + j) * nm + b] = buf[S + j];
    }
}

// One workgroup per grid row j: inverse DFT over the orders (zero padded).
template <typename real>
__global__ __launch_bounds__(kNfftNT, 1) void k_nfft_rows(NfftArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    Seq<real> buf = {lds, ld_const(&A.ffts[A.fft_ng].lds_shift)};
    const int L = A.L, ng = A.ng, S = A.stride;
    const int j = blockIdx.x;
    const int nm = 2 * L + 1;
    for (int i = threadIdx.x; i < ng; i += kNfftNT) {
        // bin i holds order m = i (i <= L) or i - ng (i >= ng - L)
        const int m = i <= L ? i : (i >= ng - L ? i - ng : L + 1);
        C2<real> vt = {0, 0}, vp = {0, 0};
        if (m <= L) {
            vt = A.g1[(size_t)j * nm + m + L];
            vp = A.g1[((size_t)ng + j) * nm + m + L];
        }
        buf[i] = vt;
        buf[S + i] = vp;
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_ng, A.tw, wR, true);
    for (int i = threadIdx.x; i < ng; i += kNfftNT) {
        A.g[(size_t)j * ng + i] = buf[i];
        A.g[((size_t)ng + j) * ng + i] = buf[S + i];
    }
}

// One lane per point (in grid-cell order): window sum of both components,
// rotation to Cartesian components, store at the caller's index.
// Gather, one workgroup per tile of kGatherTile x kGatherTile grid cells: the
// window of both grids that the tile's points touch (kGatherTile + w - 1 rows and
// columns, periodic in both) is staged in LDS once, and every point of the tile
// reads its w x w values from there.  A point whose window would leave the tile's
// (never, when the planner and the kernel agree on its first cell) reads the grids
// directly; both forms add the same terms in the same order.
constexpr int kGatherWin = kGatherTile + kNfftMaxW - 1;
template <typename real>
__global__ __launch_bounds__(256) void k_nfft_gather(NfftArgs<real> A) {
    __shared__ C2<real> win[2][kGatherWin * kGatherWin];
    const NfftTile T = ld_uniform(A.tiles + blockIdx.x);
    const int ng = A.ng, w = A.w, hw2 = w / 2;
    const int W = kGatherTile + w - 1;
    const int R0 = T.tj * kGatherTile - hw2, C0 = T.ti * kGatherTile - hw2;
    for (int e = threadIdx.x; e < W * W; e += 256) {
        const int r = e / W, c = e - (e / W) * W;
        int gr = (R0 + r) % ng, gc = (C0 + c) % ng;
        if (gr < 0) gr += ng;
        if (gc < 0) gc += ng;
        win[0][r * kGatherWin + c] = A.g[(size_t)gr * ng + gc];
        win[1][r * kGatherWin + c] = A.g[((size_t)ng + gr) * ng + gc];
    }
    __syncthreads();
    const double hw = 0.5 * w;
    for (int t = threadIdx.x; t < T.count; t += 256) {
        const NfftPoint P = A.pts[T.start + t];
        const double u = P.theta / A.h, v = P.phi / A.h;
        const int j0 = (int)ceil(u - hw), i0 = (int)ceil(v - hw);
        real wt[kNfftMaxW], wp[kNfftMaxW];
#pragma unroll
        for (int a = 0; a < kNfftMaxW; ++a) {
            wt[a] = wp[a] = 0;
            if (a < w) {
                const double dt = (u - (j0 + a)) / hw, dp = (v - (i0 + a)) / hw;
                wt[a] = (real)(fabs(dt) < 1.0 ? exp(A.beta * (sqrt((1.0 - dt) * (1.0 + dt)) - 1.0)) : 0.0);
                wp[a] = (real)(fabs(dp) < 1.0 ? exp(A.beta * (sqrt((1.0 - dp) * (1.0 + dp)) - 1.0)) : 0.0);
            }
        }
        real thr = 0, thi = 0, phr = 0, phi_ = 0;
        const int lr = j0 - R0, lc = i0 - C0;
        if (lr >= 0 && lr < kGatherTile && lc >= 0 && lc < kGatherTile) {
#pragma unroll
            for (int a = 0; a < kNfftMaxW; ++a) {
                if (a < w) {
                    const C2<real> *rt = win[0] + (lr + a) * kGatherWin + lc;
                    const C2<real> *rp = win[1] + (lr + a) * kGatherWin + lc;
                    real str = 0, sti = 0, spr = 0, spi = 0;
#pragma unroll
                    for (int c = 0; c < kNfftMaxW; ++c) {
                        if (c < w) {
                            const C2<real> gt = rt[c], gp = rp[c];
                            str += wp[c] * gt.x;
                            sti += wp[c] * gt.y;
                            spr += wp[c] * gp.x;
                            spi += wp[c] * gp.y;
                        }
                    }
                    thr += wt[a] * str;
                    thi += wt[a] * sti;
                    phr += wt[a] * spr;
                    phi_ += wt[a] * spi;
                }
            }
        } else {
            int jr = j0 % ng;
            if (jr < 0) jr += ng;
            int ir0 = i0 % ng;
            if (ir0 < 0) ir0 += ng;
            for (int a = 0; a < w; ++a) {
                const C2<real> *rt = A.g + (size_t)jr * ng;
                const C2<real> *rp = A.g + ((size_t)ng + jr) * ng;
                real str = 0, sti = 0, spr = 0, spi = 0;
                int ir = ir0;
                for (int c = 0; c < w; ++c) {
                    const C2<real> gt = rt[ir], gp = rp[ir];
                    str += wp[c] * gt.x;
                    sti += wp[c] * gt.y;
                    spr += wp[c] * gp.x;
                    spi += wp[c] * gp.y;
                    if (++ir == ng) ir = 0;
                }
                thr += wt[a] * str;
                thi += wt[a] * sti;
                phr += wt[a] * spr;
                phi_ += wt[a] * spi;
                if (++jr == ng) jr = 0;
            }
        }
        const real z = (real)P.z, s = (real)P.s, c = (real)P.c, sn = (real)P.sn;
        real sc = 1;
        if (A.weighted) sc = (real)A.weights[P.idx];
        C2<real> *o = A.Tout + 3 * P.idx;
        o[0] = {sc * (z * c * thr - sn * phr), sc * (z * c * thi - sn * phi_)};
        o[1] = {sc * (z * sn * thr + c * phr), sc * (z * sn * thi + c * phi_)};
        o[2] = {sc * (-s * thr), sc * (-s * thi)};
    }
}

// ---------------------------------------------------------------------------
// Forward transform at scattered points: the conjugate transpose, stage by
// stage, of the adjoint above (weights applied at the points).  Spreading
// (transpose of the gather) adds w_k psi psi (e_theta . T_k, e_phi . T_k) into
// the grid with vector atomics; the row and column passes take forward DFTs
// and keep |m|, |k| <= L; the conjugate deconvolution factors and an inverse
// DFT of length nt give the values at the virtual colatitudes, whose
// doubled-circle images are folded back (transpose of the extension), and the
// result, divided by sin(theta), fills the ring buffer of the virtual rings
// for the Legendre analysis.
// ---------------------------------------------------------------------------
template <typename real>
__global__ __launch_bounds__(256) void k_fill_zero(real *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <typename real>
__global__ __launch_bounds__(256) void k_nfft_spread(NfftArgs<real> A) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= A.n) return;
    const NfftPoint P = A.pts[k];
    const int ng = A.ng, w = A.w;
    const double hw = 0.5 * w;
    const double u = P.theta / A.h, v = P.phi / A.h;
    const int j0 = (int)ceil(u - hw), i0 = (int)ceil(v - hw);
    real wt[kNfftMaxW], wp[kNfftMaxW];
#pragma unroll
    for (int a = 0; a < kNfftMaxW; ++a) {
        wt[a] = wp[a] = 0;
        if (a < w) {
            const double dt = (u - (j0 + a)) / hw, dp = (v - (i0 + a)) / hw;
            wt[a] = (real)(fabs(dt) < 1.0 ? exp(A.beta * (sqrt((1.0 - dt) * (1.0 + dt)) - 1.0)) : 0.0);
            wp[a] = (real)(fabs(dp) < 1.0 ? exp(A.beta * (sqrt((1.0 - dp) * (1.0 + dp)) - 1.0)) : 0.0);
        }
    }
    const C2<real> *t = A.Tin + 3 * P.idx;
    const real z = (real)P.z, s = (real)P.s, c = (real)P.c, sn = (real)P.sn;
    real sc = 1;
    if (A.weighted) sc = (real)A.weights[P.idx];
    // e_theta = (z c, z sn, -s), e_phi = (-sn, c, 0)
    const real ttr = sc * (z * c * t[0].x + z * sn * t[1].x - s * t[2].x);
    const real tti = sc * (z * c * t[0].y + z * sn * t[1].y - s * t[2].y);
    const real tpr = sc * (-sn * t[0].x + c * t[1].x);
    const real tpi = sc * (-sn * t[0].y + c * t[1].y);
    int jr = j0 % ng;
    if (jr < 0) jr += ng;
    int ir0 = i0 % ng;
    if (ir0 < 0) ir0 += ng;
#pragma unroll
    for (int a = 0; a < kNfftMaxW; ++a) {
        if (a < w) {
            real *rt = reinterpret_cast<real *>(A.g + (size_t)jr * ng);
            real *rp = reinterpret_cast<real *>(A.g + ((size_t)ng + jr) * ng);
            int ir = ir0;
#pragma unroll
            for (int cc = 0; cc < kNfftMaxW; ++cc) {
                if (cc < w) {
                    const real f = wt[a] * wp[cc];
                    atomicAdd(rt + 2 * ir, f * ttr);
                    atomicAdd(rt + 2 * ir + 1, f * tti);
                    atomicAdd(rp + 2 * ir, f * tpr);
                    atomicAdd(rp + 2 * ir + 1, f * tpi);
                    if (++ir == ng) ir = 0;
                }
            }
            if (++jr == ng) jr = 0;
        }
    }
}

// One workgroup per grid row j: forward DFT over phi, keep |m| <= L.
template <typename real>
__global__ __launch_bounds__(kNfftNT, 1) void k_nfft_rows_fwd(NfftArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    Seq<real> buf = {lds, ld_const(&A.ffts[A.fft_ng].lds_shift)};
    const int L = A.L, ng = A.ng, S = A.stride;
    const int j = blockIdx.x;
    const int nm = 2 * L + 1;
    for (int i = threadIdx.x; i < ng; i += kNfftNT) {
        buf[i] = A.g[(size_t)j * ng + i];
        buf[S + i] = A.g[((size_t)ng + j) * ng + i];
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_ng, A.tw, wR, false);
    for (int b = threadIdx.x; b < nm; b += kNfftNT) {
        const int m = b - L;
        const int src = m >= 0 ? m : ng + m;
        A.g1[(size_t)j * nm + b] = buf[src];
        A.g1[((size_t)ng + j) * nm + b] = buf[S + src];
    }
}

// One workgroup per order m in [-L, L]: forward DFT over theta of column m,
// conjugate deconvolution, inverse DFT of length nt, fold and store into the
// virtual rings' buffer.
template <typename real>
__global__ __launch_bounds__(kNfftNT, 1) void k_nfft_cols_fwd(NfftArgs<real> A) {
    extern __shared__ unsigned char smem_raw[];
    CD *wR = reinterpret_cast<CD *>(smem_raw);
    C2<real> *lds = reinterpret_cast<C2<real> *>(smem_raw + kSmallTab * sizeof(CD));
    Seq<real> buf = {lds, ld_const(&A.ffts[A.fft_ng].lds_shift)};
    const int L = A.L, nt = A.nt, ng = A.ng, S = A.stride;
    const int b = blockIdx.x;
    const int m = b - L;
    const int am = m < 0 ? -m : m;
    const int slot = m < 0 ? 2 : 0;
    const real ext = (am & 1) ? (real)1 : (real)-1;
    const int nm = 2 * L + 1;
    for (int j = threadIdx.x; j < ng; j += kNfftNT) {
        buf[j] = A.g1[(size_t)j * nm + b];
        buf[S + j] = A.g1[((size_t)ng + j) * nm + b];
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_ng, A.tw, wR, false);
    C2<real> dk[kNfftMaxK][2];
#pragma unroll
    for (int q = 0; q < kNfftMaxK; ++q) {
        const int k = threadIdx.x + q * kNfftNT - L;
        if (k <= L) {
            const int src = k >= 0 ? k : ng + k;
            double sp, cp;
            sincos(M_PI * (double)k / (double)nt, &sp, &cp);  // conjugate of the adjoint's phase
            const double sc = A.h * A.h / ((double)nt * A.psihat[k + L] * A.psihat[m + L]);
            const CD ph = {cp * sc, sp * sc};
            dk[q][0] = cmul_d(buf[src], ph);
            dk[q][1] = cmul_d(buf[S + src], ph);
        }
    }
    __syncthreads();
    buf.ps = ld_const(&A.ffts[A.fft_nt].lds_shift);  // layout of the second DFT
    for (int i = threadIdx.x; i < nt; i += kNfftNT) {
        buf[i] = {0, 0};
        buf[S + i] = {0, 0};
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kNfftMaxK; ++q) {
        const int k = threadIdx.x + q * kNfftNT - L;
        if (k <= L) {
            const int dst = k >= 0 ? k : nt + k;
            buf[dst] = dk[q][0];
            buf[S + dst] = dk[q][1];
        }
    }
    __syncthreads();
    fft_lds<real, kNfftNT>(buf, S, A.ffts, A.ffts + A.fft_nt, A.tw, wR, true);
    // virtual ring t < nt/2 (pair p = t or nt/2 - 1 - t): its value plus its doubled-circle image
    const int NRv = nt / 2;
    for (int t = threadIdx.x; t < NRv; t += kNfftNT) {
        const int p = t < nt / 4 ? t : nt / 2 - 1 - t;
        const real f = (real)1 / (real)A.vs[p];
        const C2<real> a0 = buf[t], a1 = buf[nt - 1 - t];
        const C2<real> b0 = buf[S + t], b1 = buf[S + nt - 1 - t];
        C2<real> *o = reinterpret_cast<C2<real> *>(A.RB + ((size_t)am * NRv + t) * 8);
        const C2<real> vt = {(a0.x + ext * a1.x) * f, (a0.y + ext * a1.y) * f};
        const C2<real> vp = {(b0.x + ext * b1.x) * f, (b0.y + ext * b1.y) * f};
        o[slot] = vt;
        o[slot + 1] = vp;
        if (m == 0) {  // the -0 columns repeat +0 (unused by the recombination)
            o[2] = vt;
            o[3] = vp;
        }
    }
}

// ===========================================================================
// Batched stages: one launch per stage (and per workgroup shape) covers every
// field of a batch.  Workgroup i runs work item work[i] = (field, x, y) with the
// field's own argument block; the bodies are those of the single-field kernels.
// The first stage of each direction stamps its items' start and the last stage
// its items' end (wall clock) into `stamp`, from which per-field latencies are
// read.
// ===========================================================================
__device__ __forceinline__ void stamp_now(unsigned long long *stamp) {
    if (stamp && threadIdx.x == 0) stamp[blockIdx.x] = wall_clock64();
}

template <typename real>
__global__ __launch_bounds__(256) void kb_prep(const CoefArgs<real> *__restrict__ args,
                                               const WorkItem *__restrict__ work,
                                               unsigned long long *stamp) {
    const WorkItem w = ld_const(work + blockIdx.x);
    stamp_now(stamp);
    const CoefArgs<real> A = ld_const(args + w.f);
    prep_body(A, w.x, w.y);
}

template <typename real>
__global__ __launch_bounds__(256) void kb_recombine(const CoefArgs<real> *__restrict__ args,
                                                    const WorkItem *__restrict__ work,
                                                    unsigned long long *stamp) {
    const WorkItem w = ld_const(work + blockIdx.x);
    const CoefArgs<real> A = ld_const(args + w.f);
    recombine_body(A, w.x, w.y);
    __syncthreads();
    stamp_now(stamp);
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, 2) void kb_ring_fwd(const RingArgs<real> *__restrict__ args,
                                                          const WorkItem *__restrict__ work,
                                                          unsigned long long *stamp) {
    extern __shared__ unsigned char smem_raw[];
    const WorkItem w = ld_const(work + blockIdx.x);
    stamp_now(stamp);
    const RingArgs<real> A = ld_const(args + w.f);
    ring_fwd_body<real, NT>(A, w.x, smem_raw);
}

template <typename real, int NT>
__global__ __launch_bounds__(NT, 2) void kb_ring_adj(const RingArgs<real> *__restrict__ args,
                                                          const WorkItem *__restrict__ work,
                                                          unsigned long long *stamp) {
    extern __shared__ unsigned char smem_raw[];
    const WorkItem w = ld_const(work + blockIdx.x);
    const RingArgs<real> A = ld_const(args + w.f);
    ring_adj_body<real, NT>(A, w.x, smem_raw);
    __syncthreads();
    stamp_now(stamp);
}

// work item (field, m, -): every tile of the field's pairs in one workgroup
template <typename real, int kBf16>
__global__ __launch_bounds__(1024) void kb_leg_fwd(const LegFwdArgs<real> *__restrict__ args,
                                                   const WorkItem *__restrict__ work,
                                                   unsigned long long *) {
    extern __shared__ unsigned char smem_raw[];
    const WorkItem w = ld_const(work + blockIdx.x);
    const LegFwdArgs<real> A = ld_const(args + w.f);
    if constexpr (kBf16 != 0)
        leg_fwd_bf16_body<kBf16>(A, w.x, 0, smem_raw);
    else if constexpr (sizeof(real) == 8)
        leg_fwd_f64q_body(A, w.x, 0, smem_raw);
    else
        leg_fwd_body(A, w.x, 0, smem_raw);
}

// work item (field, x, m): the synthesis workgroup column x of order m (leg_adj_group)
template <typename real, int kBf16>
__global__ __launch_bounds__(256, kBf16 == 0 ? 4 : 1) void kb_leg_adj(const LegArgs<real> *__restrict__ args,
                                                  const WorkItem *__restrict__ work,
                                                  unsigned long long *) {
    extern __shared__ unsigned char smem_raw[];
    const WorkItem w = ld_const(work + blockIdx.x);
    const LegArgs<real> A = ld_const(args + w.f);
    leg_adj_group<real, kBf16>(A, w.y, w.x, smem_raw);
}

template <typename real>
__global__ __launch_bounds__(256) void kb_equator_adj(const LegArgs<real> *__restrict__ args,
                                                     const WorkItem *__restrict__ work,
                                                     unsigned long long *) {
    const WorkItem w = ld_const(work + blockIdx.x);
    const LegArgs<real> A = ld_const(args + w.f);
    equator_adj_body(A, w.x);
}

// ---------------------------------------------------------------------------
// Scalar transforms (FwdSHT and AdjSHT) on the same stages.  Lambda_{l,m} is
// normalised so that Y_{l,m} = Lambda_{l,m} e^{i m phi} (the 1/sqrt(4 pi) and the
// Condon-Shortley phase are in the seeds), and Y_{l,-m} = (-1)^m conj(Y_{l,m}).  The
// theta column of the spin-frame analysis of T_theta = s f is then
// F_{l,+m} = sum_k w_k f_k Lambda_{l,m} e^{-i m phi_k} = f_{l,m}, and its -m slot holds
// (-1)^m f_{l,-m}; the synthesis from g^th = f_{l,m} (and g^ph = 0) gives
// s T_theta = S_L(f).  Coefficients f_{l,m}, 0 <= l <= L, |m| <= l, at index l^2 + l + m.
// ---------------------------------------------------------------------------
template <typename real>
struct ShtArgs {
    const C2<real> *flm_in;
    C2<real> *flm_out;
    C2<real> *FG;           // [tri][4]
    double *FG64;           // binary32 paths: FG in binary64 (see prep_body)
    const double *cscale;   // [tri] c_{l',m}
    int L;
};

// one thread per triangle row (m, l'), l' = m .. L+1: FG from f_{l',+-m}
template <typename real>
__global__ __launch_bounds__(256) void k_sht_coef_to_fg(ShtArgs<real> A) {
    const int L = A.L;
    const int m = blockIdx.y;
    const int lp = m + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m > L || lp > L + 1) return;
    const int64_t ti = tri_offset(L, m) + lp - m;
    C2<double> gp = {0, 0}, gm = {0, 0};
    if (lp <= L) {
        const double sc = A.cscale[ti];
        const C2<real> fp = A.flm_in[(int64_t)lp * lp + lp + m];
        gp = {sc * (double)fp.x, sc * (double)fp.y};
        if (m > 0) {
            const C2<real> fm = A.flm_in[(int64_t)lp * lp + lp - m];
            const double sg = (m & 1) ? -sc : sc;
            gm = {sg * (double)fm.x, sg * (double)fm.y};
        }
    }
    C2<real> *o = A.FG + ti * 4;
    const C2<real> hp = {(real)gp.x, (real)gp.y}, hm = {(real)gm.x, (real)gm.y};
    o[0] = hp;
    o[1] = {0, 0};
    o[2] = hm;
    o[3] = {0, 0};
    if constexpr (sizeof(real) == 4) {
        C2<double> *o64 = reinterpret_cast<C2<double> *>(A.FG64) + ti * 4;
        o64[0] = gp;
        o64[1] = {0, 0};
        o64[2] = gm;
        o64[3] = {0, 0};
    }
}

// one thread per (m, l), l = m .. L: f_{l,+-m} from the theta columns of FG
template <typename real>
__global__ __launch_bounds__(256) void k_sht_fg_to_coef(ShtArgs<real> A) {
    const int L = A.L;
    const int m = blockIdx.y;
    const int l = m + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (m > L || l > L) return;
    const int64_t ti = tri_offset(L, m) + l - m;
    const C2<real> *r = A.FG + ti * 4;
    A.flm_out[(int64_t)l * l + l + m] = r[0];
    if (m > 0) {
        const C2<real> v = r[2];
        A.flm_out[(int64_t)l * l + l - m] = (m & 1) ? C2<real>{-v.x, -v.y} : v;
    }
}

// ===========================================================================
// launchers
// ===========================================================================
static size_t ring_lds_bytes_len(int64_t len, size_t real_size) {
    static_assert(sizeof(CD) == 2 * sizeof(double), "cos/sin table entries are two binary64");
    return ring_lds_bytes_for(len, real_size);
}
static size_t ring_lds_bytes(const Plan &p, size_t real_size) { return ring_lds_bytes_len(p.max_fft_len, real_size); }

template <typename real>
static RingArgs<real> make_ring_args(const Plan &p, const void *Tin, void *Tout, bool weighted) {
    RingArgs<real> R{};
    R.Tin = static_cast<const C2<real> *>(Tin);
    R.Tout = static_cast<C2<real> *>(Tout);
    R.weights = p.d_weights;
    R.buf = static_cast<C2<real> *>(p.d_pb);
    R.rings = p.d_rings;
    R.pairs = p.d_pairs;
    R.ffts = p.d_ffts;
    R.tw = p.d_tw;
    R.L = p.L;
    R.NP = (int)p.n_pairs;
    R.NR = (int)p.n_rings;
    R.weighted = weighted ? 1 : 0;
    R.scalar = 0;
    return R;
}

static int pairs_in_tiles(const Plan &p) { return (int)(p.n_pairs - (p.eq_ring >= 0 ? 1 : 0)); }
static int tiles_of(const Plan &p) { return (pairs_in_tiles(p) + kTileP - 1) / kTileP; }
// Products per product of a split-bf16 precision (0 for binary64 and binary32).
static int bf16_products(int precision) {
    return precision == VSHT_BF16X3 ? 3 : precision == VSHT_BF16X6 ? 6 : 0;
}

// Analysis grid: one workgroup per order m holds up to 16 tiles (waves); plans
// with more tiles split them over `groups` workgroups, each writing a partial
// triangle into the plan's group buffer, which k_sum_groups adds up in a fixed order.
static int fwd_groups(const Plan &p) { return analysis_groups(p.n_pairs, p.eq_ring); }

template <typename real>
static LegFwdArgs<real> make_leg_fwd_args(const Plan &p, int groups) {
    LegFwdArgs<real> G{};
    G.RB = static_cast<const real *>(p.d_pb);
    G.F = static_cast<real *>(groups > 1 ? p.d_fpart : p.d_fg);
    G.gstride = groups > 1 ? p.tri_size * 8 : 0;
    G.pairs = p.d_pairs;
    G.seeds = p.d_seeds;
    G.start = p.d_start;
    G.sblk = p.d_sblk;
    G.pz = p.d_pair_z;
    G.aprime = p.d_aprime;
    G.cscale = p.d_cscale;
    G.L = p.L;
    G.NP = (int)p.n_pairs;
    G.NPT = pairs_in_tiles(p);
    G.NR = (int)p.n_rings;
    G.eq_ring = p.eq_ring;
    return G;
}

template <typename real>
static LegArgs<real> make_leg_adj_args(const Plan &p) {
    LegArgs<real> G{};
    G.FG = static_cast<const real *>(p.d_fg);
    G.FG64 = p.precision == VSHT_FP64 ? static_cast<const double *>(p.d_fg) : static_cast<const double *>(p.d_fg64);

    G.PB = static_cast<real *>(p.d_pb);
    G.seeds = p.d_seeds;
    G.start = p.d_start;
    G.sblk = p.d_sblk;
    G.pz = p.d_pair_z;
    G.aprime = p.d_aprime;
    G.L = p.L;
    G.NP = (int)p.n_pairs;
    G.NPT = pairs_in_tiles(p);
    return G;
}

// recombine (forward): FG -> aout, bout;  prep (adjoint): ain, bin -> FG
template <typename real>
static CoefArgs<real> make_coef_args(const Plan &p, const void *ain, const void *bin, void *aout, void *bout) {
    CoefArgs<real> C{};
    C.FG = static_cast<const C2<real> *>(p.d_fg);
    C.FGout = static_cast<C2<real> *>(p.d_fg);
    C.ain = static_cast<const C2<real> *>(ain);
    C.bin = static_cast<const C2<real> *>(bin);
    C.aout = static_cast<C2<real> *>(aout);
    C.bout = static_cast<C2<real> *>(bout);
    C.cscale = p.d_cscale;
    C.etab = p.d_etab;
    C.rsq = p.d_rsq;
    C.FG64 = static_cast<double *>(p.d_fg64);
    // the binary32 synthesis reads only FG64; the split-bf16 tiles and the direct
    // scattered evaluation read the binary32 triangle
    C.fg32 = p.precision != VSHT_FP32 || (p.kind == VSHT_PLAN_SCATTERED && !p.nfft.on);
    C.L = p.L;
    return C;
}

static size_t leg_fwd_lds(int nw, size_t rsz) { return (size_t)nw * (kRowsB * kTileP + 2 * 128) * rsz; }

// Synthesis grid: workgroup columns x orders.
template <typename real>
static dim3 adj_grid(const LegArgs<real> &G, int nprod) {
    return dim3((unsigned)adj_columns(G.NPT, nprod), (unsigned)(G.L + 1));
}

// Analysis and synthesis launches in the plan's arithmetic.
template <typename real>
static void launch_leg_fwd(const LegFwdArgs<real> &G, dim3 grid, int nw, int nprod, hipStream_t st) {
    if constexpr (sizeof(real) == 4) {
        if (nprod == 3)
            hipLaunchKernelGGL(k_leg_fwd_bf16<3>, grid, dim3(nw * 64), leg_fwd_lds(nw, 4), st, G);
        else if (nprod == 6)
            hipLaunchKernelGGL(k_leg_fwd_bf16<6>, grid, dim3(nw * 64), leg_fwd_lds(nw, 4), st, G);
        else
            hipLaunchKernelGGL(k_leg_fwd_mfma<real>, grid, dim3(nw * 64), leg_fwd_lds(nw, 4), st, G);
    } else {
        hipLaunchKernelGGL(k_leg_fwd_mfma<real>, grid, dim3(nw * 64), leg_fwd_lds(nw, 8), st, G);
    }
}
template <typename real>
static void launch_leg_adj(const LegArgs<real> &G, dim3 grid, int nprod, hipStream_t st) {
    if constexpr (sizeof(real) == 4) {
        if (nprod == 3)
            hipLaunchKernelGGL((k_leg_adj<float, 3>), grid, dim3(256), adj_lds_block<3>(), st, G);
        else if (nprod == 6)
            hipLaunchKernelGGL((k_leg_adj<float, 6>), grid, dim3(256), adj_lds_block<6>(), st, G);
        else
            hipLaunchKernelGGL((k_leg_adj<float, 0>), grid, dim3(64 * adj_waves(G.NPT, 0)), adj_lds_block<0>(), st,
                               G);
    } else {
        hipLaunchKernelGGL((k_leg_adj<double, 0>), grid, dim3(64 * adj_waves(G.NPT, 0)), adj_lds_block<0>(), st, G);
    }
}

template <typename real>
static NfftArgs<real> make_nfft_args(const Plan &p, const void *Tin, void *Tout, bool weighted) {
    const NfftPlan &nf = p.nfft;
    NfftArgs<real> N{};
    N.PB = static_cast<const real *>(nf.d_vpb);
    N.RB = static_cast<real *>(nf.d_vpb);
    N.g1 = static_cast<C2<real> *>(nf.d_g1);
    N.g = static_cast<C2<real> *>(nf.d_g);
    N.vs = nf.d_vs;
    N.psihat = nf.d_psihat;
    N.ffts = nf.d_ffts;
    N.tw = nf.d_tw;
    N.pts = nf.d_pts;
    N.tiles = nf.d_tiles;
    N.weights = p.d_weights;
    N.Tin = static_cast<const C2<real> *>(Tin);
    N.Tout = static_cast<C2<real> *>(Tout);
    N.n = p.n;
    N.beta = nf.beta;
    N.h = 2.0 * M_PI / nf.ng;
    N.fft_nt = nf.fft_nt;
    N.fft_ng = nf.fft_ng;
    N.L = p.L;
    N.nt = nf.nt;
    N.npv = nf.npv;
    N.ng = nf.ng;
    N.w = nf.w;
    N.stride = (int)nf.lds_stride;
    N.weighted = weighted ? 1 : 0;
    return N;
}

// Intermediate buffers of a forward transform: the plan's workspace, or the
// static scratch array (allocation-free entry point, no stage timing).
// Buffers of one launch sequence.  count fields run together (blockIdx.z); field f
// uses the workspace at f times the per-field strides (bytes) and the caller's
// field and coefficients at f times their strides (complex elements).
struct FwdWork {
    void *rb, *fg, *fpart;
    bool timed;
    int count = 1;
    int64_t zb_rb = 0, zb_fg = 0, zb_fpart = 0;
    int64_t zs_T = 0, zs_coef = 0;
};
struct AdjWork {
    void *pb, *fg, *fg64;
    int count = 1;
    int64_t zb_pb = 0, zb_fg = 0, zb_fg64 = 0;
    int64_t zs_T = 0, zs_coef = 0;
};

template <typename real>
static hipError_t forward_impl(const Plan &p, const FwdWork &ws, const void *T, void *a, void *b, bool weighted,
                               hipStream_t st) {
    const int nprod = bf16_products(p.precision);
    if (p.kind == VSHT_PLAN_SCATTERED) {
        // scattered points: spread, grid DFTs, virtual-ring values, then the ring analysis
        const NfftPlan &nf = p.nfft;
        const NfftArgs<real> N = make_nfft_args<real>(p, T, nullptr, weighted);
        const size_t lds = ring_lds_bytes_len(nf.lds_stride, sizeof(real));
        {
            StageScope sc(p, VSHT_STAGE_SCATTERED, st);
            const int64_t gsize = (int64_t)2 * nf.ng * nf.ng * 2;
            hipLaunchKernelGGL(k_fill_zero<real>, dim3((unsigned)((gsize + 255) / 256)), dim3(256), 0, st,
                               static_cast<real *>(nf.d_g), gsize);
            hipLaunchKernelGGL(k_nfft_spread<real>, dim3((unsigned)((p.n + 255) / 256)), dim3(256), 0, st, N);
            hipLaunchKernelGGL(k_nfft_rows_fwd<real>, dim3(nf.ng), dim3(kNfftNT), lds, st, N);
            hipLaunchKernelGGL(k_nfft_cols_fwd<real>, dim3(2 * p.L + 1), dim3(kNfftNT), lds, st, N);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        LegFwdArgs<real> G{};
        G.RB = static_cast<const real *>(nf.d_vpb);
        G.F = static_cast<real *>(p.d_fg);
        G.pairs = nf.d_vpairs;
        G.seeds = nf.d_vseeds;
        G.start = nf.d_vstart;
        G.sblk = nf.d_vsblk;
        G.pz = nf.d_vz;
        G.aprime = p.d_aprime;
        G.cscale = p.d_cscale;
        G.L = p.L;
        G.NP = nf.npv;
        G.NPT = nf.npv;
        G.NR = nf.nt / 2;
        G.eq_ring = -1;
        G.gstride = 0;
        {
            const int ntile = (nf.npv + kTileP - 1) / kTileP;  // <= 16 for the bandlimits served
            StageScope sc(p, VSHT_STAGE_LEG_FWD, st);
            launch_leg_fwd<real>(G, dim3(p.L + 1, 1), ntile, nprod, st);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const CoefArgs<real> C = make_coef_args<real>(p, nullptr, nullptr, a, b);
        {
            StageScope sc(p, VSHT_STAGE_RECOMBINE, st);
            hipLaunchKernelGGL(k_recombine<real>, dim3((p.L + kTL - 1) / kTL, (p.L + 1 + kTM - 1) / kTM),
                               dim3(256), 0, st, C);
        }
        return hipGetLastError();
    }
    const unsigned nf = (unsigned)ws.count;
    RingArgs<real> R = make_ring_args<real>(p, T, nullptr, weighted);
    R.buf = static_cast<C2<real> *>(ws.rb);
    R.zs_T = ws.zs_T;
    R.zs_buf = ws.zb_rb / (int64_t)sizeof(C2<real>);
    {
        StageScope sc(p, VSHT_STAGE_RING_FWD, st, ws.timed);
        if (p.ring_nt_min == kRingNTSmall && p.max_fft_len <= kMaxLenSmallRing)
            hipLaunchKernelGGL((k_ring_fwd<real, kRingNTSmall>), dim3((unsigned)p.n_rings, 1, nf),
                               dim3(kRingNTSmall), ring_lds_bytes(p, sizeof(real)), st, R);
        else
            hipLaunchKernelGGL((k_ring_fwd<real, kRingNT>), dim3((unsigned)p.n_rings, 1, nf), dim3(kRingNT),
                               ring_lds_bytes(p, sizeof(real)), st, R);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int ntile = tiles_of(p);
        const int ngroup = fwd_groups(p);  // at most 16 waves per workgroup
        const int nw = ntile > 0 ? (ntile + ngroup - 1) / ngroup : 1;
        LegFwdArgs<real> G = make_leg_fwd_args<real>(p, ngroup);
        G.RB = static_cast<const real *>(ws.rb);
        G.F = static_cast<real *>(ngroup > 1 ? ws.fpart : ws.fg);
        G.zs_RB = ws.zb_rb / (int64_t)sizeof(real);
        G.zs_F = (ngroup > 1 ? ws.zb_fpart : ws.zb_fg) / (int64_t)sizeof(real);
        StageScope sc(p, VSHT_STAGE_LEG_FWD, st, ws.timed);
        launch_leg_fwd<real>(G, dim3(p.L + 1, ngroup, nf), nw, nprod, st);
        if (ngroup > 1)
            hipLaunchKernelGGL(k_sum_groups<real>, dim3((unsigned)((p.tri_size * 8 + 255) / 256), 1, nf), dim3(256),
                               0, st, static_cast<const real *>(ws.fpart), static_cast<real *>(ws.fg),
                               p.tri_size * 8, ngroup, ws.zb_fpart / (int64_t)sizeof(real),
                               ws.zb_fg / (int64_t)sizeof(real));
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    CoefArgs<real> C = make_coef_args<real>(p, nullptr, nullptr, a, b);
    C.FG = static_cast<const C2<real> *>(ws.fg);
    C.zs_FG = ws.zb_fg / (int64_t)sizeof(C2<real>);
    C.zs_coef = ws.zs_coef;
    {
        StageScope sc(p, VSHT_STAGE_RECOMBINE, st, ws.timed);
        hipLaunchKernelGGL(k_recombine<real>, dim3((p.L + kTL - 1) / kTL, (p.L + 1 + kTM - 1) / kTM, nf),
                           dim3(256), 0, st, C);
    }
    return hipGetLastError();
}

template <typename real>
static hipError_t adjoint_impl(const Plan &p, const AdjWork &ws, const void *a, const void *b, void *T,
                               bool weighted, hipStream_t st) {
    const int nprod = bf16_products(p.precision);
    const unsigned nf = (unsigned)ws.count;
    CoefArgs<real> C = make_coef_args<real>(p, a, b, nullptr, nullptr);
    C.FG = static_cast<const C2<real> *>(ws.fg);
    C.FGout = static_cast<C2<real> *>(ws.fg);
    C.FG64 = static_cast<double *>(ws.fg64);
    C.zs_FG = ws.zb_fg / (int64_t)sizeof(C2<real>);
    C.zs_coef = ws.zs_coef;
    C.zs_FG64 = ws.zb_fg64 / (int64_t)sizeof(double);
    {
        StageScope sc(p, VSHT_STAGE_PREP, st);
        hipLaunchKernelGGL(k_prep<real>, dim3((p.L + 2 + kTL - 1) / kTL, (p.L + 1 + kTM - 1) / kTM, nf),
                           dim3(256), 0, st, C);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;

    if (p.kind == VSHT_PLAN_SCATTERED && p.nfft.on) {
        const NfftPlan &nf = p.nfft;
        LegArgs<real> G{};
        G.FG = static_cast<const real *>(p.d_fg);
        G.PB = static_cast<real *>(nf.d_vpb);
        G.seeds = nf.d_vseeds;
        G.start = nf.d_vstart;
        G.sblk = nf.d_vsblk;
        G.pz = nf.d_vz;
        G.aprime = p.d_aprime;
        G.L = p.L;
        G.NP = nf.npv;
        G.NPT = nf.npv;
        G.FG64 = p.precision == VSHT_FP64 ? static_cast<const double *>(p.d_fg)
                                          : static_cast<const double *>(p.d_fg64);
        {
            StageScope sc(p, VSHT_STAGE_LEG_ADJ, st);
            launch_leg_adj<real>(G, adj_grid(G, nprod), nprod, st);
        }
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        const NfftArgs<real> N = make_nfft_args<real>(p, nullptr, T, weighted);
        const size_t lds = ring_lds_bytes_len(nf.lds_stride, sizeof(real));
        StageScope sc(p, VSHT_STAGE_SCATTERED, st);
        hipLaunchKernelGGL(k_nfft_cols<real>, dim3(2 * p.L + 1), dim3(kNfftNT), lds, st, N);
        hipLaunchKernelGGL(k_nfft_rows<real>, dim3(nf.ng), dim3(kNfftNT), lds, st, N);
        hipLaunchKernelGGL(k_nfft_gather<real>, dim3((unsigned)nf.ntiles), dim3(256), 0, st, N);
        return hipGetLastError();
    }

    if (p.kind == VSHT_PLAN_SCATTERED) {
        ScatArgs<real> S{};
        S.FG = static_cast<const C2<real> *>(p.d_fg);
        S.xyz = p.d_xyz;
        S.aprime = p.d_aprime;
        S.cscale = p.d_cscale;
        S.Tout = static_cast<C2<real> *>(T);
        S.weights = p.d_weights;
        S.n = p.n;
        S.L = p.L;
        S.weighted = weighted ? 1 : 0;
        StageScope sc(p, VSHT_STAGE_SCATTERED, st);
        hipLaunchKernelGGL(k_adj_scattered<real>, dim3((unsigned)((p.n + 63) / 64)), dim3(64), 0,
                           st, S);
        return hipGetLastError();
    }

    LegArgs<real> G = make_leg_adj_args<real>(p);
    G.FG = static_cast<const real *>(ws.fg);
    G.FG64 = p.precision == VSHT_FP64 ? static_cast<const double *>(ws.fg) : static_cast<const double *>(ws.fg64);
    G.PB = static_cast<real *>(ws.pb);
    G.zs_FG = ws.zb_fg / (int64_t)sizeof(real);
    G.zs_FG64 = (p.precision == VSHT_FP64 ? ws.zb_fg : ws.zb_fg64) / (int64_t)sizeof(double);
    G.zs_PB = ws.zb_pb / (int64_t)sizeof(real);
    {
        StageScope sc(p, VSHT_STAGE_LEG_ADJ, st);
        dim3 grid = adj_grid(G, nprod);
        grid.z = nf;
        launch_leg_adj<real>(G, grid, nprod, st);
        if (p.eq_ring >= 0 && nprod != 0)  // the vector-unit synthesis forms the equator itself
            hipLaunchKernelGGL(k_equator_adj<real>, dim3(p.L + 1, 1, nf), dim3(256), 0, st, G);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;

    RingArgs<real> R = make_ring_args<real>(p, nullptr, T, weighted);
    R.buf = static_cast<C2<real> *>(ws.pb);
    R.zs_T = ws.zs_T;
    R.zs_buf = ws.zb_pb / (int64_t)sizeof(C2<real>);
    {
        StageScope sc(p, VSHT_STAGE_RING_ADJ, st);
        const dim3 grid((unsigned)(16 * ((p.n_pairs + 7) / 8)), 1, nf);  // ring_of_block's layout
        if (p.ring_nt_min == kRingNTSmall && p.max_fft_len <= kMaxLenSmallRing)
            hipLaunchKernelGGL((k_ring_adj<real, kRingNTSmall>), grid, dim3(kRingNTSmall),
                               ring_lds_bytes(p, sizeof(real)), st, R);
        else
            hipLaunchKernelGGL((k_ring_adj<real, kRingNT>), grid, dim3(kRingNT),
                               ring_lds_bytes(p, sizeof(real)), st, R);
    }
    return hipGetLastError();
}

hipError_t launch_forward(const Plan &p, const void *T, void *a, void *b, bool weighted,
                          hipStream_t st) {
    const FwdWork ws{p.d_pb, p.d_fg, p.d_fpart, true};
    if (p.precision == VSHT_FP64) return forward_impl<double>(p, ws, T, a, b, weighted, st);
    return forward_impl<float>(p, ws, T, a, b, weighted, st);
}

hipError_t launch_adjoint(const Plan &p, const void *a, const void *b, void *T, bool weighted,
                          hipStream_t st) {
    const AdjWork ws{p.d_pb, p.d_fg, p.d_fg64};
    if (p.precision == VSHT_FP64) return adjoint_impl<double>(p, ws, a, b, T, weighted, st);
    return adjoint_impl<float>(p, ws, a, b, T, weighted, st);
}

// count fields of a ring plan in one launch per stage, with the per-field workspace
// (field_ws_bytes(p) each) at ws, laid out as [count][pb], [count][fg], [count][fg64],
// [count][fpart].
static void many_layout(const Plan &p, int count, void *ws, FwdWork *fw, AdjWork *aw) {
    const ManyWs z = field_ws(p);
    char *base = static_cast<char *>(ws);
    char *pb = base, *fg = pb + (size_t)count * z.pb, *fg64 = fg + (size_t)count * z.fg;
    char *fpart = fg64 + (size_t)count * z.fg64;
    const int64_t zs_T = p.n * 3, zs_coef = (int64_t)p.L * (p.L + 2);
    if (fw) {
        *fw = FwdWork{pb, fg, z.fpart ? fpart : nullptr, true};
        fw->count = count;
        fw->zb_rb = (int64_t)z.pb;
        fw->zb_fg = (int64_t)z.fg;
        fw->zb_fpart = (int64_t)z.fpart;
        fw->zs_T = zs_T;
        fw->zs_coef = zs_coef;
    }
    if (aw) {
        *aw = AdjWork{pb, fg, z.fg64 ? fg64 : nullptr};
        aw->count = count;
        aw->zb_pb = (int64_t)z.pb;
        aw->zb_fg = (int64_t)z.fg;
        aw->zb_fg64 = (int64_t)z.fg64;
        aw->zs_T = zs_T;
        aw->zs_coef = zs_coef;
    }
}

hipError_t launch_forward_many(const Plan &p, int count, void *ws, const void *T, void *a, void *b,
                               bool weighted, hipStream_t st) {
    FwdWork w{};
    many_layout(p, count, ws, &w, nullptr);
    if (p.precision == VSHT_FP64) return forward_impl<double>(p, w, T, a, b, weighted, st);
    return forward_impl<float>(p, w, T, a, b, weighted, st);
}

hipError_t launch_adjoint_many(const Plan &p, int count, void *ws, const void *a, const void *b, void *T,
                               bool weighted, hipStream_t st) {
    AdjWork w{};
    many_layout(p, count, ws, nullptr, &w);
    if (p.precision == VSHT_FP64) return adjoint_impl<double>(p, w, a, b, T, weighted, st);
    return adjoint_impl<float>(p, w, a, b, T, weighted, st);
}

// Scalar transforms on ring plans: the ring and Legendre stages of the vector
// path with the scalar ring input/output and the coefficient kernels above.
template <typename real>
static hipError_t sht_forward_impl(const Plan &p, const void *f, void *flm, hipStream_t st) {
    const int nprod = bf16_products(p.precision);
    RingArgs<real> R = make_ring_args<real>(p, f, nullptr, true);
    R.scalar = 1;
    {
        StageScope sc(p, VSHT_STAGE_RING_FWD, st);
        if (p.ring_nt_min == kRingNTSmall && p.max_fft_len <= kMaxLenSmallRing)
            hipLaunchKernelGGL((k_ring_fwd<real, kRingNTSmall>), dim3((unsigned)p.n_rings), dim3(kRingNTSmall),
                               ring_lds_bytes(p, sizeof(real)), st, R);
        else
            hipLaunchKernelGGL((k_ring_fwd<real, kRingNT>), dim3((unsigned)p.n_rings), dim3(kRingNT),
                               ring_lds_bytes(p, sizeof(real)), st, R);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    {
        const int ntile = tiles_of(p);
        const int ngroup = fwd_groups(p);  // at most 16 waves per workgroup
        const int nw = ntile > 0 ? (ntile + ngroup - 1) / ngroup : 1;
        const LegFwdArgs<real> G = make_leg_fwd_args<real>(p, ngroup);
        StageScope sc(p, VSHT_STAGE_LEG_FWD, st);
        launch_leg_fwd<real>(G, dim3(p.L + 1, ngroup), nw, nprod, st);
        if (ngroup > 1)
            hipLaunchKernelGGL(k_sum_groups<real>, dim3((unsigned)((p.tri_size * 8 + 255) / 256)), dim3(256), 0,
                               st, static_cast<const real *>(p.d_fpart), static_cast<real *>(p.d_fg),
                               p.tri_size * 8, ngroup, (int64_t)0, (int64_t)0);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    ShtArgs<real> S{};
    S.flm_out = static_cast<C2<real> *>(flm);
    S.FG = static_cast<C2<real> *>(p.d_fg);
    S.cscale = p.d_cscale;
    S.L = p.L;
    StageScope sc(p, VSHT_STAGE_RECOMBINE, st);
    hipLaunchKernelGGL(k_sht_fg_to_coef<real>, dim3((p.L + 1 + 255) / 256, p.L + 1), dim3(256), 0, st, S);
    return hipGetLastError();
}

template <typename real>
static hipError_t sht_adjoint_impl(const Plan &p, const void *flm, void *f, hipStream_t st) {
    const int nprod = bf16_products(p.precision);
    ShtArgs<real> S{};
    S.flm_in = static_cast<const C2<real> *>(flm);
    S.FG = static_cast<C2<real> *>(p.d_fg);
    S.FG64 = static_cast<double *>(p.d_fg64);
    S.cscale = p.d_cscale;
    S.L = p.L;
    {
        StageScope sc(p, VSHT_STAGE_PREP, st);
        hipLaunchKernelGGL(k_sht_coef_to_fg<real>, dim3((p.L + 2 + 255) / 256, p.L + 1), dim3(256), 0, st, S);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    LegArgs<real> G = make_leg_adj_args<real>(p);
    {
        StageScope sc(p, VSHT_STAGE_LEG_ADJ, st);
        launch_leg_adj<real>(G, adj_grid(G, nprod), nprod, st);
        if (p.eq_ring >= 0 && nprod != 0)
            hipLaunchKernelGGL(k_equator_adj<real>, dim3(p.L + 1), dim3(256), 0, st, G);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    RingArgs<real> R = make_ring_args<real>(p, nullptr, f, false);
    R.scalar = 1;
    {
        StageScope sc(p, VSHT_STAGE_RING_ADJ, st);
        const dim3 grid((unsigned)(16 * ((p.n_pairs + 7) / 8)));  // ring_of_block's layout
        if (p.ring_nt_min == kRingNTSmall && p.max_fft_len <= kMaxLenSmallRing)
            hipLaunchKernelGGL((k_ring_adj<real, kRingNTSmall>), grid, dim3(kRingNTSmall),
                               ring_lds_bytes(p, sizeof(real)), st, R);
        else
            hipLaunchKernelGGL((k_ring_adj<real, kRingNT>), grid, dim3(kRingNT),
                               ring_lds_bytes(p, sizeof(real)), st, R);
    }
    return hipGetLastError();
}

hipError_t launch_sht_forward(const Plan &p, const void *f, void *flm, hipStream_t st) {
    if (p.precision == VSHT_FP64) return sht_forward_impl<double>(p, f, flm, st);
    return sht_forward_impl<float>(p, f, flm, st);
}

hipError_t launch_sht_adjoint(const Plan &p, const void *flm, void *f, hipStream_t st) {
    if (p.precision == VSHT_FP64) return sht_adjoint_impl<double>(p, flm, f, st);
    return sht_adjoint_impl<float>(p, flm, f, st);
}

// ===========================================================================
// Allocation-free forward: the ring buffer, the triangle and (over 1024 ring
// pairs) the partial triangles live in `scratch`, a static device array of
// kStaticScratchBytes that the loader reserves on every GPU the library runs
// on.  Its device address is looked up once per device (with that device
// current) and kept; host code uses only that address.  Calls that overlap on
// one GPU share the array and race.  The forward writes every element it later
// reads, so nothing needs clearing.
// ===========================================================================
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

hipError_t scratch_address(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

size_t static_forward_bytes(const Plan &p) {
    const size_t rsz = p.precision == VSHT_FP64 ? 8 : 4;
    const int groups = fwd_groups(p);
    const size_t rb = (size_t)(p.L + 1) * p.n_rings * 8 * rsz;
    const size_t fg = (size_t)(p.tri_size + kFgPadRows) * 8 * rsz;
    const size_t part = groups > 1 ? (size_t)groups * p.tri_size * 8 * rsz : 0;
    return round256(rb) + round256(fg) + round256(part);
}

hipError_t launch_forward_static(const Plan &p, const void *T, void *a, void *b, hipStream_t st) {
    if (p.kind != VSHT_PLAN_RINGS || static_forward_bytes(p) > kStaticScratchBytes) return hipErrorInvalidValue;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    unsigned char *base = nullptr;
    if ((e = scratch_address(dev, reinterpret_cast<void **>(&base))) != hipSuccess) return e;
    const size_t rsz = p.precision == VSHT_FP64 ? 8 : 4;
    const size_t rb = round256((size_t)(p.L + 1) * p.n_rings * 8 * rsz);
    const size_t fg = round256((size_t)(p.tri_size + kFgPadRows) * 8 * rsz);
    const FwdWork ws{base, base + rb, base + rb + fg, false};
    if (p.precision == VSHT_FP64) return forward_impl<double>(p, ws, T, a, b, true, st);
    return forward_impl<float>(p, ws, T, a, b, true, st);
}

// ===========================================================================
// Batches
// ===========================================================================
enum BatchStage { BS_PREP, BS_LEG_ADJ, BS_EQUATOR, BS_RING_ADJ, BS_RING_FWD, BS_LEG_FWD, BS_RECOMBINE };
static bool stage_is_adjoint(int s) { return s <= BS_RING_ADJ; }

struct BatchState {
    std::vector<const Plan *> f;
    int precision = VSHT_FP64;
    size_t rsz = 8;
    BatchConfig cfg;
    // per-field argument blocks, host copies and device tables
    std::vector<unsigned char> h_prep, h_ladj, h_radj, h_rfwd, h_lfwd, h_rec;
    void *d_prep = nullptr, *d_ladj = nullptr, *d_radj = nullptr, *d_rfwd = nullptr,
         *d_lfwd = nullptr, *d_rec = nullptr;
    // work lists: launches in execution order (adjoint stages, then forward), per chain
    struct Launch {
        int stage;
        int nw;
        int64_t off, cnt;
        size_t lds;
        int chain;
    };
    // Size-class chains: the fields are split by cost into up to kBatchChains
    // classes, each running its whole stage sequence on its own stream (parallel
    // branches of the captured graph), so that small fields do not wait for the
    // stages of the large ones.
    std::vector<int> chain_of;  // per field
    int nchains = 1;
    hipStream_t cs[kBatchChains] = {};
    hipEvent_t fork = nullptr, join[kBatchChains] = {};
    std::vector<WorkItem> work;
    std::vector<Launch> launches;
    WorkItem *d_work = nullptr;
    size_t d_work_cap = 0;
    unsigned long long *d_stamp = nullptr;
    size_t d_stamp_cap = 0;
};

template <typename T>
static hipError_t alloc_table(void **d, std::vector<unsigned char> &h, size_t count) {
    h.assign(sizeof(T) * count, 0);
    return hipMalloc(d, h.size());
}

template <typename real>
static hipError_t batch_alloc_args(BatchState *b) {
    const size_t F = b->f.size();
    hipError_t e;
    if ((e = alloc_table<CoefArgs<real>>(&b->d_prep, b->h_prep, F)) != hipSuccess) return e;
    if ((e = alloc_table<LegArgs<real>>(&b->d_ladj, b->h_ladj, F)) != hipSuccess) return e;
    if ((e = alloc_table<RingArgs<real>>(&b->d_radj, b->h_radj, F)) != hipSuccess) return e;
    if ((e = alloc_table<RingArgs<real>>(&b->d_rfwd, b->h_rfwd, F)) != hipSuccess) return e;
    if ((e = alloc_table<LegFwdArgs<real>>(&b->d_lfwd, b->h_lfwd, F)) != hipSuccess) return e;
    if ((e = alloc_table<CoefArgs<real>>(&b->d_rec, b->h_rec, F)) != hipSuccess) return e;
    // the buffer-independent blocks
    auto *la = reinterpret_cast<LegArgs<real> *>(b->h_ladj.data());
    auto *lf = reinterpret_cast<LegFwdArgs<real> *>(b->h_lfwd.data());
    for (size_t i = 0; i < F; ++i) {
        la[i] = make_leg_adj_args<real>(*b->f[i]);
        lf[i] = make_leg_fwd_args<real>(*b->f[i], 1);
    }
    if ((e = hipMemcpy(b->d_ladj, b->h_ladj.data(), b->h_ladj.size(), hipMemcpyHostToDevice)) != hipSuccess)
        return e;
    return hipMemcpy(b->d_lfwd, b->h_lfwd.data(), b->h_lfwd.size(), hipMemcpyHostToDevice);
}

hipError_t batch_create(const std::vector<const Plan *> &fields, BatchState **out) {
    *out = nullptr;
    auto *b = new (std::nothrow) BatchState();
    if (!b) return hipErrorOutOfMemory;
    b->f = fields;
    b->precision = fields.empty() ? VSHT_FP64 : fields[0]->precision;
    b->rsz = b->precision == VSHT_FP64 ? 8 : 4;
    // chains: cost (~L^3) classes of the fields; the first holds the cheapest fields up to
    // 1/8 of the batch's work, the second up to 1/2, the third the rest
    const int F = (int)fields.size();
    b->chain_of.assign(F, 0);
    if (kBatchChainsEnabled && F >= kBatchChains) {
        std::vector<int> order(F);
        for (int i = 0; i < F; ++i) order[i] = i;
        auto cost = [&](int i) { return std::pow((double)fields[i]->L + 1.0, 3.0); };
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) < cost(y); });
        double total = 0.0, acc = 0.0;
        for (int i = 0; i < F; ++i) total += cost(i);
        for (int i : order) {
            acc += cost(i);
            b->chain_of[i] = acc <= total / 8 ? 0 : acc <= total / 2 ? 1 : 2;
        }
        b->nchains = 1 + *std::max_element(b->chain_of.begin(), b->chain_of.end());
    }
    hipError_t e = hipSuccess;
    if (b->nchains > 1) {
        e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
        for (int c = 0; c < b->nchains && e == hipSuccess; ++c) {
            e = hipStreamCreateWithFlags(&b->cs[c], hipStreamNonBlocking);  // default priority
            if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join[c], hipEventDisableTiming);
        }
    }
    if (e == hipSuccess)
        e = b->precision == VSHT_FP64 ? batch_alloc_args<double>(b) : batch_alloc_args<float>(b);
    if (e == hipSuccess) e = batch_configure(b, BatchConfig{});
    if (e != hipSuccess) {
        batch_destroy(b);
        return e;
    }
    *out = b;
    return hipSuccess;
}

void batch_destroy(BatchState *b) {
    if (!b) return;
    for (int c = 0; c < kBatchChains; ++c) {
        if (b->cs[c]) (void)hipStreamDestroy(b->cs[c]);
        if (b->join[c]) (void)hipEventDestroy(b->join[c]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    void *ptrs[] = {b->d_prep, b->d_ladj, b->d_radj, b->d_rfwd, b->d_lfwd, b->d_rec, b->d_work, b->d_stamp};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    delete b;
}

BatchConfig batch_config(const BatchState *b) { return b->cfg; }


// Work lists for a configuration.  Item costs (for the longest-first order):
// ring stages n_phi, Legendre stages (degrees of the order) x (tiles in the
// workgroup), coefficient tiles 1.
hipError_t batch_configure(BatchState *b, const BatchConfig &cfg) {
    if (cfg.adj_nw != 1 && cfg.adj_nw != 2 && cfg.adj_nw != 4) return hipErrorInvalidValue;
    if (cfg.ring_nt != kRingNTSmall && cfg.ring_nt != kRingNT) return hipErrorInvalidValue;
    b->cfg = cfg;
    b->work.clear();
    b->launches.clear();
    const size_t rsz = b->rsz;
    const int nprod = bf16_products(b->precision);
    struct Item {
        WorkItem w;
        double cost;
    };
    const int nchains = cfg.chains ? b->nchains : 1;
    int chain = 0;
    auto emit = [&](int stage, int nw, std::vector<Item> &items, size_t lds) {
        if (items.empty()) return;
        if (cfg.lpt)
            std::stable_sort(items.begin(), items.end(),
                             [](const Item &x, const Item &y) { return x.cost > y.cost; });
        BatchState::Launch l{stage, nw, (int64_t)b->work.size(), (int64_t)items.size(), lds, chain};
        for (auto &it : items) b->work.push_back(it.w);
        b->launches.push_back(l);
    };
    const int F = (int)b->f.size();
    std::vector<Item> items;
    for (chain = 0; chain < nchains; ++chain) {
        // the fields of this chain
        auto skip = [&](int i) { return nchains > 1 && b->chain_of[i] != chain; };
        // prep
        for (int i = 0; i < F; ++i) {
            if (skip(i)) continue;
            const int L = b->f[i]->L;
            for (int by = 0; by * kTM <= L; ++by)
                for (int bx = 0; bx * kTL < L + 2; ++bx)
                    if (!(by * kTM > bx * kTL + kTL - 1)) items.push_back({{i, bx, by, 0}, 1.0});
        }
        emit(BS_PREP, 4, items, 0);
        items.clear();
        // Legendre synthesis: the single plans' workgroups of every field, one launch per
        // workgroup width (the vector-unit form sizes its workgroups to the field's pairs)
        for (int nw = 1; nw <= 4; ++nw) {
            for (int i = 0; i < F; ++i) {
                const Plan &p = *b->f[i];
                if (skip(i) || adj_waves(pairs_in_tiles(p), nprod) != nw) continue;
                const int cols = adj_columns(pairs_in_tiles(p), nprod);
                for (int x = 0; x < cols; ++x)
                    for (int m = 0; m <= p.L; ++m) items.push_back({{i, x, m, 0}, (double)(p.L + 2 - m) * nw});
            }
            emit(BS_LEG_ADJ, nw, items,
                 nprod == 3 ? adj_lds_block<3>() : nprod == 6 ? adj_lds_block<6>() : adj_lds_block<0>());
            items.clear();
        }
        for (int i = 0; i < F; ++i)
            if (!skip(i) && b->f[i]->eq_ring >= 0 && nprod != 0)  // the vector-unit synthesis forms the equator itself
                for (int m = 0; m <= b->f[i]->L; ++m) items.push_back({{i, m, 0, 0}, (double)(b->f[i]->L + 2 - m)});
        emit(BS_EQUATOR, 4, items, 0);
        items.clear();
        // ring stages: one launch per class of stored DFT length (its LDS size) and
        // workgroup width; fields whose length exceeds the narrow width's limit use 512
        const int64_t bounds[] = {256, 512, 1024, 2048, 1 << 30};
        for (int dir = 0; dir < 2; ++dir) {
            int64_t lo = 0;
            for (int64_t hi : bounds) {
                for (int nt : {kRingNTSmall, kRingNT}) {
                    int64_t maxlen = 0;
                    for (int i = 0; i < F; ++i) {
                        const Plan &p = *b->f[i];
                        if (skip(i) || p.max_fft_len <= lo || p.max_fft_len > hi) continue;
                        const int want = (cfg.ring_nt == kRingNTSmall && p.ring_nt_min == kRingNTSmall &&
                                          p.max_fft_len <= kMaxLenSmallRing)
                                             ? kRingNTSmall : kRingNT;
                        if (want != nt) continue;
                        maxlen = std::max(maxlen, p.max_fft_len);
                        for (int r = 0; r < p.n_rings; ++r) items.push_back({{i, r, 0, 0}, (double)p.max_fft_len});
                    }
                    emit(dir == 0 ? BS_RING_ADJ : BS_RING_FWD, nt / 64, items, ring_lds_bytes_len(maxlen, rsz));
                    items.clear();
                }
                lo = hi;
            }
        }
        // Legendre analysis: one workgroup per (field, m) holding all of the field's
        // tiles; fields grouped by tile count, or merged into the widest shape
        int maxt = 1;
        for (int i = 0; i < F; ++i)
            if (!skip(i)) maxt = std::max(maxt, std::max(1, tiles_of(*b->f[i])));
        for (int nw = 1; nw <= maxt; ++nw) {
            for (int i = 0; i < F; ++i) {
                if (skip(i)) continue;
                const Plan &p = *b->f[i];
                const int nt = std::max(1, tiles_of(p));
                if (!cfg.fwd_merge && nt != nw) continue;
                if (cfg.fwd_merge && nw != maxt) continue;
                for (int m = 0; m <= p.L; ++m) items.push_back({{i, m, 0, 0}, (double)(p.L + 2 - m) * nt});
            }
            emit(BS_LEG_FWD, nw, items, leg_fwd_lds(nw, rsz));
            items.clear();
        }
        // recombine
        for (int i = 0; i < F; ++i) {
            if (skip(i)) continue;
            const int L = b->f[i]->L;
            for (int by = 0; by * kTM <= L; ++by)
                for (int bx = 0; bx * kTL < L; ++bx)
                    if (!(by * kTM > 1 + bx * kTL + kTL - 1)) items.push_back({{i, bx, by, 0}, 1.0});
        }
        emit(BS_RECOMBINE, 4, items, 0);
        items.clear();
    }
    // device copies
    const size_t need = b->work.size();
    if (need > b->d_work_cap) {
        if (b->d_work) (void)hipFree(b->d_work);
        if (b->d_stamp) (void)hipFree(b->d_stamp);
        b->d_work = nullptr;
        b->d_stamp = nullptr;
        b->d_work_cap = b->d_stamp_cap = 0;
        hipError_t e = hipMalloc((void **)&b->d_work, need * sizeof(WorkItem));
        if (e != hipSuccess) return e;
        b->d_work_cap = need;
        e = hipMalloc((void **)&b->d_stamp, need * sizeof(unsigned long long));
        if (e != hipSuccess) return e;
        b->d_stamp_cap = need;
    }
    return hipMemcpy(b->d_work, b->work.data(), need * sizeof(WorkItem), hipMemcpyHostToDevice);
}

template <typename real>
static void fill_adjoint_args(BatchState *b, const void *const *a, const void *const *bb, void *const *T) {
    auto *pr = reinterpret_cast<CoefArgs<real> *>(b->h_prep.data());
    auto *ra = reinterpret_cast<RingArgs<real> *>(b->h_radj.data());
    for (size_t i = 0; i < b->f.size(); ++i) {
        pr[i] = make_coef_args<real>(*b->f[i], a[i], bb[i], nullptr, nullptr);
        ra[i] = make_ring_args<real>(*b->f[i], nullptr, T[i], false);
    }
}

template <typename real>
static void fill_forward_args(BatchState *b, const void *const *T, void *const *a, void *const *bb) {
    auto *rf = reinterpret_cast<RingArgs<real> *>(b->h_rfwd.data());
    auto *rc = reinterpret_cast<CoefArgs<real> *>(b->h_rec.data());
    for (size_t i = 0; i < b->f.size(); ++i) {
        rf[i] = make_ring_args<real>(*b->f[i], T[i], nullptr, true);
        rc[i] = make_coef_args<real>(*b->f[i], nullptr, nullptr, a[i], bb[i]);
    }
}

// Upload the argument blocks that hold the caller's buffers (synchronous on st).
hipError_t batch_bind_adjoint(BatchState *b, const void *const *a, const void *const *bb, void *const *T,
                              hipStream_t st) {
    if (b->precision == VSHT_FP64) fill_adjoint_args<double>(b, a, bb, T);
    else fill_adjoint_args<float>(b, a, bb, T);
    hipError_t e = hipMemcpyAsync(b->d_prep, b->h_prep.data(), b->h_prep.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_radj, b->h_radj.data(), b->h_radj.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

hipError_t batch_bind_forward(BatchState *b, const void *const *T, void *const *a, void *const *bb,
                              hipStream_t st) {
    if (b->precision == VSHT_FP64) fill_forward_args<double>(b, T, a, bb);
    else fill_forward_args<float>(b, T, a, bb);
    hipError_t e = hipMemcpyAsync(b->d_rfwd, b->h_rfwd.data(), b->h_rfwd.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_rec, b->h_rec.data(), b->h_rec.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    return e;
}

template <typename real, int kBf16>
static hipError_t batch_launch_impl(const BatchState *b, int dirs, hipStream_t st0) {
    // chains fork from st0 onto their own streams and join back into it
    const bool forked = b->cfg.chains && b->nchains > 1;
    if (forked) {
        hipError_t e = hipEventRecord(b->fork, st0);
        for (int c = 0; c < b->nchains && e == hipSuccess; ++c) e = hipStreamWaitEvent(b->cs[c], b->fork, 0);
        if (e != hipSuccess) return e;
    }
    for (const auto &l : b->launches) {
        const bool adj = stage_is_adjoint(l.stage);
        if (adj && !(dirs & 1)) continue;
        if (!adj && !(dirs & 2)) continue;
        hipStream_t st = forked ? b->cs[l.chain] : st0;
        const WorkItem *w = b->d_work + l.off;
        unsigned long long *stamp = b->d_stamp + l.off;
        const dim3 grid((unsigned)l.cnt);
        switch (l.stage) {
            case BS_PREP:
                hipLaunchKernelGGL(kb_prep<real>, grid, dim3(256), 0, st,
                                   static_cast<const CoefArgs<real> *>(b->d_prep), w, stamp);
                break;
            case BS_LEG_ADJ:
                hipLaunchKernelGGL((kb_leg_adj<real, kBf16>), grid, dim3(64 * l.nw), l.lds, st,
                                   static_cast<const LegArgs<real> *>(b->d_ladj), w, stamp);
                break;
            case BS_EQUATOR:
                hipLaunchKernelGGL(kb_equator_adj<real>, grid, dim3(256), 0, st,
                                   static_cast<const LegArgs<real> *>(b->d_ladj), w, stamp);
                break;
            case BS_RING_ADJ:
                if (l.nw * 64 == kRingNTSmall)
                    hipLaunchKernelGGL((kb_ring_adj<real, kRingNTSmall>), grid, dim3(kRingNTSmall), l.lds, st,
                                       static_cast<const RingArgs<real> *>(b->d_radj), w, stamp);
                else
                    hipLaunchKernelGGL((kb_ring_adj<real, kRingNT>), grid, dim3(kRingNT), l.lds, st,
                                       static_cast<const RingArgs<real> *>(b->d_radj), w, stamp);
                break;
            case BS_RING_FWD:
                if (l.nw * 64 == kRingNTSmall)
                    hipLaunchKernelGGL((kb_ring_fwd<real, kRingNTSmall>), grid, dim3(kRingNTSmall), l.lds, st,
                                       static_cast<const RingArgs<real> *>(b->d_rfwd), w, stamp);
                else
                    hipLaunchKernelGGL((kb_ring_fwd<real, kRingNT>), grid, dim3(kRingNT), l.lds, st,
                                       static_cast<const RingArgs<real> *>(b->d_rfwd), w, stamp);
                break;
            case BS_LEG_FWD:
                hipLaunchKernelGGL((kb_leg_fwd<real, kBf16>), grid, dim3(64 * l.nw), l.lds, st,
                                   static_cast<const LegFwdArgs<real> *>(b->d_lfwd), w, stamp);
                break;
            case BS_RECOMBINE:
                hipLaunchKernelGGL(kb_recombine<real>, grid, dim3(256), 0, st,
                                   static_cast<const CoefArgs<real> *>(b->d_rec), w, stamp);
                break;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    if (forked)
        for (int c = 0; c < b->nchains; ++c) {
            hipError_t e = hipEventRecord(b->join[c], b->cs[c]);
            if (e == hipSuccess) e = hipStreamWaitEvent(st0, b->join[c], 0);
            if (e != hipSuccess) return e;
        }
    return hipSuccess;
}

hipError_t batch_launch(const BatchState *b, int dirs, hipStream_t st) {
    if (b->precision == VSHT_FP64) return batch_launch_impl<double, 0>(b, dirs, st);
    if (b->precision == VSHT_BF16X3) return batch_launch_impl<float, 3>(b, dirs, st);
    if (b->precision == VSHT_BF16X6) return batch_launch_impl<float, 6>(b, dirs, st);
    return batch_launch_impl<float, 0>(b, dirs, st);
}

// Per-field first start and last end (device wall clock, microseconds) of the
// stages of `dirs`, from the stamps of the last run.  Synchronous.
hipError_t batch_field_times(const BatchState *b, int dirs, std::vector<double> &start_us,
                             std::vector<double> &end_us) {
    const size_t F = b->f.size();
    std::vector<unsigned long long> st(b->work.size());
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(st.data(), b->d_stamp, st.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return e;
    int dev = 0, khz = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev)) != hipSuccess) return e;
    const int first = (dirs & 1) ? BS_PREP : BS_RING_FWD;
    const int last = (dirs & 2) ? BS_RECOMBINE : BS_RING_ADJ;
    std::vector<unsigned long long> lo(F, ~0ull), hi(F, 0);
    for (const auto &l : b->launches) {
        if (l.stage != first && l.stage != last) continue;
        for (int64_t k = 0; k < l.cnt; ++k) {
            const WorkItem &w = b->work[l.off + k];
            const unsigned long long t = st[l.off + k];
            if (l.stage == first) lo[w.f] = std::min(lo[w.f], t);
            if (l.stage == last) hi[w.f] = std::max(hi[w.f], t);
        }
    }
    unsigned long long t0 = ~0ull;
    for (size_t i = 0; i < F; ++i) t0 = std::min(t0, lo[i]);
    start_us.resize(F);
    end_us.resize(F);
    const double us_per_tick = 1000.0 / (double)khz;
    for (size_t i = 0; i < F; ++i) {
        start_us[i] = (double)(lo[i] - t0) * us_per_tick;
        end_us[i] = (double)(hi[i] - t0) * us_per_tick;
    }
    return hipSuccess;
}

hipError_t launch_start_kernel(const double *pair_z, const double *pair_s, int NP, int L,
                               const double *aprime, const double *cscale, LegStart *start,
                               int *sblk, int *bad, hipStream_t st) {
    hipLaunchKernelGGL(k_leg_start, dim3((NP + 63) / 64, L + 1), dim3(64), 0, st, pair_z, pair_s, NP, L,
                       aprime, cscale, start, sblk, bad);
    return hipGetLastError();
}

hipError_t launch_seed_kernel(const double *pair_s, int NP, int L, double *seeds, hipStream_t st) {
    hipLaunchKernelGGL(k_seeds, dim3((NP + 127) / 128), dim3(128), 0, st, pair_s, NP, L, seeds);
    return hipGetLastError();
}

// Let kernel k take dynamic LDS up to `total` bytes less its static LDS.
static hipError_t allow_lds(const void *k, int total) {
    hipFuncAttributes fa{};
    hipError_t e = hipFuncGetAttributes(&fa, k);
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, total - (int)fa.sharedSizeBytes);
}

hipError_t set_kernel_attributes() {
    hipError_t e;
    const int big = 160 * 1024;
    const void *batched[] = {(const void *)kb_ring_fwd<double, kRingNT>, (const void *)kb_ring_fwd<float, kRingNT>,
                             (const void *)kb_ring_adj<double, kRingNT>, (const void *)kb_ring_adj<float, kRingNT>,
                             (const void *)kb_ring_fwd<double, kRingNTSmall>,
                             (const void *)kb_ring_fwd<float, kRingNTSmall>,
                             (const void *)kb_ring_adj<double, kRingNTSmall>,
                             (const void *)kb_ring_adj<float, kRingNTSmall>,
                             (const void *)k_ring_fwd<double, kRingNTSmall>, (const void *)k_ring_fwd<float, kRingNTSmall>,
                             (const void *)k_ring_adj<double, kRingNTSmall>, (const void *)k_ring_adj<float, kRingNTSmall>,
                             (const void *)kb_leg_fwd<double, 0>, (const void *)kb_leg_fwd<float, 0>,
                             (const void *)kb_leg_fwd<float, 3>, (const void *)kb_leg_fwd<float, 6>,
                             (const void *)kb_leg_adj<double, 0>, (const void *)kb_leg_adj<float, 0>,
                             (const void *)kb_leg_adj<float, 3>, (const void *)kb_leg_adj<float, 6>};
    const void *nfft_kernels[] = {(const void *)k_nfft_cols<double>, (const void *)k_nfft_cols<float>,
                                  (const void *)k_nfft_rows<double>, (const void *)k_nfft_rows<float>,
                                  (const void *)k_nfft_cols_fwd<double>, (const void *)k_nfft_cols_fwd<float>,
                                  (const void *)k_nfft_rows_fwd<double>, (const void *)k_nfft_rows_fwd<float>};
    for (const void *k : nfft_kernels) {
        e = allow_lds(k, big);
        if (e != hipSuccess) return e;
    }
    for (const void *k : batched) {
        e = allow_lds(k, big);
        if (e != hipSuccess) return e;
    }
    e = allow_lds((const void *)k_ring_fwd<double, kRingNT>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_ring_fwd<float, kRingNT>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_ring_adj<double, kRingNT>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_ring_adj<float, kRingNT>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_fwd_mfma<double>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_fwd_mfma<float>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_adj<double, 0>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_fwd_bf16<3>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_fwd_bf16<6>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_adj<float, 3>, big);
    if (e != hipSuccess) return e;
    e = allow_lds((const void *)k_leg_adj<float, 6>, big);
    if (e != hipSuccess) return e;
    return allow_lds((const void *)k_leg_adj<float, 0>, big);
}

}  // namespace vsht
