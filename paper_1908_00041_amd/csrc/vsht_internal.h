// vsht_internal.h -- plan structure and kernel launch interface shared by the
// host code (vsht_plan.cpp, vsht_api.cpp) and the gfx950 kernels (*.hip).
//
// Formulation used by every kernel:
// with Lambda_{l,m}(z) the 4pi-normalised associated Legendre function
// (Condon-Shortley phase; Lambda_{l,-m} = (-1)^m Lambda_{l,m}) and
// e_{l,m} = sqrt((l^2-m^2)/(4l^2-1)), the polar derivative obeys
//     s dLambda_{l,m}/dtheta = l e_{l+1,m} Lambda_{l+1,m} - (l+1) e_{l,m} Lambda_{l-1,m}.
// Writing the tangent field in the (e_theta, e_phi) frame, Y^div = grad* Y /
// sqrt(l(l+1)) and Y^curl = x cross Y^div (the Clebsch-Gordan vectors of
// Definition 3.1 reduce to these), the forward transform becomes two scalar
// spin-frame transforms of degree L+1,
//     F^{theta,phi}_{l',m} = sum_k (w_k / s_k) Lambda_{l',m}(z_k) e^{-i m phi_k} T^{theta,phi}_k,
// followed by a three-term recombination in l', and the adjoint is the
// transpose: three-term "prep" in l', then scalar syntheses divided by s.
// Both Legendre stages therefore contract against Lambda only, one real
// value per (m, l', ring pair), with four complex columns (theta/phi x +-m).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "vsht.h"

namespace vsht {

// Per ring (iso-latitude circle of equispaced points).
struct RingDesc {
    double z;        // cos(theta), identical for every point of the ring
    double s;        // sin(theta) = sqrt((1-z)(1+z)) > 0
    double w;        // common weight of the ring's points (if uniform_w)
    double c0, s0;   // cos(phi_0), sin(phi_0)
    double phi0;     // first longitude
    int64_t offset;  // index of the first point
    int32_t nphi;    // points on the ring
    int32_t fft;     // index of the FFT descriptor for nphi
    int32_t uniform_w;
    int32_t pair;    // index of the ring's north/south pair
    int32_t south;   // 1 if the ring is the southern member of its pair
    int32_t pad;
};

// North/south pair of rings with z_S == -z_N bitwise; rs < 0 for an unpaired ring.
struct PairDesc {
    int32_t rn, rs;
};

// Limits of the ring DFT stages (shared by the kernels and the plan's check
// that every stage of a length fits a workgroup width).
constexpr int kKP = 2;           // output pairs per work item of a generic odd radix
constexpr int kSmallTab = 128;   // largest odd radix whose cos/sin table is staged in LDS
constexpr int kMaxItemsSmall = 4;  // work items per thread of a radix-2..5 stage
constexpr int kMaxItemsOdd = 2;    // work items per thread of a generic odd stage
constexpr int kKU = 5;             // output pairs per work item of the first odd stage
constexpr int kMaxRoundsFirst = 2; // waves per wave slot of a workgroup in that stage

// Mixed-radix Stockham descriptor for one DFT length.
constexpr int kMaxFactors = 24;
struct FftDesc {
    int32_t n;
    int32_t nfac;
    int64_t tw_offset;  // offset (in complex entries) of e^{-2 pi i k / n}, k < n (every descriptor)
    int32_t fac[kMaxFactors];
    // Bluestein form (lengths with a large prime factor): a cyclic convolution
    // of power-of-two length M through the descriptor mdesc
    int32_t blue;
    int32_t M;
    int32_t mdesc;
    int32_t lds_shift;     // LDS layout of the sequences: element i at i + (i >> lds_shift)
    int64_t chirp_offset;  // w_k = e^{-i pi k^2 / n}, k < n
    int64_t bhat_offset;   // DFT_M of conj(w) (forward), then of w (inverse), each / M: 2M entries
    // first radix R = fac[0] when 5 < R <= kSmallTab: e^{-2 pi i q / R}, q < R, as R complex
    // binary64 values, then the same as R complex binary32 values in the next R entries
    int64_t rtab_offset;
};

// LDS bytes of a workgroup that transforms two sequences of stored length len
// (the kernels' cos/sin table of an odd radix, then the padded sequences).
inline size_t ring_lds_bytes_for(int64_t len, size_t real_size) {
    const size_t elems = 2 * (size_t)len;
    return kSmallTab * 2 * sizeof(double) + (elems + elems / 16 + 1) * 2 * real_size;
}
constexpr size_t kLdsPerWorkgroup = 160 * 1024;

// Waves of the first odd stage of radix R on a ring's two sequences of length n:
// one group of kKU output pairs per wave, over the 2 n / R columns of both sequences.
__host__ __device__ inline int first_stage_waves(int n, int R) {
    return ((R - 1) / 2 + kKU - 1) / kKU * ((2 * (n / R) + 63) / 64);
}

// A scattered point as the double-Fourier-sphere stages see it (sorted by grid cell).
struct NfftPoint {
    double theta, phi;   // colatitude in [0, pi], longitude in [0, 2 pi) (0 at a pole)
    double z, s, c, sn;  // cos theta, sin theta, cos phi, sin phi
    int64_t idx;         // position in the caller's point order
};

// Gather tiles of the double-Fourier-sphere adjoint: a point whose window starts at
// grid cell (j0, i0) (the first row and column its width-w kernel touches) belongs
// to tile (tj, ti) = ((j0 + w/2) / kGatherTile, (i0 + w/2) / kGatherTile); the
// tile's workgroup stages rows and columns [t kGatherTile - w/2, + kGatherTile + w - 1)
// of both grids in LDS and gathers its points from there.
constexpr int kGatherTile = 16;
struct NfftTile {
    int32_t tj, ti, count, pad;
    int64_t start;  // first point (index into the sorted points)
};

// Where each (order m, ring pair p) enters the Legendre stages.  Degrees are
// taken in blocks of kStartBlock from l' = m; (m, p) starts at block b with the
// recurrence state (Q_{l0-1}, Q_{l0-2}), l0 = m + kStartBlock b, and adds
// nothing before it.  b is the last block boundary at or below the first degree
// where |Lambda_{l',m}(z_p)| >= 2^kSignificantExp2, or kStartNever when no degree
// up to L+1 gets there.  The state is computed with a carried exponent, so it
// exists even where the seed Lambda_{m,m} = O(s^m) lies below binary64's range,
// and it is bitwise the state the recurrence from the seed would reach if
// binary64 had no exponent limit (a start at b = 0 is (0, -Lambda_{m,m})).
struct alignas(16) LegStart {
    double q1, q2;
};
constexpr int kStartBlock = 32;
constexpr int kStartNever = 1 << 24;
constexpr int kSignificantExp2 = -64;

// Scattered points through the double Fourier sphere: the synthesis runs on
// nt equispaced colatitudes theta_t = 2 pi (t + 1/2) / nt of the doubled
// circle (nt/4 virtual north/south ring pairs), a DFT in theta gives the 2-D
// Fourier coefficients of the spin-frame components, which are deconvolved by
// the window transform and taken to an ng x ng grid; each point then gathers a
// w x w window with the exponential-of-semicircle kernel
// psi(u) = exp(beta (sqrt(1 - (2u / (w h))^2) - 1)), h = 2 pi / ng.
struct NfftPlan {
    int on = 0;
    int nt = 0, npv = 0, ng = 0, w = 0;
    double beta = 0.0;
    int fft_nt = 0, fft_ng = 0;       // descriptors in d_ffts
    int64_t lds_stride = 0;           // LDS sequence stride of the theta/grid DFTs
    FftDesc *d_ffts = nullptr;
    double *d_tw = nullptr;
    PairDesc *d_vpairs = nullptr;     // virtual ring pairs (north t, south nt/2 - 1 - t)
    double *d_vz = nullptr;           // z of each virtual pair's northern colatitude
    double *d_vs = nullptr;           // its sin theta
    double *d_vseeds = nullptr;       // Lambda_{m,m}, [(L+1)][npv]
    LegStart *d_vstart = nullptr;     // start states, [(L+1)][npv]
    int *d_vsblk = nullptr;           // start blocks, [(L+1)][npv]
    double *d_psihat = nullptr;       // window transform at k = -L..L
    NfftPoint *d_pts = nullptr;       // points sorted by gather tile, then by grid cell
    NfftTile *d_tiles = nullptr;      // the non-empty gather tiles (point ranges of d_pts)
    int ntiles = 0;
    void *d_vpb = nullptr;            // virtual pair buffer [(L+1)][npv][16] reals (adjoint),
                                      // virtual ring buffer [(L+1)][nt/2][8] reals (forward)
    void *d_g1 = nullptr;             // column pass output [2][ng][2L+1] complex
    void *d_g = nullptr;              // grid [2][ng][ng] complex
};

// Workspace layout (all in the plan's real type):
//  RB   ring buffer (forward)  [(L+1)][NR][4] complex, the ring DFTs scaled by
//       e^{-+i m phi_0} w / s: (theta,+m) (phi,+m) (theta,-m) (phi,-m)
//  PB   pair buffer (adjoint)  [(L+1)][NP][2][4] complex: slot 0 = sum over
//       even l'+m, slot 1 = sum over odd l'+m, same 4 columns
//  RB and PB share one allocation.
//  FG   triangle buffer [tri(L)][4] complex, tri index (m, l') for
//       0 <= m <= L, m <= l' <= L+1: forward F, adjoint prep g; followed by
//       kFgPadRows rows that the synthesis may load (never use) past the end.
//  FG64 (binary32 paths) the adjoint's g in binary64, FG's layout: the synthesis
//       runs in binary64 on the vector unit (binary32 path) or, for the pairs next
//       to the poles, in a binary64 polar wave (split-bf16 paths).
constexpr int kFgPadRows = 8;

// Workgroups per order of the ring analysis: up to 16 tiles of 64 ring pairs
// (the equator excluded) in one workgroup, more split over several.
inline int analysis_groups(int64_t n_pairs, int eq_ring) {
    const int64_t tiles = (n_pairs - (eq_ring >= 0 ? 1 : 0) + 63) / 64;
    return tiles > 16 ? (int)((tiles + 15) / 16) : 1;
}

struct Plan {
    int L = 0;
    int precision = VSHT_FP64;
    int device = 0;
    int kind = VSHT_PLAN_RINGS;
    int has_weights = 0;
    int64_t n = 0;
    int64_t n_rings = 0, n_pairs = 0;
    int64_t max_nphi = 0;
    int64_t max_fft_len = 0;   // longest stored DFT sequence (n, or M for Bluestein rings)
    int ring_nt_min = 256;     // narrowest ring workgroup (256 or 512) every ring's DFT stages fit
    int64_t tri_size = 0;
    int eq_ring = -1;       // ring at z = 0 (always the last pair), handled in closed form

    // device tables
    RingDesc *d_rings = nullptr;
    PairDesc *d_pairs = nullptr;
    FftDesc *d_ffts = nullptr;
    double *d_tw = nullptr;        // twiddles, complex as (re, im)
    double *d_pair_z = nullptr;    // z of each pair's northern ring
    double *d_aprime = nullptr;    // scaled recurrence Q_l = a'_l z Q_{l-1} - Q_{l-2}, [tri]
    double *d_cscale = nullptr;    // Lambda_{l,m} = c_{l,m} Q_{l,m}, [tri]
    double *d_etab = nullptr;      // e_{l,m} = sqrt((l^2-m^2)/(4l^2-1)), [tri]
    double *d_rsq = nullptr;       // 1/sqrt(l(l+1)), [L+2] (0 at l = 0)
    double *d_seeds = nullptr;     // Lambda_{m,m}(z_p), [(L+1)][NP]
    LegStart *d_start = nullptr;   // start states of the Legendre stages, [(L+1)][NP]
    int *d_sblk = nullptr;         // start blocks, [(L+1)][NP]
    double *d_weights = nullptr;   // per-point weights (rings with non-uniform weights)
    double *d_xyz = nullptr;       // points (scattered plans)
    size_t table_bytes = 0;

    NfftPlan nfft;                 // scattered plans evaluated through the double Fourier sphere

    // workspace
    void *d_pb = nullptr;
    void *d_fg = nullptr;
    void *d_fg64 = nullptr;        // binary32 paths: the adjoint's g in binary64, [tri][8] double
    void *d_fpart = nullptr;       // analysis split over g > 1 workgroups per order: [g][tri][8]

    void *d_many = nullptr;        // workspace of the *_many calls: several fields at once,
    size_t many_bytes = 0;         // allocated on first use, grown as needed
    void *d_state = nullptr;       // Legendre recurrence state
    size_t workspace_bytes = 0;
    int n_ffts = 0;

    // optional per-stage event timing
    struct StageRecord {
        int stage;
        hipEvent_t start, stop;
    };
    int timing = 0;
    mutable std::vector<StageRecord> records;
};

// Record events around a kernel launch when the plan's timing is enabled.
struct StageScope {
    const Plan &p;
    hipStream_t st;
    Plan::StageRecord rec{};
    bool on;
    StageScope(const Plan &plan, int stage, hipStream_t stream, bool allowed = true) : p(plan), st(stream) {
        on = allowed && plan.timing != 0;
        if (on) {
            rec.stage = stage;
            on = hipEventCreate(&rec.start) == hipSuccess;
            if (on && hipEventCreate(&rec.stop) != hipSuccess) {
                (void)hipEventDestroy(rec.start);
                on = false;
            }
            if (on) (void)hipEventRecord(rec.start, st);
        }
    }
    ~StageScope() {
        if (on) {
            (void)hipEventRecord(rec.stop, st);
            p.records.push_back(rec);
        }
    }
};

__host__ __device__ inline int64_t tri_offset(int L, int m) {
    // sum_{m' < m} (L + 2 - m')
    return (int64_t)m * (L + 2) - (int64_t)m * (m - 1) / 2;
}
__host__ __device__ inline int64_t tri_size(int L) { return tri_offset(L, L + 1); }

// Workspace of one field of a ring plan, bytes (each rounded up to 256): the
// ring/pair buffer, the triangle FG, FG64 (binary32 plans) and the partial
// triangles of a split analysis (more than 1024 ring pairs).
struct ManyWs {
    size_t pb, fg, fg64, fpart;
    size_t total() const { return pb + fg + fg64 + fpart; }
};
inline size_t round256(size_t x) { return (x + 255) / 256 * 256; }
inline ManyWs field_ws(const Plan &P) {
    const size_t rsz = P.precision == VSHT_FP64 ? 8 : 4;
    const size_t per_m = std::max((size_t)P.n_rings * 4, (size_t)P.n_pairs * 8);
    ManyWs z{};
    z.pb = round256((size_t)(P.L + 1) * per_m * 2 * rsz);
    z.fg = round256((size_t)(P.tri_size + kFgPadRows) * 4 * 2 * rsz);
    z.fg64 = rsz == 4 ? round256((size_t)(P.tri_size + kFgPadRows) * 4 * 2 * 8) : 0;
    const int groups = analysis_groups(P.n_pairs, P.eq_ring);
    z.fpart = groups > 1 ? round256((size_t)groups * P.tri_size * 8 * rsz) : 0;
    return z;
}

// Kernel launchers (vsht_kernels.hip).  Each returns the hipError_t of the launch.
hipError_t launch_forward(const Plan &p, const void *T, void *a, void *b, bool weighted,
                          hipStream_t st);
hipError_t launch_adjoint(const Plan &p, const void *a, const void *b, void *T, bool weighted,
                          hipStream_t st);
hipError_t launch_sht_forward(const Plan &p, const void *f, void *flm, hipStream_t st);
// The weighted forward of a ring plan with its intermediate buffers in the library's
// static device array (no allocation, no stage timing).  *need receives the bytes the
// plan needs; hipErrorInvalidValue when they exceed kStaticScratchBytes.
constexpr size_t kStaticScratchBytes = (size_t)128 << 20;
size_t static_forward_bytes(const Plan &p);
hipError_t launch_forward_static(const Plan &p, const void *T, void *a, void *b, hipStream_t st);
hipError_t launch_sht_adjoint(const Plan &p, const void *flm, void *f, hipStream_t st);
// count fields of a ring plan in one launch per stage (fields along the grid's z
// dimension), with count field workspaces (field_ws) at ws; T, a and b hold count
// contiguous fields.
hipError_t launch_forward_many(const Plan &p, int count, void *ws, const void *T, void *a, void *b,
                               bool weighted, hipStream_t st);
hipError_t launch_adjoint_many(const Plan &p, int count, void *ws, const void *a, const void *b, void *T,
                               bool weighted, hipStream_t st);
hipError_t launch_seed_kernel(const double *pair_s, int NP, int L, double *seeds, hipStream_t st);
// Start blocks and states of every (m, p), p < NP; *bad (device) is set to 1 if a
// state falls outside binary64's normal range (never expected: it is at least
// 2^kSignificantExp2 divided by the growth over kStartBlock + 2 degrees).
hipError_t launch_start_kernel(const double *pair_z, const double *pair_s, int NP, int L,
                               const double *aprime, const double *cscale, LegStart *start,
                               int *sblk, int *bad, hipStream_t st);

hipError_t set_kernel_attributes();

// Batches (vsht_kernels.hip): every field of a batch in one launch per stage.
struct WorkItem {
    int32_t f, x, y, pad;  // field, block coordinates
};
struct BatchConfig {
    int adj_nw = 4;     // waves (64-pair tiles) per workgroup of the Legendre synthesis: 1, 2 or 4
    int fwd_merge = 0;  // 1: one analysis launch at the widest shape; 0: one launch per tile count
    int lpt = 1;        // 1: work items longest first; 0: field by field
    int ring_nt = 256;  // threads per ring workgroup (256 or 512; rings longer than 2048 always 512)
    int chains = 0;     // 1: size classes of fields run as parallel chains; 0: one sequence
};
constexpr int kBatchChains = 3;
// Parallel chains are switched off: one run crashed (segmentation fault in the host
// process) inside an autotune that captured and replayed the multi-branch graphs, and
// the cause is not known.  With the switch off no chain streams are created and
// vsht_batch_set_config refuses chains = 1.
constexpr bool kBatchChainsEnabled = false;
struct BatchState;
hipError_t batch_create(const std::vector<const Plan *> &fields, BatchState **out);
void batch_destroy(BatchState *b);
hipError_t batch_configure(BatchState *b, const BatchConfig &cfg);
BatchConfig batch_config(const BatchState *b);
hipError_t batch_bind_adjoint(BatchState *b, const void *const *a, const void *const *bb, void *const *T,
                              hipStream_t st);
hipError_t batch_bind_forward(BatchState *b, const void *const *T, void *const *a, void *const *bb,
                              hipStream_t st);
hipError_t batch_launch(const BatchState *b, int dirs, hipStream_t st);  // dirs: 1 adjoint, 2 forward, 3 both
hipError_t batch_field_times(const BatchState *b, int dirs, std::vector<double> &start_us,
                             std::vector<double> &end_us);

}  // namespace vsht
