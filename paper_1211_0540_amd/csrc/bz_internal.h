// Internal definitions of the bz library: mesh handle, work schedules, launchers.
// Everything here is private to libbz.so; the public interface is include/bz.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bz.h"

namespace bz {

constexpr int kMinN = 8;
constexpr int kMaxN = 32;
constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Per-axis bookkeeping of the trapezoid sum (Sec. 3.2): for an output index k
// the partner index j = k - m + N/2 must stay on the mesh, so m ranges over
// [lo(k), hi(k)] with lo = max(0, k - N/2 + 1), hi = min(N - 1, k + N/2).
// ---------------------------------------------------------------------------
__host__ __device__ inline int axis_lo(int N, int k) { return k - N / 2 + 1 > 0 ? k - N / 2 + 1 : 0; }
__host__ __device__ inline int axis_hi(int N, int k) { return k + N / 2 < N - 1 ? k + N / 2 : N - 1; }
__host__ __device__ inline int axis_cnt(int N, int k) { return axis_hi(N, k) - axis_lo(N, k) + 1; }

// ---------------------------------------------------------------------------
// T_lambda(a, b) = int_0^1 s^{lambda+2} sinc(a s) sinc(b s) ds for lambda = 0, 1
// and real a, b >= 0 (the gain integral of eq. GHat_calc in units r = L s; with
// inelastic collisions, beta < 1, its second argument is no longer the root of
// an integer).  With a >= b:
//   b >= a/2:  [F(a - b) - F(a + b)] / (2ab),  F = S (lambda 0) or U (lambda 1),
//              S(x) = sin x / x,  U(x) = int_0^1 s cos(xs) ds = S(x) - 2 sin^2(x/2)/x^2;
//   b <  a/2:  the same expression expanded with the addition theorems, which
//              removes the division by b:
//      lambda 0:  [sin a cos b - a cos a S(b)] / (a (a^2 - b^2))
//      lambda 1:  that + [2 (cos a cos b - 1) + (a^2 + b^2) sin a S(b) / a] / (a^2 - b^2)^2;
//   b = 0:     the one-sided limits, a = b = 0: 1 / (lambda + 3).
// ---------------------------------------------------------------------------
__host__ __device__ inline double sinc_d(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }
__host__ __device__ inline double ucos_d(double x) {
    if (x == 0.0) return 0.5;
    const double hs = sin(0.5 * x);
    return sin(x) / x - 2.0 * hs * hs / (x * x);
}
__host__ __device__ inline double T_real(int lam, double a, double b) {
    if (a < b) {
        const double t = a;
        a = b;
        b = t;
    }
    if (a == 0.0) return 1.0 / (lam + 3);
    if (b == 0.0) {
        const double sc = sin(a), cc = cos(a), hs = sin(0.5 * a);
        if (lam == 0) return (sc - a * cc) / (a * a * a);
        return (-cc / a + 2.0 * sc / (a * a) - 4.0 * hs * hs / (a * a * a)) / a;
    }
    if (b >= 0.5 * a) {
        if (lam == 0) return (sinc_d(a - b) - sinc_d(a + b)) / (2.0 * a * b);
        return (ucos_d(a - b) - ucos_d(a + b)) / (2.0 * a * b);
    }
    const double sa = sin(a), ca = cos(a), cb = cos(b), sb = sinc_d(b), d = a * a - b * b;
    const double t0 = (sa * cb - a * ca * sb) / (a * d);
    if (lam == 0) return t0;
    return t0 + (2.0 * (ca * cb - 1.0) + (a * a + b * b) * sa * sb / a) / (d * d);
}

// Gain part of the weight for output k and partner m of an inelastic collision (beta):
// T(beta pi |k - N/2| / 2, pi |2(m - N/2) - beta (k - N/2)| / 2).
__host__ __device__ inline double gain_beta(int lam, double beta, int h, int k1, int k2, int k3, int m1, int m2,
                                            int m3) {
    constexpr double kHalfPi = 1.57079632679489661923;
    const double y1 = k1 - h, y2 = k2 - h, y3 = k3 - h;
    const double w1 = 2.0 * (m1 - h) - beta * y1, w2 = 2.0 * (m2 - h) - beta * y2, w3 = 2.0 * (m3 - h) - beta * y3;
    return T_real(lam, beta * kHalfPi * sqrt(y1 * y1 + y2 * y2 + y3 * y3), kHalfPi * sqrt(w1 * w1 + w2 * w2 + w3 * w3));
}

// ---------------------------------------------------------------------------
// Batched ("lane = cell") schedule.
//
// A work item is one output row (k1, k2, 0..N-1) of 64 cells on the same mesh.
// The pair (m, j = k - m + N/2) and its mirror (j, m) carry the same product
// fhat_m fhat_j, and the gain weight T(na, |m - j|^2) is symmetric in them, so
// each unordered pair is visited once with the weight
//   W = s [2 T(na, nb) - T(0, 4 nc(m)) - T(0, 4 nc(j))]        (m != j)
//   W = s [  T(na, 0)  - T(0, 4 nc(m))                ]        (m == j)
// where s = 4pi (2pi)^{-3/2} L^{lambda+3} dzeta^3.  Unordered pairs are
// represented by m <= j in the lexicographic order of (m1, m2, m3); a "step"
// is one (m1, m2) with (m1, m2) <= (j1, j2), and covers all (k3, m3) of the
// row in the fixed order  for k3 in [0, N): for m3 in [axis_lo(k3), axis_hi(k3)]
// (output-major, so that the terms of one output in one step are contiguous).
// In the diagonal step (m1, m2) == (j1, j2) the pairs with m3 > j3 get W = 0.
// ---------------------------------------------------------------------------
__host__ __device__ inline int pairs_per_step(int N) { return 3 * N * N / 4; }
// offset of output k3's run in a step: sum of axis_cnt over k < k3
__host__ __device__ constexpr int step_koff(int N, int k3) {
    int s = 0;
    for (int k = 0; k < k3; ++k) {
        const int lo = k - N / 2 + 1 > 0 ? k - N / 2 + 1 : 0;
        const int hi = k + N / 2 < N - 1 ? k + N / 2 : N - 1;
        s += hi - lo + 1;
    }
    return s;
}

// Last m1 of the row: the largest m1 with 2 m1 <= k1 + N/2.
__host__ __device__ inline int cells_m1_last(int N, int k1) {
    int t = (k1 + N / 2) / 2;
    int hi = axis_hi(N, k1);
    return t < hi ? t : hi;
}
// Last m2 for a given m1 (all of the band, or up to the diagonal when m1 == j1).
__host__ __device__ inline int cells_m2_last(int N, int k1, int k2, int m1) {
    int hi = axis_hi(N, k2);
    if (2 * m1 < k1 + N / 2) return hi;
    int t = (k2 + N / 2) / 2;
    return t < hi ? t : hi;
}
__host__ __device__ inline int cells_steps(int N, int k1, int k2) {
    int lo1 = axis_lo(N, k1), lo2 = axis_lo(N, k2);
    int n = 0;
    for (int m1 = lo1; m1 <= cells_m1_last(N, k1); ++m1) n += cells_m2_last(N, k1, k2, m1) - lo2 + 1;
    return n;
}

// ---------------------------------------------------------------------------
// Conjugate-symmetric ("halved") batched schedule.
//
// f is real, so fhat(-zeta) = conj fhat(zeta): on the mesh, index k maps to
// N - k on every axis, except the planes k_d = 0 (zeta_d = -N dzeta / 2),
// whose mirror lies off the mesh.  Split the sum of an output k into interior
// pairs (every coordinate of m and j in [1, N)) and edge pairs (some
// coordinate of m or j equal to 0).  The weight is invariant under
// (k, m) -> (N - k, N - m), so the interior sum I satisfies
// I(N - k) = conj I(k) whenever every k_d >= 1, and with E the edge sum
//   Qhat(k) = I(k) + E(k),   Qhat(N - k) = conj I(k) + E(N - k).
// The library therefore evaluates
//   pass A : the interior sums of the rows (k1, k2) of the "direct" half, as
//            whole rows on a copy of fhat whose k_d = 0 planes are zeroed
//            (edge pairs then contribute nothing; the steps with m1 = 0 are
//            skipped);
//   pass E1: edge pairs with m1 = 0 or j1 = 0 (in the schedule, the steps
//            with m1 = 0 of the rows with k1 < N/2), every row;
//   pass E2: edge pairs with m2 = 0 or j2 = 0 and no axis-1 edge: the same
//            step block on a copy of fhat with axes 1 and 2 exchanged, minus
//            its first and last step (m1 = 0, j1 = 0);
//   pass E3: edge pairs with m3 = 0 or j3 = 0 and no axis-1 or axis-2 edge:
//            the block on a copy with axes ordered (3, 1, 2), minus its end
//            steps, with the weights of the inner-axis edge terms set to 0
//            (a separate weight stream);
//   pass Z : the outputs k3 = 0 of the "derived" rows (no mirror), as whole
//            rows (0, k1) of the (3, 1, 2) copy;
// and the first inverse-transform pass assembles Qhat.  The weight stream of
// a row serves every axis order because W depends on k and m only through
// |k - N/2|^2, |2m - k - N/2|^2 and |m - N/2|^2.
// ---------------------------------------------------------------------------
// rows (k1, k2) whose outputs with k3 >= 1 are mirrors of the direct rows
__host__ __device__ inline bool herm_derived_row(int N, int k1, int k2) {
    const int h = N / 2;
    return k1 >= 1 && k2 >= 1 && (k1 > h || (k1 == h && k2 > h));
}
enum ConvPassId { kPassA = 0, kPassE1 = 1, kPassE2 = 2, kPassE3 = 3, kPassZ = 4, kPasses = 5 };
// Assembly of Qhat from the passes of the conjugate-symmetric schedule, done by
// the first inverse-transform pass.  With B = G N^3 64 complex elements (one
// full buffer): pass A's nA partial sums at [0, nA B); then E1, E2 and E3, B/2
// each (rows a < N/2 only, N^3/2 64 per group); then nA partial sums of pass Z,
// B / (2N) each (rows k1 = N/2..N-1 of the k3 = 0 plane, N^2/2 64 per group).
struct HermAssembly {
    bool on;
    int nA;
};

// FP64 sum of the low-frequency core, added to every output by the first
// inverse-transform pass: core[g][k][lane] (one full output buffer) holds it
// for the outputs k with every |k_d - N/2| <= 2r of the direct rows, and of the
// derived rows at k3 = 0; NULL when the core is off.
struct CoreAdd {
    const double2 *core;         // `parts` partial sums [G][N^3][64], pstride apart (complex units)
    int r;
    int parts;
    long long pstride;
};

// ---------------------------------------------------------------------------
// Low-frequency core of the batched FP32 mode.
//
// Near the centre of the Fourier mesh |fhat| is largest, and so are the terms
// of the sum of Sec. 3.2 there; rounding fhat and the weights to FP32 leaves an
// error proportional to those terms, which for near-Maxwellian cells (whose
// terms cancel to a small Qhat) exceeds a relative 1e-5.  The pairs whose two
// partners both lie in the ball |m - N/2|^2 <= r2 (the "core") are therefore
// summed in FP64 by a separate kernel, and their weights are zero in the FP32
// stream.  The core sum is added to the outputs after the assembly of the FP32
// passes.  Same sum, split by frequency, each term evaluated once.  The core
// pairs are interior pairs, so the core sum of a derived output with k3 >= 1 is
// the conjugate of that of its mirror N - k: only the direct rows (and k3 = 0
// of the derived rows, reached when 2r >= N/2) are summed.
//
// Rows of the core: the disk (a - h)^2 + (b - h)^2 <= r2, numbered in
// lexicographic order; a core row holds the S = 2r + 1 values m3 = h - r .. h + r
// (zero outside the ball).  A core step of output row (k1, k2) is a pair of
// core rows (m1, m2) <= (j1, j2) (lexicographic) with j = k + h - m on both
// axes; its S x S weights are indexed (tm, tj) with m3 = h - r + tm,
// j3 = h - r + tj, output k3 = m3 + j3 - h, zero off the ball, off the mesh and
// for tm > tj in a diagonal step (m1, m2) = (j1, j2).
// ---------------------------------------------------------------------------
constexpr int kCoreMaxR = 8;
__host__ __device__ constexpr int core_wstride(int r) {
    // weights of one step, padded to whole KiB (128 doubles) for the direct-to-LDS copy
    return ((2 * r + 1) * (2 * r + 1) + 127) / 128 * 128;
}

// ---------------------------------------------------------------------------
// Plain ("lane = output") schedule, one cell at a time.
//
// A block holds R consecutive rows k2 = kb R .. kb R + R - 1 of one k1 plane,
// one output per lane (lane = r N + k3, R N <= 64).  All lanes walk the same
// m in the order m1 in [lo(k1), hi(k1)], m2 over the union of the rows' bands,
// m3 in [0, N); a lane whose partner leaves the mesh reads weight 0.
// ---------------------------------------------------------------------------
__host__ __device__ inline int plain_rows(int N) {
    int R = kWave / N;
    while (R > 1 && N % R) --R;
    return R;
}
__host__ __device__ inline int plain_u2_lo(int N, int kb) { return axis_lo(N, kb * plain_rows(N)); }
__host__ __device__ inline int plain_u2_hi(int N, int kb) { return axis_hi(N, kb * plain_rows(N) + plain_rows(N) - 1); }
__host__ __device__ inline long long plain_block_iters(int N, int k1, int kb) {
    return (long long)axis_cnt(N, k1) * (plain_u2_hi(N, kb) - plain_u2_lo(N, kb) + 1) * N;
}

// ---------------------------------------------------------------------------
// Mesh handle.
// ---------------------------------------------------------------------------
struct CoreSched {
    int r2 = -1;                      // radius^2 of the core ball; -1: no core
    int r = 0;                        // floor(sqrt(r2)), the per-axis half-width
    int nD = 0;                       // rows in the disk
    std::vector<int> disk_idx;        // N*N: index of row (a, b) in the disk, -1 outside
    std::vector<int> disk_ext;        // nD: the row's half-width in m3 inside the ball, floor(sqrt(r2 - rho^2))
    std::vector<int> row_steps;       // N*N: core steps of output row (k1, k2)
    std::vector<long long> row_soff;  // N*N: first step of the row in the step list
    std::vector<int> steps;           // per step: disk index of the m row | (disk index of the j row) << 16
    long long nsteps = 0;
};

struct Schedule {
    // batched: N*N rows, offsets in weights (elements), steps per row
    std::vector<long long> row_woff;
    std::vector<int> row_steps;
    long long cells_weights = 0;
    // edge-pass weights of pass E3 (rows a < N/2: the m1 = 0 block of row (a, b),
    // inner edge terms zeroed), offsets relative to the start of that stream
    std::vector<long long> e3_woff;
    long long e3_weights = 0;
    // plain: N * (N / R) blocks
    std::vector<long long> blk_woff;
    long long plain_weights = 0;
    CoreSched core;
};

}  // namespace bz

struct bz_grid_s {
    int N;
    double L, lambda, beta, dv, dzeta;
    long long pairs;
    double linv[25];  // L^{-1} with C C^T = L L^T (Cholesky), row-major; energy row zero when beta < 1
    bz::Schedule sched;
};

namespace bz {

// status helpers (thread-local message)
bz_status fail(bz_status s, const std::string &msg);
bz_status hip_fail(hipError_t e, const char *what);

#define BZ_HIP(call, what)                               \
    do {                                                 \
        hipError_t e_ = (call);                          \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ---------------------------------------------------------------------------
// Kernel launchers (defined in the .hip files).  All take a hipStream_t.
// ---------------------------------------------------------------------------
// Weight expansion from the FP64 universal table T[p * qstride + q].
// Pairs with both partners in the core ball (core_r2 >= 0) get weight 0 (they are summed in FP64).
// beta < 1 (inelastic, lambda 0 or 1): the gain parts come from gain_beta, the loss parts from T.
hipError_t launch_expand_cells(int N, const double *dT, int qstride, double scale, const long long *d_row_woff,
                               void *d_w, bool f64, int core_r2, int lam, double beta, hipStream_t s);
hipError_t launch_expand_plain(int N, const double *dT, int qstride, double scale, const long long *d_blk_woff,
                               void *d_w, bool f64, int lam, double beta, hipStream_t s);

// Forward transform of `ncells` cells of one mesh.  Cell c's f starts at
// f + f_off[c]; fhat element k of cell c is written at out + o_base[c] + k*o_stride
// (complex units) as float2 (f32) or double2.
// batched paths: cell-interleaved groups of 64; S and T are scratch buffers of
// groups * N^3 * 64 double2 each (T may be the first partial buffer of qh for
// the inverse, which reads qh only in its first pass)
// With `copies` = 4 the last pass also writes fhat with the axes ordered
// (2, 1, 3) and (3, 1, 2), and fhat with its k_d = 0 planes zeroed, after the
// first copy, G * N^3 * 64 elements apart.  Groups g with skip[g] != 0 (skip
// may be NULL) are left untouched by both directions.
// With core.cf non-NULL the last forward pass also writes the FP64 core rows (CoreSched) of every
// group to cf[g][disk row][t][lane], t = m3 - (N/2 - r).
struct CoreFill {
    double2 *cf;
    const int *disk_idx;   // device, N*N
    int nD, r, r2;
};
hipError_t launch_dft_forward_grouped(int N, double L, int ncells, const double *f, const long long *d_f_off,
                                      double2 *S, double2 *T, void *fh, bool out_f32, int copies,
                                      const CoreFill &core, const unsigned char *skip, hipStream_t s);
hipError_t launch_dft_inverse_grouped(int N, double L, int ncells, const double2 *qh, int nparts, long long pstride,
                                      const HermAssembly &herm, const CoreAdd &core, double2 *S, double2 *T,
                                      double *qt, const long long *d_q_off, const unsigned char *skip,
                                      hipStream_t s);
hipError_t launch_dft_forward(int N, double L, int ncells, const double *f, const long long *d_f_off,
                              double2 *scratch, void *out, bool out_f32, const long long *d_o_base,
                              long long o_stride, hipStream_t s);
// Inverse transform: Qhat element k of cell c at in + i_base[c] + k*i_stride,
// summed over `nparts` partial buffers spaced part_stride (complex units).
hipError_t launch_dft_inverse(int N, double L, int ncells, const double2 *in, const long long *d_i_base,
                              long long i_stride, int nparts, long long part_stride, double2 *scratch,
                              double *qt, const long long *d_q_off, hipStream_t s);

// Weight streams are padded so that the prefetch of the step after a row's last
// step (1 KiB granules) stays inside the buffer.
constexpr size_t kWeightPadBytes = 16384;

// One pass of the batched convolution: where its fhat copy, weights and
// output buffer are.  Offsets are in complex elements from fh and qh.
struct ConvPass {
    long long fh_off;            // fhat copy read by the pass
    long long out_off;           // first output buffer written by the pass
    const void *w;               // weight stream
    const long long *row_woff;   // device, N*N offsets of the rows in w (elements)
    int zero_planes;             // fhat copy has its k_d = 0 planes zeroed: skip steps with m2 = 0 or j2 = 0
    int row0;                    // first row the pass writes: row r goes to slot r - row0
    long long gstride;           // complex elements per group in the pass's output buffer
    long long pstride;           // complex elements between its partial-sum buffers
};
struct ConvPasses {
    ConvPass p[kPasses];
};

// Batched convolution over the (group, row | part << 16 | pass << 20, first
// step, end step) items of one mesh.
struct CellsLaunch {
    int N;
    const void *fh;              // [copies][G][N^3][64] float2 or double2
    const int4 *items;           // device, longest first
    int n_items;
    unsigned *counter;           // device, zeroed by the launcher's fill kernel
    double2 *qh;                 // output buffers of the passes (ConvPass.out_off, gstride, pstride)
    int variant;                 // tuning variant
    const unsigned char *skip;   // device, per group: 1 = outputs not needed (may be NULL)
    ConvPasses passes;
};
// Batched FP32 convolution of several meshes in one persistent launch: item words carry the
// mesh index (bits 24..27) into a device table of descriptors (uploaded when the weights are
// bound), ordered by cost (steps x pairs per step), longest first.
constexpr int kMaxMultiMeshes = 4;
struct MeshConvDesc {
    long long fh_bytes;          // fhat copies [copies][G][N^3][64] float2, offset in the workspace
    long long qh_bytes;          // output buffers, offset in the workspace
    int N;
    ConvPasses ps;
    // FP64 core of the mesh (core_r = 0: none): rows [G][nD][2r+1][64] and sums [G][N^3][64]
    // at these workspace offsets, core steps and core weights (device)
    long long cf_bytes, cq_bytes, cq_pstride;
    const int *core_steps;
    const int *core_ext;         // per disk row: its half-width in m3 inside the ball
    const double *core_w;
    int nD, core_r;
};
// bit 28 of an item's row word marks an FP64 core item in the one-launch queue
constexpr int kCoreItemBit = 1 << 28;
// most step pieces of one core row (bits 20..23 of a core item's row word)
constexpr int kCoreMaxParts = 4;
struct MultiLaunch {
    const int4 *items;
    int n_items;
    unsigned *counter;
    const MeshConvDesc *desc;    // device
    char *ws;                    // the call's workspace
    const unsigned char *skip;   // device, per group (one-mesh batches), may be NULL: groups to leave out
};
hipError_t launch_conv_cells_multi(const MultiLaunch &p, hipStream_t s);
hipError_t launch_build_e3(int N, const long long *d_row_woff, const long long *d_e3_woff, const void *w_main,
                           void *w_e3, bool f64, hipStream_t s);
// batched FP32 variants: count, and a rank that grows with the accuracy of the
// accumulation (more interleaved partials, then shorter fold interval)
int conv_variant_count();
int conv_variant_accuracy_rank(int v);
hipError_t launch_conv_cells(const CellsLaunch &p, bool f64, hipStream_t s);

// FP64 core sum of one mesh (CoreSched): items (group, output row | kind << 16 | piece << 20, first
// step, end step), longest first; kind 2 writes the outputs k3 - N/2 in [-2r, 2r], kind 0 those in
// [-2r, 0], kind 1 those in [1, 2r]; piece p of a row's steps writes partial sum p.
struct CoreLaunch {
    int N, r, nD;
    const double2 *cf;           // [G][nD][2r+1][64] FP64 core rows
    const int4 *items;
    int n_items;
    unsigned *counter;           // device, zeroed by the launcher's fill kernel
    const int *steps;            // device, CoreSched::steps
    const int *ext;              // device, CoreSched::disk_ext
    const double *w;             // core weight stream, core_wstride(r) doubles per step
    double2 *out;                // partial sums [piece][G][N^3][64], pstride apart (complex units)
    long long pstride;
    const unsigned char *skip;   // device, per group (may be NULL)
    int waves;                   // persistent grid in wavefronts (0: eight per CU)
};
hipError_t launch_conv_core(const CoreLaunch &p, hipStream_t s);

// Plain convolution of one cell.
struct PlainLaunch {
    int N;
    const void *fh;              // [N^3] float2 or double2
    const void *w;               // plain schedule weights
    const long long *blk_woff;   // device, N * (N / R)
    int nsplit;                  // m1 range split into nsplit partial sums
    double2 *qh;                 // [nsplit][N^3]
};
hipError_t launch_conv_plain(const PlainLaunch &p, bool f64, hipStream_t s);

// Diagnostics: per cell (f at f + off[c], mesh nn[c], spacing dvs[c]) rho, u1, u2, u3, T into
// mom[5 c ..]; the v1 marginal of one cell (f at f) into out[N].
hipError_t launch_cell_moments(int ncells, const double *f, const long long *off, const int *nn, const double *dvs,
                               double *mom, hipStream_t s);
hipError_t launch_marginal_v1(int N, double dv, const double *f, double *out, hipStream_t s);

// Projection (Sec. 3.3) of ncells cells of one mesh, in place, two passes.
hipError_t launch_project(int N, double dv, const double *linv, int ncells, double *q, const long long *d_off,
                          hipStream_t s);

// Heun helpers: out = a + c*q ; out = 0.5*(a + b + c*q); flag nonfinite.
hipError_t launch_axpy(size_t n, const double *a, const double *q, double c, double *out, unsigned *flag,
                       hipStream_t s);
hipError_t launch_heun_final(size_t n, const double *f, const double *fs, const double *q, double c, double *out,
                             unsigned *flag, hipStream_t s);
hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s);

// Gated closure helpers (bz_surrogate.hip).
// stats (may be NULL): the closure counters, whose gate cap (set by failed judges) lowers `gate`
hipError_t launch_sur_prepare(int N, double dv, int n, const double *f, const long long *f_off, double gate,
                              double s_in, int judge_every, int phase, const unsigned *stats, double *state,
                              unsigned short *x, hipStream_t s);
hipError_t launch_pack_slots(int n, const double *state, const long long *f_off, long long *slot_off,
                             unsigned char *skip, hipStream_t s);
hipError_t launch_sur_finish(int N, double dv, const double *linv, int n, const double *state, const float *y,
                             double s_out, double floor_, double tol, const long long *q_off, double *q,
                             unsigned *stats, hipStream_t s);
hipError_t launch_sur_targets(int N, int n, const double *state, const double *q, const long long *q_off,
                              double s_out, float *y, hipStream_t s);

}  // namespace bz
