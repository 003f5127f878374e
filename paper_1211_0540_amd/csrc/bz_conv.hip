// Weighted convolution of Sec. 3.2,
//   Qhat_k = sum_m Ghat(xi_m, zeta_k) fhat_m fhat_{k-m+N/2} dzeta^3,
// the O(N^6) step where the method spends its time (Sec. 3.2, Sec. 4).
//
// Two schedules:
//
// * Batched (lane = cell).  64 cells of one mesh share a wavefront, so every
//   weight is wavefront-uniform and is read once per 64 cells.  The weights of
//   a step are contiguous; while a step runs, the next step's weights are
//   copied HBM -> LDS by one coalesced direct-to-LDS load per 1 KiB
//   (global_load_lds_dwordx4) into the other half of a per-wave double buffer,
//   and the running step reads its weights with broadcast LDS reads.  (Reading
//   them through the scalar cache instead leaves only a few 64-byte requests in
//   flight and stalls every step on HBM latency.)  A work item is a range of
//   steps of one output row (k1, k2, 0..N-1) of 64 cells; it keeps
//   the row's N accumulators and, per step (m1, m2), the rows fhat(m1, m2, .)
//   and fhat(j1, j2, .) of its own cell in registers (cell-interleaved layout,
//   coalesced 512-byte loads).  Each unordered pair {m, j} is visited once
//   with the symmetrised weight (see bz_internal.h), so a step costs 6 VALU
//   operations per visited pair: 4 for the complex product fhat_m fhat_j and 2
//   FMAs that add its weighted parts to a fresh per-output partial of the step,
//   plus 2 additions per output and step into the running sums (and 2 more that
//   combine two interleaved partials, where a variant keeps two).  Work items are popped from an atomic
//   queue ordered longest first, so the launch is persistent.  Every item names
//   its pass of the conjugate-symmetric schedule (bz_internal.h): which fhat
//   copy it reads, which weight stream and which output buffer it writes; the
//   full-sum schedule uses pass A only.  Steps of pass A whose rows lie on a
//   zeroed plane of its fhat copy are skipped.
//
//   FP32 variant: products, per-step partials and a running sum over FOLD
//   steps in FP32 (the running sum takes one rounding per output and step);
//   every FOLD steps the running sum is folded into a compensated total:
//   an FP64 total in registers (COMP = 0), an FP32 (hi, lo) pair updated with
//   Knuth's error-free TwoSum (COMP = 1, Kahan-style compensation), or an FP64
//   total kept in the item's own output slot and updated by read-modify-write
//   (COMP = 2), which leaves the registers to fit two wavefronts per SIMD at
//   N = 32.  FP64 variant: everything FP64.
//
// * Plain (lane = output), one cell per launch: the lanes of a wavefront are R
//   output rows of one k1 plane; all lanes walk the same m, the weight of each
//   (lane, m) is streamed from HBM in a coalesced layout, fhat_m is uniform and
//   fhat_j is a per-lane read.  This is the paper's precompute-and-store
//   organisation; it is bound by the weight stream.
#include "bz_internal.h"

namespace bz {
namespace {

template <typename T>
struct cplx;
template <>
struct cplx<float> {
    using t = float2;
};
template <>
struct cplx<double> {
    using t = double2;
};

// TwoSum: hi + lo += p without losing the rounding error of the addition.
__device__ inline void two_sum_acc(float &hi, float &lo, float p) {
    const float s = hi + p;
    const float bp = s - hi;
    const float e = (hi - (s - bp)) + (p - bp);
    hi = s;
    lo += e;
}

// One step of the batched schedule for one row: for each output k3 its terms
// of the step are summed into fresh partials (SPLIT interleaved accumulators,
// combined pairwise), which are then added to the running sum once (one
// rounding of the running sum per output and step).
template <typename T, int N, int SPLIT, typename WP>
__device__ __forceinline__ void cells_step(const typename cplx<T>::t (&mv)[N], const typename cplx<T>::t (&jv)[N],
                                           WP w, T (&pr)[N], T (&pi)[N]) {
    constexpr int h = N / 2;
#pragma unroll
    for (int k3 = 0; k3 < N; ++k3) {
        const int mlo = k3 - h + 1 > 0 ? k3 - h + 1 : 0;
        const int mhi = k3 + h < N - 1 ? k3 + h : N - 1;
        T sr[SPLIT], si[SPLIT];
#pragma unroll
        for (int a = 0; a < SPLIT; ++a) sr[a] = si[a] = 0;
#pragma unroll
        for (int m3 = mlo; m3 <= mhi; ++m3) {
            const int j3 = k3 - m3 + h;
            const int a = (m3 - mlo) % SPLIT;
            const T wt = w[step_koff(N, k3) + (m3 - mlo)];
            // product fhat_m fhat_j first, then one rounding into a partial per term
            const T px = fma(mv[m3].x, jv[j3].x, -(mv[m3].y * jv[j3].y));
            const T py = fma(mv[m3].x, jv[j3].y, mv[m3].y * jv[j3].x);
            sr[a] = fma(wt, px, sr[a]);
            si[a] = fma(wt, py, si[a]);
        }
#pragma unroll
        for (int st = 1; st < SPLIT; st *= 2)
#pragma unroll
            for (int a = 0; a + st < SPLIT; a += 2 * st) {
                sr[a] += sr[a + st];
                si[a] += si[a + st];
            }
        pr[k3] += sr[0];
        pi[k3] += si[0];
    }
}

template <typename T, int N>
__device__ __forceinline__ void load_row(const typename cplx<T>::t *__restrict__ p, typename cplx<T>::t (&v)[N]) {
#pragma unroll
    for (int t = 0; t < N; ++t) v[t] = p[t * kWave];
}

// Copy `chunks` KiB of a step's weights from global memory to LDS: each lane
// moves 16 bytes per chunk, the wave 1 KiB, landing contiguously at dst.
typedef __attribute__((address_space(3))) char lds_char;

// LDS address of a __shared__ object, taken directly so that no generic-to-LDS
// conversion of a computed pointer is needed.
template <typename T>
__device__ __forceinline__ lds_char *lds_ptr(T *shared_obj) {
    return (lds_char *)shared_obj;
}

template <int CHUNKS>
__device__ __forceinline__ void prefetch_weights(const void *src, lds_char *dst) {
    const char *g = (const char *)src + threadIdx.x * 16;
#pragma unroll
    for (int c = 0; c < CHUNKS; ++c)
        __builtin_amdgcn_global_load_lds((const void *)(g + c * 1024), (void __attribute__((address_space(3))) *)(dst + c * 1024),
                                         16, 0, 0);
}

// Position (m1, m2) of step index s0 in the row's step enumeration.
template <int N>
__device__ __forceinline__ void seek_step(int k1, int k2, int s0, int &m1, int &m2) {
    const int lo2 = axis_lo(N, k2);
    m1 = axis_lo(N, k1);
    for (;;) {
        const int cnt = cells_m2_last(N, k1, k2, m1) - lo2 + 1;
        if (s0 < cnt) break;
        s0 -= cnt;
        ++m1;
    }
    m2 = lo2 + s0;
}

// The pass of an item (wavefront-uniform): its fhat copy, weights and output buffer.
__device__ __forceinline__ ConvPass pick_pass(const ConvPasses &ps, int pass) {
    ConvPass c = ps.p[0];
    if (pass == kPassE1) c = ps.p[kPassE1];
    if (pass == kPassE2) c = ps.p[kPassE2];
    if (pass == kPassE3) c = ps.p[kPassE3];
    if (pass == kPassZ) c = ps.p[kPassZ];
    return c;
}

__device__ inline int pop_item(unsigned *counter) {
    unsigned it = 0;
    if (threadIdx.x == 0) it = atomicAdd(counter, 1u);
    return (int)__builtin_amdgcn_readfirstlane(it);
}

// ---------------------------------------------------------------------------
// Batched FP32 with compensated accumulation.  One work item: the body is
// shared by the one-mesh kernel and by the kernel whose queue holds the items
// of several meshes (an item names its mesh; N is wavefront-uniform).
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) float lds_float;
typedef __attribute__((address_space(3))) double lds_double;

template <int N, int FOLD, int COMP, int WP, int RP, int SPLIT>
__device__ __forceinline__ void cells_f32_item(const float2 *__restrict__ fh, double2 *__restrict__ qh,
                                               const unsigned char *__restrict__ skip, const ConvPass &cp,
                                               const int4 item, lds_char *const wl, lds_char *const rl) {
    constexpr int h = N / 2, M = N * N * N, PS = 3 * N * N / 4;
    constexpr int CH = (PS * 4 + 1023) / 1024;       // KiB per step of weights
    constexpr int RCH = N * kWave * 8 / 1024;        // KiB per fhat row of 64 cells
    const int lane = threadIdx.x;
    const int g = item.x, r = item.y & 0xffff, part = (item.y >> 16) & 0xf, s0 = item.z, s1 = item.w;
    const int k1 = r / N, k2 = r - k1 * N;
    double2 *const out = qh + cp.out_off + part * cp.pstride + g * cp.gstride + (size_t)(r - cp.row0) * N * kWave + lane;
    if (skip && skip[g]) {
        // every cell of the group is served elsewhere: leave zeros in this item's outputs
#pragma unroll
        for (int t = 0; t < N; ++t) out[t * kWave] = make_double2(0.0, 0.0);
        return;
    }
    const float *w = (const float *)cp.w + cp.row_woff[r] + (long long)s0 * PS;
    const float2 *G = fh + cp.fh_off + (size_t)g * M * kWave;   // this group's fhat (copy of the pass)
    const float2 *F = G + lane;
    const lds_float *const rbuf = (const lds_float *)rl;   // rows as (re, im) float pairs

    float pr[N], pi[N];
    float hr[N], hi[N], lr[N], li[N];
    double dr[N], di[N];
#pragma unroll
    for (int t = 0; t < N; ++t) {
        pr[t] = pi[t] = 0.f;
        if (COMP == 1) hr[t] = hi[t] = lr[t] = li[t] = 0.f;
        else if (COMP == 0) dr[t] = di[t] = 0.0;
    }
    bool first = true;
    auto fold = [&]() {
        if (COMP == 2) {
            // the FP64 total lives in this item's own output slot (no other item writes it)
#pragma unroll
            for (int t = 0; t < N; ++t) {
                double2 o = make_double2(0.0, 0.0);
                if (!first) o = out[t * kWave];
                o.x += (double)pr[t];
                o.y += (double)pi[t];
                out[t * kWave] = o;
                pr[t] = pi[t] = 0.f;
            }
            first = false;
            return;
        }
#pragma unroll
        for (int t = 0; t < N; ++t) {
            if (COMP == 1) {
                two_sum_acc(hr[t], lr[t], pr[t]);
                two_sum_acc(hi[t], li[t], pi[t]);
            } else {
                dr[t] += (double)pr[t];
                di[t] += (double)pi[t];
            }
            pr[t] = pi[t] = 0.f;
        }
    };
    // rows of step (m1, m2): fhat(m1, m2, .) and fhat(j1, j2, .) of the 64 cells, N/2 KiB each
    auto prefetch_rows = [&](int a1, int a2) {
        prefetch_weights<RCH>(G + (size_t)((a1 * N + a2) * N) * kWave, rl);
        prefetch_weights<RCH>(G + (size_t)(((k1 + h - a1) * N + (k2 + h - a2)) * N) * kWave, rl + RCH * 1024);
    };

    int m1, m2;
    seek_step<N>(k1, k2, s0, m1, m2);
    const int lo2 = axis_lo(N, k2);
    prefetch_weights<CH>(w, wl);
    if (RP && s0 < s1) prefetch_rows(m1, m2);
    __builtin_amdgcn_s_waitcnt(0);
    int buf = 0, nst = 0;
    for (int s = s0; s < s1; ++s) {
        const int j1 = k1 + h - m1, j2 = k2 + h - m2;
        // on a plane-zeroed copy a step with m2 = 0 or j2 = 0 has only zero products
        const bool live = !cp.zero_planes || (m2 != 0 && j2 != 0);
        // (m1, m2) of the next step in the row's order
        int n1 = m1, n2 = m2 + 1;
        if (n2 > cells_m2_last(N, k1, k2, m1)) {
            ++n1;
            n2 = lo2;
        }
        float2 mv[N], jv[N];
        if (RP) {
#pragma unroll
            for (int t = 0; t < N; ++t) {
                const int a = 2 * (t * kWave + lane), b = 2 * (N * kWave + t * kWave + lane);
                mv[t] = make_float2(rbuf[a], rbuf[a + 1]);
                jv[t] = make_float2(rbuf[b], rbuf[b + 1]);
            }
            __builtin_amdgcn_s_waitcnt(0);        // rows are in registers: the buffer is free
            if (s + 1 < s1) prefetch_rows(n1, n2);
        } else {
            load_row<float, N>(F + (size_t)((m1 * N + m2) * N) * kWave, mv);
            load_row<float, N>(F + (size_t)((j1 * N + j2) * N) * kWave, jv);
        }
        if (WP == 0) {
            // next step's weights into the other LDS half; this step reads its half
            prefetch_weights<CH>(w + PS, wl + (buf ^ 1) * CH * 1024);
            if (live) cells_step<float, N, SPLIT>(mv, jv, (const lds_float *)(wl + buf * CH * 1024), pr, pi);
        } else if (WP == 1) {
            // next step's weights pulled into L2 (the LDS copy is discarded); this
            // step's weights, pulled last step, are read through the scalar cache
            prefetch_weights<CH>(w + PS, wl + CH * 1024);
            if (live)
                cells_step<float, N, SPLIT>(mv, jv, (const __attribute__((address_space(4))) float *)w, pr, pi);
        } else {
            // as 1, but the weights are read by uniform-address vector loads
            prefetch_weights<CH>(w + PS, wl + CH * 1024);
            if (live) cells_step<float, N, SPLIT>(mv, jv, w, pr, pi);
        }
        w += PS;
        buf ^= 1;
        if (++nst == FOLD) {
            fold();
            nst = 0;
        }
        m1 = n1;
        m2 = n2;
        __builtin_amdgcn_s_waitcnt(0);
    }
    fold();
    if (COMP == 2) return;
#pragma unroll
    for (int t = 0; t < N; ++t) {
        if (COMP == 1)
            out[t * kWave] = make_double2((double)hr[t] + (double)lr[t], (double)hi[t] + (double)li[t]);
        else
            out[t * kWave] = make_double2(dr[t], di[t]);
    }
}

template <int N, int FOLD, int COMP, int WP, int RP, int SPLIT>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(COMP == 2 ? 2 : 1)))
k_conv_cells_f32(const float2 *__restrict__ fh, const int4 *__restrict__ items, int n_items,
                 unsigned *__restrict__ counter, double2 *__restrict__ qh,
                 const unsigned char *__restrict__ skip, const ConvPasses ps) {
    constexpr int PS = 3 * N * N / 4;
    constexpr int CH = (PS * 4 + 1023) / 1024;
    __shared__ __attribute__((aligned(16))) float wbuf[2][CH * 256];
    __shared__ __attribute__((aligned(16))) float2 rbuf[RP ? 2 * N * kWave : 2];
    lds_char *const wl = lds_ptr(&wbuf[0][0]);
    lds_char *const rl = lds_ptr(&rbuf[0]);
    for (;;) {
        const int it = pop_item(counter);
        if (it >= n_items) break;
        const int4 item = items[it];
        const ConvPass cp = pick_pass(ps, (item.y >> 20) & 0xf);
        cells_f32_item<N, FOLD, COMP, WP, RP, SPLIT>(fh, qh, skip, cp, item, wl, rl);
    }
}

// ---------------------------------------------------------------------------
// FP64 core of the batched FP32 mode (CoreSched in bz_internal.h): the pairs
// whose two partners lie in the low-frequency ball carry the largest terms of
// the sum, so they are summed here in FP64 from FP64 fhat, with FP64 weights.
// Lane = cell, like the batched kernels; an item is one output row of one
// group.  A step loads its two rows (2R + 1 values each) and reads its
// (2R + 1)^2 weights from LDS, copied there during the previous step.  Item
// kinds (bits 16..17 of the row word): 2 = every output of the row
// (k3 - N/2 in [-2R, 2R]); 0 = only k3 - N/2 in [-2R, 0] (rows whose other
// outputs follow from conjugate symmetry); 1 = only [1, 2R].  A full row
// loads each row value once for 2R + 1 products.
// ---------------------------------------------------------------------------
template <int R, int KIND>
struct CoreOut {
    static constexpr int lo = KIND == 1 ? 1 : -2 * R;
    static constexpr int hi = KIND == 0 ? 0 : 2 * R;
    static constexpr int n = hi - lo + 1;
};

// am, aj: the half-widths of the two rows inside the ball (wavefront-uniform); entries beyond
// them are zero, so they are neither loaded nor multiplied.
template <int R, int KIND>
__device__ __forceinline__ void core_step(const double2 *pm, const double2 *pj, int am, int aj, const lds_double *wl,
                                          double2 (&acc)[CoreOut<R, KIND>::n]) {
    constexpr int S = 2 * R + 1, LO = CoreOut<R, KIND>::lo, HI = CoreOut<R, KIND>::hi;
    double2 jr[S];
#pragma unroll
    for (int t = 0; t < S; ++t) jr[t] = abs(t - R) <= aj ? pj[t * kWave] : make_double2(0.0, 0.0);
#pragma unroll
    for (int tm = 0; tm < S; ++tm) {
        if (abs(tm - R) > am) continue;
        const double2 mv = pm[tm * kWave];
#pragma unroll
        for (int tj = 0; tj < S; ++tj) {
            const int e = tm + tj - 2 * R;   // k3 - N/2
            if (e >= LO && e <= HI && abs(tj - R) <= aj) {
                const double wt = wl[tm * S + tj];
                const double px = fma(mv.x, jr[tj].x, -(mv.y * jr[tj].y));
                const double py = fma(mv.x, jr[tj].y, mv.y * jr[tj].x);
                acc[e - LO].x = fma(wt, px, acc[e - LO].x);
                acc[e - LO].y = fma(wt, py, acc[e - LO].y);
            }
        }
    }
}

template <int R, int KIND>
__device__ __forceinline__ void core_rows(int N, const double2 *G, const int *steps, const int *ext, const double *ws,
                                          int s0, int s1, double2 *o, lds_char *wl) {
    constexpr int S = 2 * R + 1, WS = core_wstride(R), CH = WS * 8 / 1024;
    constexpr int LO = CoreOut<R, KIND>::lo, NO = CoreOut<R, KIND>::n;
    const int h = N / 2;
    double2 acc[NO];
#pragma unroll
    for (int a = 0; a < NO; ++a) acc[a] = make_double2(0.0, 0.0);
    if (s0 < s1) prefetch_weights<CH>(ws, wl);
    __builtin_amdgcn_s_waitcnt(0);
    int buf = 0;
    for (int s = s0; s < s1; ++s) {
        const int st = steps[s], dm = st & 0xffff, dj = st >> 16;
        const double2 *pm = G + (size_t)dm * S * kWave;
        const double2 *pj = G + (size_t)dj * S * kWave;
        if (s + 1 < s1) prefetch_weights<CH>(ws + WS, wl + (buf ^ 1) * WS * 8);
        core_step<R, KIND>(pm, pj, ext[dm], ext[dj], (const lds_double *)(wl + buf * WS * 8), acc);
        ws += WS;
        buf ^= 1;
        __builtin_amdgcn_s_waitcnt(0);
    }
#pragma unroll
    for (int a = 0; a < NO; ++a) {
        const int k3 = h + LO + a;
        if (k3 >= 0 && k3 < N) o[k3 * kWave] = acc[a];
    }
}

// One core item: group g, output row, kind; rows of the group from cf, weights of
// step s at w + s * core_wstride(R), outputs into out [G][N^3][64].
template <int R>
__device__ __forceinline__ void core_item(int N, int nD, const double2 *cf, const int *steps, const int *ext,
                                          const double *w, double2 *out, long long pstride, const int4 item,
                                          lds_char *wl) {
    constexpr int S = 2 * R + 1, WS = core_wstride(R);
    const int lane = threadIdx.x;
    const int g = item.x, row = item.y & 0xffff, kind = (item.y >> 16) & 3, piece = (item.y >> 20) & 0xf;
    const int s0 = item.z, s1 = item.w;
    double2 *const o = out + (size_t)piece * pstride + ((size_t)g * N * N * N + (size_t)row * N) * kWave + lane;
    const double2 *const G = cf + (size_t)g * nD * S * kWave + lane;
    const double *ws = w + (size_t)s0 * WS;
    if (kind == 2) core_rows<R, 2>(N, G, steps, ext, ws, s0, s1, o, wl);
    else if (kind == 0) core_rows<R, 0>(N, G, steps, ext, ws, s0, s1, o, wl);
    else core_rows<R, 1>(N, G, steps, ext, ws, s0, s1, o, wl);
}

template <int R>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_conv_core(int N, int nD, const double2 *__restrict__ cf, const int4 *__restrict__ items, int n_items,
            unsigned *__restrict__ counter, const int *__restrict__ steps, const int *__restrict__ ext,
            const double *__restrict__ w, double2 *__restrict__ out, long long pstride,
            const unsigned char *__restrict__ skip) {
    __shared__ __attribute__((aligned(16))) double wbuf[2 * core_wstride(R)];
    lds_char *const wl = lds_ptr(&wbuf[0]);
    for (;;) {
        const int it = pop_item(counter);
        if (it >= n_items) break;
        const int4 item = items[it];
        if (skip && skip[item.x]) continue;   // the closure serves every cell of the group
        core_item<R>(N, nD, cf, steps, ext, w, out, pstride, item, wl);
    }
}

// Items of several meshes in one persistent launch: the mesh index sits in bits 24..27
// of the item word; its descriptor (N, buffer offsets in the workspace, one ConvPass per
// pass, its FP64 core) is read from a device table with wavefront-uniform loads.  Every
// mesh runs the output-slot accumulation with FOLD 16 and two interleaved partials
// (tuning variant 12: with the FP64 core as accurate as four, and 1% faster), two
// wavefronts per SIMD.  Items with kCoreItemBit are rows of an
// FP64 core (core_item): spread through the queue, their row loads overlap the FP32
// arithmetic of the other wavefront on the SIMD.
template <int N>
__device__ __forceinline__ void multi_item(const MeshConvDesc &d, char *ws, int pass, const int4 item, lds_char *wl) {
    const ConvPass cp = d.ps.p[pass];
    cells_f32_item<N, 16, 2, 0, 0, 2>((const float2 *)(ws + d.fh_bytes), (double2 *)(ws + d.qh_bytes), nullptr, cp,
                                      item, wl, nullptr);
}

template <int R>
__device__ __forceinline__ void multi_core(const MeshConvDesc &d, char *ws, const int4 item, lds_char *wl) {
    core_item<R>(d.N, d.nD, (const double2 *)(ws + d.cf_bytes), d.core_steps, d.core_ext, d.core_w,
                 (double2 *)(ws + d.cq_bytes), d.cq_pstride, item, wl);
}

// LDS of the one-launch kernel: the largest FP32 step's weights (N = 32: 3 KiB) or the largest
// core step's (r = 8: 17^2 doubles padded to 3 KiB), double-buffered
constexpr int kMultiLdsBytes = 2 * 3 * 1024;
static_assert(2 * core_wstride(kCoreMaxR) * 8 <= kMultiLdsBytes, "core weights exceed the one-launch LDS buffer");

__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2)))
k_conv_cells_f32_multi(const int4 *__restrict__ items, int n_items, unsigned *__restrict__ counter,
                       const MeshConvDesc *__restrict__ desc, char *__restrict__ ws,
                       const unsigned char *__restrict__ skip) {
    __shared__ __attribute__((aligned(16))) double wbuf[kMultiLdsBytes / 8];
    lds_char *const wl = lds_ptr(&wbuf[0]);
    for (;;) {
        const int it = pop_item(counter);
        if (it >= n_items) break;
        const int4 item = items[it];
        // a group whose cells are all served elsewhere: nothing reads its outputs
        if (skip && skip[item.x]) continue;
        const int mi = (item.y >> 24) & 0xf, pass = (item.y >> 20) & 0xf;
        const MeshConvDesc &d = desc[mi];
        if (item.y & kCoreItemBit) {
            const int4 ci = make_int4(item.x, item.y & 0xffffff, item.z, item.w);
            switch (d.core_r) {
            case 1: multi_core<1>(d, ws, ci, wl); break;
            case 2: multi_core<2>(d, ws, ci, wl); break;
            case 3: multi_core<3>(d, ws, ci, wl); break;
            case 4: multi_core<4>(d, ws, ci, wl); break;
            case 5: multi_core<5>(d, ws, ci, wl); break;
            case 6: multi_core<6>(d, ws, ci, wl); break;
            case 7: multi_core<7>(d, ws, ci, wl); break;
            default: multi_core<8>(d, ws, ci, wl); break;
            }
            continue;
        }
        switch (d.N) {
        case 8: multi_item<8>(d, ws, pass, item, wl); break;
        case 12: multi_item<12>(d, ws, pass, item, wl); break;
        case 16: multi_item<16>(d, ws, pass, item, wl); break;
        case 20: multi_item<20>(d, ws, pass, item, wl); break;
        case 24: multi_item<24>(d, ws, pass, item, wl); break;
        case 28: multi_item<28>(d, ws, pass, item, wl); break;
        default: multi_item<32>(d, ws, pass, item, wl); break;
        }
    }
}

// ---------------------------------------------------------------------------
// Batched FP64.
// ---------------------------------------------------------------------------
template <int N>
__global__ void __launch_bounds__(64) k_conv_cells_f64(const double2 *__restrict__ fh, const int4 *__restrict__ items,
                                                       int n_items, unsigned *__restrict__ counter,
                                                       double2 *__restrict__ qh,
                                                       const unsigned char *__restrict__ skip, const ConvPasses ps) {
    constexpr int h = N / 2, M = N * N * N, PS = 3 * N * N / 4;
    constexpr int CH = (PS * 8 + 1023) / 1024;
    __shared__ __attribute__((aligned(16))) double wbuf[2][CH * 128];
    lds_char *const wl = lds_ptr(&wbuf[0][0]);
    const int lane = threadIdx.x;
    for (;;) {
        const int it = pop_item(counter);
        if (it >= n_items) break;
        const int4 item = items[it];
        const int g = item.x, r = item.y & 0xffff, part = (item.y >> 16) & 0xf, s0 = item.z, s1 = item.w;
        const ConvPass cp = pick_pass(ps, (item.y >> 20) & 0xf);
        const int k1 = r / N, k2 = r - k1 * N;
        double2 *const out = qh + cp.out_off + part * cp.pstride + g * cp.gstride + (size_t)(r - cp.row0) * N * kWave + lane;
        if (skip && skip[g]) {
            // every cell of the group is served elsewhere: leave zeros in this item's outputs
#pragma unroll
            for (int t = 0; t < N; ++t) out[t * kWave] = make_double2(0.0, 0.0);
            continue;
        }
        const double *w = (const double *)cp.w + cp.row_woff[r] + (long long)s0 * PS;
        const double2 *F = fh + cp.fh_off + (size_t)g * M * kWave + lane;
        double pr[N], pi[N];
#pragma unroll
        for (int t = 0; t < N; ++t) pr[t] = pi[t] = 0.0;
        int m1, m2;
        seek_step<N>(k1, k2, s0, m1, m2);
        const int lo2 = axis_lo(N, k2);
        prefetch_weights<CH>(w, wl);
        __builtin_amdgcn_s_waitcnt(0);
        int buf = 0;
        for (int s = s0; s < s1; ++s) {
            const int j1 = k1 + h - m1, j2 = k2 + h - m2;
            prefetch_weights<CH>(w + PS, wl + (buf ^ 1) * CH * 1024);
            double2 mv[N], jv[N];
            load_row<double, N>(F + (size_t)((m1 * N + m2) * N) * kWave, mv);
            load_row<double, N>(F + (size_t)((j1 * N + j2) * N) * kWave, jv);
            if (!cp.zero_planes || (m2 != 0 && j2 != 0))
                cells_step<double, N, 1>(mv, jv, (const double *)wbuf[buf], pr, pi);
            w += PS;
            buf ^= 1;
            if (++m2 > cells_m2_last(N, k1, k2, m1)) {
                ++m1;
                m2 = lo2;
            }
            __builtin_amdgcn_s_waitcnt(0);
        }
#pragma unroll
        for (int t = 0; t < N; ++t) out[t * kWave] = make_double2(pr[t], pi[t]);
    }
}

// ---------------------------------------------------------------------------
// Plain schedule, one cell.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int plain_rows_c(int N) {
    int R = kWave / N;
    while (R > 1 && N % R) --R;
    return R;
}

template <typename T, int N>
__global__ void __launch_bounds__(64) k_conv_plain(const typename cplx<T>::t *__restrict__ fh,
                                                   const T *__restrict__ W, const long long *__restrict__ blk_woff,
                                                   int nsplit, double2 *__restrict__ qh) {
    using C = typename cplx<T>::t;
    constexpr int h = N / 2, R = plain_rows_c(N), NB = N / R, LN = R * N, M = N * N * N;
    const int lane = threadIdx.x;
    const int b = blockIdx.x, s = blockIdx.y;
    const int k1 = b / NB, kb = b - k1 * NB;
    const bool active = lane < LN;
    const int r = active ? lane / N : 0, k3 = active ? lane - (lane / N) * N : 0;
    const int k2 = kb * R + r;
    const int lo1 = axis_lo(N, k1), c1 = axis_cnt(N, k1);
    const int u2lo = plain_u2_lo(N, kb), U2 = plain_u2_hi(N, kb) - u2lo + 1;
    const int ma = lo1 + (s * c1) / nsplit, mb = lo1 + ((s + 1) * c1) / nsplit;
    const T *w = W + blk_woff[b] + (long long)(ma - lo1) * U2 * N * LN + (active ? lane : 0);
    double ar = 0.0, ai = 0.0;
    for (int m1 = ma; m1 < mb; ++m1) {
        const int j1 = k1 + h - m1;
        for (int m2 = u2lo; m2 < u2lo + U2; ++m2) {
            int j2 = k2 + h - m2;
            j2 = j2 < 0 ? 0 : (j2 > N - 1 ? N - 1 : j2);
            const C *rowm = fh + (m1 * N + m2) * N;
            const C *rowj = fh + (j1 * N + j2) * N;
            T pr = 0, pi = 0;
#pragma unroll
            for (int m3 = 0; m3 < N; ++m3) {
                int j3 = k3 + h - m3;
                j3 = j3 < 0 ? 0 : (j3 > N - 1 ? N - 1 : j3);
                const C a = rowm[m3];
                const C bb = rowj[j3];
                const T wt = w[m3 * LN];
                const T px = fma(a.x, bb.x, -(a.y * bb.y));
                const T py = fma(a.x, bb.y, a.y * bb.x);
                pr = fma(wt, px, pr);
                pi = fma(wt, py, pi);
            }
            w += N * LN;
            ar += (double)pr;
            ai += (double)pi;
        }
    }
    if (active) qh[(size_t)s * M + ((size_t)k1 * N + k2) * N + k3] = make_double2(ar, ai);
}

// Tuning variants of the batched FP32 kernel: (fold interval, compensation, weight path, row path).
//   0: FOLD 2, FP64 total,   LDS double-buffered weights, rows prefetched to LDS   (default)
//   1: FOLD 2, TwoSum total, LDS double-buffered weights, rows prefetched to LDS
//   2: FOLD 2, FP64 total,   LDS double-buffered weights, rows loaded per step
//   3: FOLD 2, TwoSum total, LDS double-buffered weights, rows loaded per step
//   4: FOLD 2, FP64 total,   scalar weights + L2 prefetch, rows prefetched to LDS
//   5: FOLD 4, FP64 total,   LDS double-buffered weights, rows prefetched to LDS
//   6: FOLD 2, FP64 total kept in the output slot (read-modify-write per fold), LDS
//      double-buffered weights, rows loaded per step; fits two wavefronts per SIMD
//   7: as 6 with FOLD 4
//   8: as 6 with FOLD 8
//   9: as 6 with FOLD 16
//  10: as 9 with four interleaved partials per output and step (pairwise combined)
//  11: as 10 with FOLD 8
//  12: as 10 with two interleaved partials
//  13: as 5 with four interleaved partials
//  14: as 10 with FOLD 4
//  15: as 10 with FOLD 2
// Accumulation parameters of each variant (must match the switch below): the
// autotuner prefers more interleaved partials, then a shorter fold interval.
struct VariantAcc {
    int fold, split;
};
constexpr VariantAcc kVariantAcc[] = {{2, 1}, {2, 1}, {2, 1}, {2, 1}, {2, 1},  {4, 1},  {2, 1},
                                      {4, 1}, {8, 1}, {16, 1}, {16, 4}, {8, 4}, {16, 2}, {4, 4},
                                      {4, 4}, {2, 4}};

template <int N>
hipError_t cells_f32_variant(const CellsLaunch &p, unsigned grid, hipStream_t s) {
#define BZ_CELLS_F32(F, C, WPV, RPV, SP)                                                                    \
    hipLaunchKernelGGL((k_conv_cells_f32<N, F, C, WPV, RPV, SP>), dim3(grid), dim3(64), 0, s,               \
                       (const float2 *)p.fh, p.items, p.n_items, p.counter, p.qh, p.skip, p.passes)
    switch (p.variant) {
    case 1: BZ_CELLS_F32(2, 1, 0, 1, 1); break;
    case 2: BZ_CELLS_F32(2, 0, 0, 0, 1); break;
    case 3: BZ_CELLS_F32(2, 1, 0, 0, 1); break;
    case 4: BZ_CELLS_F32(2, 0, 1, 1, 1); break;
    case 5: BZ_CELLS_F32(4, 0, 0, 1, 1); break;
    case 6: BZ_CELLS_F32(2, 2, 0, 0, 1); break;
    case 7: BZ_CELLS_F32(4, 2, 0, 0, 1); break;
    case 8: BZ_CELLS_F32(8, 2, 0, 0, 1); break;
    case 9: BZ_CELLS_F32(16, 2, 0, 0, 1); break;
    case 10: BZ_CELLS_F32(16, 2, 0, 0, 4); break;
    case 11: BZ_CELLS_F32(8, 2, 0, 0, 4); break;
    case 12: BZ_CELLS_F32(16, 2, 0, 0, 2); break;
    case 13: BZ_CELLS_F32(4, 0, 0, 1, 4); break;
    case 14: BZ_CELLS_F32(4, 2, 0, 0, 4); break;
    case 15: BZ_CELLS_F32(2, 2, 0, 0, 4); break;
    default: BZ_CELLS_F32(2, 0, 0, 1, 1); break;
    }
#undef BZ_CELLS_F32
    return hipGetLastError();
}

template <int N>
hipError_t cells_f64_launch(const CellsLaunch &p, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL((k_conv_cells_f64<N>), dim3(grid), dim3(64), 0, s, (const double2 *)p.fh, p.items,
                       p.n_items, p.counter, p.qh, p.skip, p.passes);
    return hipGetLastError();
}

template <typename T, int N>
hipError_t plain_launch(const PlainLaunch &p, hipStream_t s) {
    const int nb = N * (N / plain_rows_c(N));
    hipLaunchKernelGGL((k_conv_plain<T, N>), dim3(nb, p.nsplit), dim3(64), 0, s,
                       (const typename cplx<T>::t *)p.fh, (const T *)p.w, p.blk_woff, p.nsplit, p.qh);
    return hipGetLastError();
}

}  // namespace

int conv_variant_count() { return (int)(sizeof(kVariantAcc) / sizeof(kVariantAcc[0])); }

// The compensation form does not enter the rank: the FP64 total (in registers or in the
// output slot) and the TwoSum (hi, lo) pair both carry the folded total to at least 48
// bits, far below the FP32 rounding of the running sum between folds, which the fold
// interval and the interleaved partials set.
int conv_variant_accuracy_rank(int v) {
    if (v < 0 || v >= conv_variant_count()) return -1;
    return kVariantAcc[v].split * 1000 - kVariantAcc[v].fold;
}

// Persistent grid: enough single-wave workgroups to keep every SIMD busy.
static unsigned persistent_grid(int n_items) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    unsigned g = (unsigned)cus * 8u;
    return (unsigned)n_items < g ? (unsigned)n_items : g;
}

template <int R>
hipError_t core_launch(const CoreLaunch &p, unsigned grid, hipStream_t s) {
    hipLaunchKernelGGL(k_conv_core<R>, dim3(grid), dim3(64), 0, s, p.N, p.nD, p.cf, p.items, p.n_items, p.counter,
                       p.steps, p.ext, p.w, p.out, p.pstride, p.skip);
    return hipGetLastError();
}

hipError_t launch_conv_cells_multi(const MultiLaunch &p, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    hipError_t e = launch_fill_u32(p.counter, 1, 0u, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_conv_cells_f32_multi, dim3(persistent_grid(p.n_items)), dim3(64), 0, s, p.items, p.n_items,
                       p.counter, p.desc, p.ws, p.skip);
    return hipGetLastError();
}

hipError_t launch_conv_core(const CoreLaunch &p, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    if (p.r < 1 || p.r > kCoreMaxR) return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32(p.counter, 1, 0u, s);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int want = p.waves > 0 ? p.waves : 8 * cus;
    const unsigned grid = (unsigned)(p.n_items < want ? p.n_items : want);
    switch (p.r) {
    case 1: return core_launch<1>(p, grid, s);
    case 2: return core_launch<2>(p, grid, s);
    case 3: return core_launch<3>(p, grid, s);
    case 4: return core_launch<4>(p, grid, s);
    case 5: return core_launch<5>(p, grid, s);
    case 6: return core_launch<6>(p, grid, s);
    case 7: return core_launch<7>(p, grid, s);
    default: return core_launch<8>(p, grid, s);
    }
}

#define BZ_FOR_EACH_N(X) X(8) X(12) X(16) X(20) X(24) X(28) X(32)

hipError_t launch_conv_cells(const CellsLaunch &p, bool f64, hipStream_t s) {
    if (p.n_items <= 0) return hipSuccess;
    hipError_t e = launch_fill_u32(p.counter, 1, 0u, s);
    if (e != hipSuccess) return e;
    const unsigned grid = persistent_grid(p.n_items);
#define CASE(NN)                                                                                   \
    case NN:                                                                                       \
        return f64 ? cells_f64_launch<NN>(p, grid, s) : cells_f32_variant<NN>(p, grid, s);
    switch (p.N) {
        BZ_FOR_EACH_N(CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef CASE
}

hipError_t launch_conv_plain(const PlainLaunch &p, bool f64, hipStream_t s) {
#define CASE(NN) \
    case NN:     \
        return f64 ? plain_launch<double, NN>(p, s) : plain_launch<float, NN>(p, s);
    switch (p.N) {
        BZ_FOR_EACH_N(CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef CASE
}

}  // namespace bz
