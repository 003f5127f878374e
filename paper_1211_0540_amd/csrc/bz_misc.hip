// Conservation projection (Sec. 3.3), Heun update helpers (Sec. 3.1) and the
// expansion of the universal weight table into the schedules' weight streams
// (Sec. 2.2 eq. GHat_calc).  FP64 throughout.
#include "bz_internal.h"

namespace bz {
namespace {

// ---------------------------------------------------------------------------
// Projection.  C has rows dv^3 {1, v1, v2, v3, |v|^2}.  With C C^T = L L^T,
// the rows of E = L^{-1} C are orthonormal and the minimiser of |Qt - Q|^2
// subject to C Q = 0 is Q = Qt - E^T (E Qt), the same operator as
// Qt - C^T (C C^T)^{-1} C Qt but applied through an orthonormal basis.  Per
// cell the five raw moments s = C Qt are reduced in FP64 (per-thread sums,
// wavefront shuffles, then LDS in a fixed order), mu = L^{-1} s and
// nu = L^{-T} mu follow once per cell, and each value takes the correction
// (C^T nu)_j = dv^3 (nu_0 + nu_1 v1 + nu_2 v2 + nu_3 v3 + nu_4 |v|^2); the
// projection is applied twice, the second pass removing the rounding residue
// of the first.
// ---------------------------------------------------------------------------
struct Linv {
    double a[25];
};

// the velocity of mesh point j
__device__ inline void mesh_v(int N, double dv, int j, double &v1, double &v2, double &v3) {
    const int j1 = j / (N * N), j2 = (j / N) % N, j3 = j % N;
    v1 = dv * (j1 - N / 2);
    v2 = dv * (j2 - N / 2);
    v3 = dv * (j3 - N / 2);
}

__device__ inline double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Two layouts of the cell over a block's threads, both keeping every value in registers through
// both passes (the cell is read and written once).
// N <= 24: one block per cell, N^2 threads rounded up to whole wavefronts: thread t < N^2 owns
// the column (j2, j3) = (t / N, t % N), its N values j = t + N^2 j1, so v2 and v3 are fixed per
// thread and v1 = dv (j1 - N/2) needs no index arithmetic; the threads past N^2 hold zeros.
// Smaller blocks also let a CU hold several cells, whose phases (loads, reductions, stores)
// then overlap: 16 against 36 us at N=16 and 36 against 45 us at N=24 for the flat layout
// below.  From N = 28 on, N values per thread no longer fit the registers of the wider block
// without spilling, and the flat layout is faster.
constexpr int kProjThreads = 1024;
template <int N>
constexpr int proj_threads() {
    return (N * N + 63) / 64 * 64;
}
template <int N>
__global__ void __launch_bounds__(proj_threads<N>()) k_project_cols(double dv, Linv li, double *__restrict__ q,
                                                               const long long *__restrict__ off) {
    constexpr int P = N * N;
    static_assert(proj_threads<N>() <= kProjThreads, "one thread per column");
    __shared__ double red[kProjThreads / 64][5];
    __shared__ double nu[5];
    double *Q = q + off[blockIdx.x];
    const int t = threadIdx.x, wid = t >> 6, lane = t & 63;
    const bool own = t < P;
    const double v2 = dv * (t / N - N / 2), v3 = dv * (t % N - N / 2), r23 = v2 * v2 + v3 * v3;
    double x[N];
#pragma unroll
    for (int i = 0; i < N; ++i) x[i] = own ? Q[t + P * i] : 0.0;
    const double w = dv * dv * dv;
    for (int pass = 0; pass < 2; ++pass) {
        // dv and each v1 through an empty asm, so that the N values of v1 (and v1^2) are
        // computed one at a time where they are used rather than kept live together
        double s[5] = {0, 0, 0, 0, 0};
        double dva = dv;
        asm volatile("" : "+v"(dva));
#pragma unroll
        for (int i = 0; i < N; ++i) {
            double v1 = dva * (i - N / 2);
            asm volatile("" : "+v"(v1));
            s[0] += x[i];
            s[1] = fma(v1, x[i], s[1]);
            s[2] = fma(v2, x[i], s[2]);
            s[3] = fma(v3, x[i], s[3]);
            s[4] = fma(fma(v1, v1, r23), x[i], s[4]);
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            double u = wave_sum(s[a]);
            if (lane == 0) red[wid][a] = u;
        }
        __syncthreads();
        if (t == 0) {
            double tt[5], m[5];
            for (int b = 0; b < 5; ++b) {
                double u = 0.0;
                for (int v = 0; v < (int)(blockDim.x >> 6); ++v) u += red[v][b];
                tt[b] = u * w;   // C Qt
            }
            for (int a = 0; a < 5; ++a) {   // mu = L^{-1} C Qt
                double u = 0.0;
                for (int b = 0; b <= a; ++b) u = fma(li.a[a * 5 + b], tt[b], u);
                m[a] = u;
            }
            for (int b = 0; b < 5; ++b) {   // nu = L^{-T} mu, dv^3 folded in
                double u = 0.0;
                for (int a = b; a < 5; ++a) u = fma(li.a[a * 5 + b], m[a], u);
                nu[b] = u * w;
            }
        }
        __syncthreads();
        // (the threads past N^2 keep their zeros for the second pass's sums)
        const double c0 = fma(nu[3], v3, fma(nu[2], v2, nu[0]));
        double dvb = dv;
        asm volatile("" : "+v"(dvb));
        if (own) {
#pragma unroll
            for (int i = 0; i < N; ++i) {
                double v1 = dvb * (i - N / 2);
                asm volatile("" : "+v"(v1));
                x[i] -= fma(nu[4], fma(v1, v1, r23), fma(nu[1], v1, c0));
            }
        }
        __syncthreads();
    }
    if (own) {
#pragma unroll
        for (int i = 0; i < N; ++i) Q[t + P * i] = x[i];
    }
}

// N >= 28: one block of kProjThreads threads per cell.  Thread t owns the values j = t + i kProjThreads,
// i < PER = ceil(N^3 / kProjThreads), and keeps them in registers through both passes, so the
// cell is read and written once.  Indices and velocities are recomputed in every loop (the
// empty asm hides the thread index from common-subexpression elimination, which would otherwise
// keep PER indices and 3 PER velocities live across the passes and spill them).
template <int N>
__global__ void __launch_bounds__(kProjThreads) k_project_flat(double dv, Linv li, double *__restrict__ q,
                                                          const long long *__restrict__ off) {
    constexpr int M = N * N * N, PER = (M + kProjThreads - 1) / kProjThreads;
    __shared__ double red[kProjThreads / 64][5];
    __shared__ double nu[5];
    double *Q = q + off[blockIdx.x];
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    double x[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = threadIdx.x + i * kProjThreads;
        x[i] = j < M ? Q[j] : 0.0;
    }
    const double w = dv * dv * dv;
    for (int pass = 0; pass < 2; ++pass) {
        double s[5] = {0, 0, 0, 0, 0};
        int tr = threadIdx.x;
        asm volatile("" : "+v"(tr));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = tr + i * kProjThreads;
            if (j < M) {
                double v1, v2, v3;
                mesh_v(N, dv, j, v1, v2, v3);
                s[0] += x[i];
                s[1] = fma(v1, x[i], s[1]);
                s[2] = fma(v2, x[i], s[2]);
                s[3] = fma(v3, x[i], s[3]);
                s[4] = fma(v1 * v1 + v2 * v2 + v3 * v3, x[i], s[4]);
            }
        }
#pragma unroll
        for (int a = 0; a < 5; ++a) {
            double t = wave_sum(s[a]);
            if (lane == 0) red[wid][a] = t;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t[5], m[5];
            for (int b = 0; b < 5; ++b) {
                double u = 0.0;
                for (int v = 0; v < (int)(blockDim.x >> 6); ++v) u += red[v][b];
                t[b] = u * w;   // C Qt
            }
            for (int a = 0; a < 5; ++a) {   // mu = L^{-1} C Qt
                double u = 0.0;
                for (int b = 0; b <= a; ++b) u = fma(li.a[a * 5 + b], t[b], u);
                m[a] = u;
            }
            for (int b = 0; b < 5; ++b) {   // nu = L^{-T} mu, dv^3 folded in
                double u = 0.0;
                for (int a = b; a < 5; ++a) u = fma(li.a[a * 5 + b], m[a], u);
                nu[b] = u * w;
            }
        }
        __syncthreads();
        int tc = threadIdx.x;
        asm volatile("" : "+v"(tc));
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int j = tc + i * kProjThreads;
            if (j < M) {
                double v1, v2, v3;
                mesh_v(N, dv, j, v1, v2, v3);
                const double corr = fma(nu[4], v1 * v1 + v2 * v2 + v3 * v3,
                                        fma(nu[3], v3, fma(nu[2], v2, fma(nu[1], v1, nu[0]))));
                x[i] -= corr;
            }
        }
        __syncthreads();
    }
    int ts = threadIdx.x;
    asm volatile("" : "+v"(ts));
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = ts + i * kProjThreads;
        if (j < M) Q[j] = x[i];
    }
}

// ---------------------------------------------------------------------------
// Heun helpers and flag fill.
// ---------------------------------------------------------------------------
__global__ void k_axpy(size_t n, const double *__restrict__ a, const double *__restrict__ q, double c,
                       double *__restrict__ out, unsigned *flag) {
    bool bad = false;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double y = fma(c, q[i], a[i]);
        out[i] = y;
        bad |= !isfinite(y);
    }
    if (__syncthreads_or(bad ? 1 : 0) && threadIdx.x == 0) atomicOr(flag, 1u);
}

__global__ void k_heun_final(size_t n, const double *__restrict__ f, const double *__restrict__ fs,
                             const double *__restrict__ q, double c, double *__restrict__ out, unsigned *flag) {
    bool bad = false, neg = false;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        double y = 0.5 * (f[i] + fma(c, q[i], fs[i]));
        out[i] = y;
        bad |= !isfinite(y);
        neg |= y < 0.0;
    }
    // negative values are common in the far tails: one test per block, and the atomic only
    // when the flag lacks the bit (atomics of every block on one word serialise the grid)
    const int any_bad = __syncthreads_or(bad ? 1 : 0), any_neg = __syncthreads_or(neg ? 1 : 0);
    if (threadIdx.x == 0 && (any_bad || any_neg)) {
        const unsigned bits = (any_bad ? 1u : 0u) | (any_neg ? 2u : 0u);
        if ((__atomic_load_n(flag, __ATOMIC_RELAXED) & bits) != bits) atomicOr(flag, bits);
    }
}

__global__ void k_fill_u32(unsigned *p, int n, unsigned v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Diagnostics (Sec. 5: bulk velocity, marginal near the wall).  One block of
// 256 threads per cell, fixed reduction order: density and bulk velocity in a
// first pass, the temperature about that velocity in a second.
// ---------------------------------------------------------------------------
__device__ inline double block_sum256(double x, double *red) {
    x = wave_sum(x);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    return red[0] + red[1] + red[2] + red[3];
}

__global__ void __launch_bounds__(256) k_cell_moments(const double *__restrict__ f, const long long *__restrict__ off,
                                                      const int *__restrict__ nn, const double *__restrict__ dvs,
                                                      double *__restrict__ mom) {
    __shared__ double red[4];
    const int c = blockIdx.x, N = nn[c], M = N * N * N, h = N / 2;
    const double dv = dvs[c];
    const double *F = f + off[c];
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) {
        const double x = F[k];
        a0 += x;
        a1 = fma(dv * (k / (N * N) - h), x, a1);
        a2 = fma(dv * ((k / N) % N - h), x, a2);
        a3 = fma(dv * (k % N - h), x, a3);
    }
    const double rho = block_sum256(a0, red);
    const double u1 = block_sum256(a1, red) / rho, u2 = block_sum256(a2, red) / rho, u3 = block_sum256(a3, red) / rho;
    double e = 0.0;
    for (int k = threadIdx.x; k < M; k += 256) {
        const double w1 = dv * (k / (N * N) - h) - u1, w2 = dv * ((k / N) % N - h) - u2, w3 = dv * (k % N - h) - u3;
        e = fma(w1 * w1 + w2 * w2 + w3 * w3, F[k], e);
    }
    const double E = block_sum256(e, red);
    if (threadIdx.x == 0) {
        double *o = mom + 5 * (size_t)c;
        o[0] = rho * dv * dv * dv;
        o[1] = u1;
        o[2] = u2;
        o[3] = u3;
        o[4] = E / (3.0 * rho);
    }
}

// marginal of one cell in v1: out[k1] = dv^2 sum_{k2,k3} f(k1, k2, k3); one wavefront per k1
__global__ void __launch_bounds__(256) k_marginal_v1(int N, double dv, const double *__restrict__ F,
                                                     double *__restrict__ out) {
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int k1 = wid; k1 < N; k1 += 4) {
        double s = 0.0;
        for (int t = lane; t < N * N; t += 64) s += F[(size_t)k1 * N * N + t];
        s = wave_sum(s);
        if (lane == 0) out[k1] = s * dv * dv;
    }
}

// ---------------------------------------------------------------------------
// Weight expansion.  T[p * qs + q] = T_lambda(p, q) of the universal table;
// scale = 4pi (2pi)^{-3/2} L^{lambda+3} dzeta^3.
// ---------------------------------------------------------------------------
__device__ inline int sq3(int a, int b, int c) { return a * a + b * b + c * c; }

template <typename W>
__global__ void __launch_bounds__(256) k_expand_cells(int N, const double *__restrict__ T, int qs, double scale,
                                                      const long long *__restrict__ row_woff, W *__restrict__ w,
                                                      int core_r2, int lam, double beta) {
    const int h = N / 2;
    const int r = blockIdx.x;
    const int k1 = r / N, k2 = r % N;
    const int PS = pairs_per_step(N);
    W *out = w + row_woff[r];
    long long step = 0;
    for (int m1 = axis_lo(N, k1); m1 <= cells_m1_last(N, k1); ++m1) {
        const int j1 = k1 + h - m1;
        for (int m2 = axis_lo(N, k2); m2 <= cells_m2_last(N, k1, k2, m1); ++m2, ++step) {
            const int j2 = k2 + h - m2;
            for (int t = threadIdx.x; t < PS; t += blockDim.x) {
                // locate (k3, m3) of flat pair index t in the output-major step order
                int k3 = 0, base = 0;
                for (;; ++k3) {
                    const int cnt = axis_cnt(N, k3);
                    if (t < base + cnt) break;
                    base += cnt;
                }
                const int m3 = axis_lo(N, k3) + (t - base);
                const int j3 = k3 + h - m3;
                const int na = sq3(k1 - h, k2 - h, k3 - h);
                const int nb = sq3(m1 - j1, m2 - j2, m3 - j3);
                const int ncm = sq3(m1 - h, m2 - h, m3 - h);
                const int ncj = sq3(j1 - h, j2 - h, j3 - h);
                double v;
                const bool diag = (m1 == j1) && (m2 == j2);
                if (beta != 1.0) {
                    // inelastic: the gain of (k, m) and of (k, j) differ
                    const double gm = gain_beta(lam, beta, h, k1, k2, k3, m1, m2, m3);
                    if (diag && m3 == j3)
                        v = gm - T[4 * ncm];
                    else if (diag && m3 > j3)
                        v = 0.0;
                    else
                        v = gm + gain_beta(lam, beta, h, k1, k2, k3, j1, j2, j3) - T[4 * ncm] - T[4 * ncj];
                } else if (diag && m3 == j3)
                    v = T[(size_t)na * qs] - T[4 * ncm];
                else if (diag && m3 > j3)
                    v = 0.0;
                else
                    v = 2.0 * T[(size_t)na * qs + nb] - T[4 * ncm] - T[4 * ncj];
                // both partners in the low-frequency core: summed in FP64 by the core kernel
                if (core_r2 >= 0 && ncm <= core_r2 && ncj <= core_r2) v = 0.0;
                out[step * PS + t] = (W)(scale * v);
            }
        }
    }
}

template <typename W>
__global__ void __launch_bounds__(256) k_expand_plain(int N, const double *__restrict__ T, int qs, double scale,
                                                      const long long *__restrict__ blk_woff, W *__restrict__ w,
                                                      int lam, double beta) {
    const int h = N / 2;
    const int R = plain_rows(N), NB = N / R, LN = R * N;
    const int b = blockIdx.x;
    const int k1 = b / NB, kb = b % NB;
    const int lo1 = axis_lo(N, k1), c1 = axis_cnt(N, k1);
    const int u2lo = plain_u2_lo(N, kb), U2 = plain_u2_hi(N, kb) - u2lo + 1;
    const long long iters = (long long)c1 * U2 * N;
    W *out = w + blk_woff[b];
    for (long long e = threadIdx.x; e < iters * LN; e += blockDim.x) {
        const int lane = (int)(e % LN);
        const long long it = e / LN;
        const int m3 = (int)(it % N);
        const int m2 = u2lo + (int)((it / N) % U2);
        const int m1 = lo1 + (int)(it / ((long long)N * U2));
        const int r = lane / N, k3 = lane % N, k2 = kb * R + r;
        const int j1 = k1 + h - m1, j2 = k2 + h - m2, j3 = k3 + h - m3;
        double v = 0.0;
        if (j2 >= 0 && j2 < N && j3 >= 0 && j3 < N && j1 >= 0 && j1 < N) {
            const int na = sq3(k1 - h, k2 - h, k3 - h);
            const int nb = sq3(m1 - j1, m2 - j2, m3 - j3);
            const int ncm = sq3(m1 - h, m2 - h, m3 - h);
            const double g = beta != 1.0 ? gain_beta(lam, beta, h, k1, k2, k3, m1, m2, m3) : T[(size_t)na * qs + nb];
            v = g - T[4 * ncm];
        }
        out[e] = (W)(scale * v);
    }
}

}  // namespace


template <int N>
static void project_launch(int ncells, double dv, const Linv &li, double *q, const long long *d_off, hipStream_t s) {
    if constexpr (N <= 24)
        hipLaunchKernelGGL(k_project_cols<N>, dim3(ncells), dim3(proj_threads<N>()), 0, s, dv, li, q, d_off);
    else
        hipLaunchKernelGGL(k_project_flat<N>, dim3(ncells), dim3(kProjThreads), 0, s, dv, li, q, d_off);
}

hipError_t launch_project(int N, double dv, const double *linv, int ncells, double *q, const long long *d_off,
                          hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
    Linv li;
    for (int i = 0; i < 25; ++i) li.a[i] = linv[i];
    switch (N) {
#define BZ_PROJ(n) \
    case n: project_launch<n>(ncells, dv, li, q, d_off, s); break;
        BZ_PROJ(8) BZ_PROJ(12) BZ_PROJ(16) BZ_PROJ(20) BZ_PROJ(24) BZ_PROJ(28) BZ_PROJ(32)
#undef BZ_PROJ
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

static inline unsigned blocks_for(size_t n) {
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 8192 ? 8192 : (b < 1 ? 1 : b));
}

hipError_t launch_axpy(size_t n, const double *a, const double *q, double c, double *out, unsigned *flag,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_for(n)), dim3(256), 0, s, n, a, q, c, out, flag);
    return hipGetLastError();
}

hipError_t launch_heun_final(size_t n, const double *f, const double *fs, const double *q, double c, double *out,
                             unsigned *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_heun_final, dim3(blocks_for(n)), dim3(256), 0, s, n, f, fs, q, c, out, flag);
    return hipGetLastError();
}

hipError_t launch_fill_u32(unsigned *p, int n, unsigned v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 255) / 256), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Weights of edge pass E3 of the conjugate-symmetric schedule: for each row
// (a, b) with a < N/2, the block of steps with m1 = 0 copied from the main
// stream, with the terms whose inner partner sits on an edge plane (k3 < N/2
// and m3 = 0 or j3 = 0, i.e. m3 = k3 + N/2) set to zero.
template <typename W>
__global__ void __launch_bounds__(256) k_build_e3(int N, const long long *__restrict__ row_woff,
                                                  const long long *__restrict__ e3_woff, const W *__restrict__ w,
                                                  W *__restrict__ e3) {
    const int h = N / 2;
    const int r = blockIdx.x;  // a * N + b, a < N/2
    const int b = r % N;
    const int PS = pairs_per_step(N);
    const long long n = (long long)axis_cnt(N, b) * PS;
    const W *src = w + row_woff[r];
    W *dst = e3 + e3_woff[r];
    for (long long i = threadIdx.x; i < n; i += blockDim.x) {
        const int t = (int)(i % PS);
        int k3 = 0, base = 0;
        for (;; ++k3) {
            const int cnt = axis_cnt(N, k3);
            if (t < base + cnt) break;
            base += cnt;
        }
        const int m3 = axis_lo(N, k3) + (t - base);
        const bool edge = k3 < h && (m3 == 0 || m3 == k3 + h);
        dst[i] = edge ? (W)0 : src[i];
    }
}

hipError_t launch_build_e3(int N, const long long *d_row_woff, const long long *d_e3_woff, const void *w_main,
                           void *w_e3, bool f64, hipStream_t s) {
    const dim3 grid(N / 2 * N);
    if (f64)
        hipLaunchKernelGGL(k_build_e3<double>, grid, dim3(256), 0, s, N, d_row_woff, d_e3_woff,
                           (const double *)w_main, (double *)w_e3);
    else
        hipLaunchKernelGGL(k_build_e3<float>, grid, dim3(256), 0, s, N, d_row_woff, d_e3_woff,
                           (const float *)w_main, (float *)w_e3);
    return hipGetLastError();
}

hipError_t launch_cell_moments(int ncells, const double *f, const long long *off, const int *nn, const double *dvs,
                               double *mom, hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cell_moments, dim3(ncells), dim3(256), 0, s, f, off, nn, dvs, mom);
    return hipGetLastError();
}

hipError_t launch_marginal_v1(int N, double dv, const double *f, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_marginal_v1, dim3(1), dim3(256), 0, s, N, dv, f, out);
    return hipGetLastError();
}

hipError_t launch_expand_cells(int N, const double *dT, int qstride, double scale, const long long *d_row_woff,
                               void *d_w, bool f64, int core_r2, int lam, double beta, hipStream_t s) {
    if (f64)
        hipLaunchKernelGGL(k_expand_cells<double>, dim3(N * N), dim3(256), 0, s, N, dT, qstride, scale, d_row_woff,
                           (double *)d_w, core_r2, lam, beta);
    else
        hipLaunchKernelGGL(k_expand_cells<float>, dim3(N * N), dim3(256), 0, s, N, dT, qstride, scale, d_row_woff,
                           (float *)d_w, core_r2, lam, beta);
    return hipGetLastError();
}

hipError_t launch_expand_plain(int N, const double *dT, int qstride, double scale, const long long *d_blk_woff,
                               void *d_w, bool f64, int lam, double beta, hipStream_t s) {
    const int nb = N * (N / plain_rows(N));
    if (f64)
        hipLaunchKernelGGL(k_expand_plain<double>, dim3(nb), dim3(256), 0, s, N, dT, qstride, scale, d_blk_woff,
                           (double *)d_w, lam, beta);
    else
        hipLaunchKernelGGL(k_expand_plain<float>, dim3(nb), dim3(256), 0, s, N, dT, qstride, scale, d_blk_woff,
                           (float *)d_w, lam, beta);
    return hipGetLastError();
}

}  // namespace bz
