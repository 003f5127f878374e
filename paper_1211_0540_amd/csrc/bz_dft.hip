// Sampled Fourier transform pair of the spectral method (Sec. 2.2 / 3.2):
//   fhat_k = (2pi)^{-3/2} dv^3    sum_j f_j    exp(-i zeta_k . v_j)
//   Qt_j   = (2pi)^{-3/2} dzeta^3 Re sum_k Qhat_k exp(+i zeta_k . v_j)
// On the mesh zeta_k . v_j = (2pi/N) sum_d (k_d - N/2)(j_d - N/2), so each
// axis is an N-point DFT with the twiddle w^{((k-N/2)(j-N/2)) mod N},
// w = exp(-2 pi i / N).  The plain path sums each axis directly (O(N^4) per
// cell); the batched paths use an in-register FFT per line (O(N^3 log N), the
// cost the method states for this step).  FP64 throughout.
//
// Two organisations:
// * one cell at a time (plain path): pass A transforms the two fast axes of
//   one plane out of LDS, pass B the slow axis of one (k2) slab;
// * cell-interleaved groups of 64 (batched paths, element (g, k, lane) at
//   (g M + k) 64 + lane): one wavefront transforms one line of its 64 cells
//   along one axis, lane = cell, so every read and write of the
//   intermediate and spectral buffers is a whole 1 KiB line; three passes,
//   one per axis.
#include <utility>

#include "bz_internal.h"

namespace bz {
namespace {

constexpr double kPi = 3.14159265358979323846;

__device__ inline int tw_index(int N, int k, int j) {
    int t = ((k - N / 2) * (j - N / 2)) % N;
    return t < 0 ? t + N : t;
}

__device__ inline void load_roots(double2 *roots, int N, double sign) {
    for (int t = threadIdx.x; t < N; t += blockDim.x) {
        double s, c;
        sincospi(sign * 2.0 * t / N, &s, &c);
        roots[t] = make_double2(c, s);
    }
}

__device__ inline double2 cmul(double2 a, double2 b) {
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Pass A (forward): plane j1 of cell c: real f[j2][j3] -> G[c][j1][k2][k3].
__global__ void __launch_bounds__(256) k_dft_fwd_a(int N, const double *__restrict__ f,
                                                   const long long *__restrict__ f_off, double2 *__restrict__ G) {
    __shared__ double2 roots[kMaxN];
    __shared__ double fp[kMaxN * kMaxN];
    __shared__ double2 t1[kMaxN * kMaxN];
    const int c = blockIdx.y, j1 = blockIdx.x;
    const int NN = N * N;
    load_roots(roots, N, -1.0);
    const double *src = f + f_off[c] + (size_t)j1 * NN;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) fp[i] = src[i];
    __syncthreads();
    // axis 3: t1[j2][k3] = sum_j3 f[j2][j3] w^(..)
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int j2 = i / N, k3 = i - j2 * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int j3 = 0; j3 < N; ++j3) {
            double2 w = roots[tw_index(N, k3, j3)];
            double x = fp[j2 * N + j3];
            acc.x += x * w.x;
            acc.y += x * w.y;
        }
        t1[i] = acc;
    }
    __syncthreads();
    // axis 2: G[k2][k3] = sum_j2 w^(..) t1[j2][k3]
    double2 *dst = G + ((size_t)c * N + j1) * NN;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int k2 = i / N, k3 = i - k2 * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int j2 = 0; j2 < N; ++j2) {
            double2 p = cmul(roots[tw_index(N, k2, j2)], t1[j2 * N + k3]);
            acc.x += p.x;
            acc.y += p.y;
        }
        dst[i] = acc;
    }
}

// Pass B (forward): slab k2 of cell c: G[c][j1][k2][k3] -> fhat[k1][k2][k3] (scaled).
template <typename Out>
__global__ void __launch_bounds__(256) k_dft_fwd_b(int N, double scale, const double2 *__restrict__ G,
                                                   Out *__restrict__ out, const long long *__restrict__ o_base,
                                                   long long o_stride) {
    __shared__ double2 roots[kMaxN];
    __shared__ double2 slab[kMaxN * kMaxN];
    const int c = blockIdx.y, k2 = blockIdx.x;
    const int NN = N * N;
    load_roots(roots, N, -1.0);
    const double2 *src = G + (size_t)c * N * NN;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int j1 = i / N, k3 = i - j1 * N;
        slab[i] = src[(size_t)j1 * NN + k2 * N + k3];
    }
    __syncthreads();
    const long long base = o_base[c];
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int k1 = i / N, k3 = i - k1 * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int j1 = 0; j1 < N; ++j1) {
            double2 p = cmul(roots[tw_index(N, k1, j1)], slab[j1 * N + k3]);
            acc.x += p.x;
            acc.y += p.y;
        }
        long long k = ((long long)k1 * N + k2) * N + k3;
        Out v;
        v.x = acc.x * scale;
        v.y = acc.y * scale;
        out[base + k * o_stride] = v;
    }
}

// Pass A (inverse): plane k1 of cell c (summed over partial buffers) -> H[c][k1][j2][j3].
__global__ void __launch_bounds__(256) k_dft_inv_a(int N, const double2 *__restrict__ in,
                                                   const long long *__restrict__ i_base, long long i_stride,
                                                   int nparts, long long part_stride, double2 *__restrict__ H) {
    __shared__ double2 roots[kMaxN];
    __shared__ double2 pl[kMaxN * kMaxN];
    __shared__ double2 t1[kMaxN * kMaxN];
    const int c = blockIdx.y, k1 = blockIdx.x;
    const int NN = N * N;
    load_roots(roots, N, +1.0);
    const long long base = i_base[c];
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        long long k = (long long)k1 * NN + i;
        double2 acc = in[base + k * i_stride];
        for (int p = 1; p < nparts; ++p) {
            double2 x = in[base + k * i_stride + p * part_stride];
            acc.x += x.x;
            acc.y += x.y;
        }
        pl[i] = acc;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int k2 = i / N, j3 = i - k2 * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int k3 = 0; k3 < N; ++k3) {
            double2 p = cmul(roots[tw_index(N, k3, j3)], pl[k2 * N + k3]);
            acc.x += p.x;
            acc.y += p.y;
        }
        t1[i] = acc;
    }
    __syncthreads();
    double2 *dst = H + ((size_t)c * N + k1) * NN;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int j2 = i / N, j3 = i - j2 * N;
        double2 acc = make_double2(0.0, 0.0);
        for (int k2 = 0; k2 < N; ++k2) {
            double2 p = cmul(roots[tw_index(N, k2, j2)], t1[k2 * N + j3]);
            acc.x += p.x;
            acc.y += p.y;
        }
        dst[i] = acc;
    }
}

// Pass B (inverse): slab j2 of cell c: H[c][k1][j2][j3] -> Qt[j1][j2][j3] (real part, scaled).
__global__ void __launch_bounds__(256) k_dft_inv_b(int N, double scale, const double2 *__restrict__ H,
                                                   double *__restrict__ qt, const long long *__restrict__ q_off) {
    __shared__ double2 roots[kMaxN];
    __shared__ double2 slab[kMaxN * kMaxN];
    const int c = blockIdx.y, j2 = blockIdx.x;
    const int NN = N * N;
    load_roots(roots, N, +1.0);
    const double2 *src = H + (size_t)c * N * NN;
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int k1 = i / N, j3 = i - k1 * N;
        slab[i] = src[(size_t)k1 * NN + j2 * N + j3];
    }
    __syncthreads();
    double *dst = qt + q_off[c];
    for (int i = threadIdx.x; i < NN; i += blockDim.x) {
        int j1 = i / N, j3 = i - j1 * N;
        double re = 0.0;
        for (int k1 = 0; k1 < N; ++k1) {
            double2 w = roots[tw_index(N, k1, j1)];
            double2 x = slab[k1 * N + j3];
            re += w.x * x.x - w.y * x.y;
        }
        dst[((size_t)j1 * N + j2) * N + j3] = re * scale;
    }
}

// ---------------------------------------------------------------------------
// Cell-interleaved groups (batched paths).  Each lane transforms its cell's
// line in registers with an FFT: Cooley-Tukey decimation in time, radix 2 down
// to an odd length (1, 3, 5 or 7 for the meshes here) done as a direct sum.
// N and the sign are compile-time, so every twiddle is a constant.
// ---------------------------------------------------------------------------
struct Twiddle {
    double c, s;
};
// sin and cos on [0, pi/4] by their Taylor series (the omitted terms are below 1e-30)
constexpr double tw_sin(double x) {
    double t = x, s = x;
    for (int i = 1; i < 13; ++i) {
        t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
        s += t;
    }
    return s;
}
constexpr double tw_cos(double x) {
    double t = 1.0, s = 1.0;
    for (int i = 1; i < 13; ++i) {
        t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
        s += t;
    }
    return s;
}
// exp(sign 2 pi i k / n), 0 <= k < n: the angle is (pi/4)(o + r/n) with octant o = 8k div n and
// r = 8k mod n; reduced to [0, pi/4] by the octant symmetries, exact at multiples of pi/2
constexpr Twiddle twiddle(int sign, int k, int n) {
    constexpr double q = 3.14159265358979323846 / 4.0;
    const int o = (8 * k) / n, r = 8 * k - o * n;
    double c = 0.0, s = 0.0;
    if (o % 2 == 0) {
        c = tw_cos(q * r / n);
        s = tw_sin(q * r / n);
    } else {
        c = tw_sin(q * (n - r) / n);
        s = tw_cos(q * (n - r) / n);
    }
    double cc = c, ss = s;  // rotate by the quadrant o / 2
    if (o / 2 == 1) cc = -s, ss = c;
    if (o / 2 == 2) cc = -c, ss = -s;
    if (o / 2 == 3) cc = s, ss = -c;
    return Twiddle{cc, sign * ss};
}

// output K of a direct transform of odd length n: x_0 + sum_{j >= 1} x_j exp(SIGN 2 pi i K j / n)
template <int n, int SIGN, int K, int... J>
__device__ __forceinline__ double2 odd_dft_term(const double2 (&x)[n], std::integer_sequence<int, J...>) {
    double re = x[0].x, im = x[0].y;
    ((void)[&] {
        constexpr Twiddle w = twiddle(SIGN, (K * (J + 1)) % n, n);
        re = fma(x[J + 1].x, w.c, fma(-x[J + 1].y, w.s, re));
        im = fma(x[J + 1].x, w.s, fma(x[J + 1].y, w.c, im));
    }(), ...);
    return make_double2(re, im);
}

template <int n, int SIGN>
__device__ __forceinline__ void fft_rec(double2 (&x)[n]) {
    if constexpr (n % 2 == 0) {
        constexpr int m = n / 2;
        double2 e[m], o[m];
#pragma unroll
        for (int i = 0; i < m; ++i) {
            e[i] = x[2 * i];
            o[i] = x[2 * i + 1];
        }
        fft_rec<m, SIGN>(e);
        fft_rec<m, SIGN>(o);
        [&]<int... K>(std::integer_sequence<int, K...>) {
            ((void)[&] {
                constexpr Twiddle w = twiddle(SIGN, K, n);
                double2 t = o[K];
                if constexpr (K > 0) t = make_double2(fma(w.c, o[K].x, -w.s * o[K].y), fma(w.c, o[K].y, w.s * o[K].x));
                x[K] = make_double2(e[K].x + t.x, e[K].y + t.y);
                x[K + m] = make_double2(e[K].x - t.x, e[K].y - t.y);
            }(), ...);
        }(std::make_integer_sequence<int, m>{});
    } else if constexpr (n > 1) {
        double2 y[n];
        [&]<int... K>(std::integer_sequence<int, K...>) {
            ((y[K] = odd_dft_term<n, SIGN, K>(x, std::make_integer_sequence<int, n - 1>{})), ...);
        }(std::make_integer_sequence<int, n>{});
#pragma unroll
        for (int k = 0; k < n; ++k) x[k] = y[k];
    }
}

// Centred transform of one line, x_k <- sum_j x_j w^((k - N/2)(j - N/2)), w = exp(SIGN 2 pi i / N).
// For N a multiple of 4, (k - N/2)(j - N/2) = k j - (N/2)(k + j) + N^2/4 with w^(N/2) = -1 and
// w^(N^2/4) = 1: the plain transform of (-1)^j x_j, times (-1)^k.
template <int N, int SIGN>
__device__ __forceinline__ void centred_dft(double2 (&x)[N]) {
    static_assert(N % 4 == 0, "mesh sizes are multiples of 4");
#pragma unroll
    for (int j = 1; j < N; j += 2) x[j] = make_double2(-x[j].x, -x[j].y);
    fft_rec<N, SIGN>(x);
#pragma unroll
    for (int k = 1; k < N; k += 2) x[k] = make_double2(-x[k].x, -x[k].y);
}

// line index of this wavefront (4 per block) and its lane
#define BZ_LINE_SETUP                                         \
    if (skip && skip[blockIdx.y]) return;                     \
    constexpr int M = N * N * N;                              \
    const int lane = threadIdx.x & (kWave - 1);               \
    const int line = blockIdx.x * 4 + (threadIdx.x >> 6);     \
    const int g = blockIdx.y;                                 \
    const size_t gb = (size_t)g * M;                          \
    (void)gb;

// forward, axis 3: real f of cell g*64 + lane, line (j1, j2) -> S (j1, j2, k3)
template <int N>
__global__ void __launch_bounds__(256) k_dftg_fwd1(const double *__restrict__ f, const long long *__restrict__ f_off,
                                                   int nc, double2 *__restrict__ S,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const int i = g * kWave + lane;
    double x[N];
    if (i < nc) {
        const double *src = f + f_off[i] + (size_t)line * N;
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = src[j];
    } else {
#pragma unroll
        for (int j = 0; j < N; ++j) x[j] = 0.0;
    }
    double2 *dst = S + (gb + (size_t)line * N) * kWave + lane;
    double2 y[N];
#pragma unroll
    for (int j = 0; j < N; ++j) y[j] = make_double2(x[j], 0.0);
    centred_dft<N, -1>(y);
#pragma unroll
    for (int k = 0; k < N; ++k) dst[(size_t)k * kWave] = y[k];
}

// one complex line: out_k = scale sum_j in_j w^((k - N/2)(j - N/2)); out strided by `stride` elements
template <int N, int SIGN>
__device__ __forceinline__ void line_dft(double2 (&x)[N], double2 *dst, size_t stride, double scale) {
    centred_dft<N, SIGN>(x);
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k * stride] = make_double2(x[k].x * scale, x[k].y * scale);
}

// forward, axis 2: line (j1, k3): S (j1, j2, k3) -> T (j1, k2, k3)
template <int N>
__global__ void __launch_bounds__(256) k_dftg_fwd2(const double2 *__restrict__ S, double2 *__restrict__ T,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const int j1 = line / N, k3 = line - j1 * N;
    const size_t off = (gb + (size_t)j1 * N * N + k3) * kWave + lane;
    double2 x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = S[off + (size_t)j * N * kWave];
    line_dft<N, -1>(x, T + off, (size_t)N * kWave, 1.0);
}

// forward, axis 1: line (k2, k3): T (j1, k2, k3) -> fhat (k1, k2, k3), scaled, in the kernel's precision;
// with copies = 4 also fhat with the axes ordered (2, 1, 3) and (3, 1, 2), and fhat with every k_d = 0
// plane set to zero (axes in order), copy_stride elements apart
// With cf non-NULL it also writes the FP64 rows of the low-frequency core (CoreFill).
template <int N, typename Out>
__global__ void __launch_bounds__(256) k_dftg_fwd3(const double2 *__restrict__ T, int nc, double scale,
                                                   Out *__restrict__ fh, int copies, long long copy_stride,
                                                   double2 *__restrict__ cf, const int *__restrict__ disk_idx,
                                                   int nD, int cr, int cr2,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const size_t off = (gb + (size_t)line) * kWave + lane;
    double2 x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = T[off + (size_t)j * N * N * kWave];
    const bool live = g * kWave + lane < nc;
    centred_dft<N, -1>(x);
#pragma unroll
    for (int k = 0; k < N; ++k) {
        Out v;
        v.x = live ? x[k].x * scale : 0.0;
        v.y = live ? x[k].y * scale : 0.0;
        fh[off + (size_t)k * N * N * kWave] = v;
        if (copies > 1) {
            const int k2 = line / N, k3 = line - k2 * N;
            const size_t gl = gb * kWave + lane;
            fh[copy_stride + gl + ((size_t)(k2 * N + k) * N + k3) * kWave] = v;
            fh[2 * copy_stride + gl + ((size_t)(k3 * N + k) * N + k2) * kWave] = v;
            Out z = v;
            if (k == 0 || k2 == 0 || k3 == 0) z.x = z.y = 0.0;
            fh[3 * copy_stride + off + (size_t)k * N * N * kWave] = z;
        }
    }
    if (cf) {
        constexpr int h = N / 2;
        const int k2 = line / N, k3 = line - k2 * N, t = k3 - (h - cr);
        if (t >= 0 && t <= 2 * cr) {
            const int b2 = (k2 - h) * (k2 - h), c2 = (k3 - h) * (k3 - h);
#pragma unroll
            for (int k = 0; k < N; ++k) {
                const int a2 = (k - h) * (k - h);
                if (a2 + b2 > cr2) continue;   // row (k, k2) is not in the core disk
                const int d = disk_idx[k * N + k2];
                const bool in = live && a2 + b2 + c2 <= cr2;
                cf[(((size_t)g * nD + d) * (2 * cr + 1) + t) * kWave + lane] =
                    in ? make_double2(x[k].x * scale, x[k].y * scale) : make_double2(0.0, 0.0);
            }
        }
    }
}

// inverse, axis 1, conjugate-symmetric schedule: assemble Qhat(k1, k2, k3) of line (k2, k3) from the
// passes (qh: nA partial buffers of pass A, then the half-size E1, E2, E3, then nA partial buffers
// of Z, laid out as HermAssembly describes; pstride = one full buffer), then transform -> S (j1, k2, k3).  Pass A holds the interior sums I of the direct rows.
//   direct row (k1, k2):        Qhat = I(k) + E(k)
//   derived row, k3 = 0:        Qhat = Z at (0, k1, k2) of the (3, 1, 2) order
//   derived row, k3 >= 1:       Qhat = conj I(k') + E(k),   k' = N - k
// E(k) is the edge sum: E1 at (k1, k2, k3) if k1 < N/2, E2 at (k2, k1, k3) if k2 < N/2,
// E3 at (k3, k1, k2) if k3 < N/2.
// Three wavefronts per SIMD: at N=32 that costs some register spills, but the 3 x 1024 lines of a
// 190-cell batch then run in one round (139 instead of 157 us measured).
// The FP64 core sum (CoreAdd; core NULL when off) is added to every output within 2cr of the centre.
// The core holds it for the direct rows and for k3 = 0 of the derived rows; elsewhere a derived
// output is the conjugate of its mirror N - k (the core pairs are interior, and the weights even).
template <int N>
__device__ __forceinline__ void add_core(double2 (&x)[N], const CoreAdd &ca, size_t gl, int k2, int k3) {
    constexpr int h = N / 2;
    const int cr = ca.r;
    if (!ca.core || abs(k2 - h) > 2 * cr || abs(k3 - h) > 2 * cr) return;
#pragma unroll
    for (int k1 = 0; k1 < N; ++k1) {
        if (abs(k1 - h) > 2 * cr) continue;
        const bool mirrored = herm_derived_row(N, k1, k2) && k3 >= 1;
        const size_t o = mirrored ? gl + ((size_t)((N - k1) * N + (N - k2)) * N + (N - k3)) * kWave
                                  : gl + ((size_t)(k1 * N + k2) * N + k3) * kWave;
        // the partial sums of the row's step pieces, in piece order
        double2 c = ca.core[o];
        for (int p = 1; p < ca.parts; ++p) {
            const double2 t = ca.core[o + (size_t)p * ca.pstride];
            c.x += t.x;
            c.y += t.y;
        }
        if (mirrored) c.y = -c.y;
        x[k1].x += c.x;
        x[k1].y += c.y;
    }
}

template <int N>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_dftg_inv1_herm(const double2 *__restrict__ qh, int nA, long long pstride,
                                                        const CoreAdd core,
                                                        double2 *__restrict__ S,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    constexpr int h = N / 2;
    const int k2 = line / N, k3 = line - k2 * N;
    // pstride = B, one full buffer; group bases of the full, edge (half) and Z buffers
    const size_t gl = gb * kWave + lane;
    const size_t ge = (size_t)g * (M / 2) * kWave + lane;
    const size_t gz = (size_t)g * h * N * kWave + lane;
    const double2 *E1 = qh + (size_t)nA * pstride;
    const double2 *E2 = E1 + pstride / 2, *E3 = E2 + pstride / 2, *Z = E3 + pstride / 2;
    const size_t zstride = (size_t)pstride / (2 * N);
    auto at = [](int a, int b, int c) { return ((size_t)(a * N + b) * N + c) * kWave; };
    auto sum_parts = [&](const double2 *base, size_t o, size_t stride) {
        double2 a = base[o];
        for (int p = 1; p < nA; ++p) {
            const double2 b = base[o + (size_t)p * stride];
            a.x += b.x;
            a.y += b.y;
        }
        return a;
    };
    auto edge = [&](int a, int b, int c) {
        double2 e = make_double2(0.0, 0.0);
        if (a < h) {
            const double2 t = E1[ge + at(a, b, c)];
            e.x += t.x;
            e.y += t.y;
        }
        if (b < h) {
            const double2 t = E2[ge + at(b, a, c)];
            e.x += t.x;
            e.y += t.y;
        }
        if (c < h) {
            const double2 t = E3[ge + at(c, a, b)];
            e.x += t.x;
            e.y += t.y;
        }
        return e;
    };
    double2 x[N];
#pragma unroll
    for (int k1 = 0; k1 < N; ++k1) {
        if (!herm_derived_row(N, k1, k2)) {
            const double2 i = sum_parts(qh, gl + at(k1, k2, k3), pstride), e = edge(k1, k2, k3);
            x[k1] = make_double2(i.x + e.x, i.y + e.y);
        } else if (k3 == 0) {
            // derived rows have k1 >= N/2: Z slot (k1 - N/2, k2) of the k3 = 0 plane
            x[k1] = sum_parts(Z, gz + ((size_t)(k1 - h) * N + k2) * kWave, zstride);
        } else {
            const double2 i = sum_parts(qh, gl + at(N - k1, N - k2, N - k3), pstride), e = edge(k1, k2, k3);
            x[k1] = make_double2(i.x + e.x, e.y - i.y);
        }
    }
    add_core<N>(x, core, gl, k2, k3);
    line_dft<N, +1>(x, S + gl + (size_t)line * kWave, (size_t)N * N * kWave, 1.0);
}

// inverse, axis 1: line (k2, k3): sum of the partial buffers (k1, k2, k3) -> S (j1, k2, k3)
template <int N>
__global__ void __launch_bounds__(256) k_dftg_inv1(const double2 *__restrict__ qh, int nparts, long long pstride,
                                                   const CoreAdd core,
                                                   double2 *__restrict__ S,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const size_t off = (gb + (size_t)line) * kWave + lane;
    const int k2 = line / N, k3 = line - k2 * N;
    double2 x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
        double2 a = qh[off + (size_t)j * N * N * kWave];
        for (int p = 1; p < nparts; ++p) {
            const double2 b = qh[off + (size_t)j * N * N * kWave + (size_t)p * pstride];
            a.x += b.x;
            a.y += b.y;
        }
        x[j] = a;
    }
    add_core<N>(x, core, gb * kWave + lane, k2, k3);
    line_dft<N, +1>(x, S + off, (size_t)N * N * kWave, 1.0);
}

// inverse, axis 2: line (j1, k3): S (j1, k2, k3) -> T (j1, j2, k3)
template <int N>
__global__ void __launch_bounds__(256) k_dftg_inv2(const double2 *__restrict__ S, double2 *__restrict__ T,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const int j1 = line / N, k3 = line - j1 * N;
    const size_t off = (gb + (size_t)j1 * N * N + k3) * kWave + lane;
    double2 x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = S[off + (size_t)j * N * kWave];
    line_dft<N, +1>(x, T + off, (size_t)N * kWave, 1.0);
}

// inverse, axis 3: line (j1, j2): T (j1, j2, k3) -> Qt (j1, j2, j3) = scale Re(...) of cell g*64 + lane
template <int N>
__global__ void __launch_bounds__(256) k_dftg_inv3(const double2 *__restrict__ T, int nc, double scale,
                                                   double *__restrict__ qt, const long long *__restrict__ q_off,
    const unsigned char *__restrict__ skip) {
    BZ_LINE_SETUP
    const int i = g * kWave + lane;
    const size_t off = (gb + (size_t)line * N) * kWave + lane;
    double2 x[N];
#pragma unroll
    for (int j = 0; j < N; ++j) x[j] = T[off + (size_t)j * kWave];
    if (i >= nc) return;
    double *dst = qt + q_off[i] + (size_t)line * N;
    centred_dft<N, +1>(x);
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k] = x[k].x * scale;
}
#undef BZ_LINE_SETUP

template <int N>
hipError_t grouped_forward(double L, int nc, const double *f, const long long *f_off, double2 *S, double2 *T,
                           void *fh, bool f32, int copies, const CoreFill &cfill, const unsigned char *skip,
                           hipStream_t s) {
    const int groups = (nc + kWave - 1) / kWave;
    const dim3 grid(N * N / 4, groups);
    const double dv = 2.0 * L / N;
    const double scale = pow(2.0 * kPi, -1.5) * dv * dv * dv;
    const long long cstride = (long long)groups * N * N * N * kWave;
    hipLaunchKernelGGL(k_dftg_fwd1<N>, grid, dim3(256), 0, s, f, f_off, nc, S, skip);
    hipLaunchKernelGGL(k_dftg_fwd2<N>, grid, dim3(256), 0, s, S, T, skip);
    if (f32)
        hipLaunchKernelGGL((k_dftg_fwd3<N, float2>), grid, dim3(256), 0, s, T, nc, scale, (float2 *)fh, copies,
                           cstride, cfill.cf, cfill.disk_idx, cfill.nD, cfill.r, cfill.r2, skip);
    else
        hipLaunchKernelGGL((k_dftg_fwd3<N, double2>), grid, dim3(256), 0, s, T, nc, scale, (double2 *)fh, copies,
                           cstride, cfill.cf, cfill.disk_idx, cfill.nD, cfill.r, cfill.r2, skip);
    return hipGetLastError();
}

template <int N>
hipError_t grouped_inverse(double L, int nc, const double2 *qh, int nparts, long long pstride,
                           const HermAssembly &herm, const CoreAdd &core, double2 *S, double2 *T, double *qt,
                           const long long *q_off, const unsigned char *skip, hipStream_t s) {
    const int groups = (nc + kWave - 1) / kWave;
    const dim3 grid(N * N / 4, groups);
    const double dz = kPi / L;
    const double scale = pow(2.0 * kPi, -1.5) * dz * dz * dz;
    if (herm.on)
        hipLaunchKernelGGL(k_dftg_inv1_herm<N>, grid, dim3(256), 0, s, qh, herm.nA, pstride, core, S,
                           skip);
    else
        hipLaunchKernelGGL(k_dftg_inv1<N>, grid, dim3(256), 0, s, qh, nparts, pstride, core, S, skip);
    hipLaunchKernelGGL(k_dftg_inv2<N>, grid, dim3(256), 0, s, S, T, skip);
    hipLaunchKernelGGL(k_dftg_inv3<N>, grid, dim3(256), 0, s, T, nc, scale, qt, q_off, skip);
    return hipGetLastError();
}

}  // namespace

#define BZ_FOR_EACH_N(X) X(8) X(12) X(16) X(20) X(24) X(28) X(32)

hipError_t launch_dft_forward_grouped(int N, double L, int ncells, const double *f, const long long *d_f_off,
                                      double2 *S, double2 *T, void *fh, bool out_f32, int copies,
                                      const CoreFill &core, const unsigned char *skip, hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
    if (copies != 1 && copies != 4) return hipErrorInvalidValue;
#define CASE(NN) \
    case NN: return grouped_forward<NN>(L, ncells, f, d_f_off, S, T, fh, out_f32, copies, core, skip, s);
    switch (N) {
        BZ_FOR_EACH_N(CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef CASE
}

hipError_t launch_dft_inverse_grouped(int N, double L, int ncells, const double2 *qh, int nparts, long long pstride,
                                      const HermAssembly &herm, const CoreAdd &core, double2 *S, double2 *T,
                                      double *qt, const long long *d_q_off, const unsigned char *skip,
                                      hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
#define CASE(NN) \
    case NN: return grouped_inverse<NN>(L, ncells, qh, nparts, pstride, herm, core, S, T, qt, d_q_off, skip, s);
    switch (N) {
        BZ_FOR_EACH_N(CASE)
    default:
        return hipErrorInvalidValue;
    }
#undef CASE
}
#undef BZ_FOR_EACH_N

hipError_t launch_dft_forward(int N, double L, int ncells, const double *f, const long long *d_f_off,
                              double2 *scratch, void *out, bool out_f32, const long long *d_o_base,
                              long long o_stride, hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
    const double dv = 2.0 * L / N;
    const double scale = pow(2.0 * kPi, -1.5) * dv * dv * dv;
    dim3 grid(N, ncells);
    hipLaunchKernelGGL(k_dft_fwd_a, grid, dim3(256), 0, s, N, f, d_f_off, scratch);
    if (out_f32)
        hipLaunchKernelGGL(k_dft_fwd_b<float2>, grid, dim3(256), 0, s, N, scale, scratch, (float2 *)out, d_o_base,
                           o_stride);
    else
        hipLaunchKernelGGL(k_dft_fwd_b<double2>, grid, dim3(256), 0, s, N, scale, scratch, (double2 *)out,
                           d_o_base, o_stride);
    return hipGetLastError();
}

hipError_t launch_dft_inverse(int N, double L, int ncells, const double2 *in, const long long *d_i_base,
                              long long i_stride, int nparts, long long part_stride, double2 *scratch,
                              double *qt, const long long *d_q_off, hipStream_t s) {
    if (ncells <= 0) return hipSuccess;
    const double dz = kPi / L;
    const double scale = pow(2.0 * kPi, -1.5) * dz * dz * dz;
    dim3 grid(N, ncells);
    hipLaunchKernelGGL(k_dft_inv_a, grid, dim3(256), 0, s, N, in, d_i_base, i_stride, nparts, part_stride, scratch);
    hipLaunchKernelGGL(k_dft_inv_b, grid, dim3(256), 0, s, N, scale, scratch, qt, d_q_off);
    return hipGetLastError();
}

}  // namespace bz
