// Sampled Fourier transform pair of the spectral method (Sec. 2.2 / 3.2):
//   fhat_k = (2pi)^{-3/2} dv^3    sum_j f_j    exp(-i zeta_k . v_j)
//   Qt_j   = (2pi)^{-3/2} dzeta^3 Re sum_k Qhat_k exp(+i zeta_k . v_j)
// On the mesh zeta_k . v_j = (2pi/N) sum_d (k_d - N/2)(j_d - N/2), so each
// axis is an N-point DFT with the twiddle w^{((k-N/2)(j-N/2)) mod N},
// w = exp(-2 pi i / N).  N <= 32 is small, so each axis is a direct sum done
// out of LDS: pass A transforms the two fast axes of one plane, pass B the
// slow axis of one (k2) slab.  FP64 throughout; the cost is O(N^4) per cell,
// about 1% of the convolution.
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

}  // namespace

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
