// Gated learned closure around the collision step.
//
// For every cell:  rho, u, T (FP64 moments on the mesh), the local Maxwellian
// M = rho (2 pi T)^{-3/2} exp(-|v-u|^2 / 2T), the deviation d = |f - M|_2 / |M|_2
// and the gate d < gate.  The network input x (BF16) is the direction of f - M,
// scaled to unit RMS, with the amplitude d / s_in in the corner entry
// v = (-L, -L, -L); its output y (FP32) gives the closure
// Q_s = rho |f - M|_2 s_out y.  Near equilibrium Q is linear in f - M with a
// coefficient proportional to rho, so y depends on the direction, on d only
// through the quadratic part, and vanishes with f - M.  Gated cells take Q_s,
// the others the weighted
// convolution; the gated cells of one 64-cell group in judge_every (rotating
// over evaluations, "judged" cells) are also convolved and compared after
// projection,
//   err = |P(Q_s - Q_c)|_2 / (|P Q_c|_2 + floor rho |M|_2),
// (the floor is on the scale of the loss term rho nu f, so that cells at
// equilibrium, whose Q is only the discretisation residual, are judged
// against the collision rate rather than against that residual)
// and keeps the convolution result (fallback).  A failed judge also caps the
// gate of later evaluations at that cell's deviation (no cell at least as far
// from equilibrium is served again), and the cells served in an evaluation
// with a failed judge are counted as unbounded.  The FP64 projection of
// Sec. 3.3 is applied to every cell afterwards.  The batched modes pack the
// cells that need the convolution into the first 64-cell groups of the launch
// and skip the groups left with served cells only.
#include <cmath>
#include <new>

#include "bz_internal.h"

namespace bz {
namespace {

constexpr int kState = 10;  // rho, u1, u2, u3, T, d, gated, judged, |M|_2, unused
// closure counters (unsigned words): total served, judged, max err (float bits), failed; this
// evaluation's served and failed; unbounded served; pad; at words 8..9 the gate cap as the
// complement of its double's bits (0: no cap), so that a smaller cap is a larger word
enum { kStServed = 0, kStJudged = 1, kStMaxErr = 2, kStFailed = 3, kStEvalServed = 4, kStEvalFailed = 5,
       kStUnbounded = 6, kStCap = 8 };

__device__ inline double block_sum(double x, double *red) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = x;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
    return t;
}

__device__ inline unsigned short f2bf(float x) {
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

// One block of kSurThreads per cell; every thread keeps its PER values of f (then f - M) in
// registers, so f is read once and the Maxwellian evaluated once per point.
constexpr int kSurThreads = 1024;
template <int N>
__global__ void __launch_bounds__(kSurThreads) k_prepare(double dv, const double *__restrict__ f,
                                                         const long long *__restrict__ f_off, double gate,
                                                         double inv_s_in, int judge_every, int phase,
                                                         const unsigned *__restrict__ stats,
                                                         double *__restrict__ state, unsigned short *__restrict__ x) {
    constexpr int M = N * N * N, PER = (M + kSurThreads - 1) / kSurThreads;
    __shared__ double red[kSurThreads / 64];
    const int c = blockIdx.x;
    const double *F = f + f_off[c];
    const double w = dv * dv * dv;
    double fv[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = threadIdx.x + i * kSurThreads;
        fv[i] = j < M ? F[j] : 0.0;
    }
    // each pass recomputes its indices and velocities from an opaque copy of the thread index,
    // so that the compiler does not keep them live across the passes (and spill them)
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0, s4 = 0;
    int t0 = threadIdx.x;
    asm volatile("" : "+v"(t0));
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = t0 + i * kSurThreads;
        if (j >= M) continue;
        const double v1 = dv * (j / (N * N) - N / 2), v2 = dv * ((j / N) % N - N / 2), v3 = dv * (j % N - N / 2);
        const double q = fv[i];
        s0 += q;
        s1 += v1 * q;
        s2 += v2 * q;
        s3 += v3 * q;
        s4 += (v1 * v1 + v2 * v2 + v3 * v3) * q;
    }
    const double rho = block_sum(s0, red) * w;
    const double u1 = block_sum(s1, red) * w / rho, u2 = block_sum(s2, red) * w / rho, u3 = block_sum(s3, red) * w / rho;
    const double e = block_sum(s4, red) * w / rho;
    const double T = (e - (u1 * u1 + u2 * u2 + u3 * u3)) / 3.0;
    const double nrm = rho * pow(2.0 * M_PI * T, -1.5);
    double dd = 0, mm = 0;
    int t1 = threadIdx.x;
    asm volatile("" : "+v"(t1));
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = t1 + i * kSurThreads;
        if (j >= M) continue;
        const double a = dv * (j / (N * N) - N / 2) - u1, b = dv * ((j / N) % N - N / 2) - u2,
                     cc = dv * (j % N - N / 2) - u3;
        const double Mj = nrm * exp(-(a * a + b * b + cc * cc) / (2.0 * T));
        fv[i] -= Mj;   // f - M from here on
        dd += fv[i] * fv[i];
        mm += Mj * Mj;
    }
    const double D2 = block_sum(dd, red), M2 = block_sum(mm, red);
    const double d = sqrt(D2 / M2);
    // network input: the direction of f - M scaled to unit RMS, and in the corner entry
    // (v = (-L, -L, -L), where f - M is negligible) the amplitude d / s_in
    const double sx = D2 > 0 ? sqrt((double)M / D2) : 0.0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int j = threadIdx.x + i * kSurThreads;
        if (j < M) x[(size_t)c * M + j] = f2bf((float)(j == 0 ? d * inv_s_in : fv[i] * sx));
    }
    if (threadIdx.x == 0) {
        if (stats) {
            const unsigned long long cap = *(const unsigned long long *)(stats + kStCap);
            if (cap) gate = fmin(gate, __longlong_as_double((long long)~cap));
        }
        const bool gated = d < gate && rho > 0 && T > 0;
        // judge the gated cells of one 64-cell index range in judge_every per evaluation
        // (rotating), so that at most 64 served cells per evaluation are also convolved
        const bool judged = gated && judge_every > 0 && ((c / kWave) % judge_every) == (phase % judge_every);
        double *st = state + (size_t)c * kState;
        st[0] = rho;
        st[1] = u1;
        st[2] = u2;
        st[3] = u3;
        st[4] = T;
        st[5] = d;
        st[6] = gated ? 1.0 : 0.0;
        st[7] = judged ? 1.0 : 0.0;
        st[8] = sqrt(M2);
        st[9] = 0.0;
    }
}

// Slot order of the convolution: the cells that need it (not gated, or judged) first, then the
// served ones, each in index order.  slot_off[s] = f_off of the cell in slot s; skip[g] = 1 for
// the groups of 64 slots that hold served cells only.  Every cell keeps its own lane arithmetic,
// so only the number of convolved groups changes.  One block of kPackThreads; thread t owns a
// contiguous chunk of cells, and a scan over the chunks gives each its first slot.
constexpr int kPackThreads = 1024;
__global__ void __launch_bounds__(kPackThreads) k_pack_slots(int n, const double *__restrict__ state,
                                                              const long long *__restrict__ f_off,
                                                              long long *__restrict__ slot_off,
                                                              unsigned char *__restrict__ skip) {
    __shared__ int scan[kPackThreads];
    const int t = threadIdx.x;
    const int chunk = (n + kPackThreads - 1) / kPackThreads;
    const int c0 = min(n, t * chunk), c1 = min(n, c0 + chunk);
    auto needs = [&](int c) {
        const double *st = state + (size_t)c * kState;
        return st[6] == 0.0 || st[7] != 0.0;
    };
    int cnt = 0;
    for (int c = c0; c < c1; ++c) cnt += needs(c) ? 1 : 0;
    scan[t] = cnt;
    __syncthreads();
    for (int o = 1; o < kPackThreads; o <<= 1) {  // inclusive scan of the chunk counts
        const int v = t >= o ? scan[t - o] : 0;
        __syncthreads();
        scan[t] += v;
        __syncthreads();
    }
    const int n0 = scan[kPackThreads - 1];  // cells that need the convolution
    int a = scan[t] - cnt;                   // their slots before this chunk
    int b = n0 + (c0 - a);                   // served slots: after all of them, in index order
    for (int c = c0; c < c1; ++c) {
        if (needs(c)) slot_off[a++] = f_off[c];
        else slot_off[b++] = f_off[c];
    }
    for (int g = t; g * kWave < n; g += kPackThreads) skip[g] = g * kWave >= n0 ? 1 : 0;
}

struct Basis {
    double a[25];
};

template <int N>
__device__ inline void basis5(double dv, const Basis &li, int j, double e[5]) {
    const int j1 = j / (N * N), j2 = (j / N) % N, j3 = j % N;
    const double v1 = dv * (j1 - N / 2), v2 = dv * (j2 - N / 2), v3 = dv * (j3 - N / 2);
    const double w = dv * dv * dv;
    const double c[5] = {w, v1 * w, v2 * w, v3 * w, (v1 * v1 + v2 * v2 + v3 * v3) * w};
    for (int a = 0; a < 5; ++a) {
        double s = 0.0;
        for (int b = 0; b <= a; ++b) s = fma(li.a[a * 5 + b], c[b], s);
        e[a] = s;
    }
}

// one block per cell: select the closure or the convolution, judge sampled cells
template <int N>
__global__ void __launch_bounds__(kSurThreads) k_finish(double dv, Basis li, const double *__restrict__ state,
                                                        const float *__restrict__ y, double s_out, double floor_,
                                                        double tol, const long long *__restrict__ q_off,
                                                        double *__restrict__ q, unsigned *__restrict__ stats) {
    __shared__ double red[kSurThreads / 64];
    const int c = blockIdx.x, M = N * N * N;
    const double *st = state + (size_t)c * kState;
    const bool gated = st[6] != 0.0, judged = st[7] != 0.0;
    if (!gated) return;
    double *Q = q + q_off[c];
    const double sc = st[0] * st[5] * st[8] * s_out;   // rho |f - M|_2 s_out
    const float *Y = y + (size_t)c * M;
    if (!judged) {
        for (int j = threadIdx.x; j < M; j += blockDim.x) Q[j] = sc * (double)Y[j];
        if (threadIdx.x == 0) {
            atomicAdd(&stats[kStServed], 1u);
            atomicAdd(&stats[kStEvalServed], 1u);
        }
        return;
    }
    // judged: |P D|^2 = |D|^2 - sum_a (e_a . D)^2 with D = Q_s - Q_c, same for Q_c
    double dd = 0, cc = 0, md[5] = {0, 0, 0, 0, 0}, mc[5] = {0, 0, 0, 0, 0};
    for (int j = threadIdx.x; j < M; j += blockDim.x) {
        double e[5];
        basis5<N>(dv, li, j, e);
        const double qc = Q[j], dj = sc * (double)Y[j] - qc;
        dd += dj * dj;
        cc += qc * qc;
        for (int a = 0; a < 5; ++a) {
            md[a] = fma(e[a], dj, md[a]);
            mc[a] = fma(e[a], qc, mc[a]);
        }
    }
    double D2 = block_sum(dd, red), C2 = block_sum(cc, red);
    for (int a = 0; a < 5; ++a) {
        const double ta = block_sum(md[a], red), tc = block_sum(mc[a], red);
        D2 -= ta * ta;
        C2 -= tc * tc;
    }
    if (threadIdx.x == 0) {
        const double err = sqrt(fmax(D2, 0.0)) / (sqrt(fmax(C2, 0.0)) + floor_ * st[0] * st[8]);
        const float ef = (float)err;
        atomicMax(&stats[kStMaxErr], __float_as_uint(ef));  // non-negative floats order as unsigned
        atomicAdd(&stats[kStJudged], 1u);
        if (err > tol) {
            atomicAdd(&stats[kStFailed], 1u);
            atomicAdd(&stats[kStEvalFailed], 1u);
            // cap the gate at this cell's deviation: the complement of the bits of a smaller
            // positive double is a larger word
            atomicMax((unsigned long long *)(stats + kStCap), ~(unsigned long long)__double_as_longlong(st[5]));
        }
    }
    // the judged cell keeps the convolution result (fallback)
}

// After the selection of an evaluation: its served cells are unbounded if one of its judges
// failed; the evaluation's counters restart.
__global__ void k_judge_close(unsigned *__restrict__ stats) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (stats[kStEvalFailed]) stats[kStUnbounded] += stats[kStEvalServed];
        stats[kStEvalServed] = 0;
        stats[kStEvalFailed] = 0;
    }
}

// y = Q / (rho |f - M|_2 s_out) for harvesting training targets (0 where f = M)
template <int N>
__global__ void k_targets(const double *__restrict__ state, const double *__restrict__ q,
                          const long long *__restrict__ q_off, double inv_s_out, float *__restrict__ y) {
    const int c = blockIdx.y, M = N * N * N;
    const double *st = state + (size_t)c * kState;
    const double a = st[0] * st[5] * st[8];
    const double sc = a > 0 ? inv_s_out / a : 0.0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < M; j += gridDim.x * blockDim.x)
        y[(size_t)c * M + j] = (float)(q[q_off[c] + j] * sc);
}

}  // namespace

// the mesh sizes the library accepts (multiples of 4 from 8 to 32)
#define BZ_SUR_FOR_N(CALL)                                   \
    switch (N) {                                             \
    case 8: CALL(8); break;                                  \
    case 12: CALL(12); break;                                \
    case 16: CALL(16); break;                                \
    case 20: CALL(20); break;                                \
    case 24: CALL(24); break;                                \
    case 28: CALL(28); break;                                \
    case 32: CALL(32); break;                                \
    default: return hipErrorInvalidValue;                    \
    }

hipError_t launch_sur_prepare(int N, double dv, int n, const double *f, const long long *f_off, double gate,
                              double s_in, int judge_every, int phase, const unsigned *stats, double *state,
                              unsigned short *x, hipStream_t s) {
#define BZ_PREP(NN)                                                                                             \
    hipLaunchKernelGGL(k_prepare<NN>, dim3(n), dim3(kSurThreads), 0, s, dv, f, f_off, gate, 1.0 / s_in,      \
                       judge_every, phase, stats, state, x)
    BZ_SUR_FOR_N(BZ_PREP)
#undef BZ_PREP
    return hipGetLastError();
}

hipError_t launch_pack_slots(int n, const double *state, const long long *f_off, long long *slot_off,
                             unsigned char *skip, hipStream_t s) {
    hipLaunchKernelGGL(k_pack_slots, dim3(1), dim3(kPackThreads), 0, s, n, state, f_off, slot_off, skip);
    return hipGetLastError();
}

hipError_t launch_sur_finish(int N, double dv, const double *linv, int n, const double *state, const float *y,
                             double s_out, double floor_, double tol, const long long *q_off, double *q,
                             unsigned *stats, hipStream_t s) {
    Basis li;
    for (int i = 0; i < 25; ++i) li.a[i] = linv[i];
#define BZ_FIN(NN)                                                                                              \
    hipLaunchKernelGGL(k_finish<NN>, dim3(n), dim3(kSurThreads), 0, s, dv, li, state, y, s_out, floor_, tol,  \
                       q_off, q, stats)
    BZ_SUR_FOR_N(BZ_FIN)
#undef BZ_FIN
    hipLaunchKernelGGL(k_judge_close, dim3(1), dim3(64), 0, s, stats);
    return hipGetLastError();
}

hipError_t launch_sur_targets(int N, int n, const double *state, const double *q, const long long *q_off,
                              double s_out, float *y, hipStream_t s) {
#define BZ_TGT(NN) hipLaunchKernelGGL(k_targets<NN>, dim3(16, n), dim3(256), 0, s, state, q, q_off, 1.0 / s_out, y)
    BZ_SUR_FOR_N(BZ_TGT)
#undef BZ_TGT
    return hipGetLastError();
}
#undef BZ_SUR_FOR_N

}  // namespace bz
