// Learned closure: a 3-layer perceptron n_in -> n_hid -> n_hid -> n_out with
// exact-erf GELU, BF16 operands and FP32 accumulation on the CDNA4 matrix
// cores, trained with mean-squared error and Adam (FP32 master weights).
//
// One GEMM form serves forward and backward: C[M x N] = alpha * A[M x K] B^T,
// A [M x K] and B [N x K] both row-major BF16 with K contiguous, so that the
// fragments of v_mfma_f32_16x16x32_bf16 (8 consecutive k per lane: A row
// lane%16, B column lane%16, k block lane/16) are single 16-byte LDS reads.
//   forward   Z1 = X W1^T, Z2 = A1 W2^T, Y = A2 W3^T         (weights stored [out][in])
//   backward  dA2 = dY W3, dA1 = dZ2 W2                       (transposed copies W3, W2)
//             dW3 = dY^T A2, dW2 = dZ2^T A1, dW1 = dZ1^T X     (transposed activations)
// Tile 128 x 128 per 256-thread workgroup (4 waves of 64 x 64, 16 MFMAs each per
// 32-deep k tile), the k tiles staged through LDS by direct-to-LDS loads, several
// tiles in flight (k_gemm_nt).  K must be a multiple of 32.
#include <cmath>
#include <new>
#include <vector>

#include "bz_internal.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

struct bz_mlp_s {
    int n_in = 0, n_hid = 0, n_out = 0;
    // offsets (elements) into the FP32 master block
    size_t oW1 = 0, ob1 = 0, oW2 = 0, ob2 = 0, oW3 = 0, ob3 = 0, n_params = 0;
};

namespace bz {
namespace {

__device__ inline unsigned short f2bf(float x) {
    // round to nearest even (finite inputs)
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_prime(float z) {
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.3989422804014327f;
}

enum { EPI_F32 = 0, EPI_GELU = 1, EPI_PARTIAL = 2 };

constexpr int TBM = 128, TBN = 128, TBK = 32;
constexpr int kXcds = 8;   // accelerator complex dies of the chip, each with its own L2

// Tile (tm, tn) and split slice tz of this workgroup.  Workgroup w of the launch (x fastest,
// then y, then z) runs on XCD w % 8, and the eight XCDs have their own L2, so each XCD takes a
// contiguous range of the tiles, ordered split slice slowest and, within a slice, along the
// smaller operand fastest: the workgroups of one XCD then share the tiles of the larger
// operand, which is read from memory about once instead of once per XCD.
__device__ __forceinline__ void gemm_tile(int M, int N, int &tm, int &tn, int &tz) {
    const int Tn = gridDim.x, Tm = gridDim.y, T = Tn * Tm * gridDim.z;
    const int w = blockIdx.x + Tn * (blockIdx.y + Tm * blockIdx.z);
    const int q = T / kXcds, r = T % kXcds, x = w % kXcds, l = w / kXcds;
    const int t = x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
    const int mn = t % (Tm * Tn);
    tz = t / (Tm * Tn);
    if (N > M) {
        tm = mn % Tm;
        tn = mn / Tm;
    } else {
        tn = mn % Tn;
        tm = mn / Tn;
    }
}

// Epilogue of a 128 x 128 tile: wave (wm, wn) holds the 64 x 64 block acc[i][j] (16 x 16
// MFMA tiles; lane l holds column l % 16, rows 4 (l / 16) .. 4 (l / 16) + 3).
template <int EPI>
__device__ __forceinline__ void gemm_epilogue(const f32x4 (&acc)[4][4], int M, int N, int m0, int n0, int tz, int wm,
                                              int wn, int lane, float alpha, const float *__restrict__ bias,
                                              float *__restrict__ C32, int ldc, unsigned short *__restrict__ Cbf,
                                              int ldcb) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int col = n0 + wn * 64 + j * 16 + (lane & 15);
            if (col >= N) continue;
            const float bcol = bias ? bias[col] : 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + r;
                if (row >= M) continue;
                if (EPI == EPI_PARTIAL) {
                    C32[((size_t)tz * M + row) * ldc + col] = acc[i][j][r];
                    continue;
                }
                const float z = alpha * acc[i][j][r] + bcol;
                if (EPI == EPI_GELU) {
                    C32[(size_t)row * ldc + col] = z;
                    Cbf[(size_t)row * ldcb + col] = f2bf(gelu(z));
                } else {
                    C32[(size_t)row * ldc + col] = z;
                }
            }
        }
}

// k tiles of 128 x 32 per operand (rows of 64 bytes: four 16-byte chunks) are copied
// global -> LDS by direct-to-LDS loads (global_load_lds_dwordx4: each lane moves 16 bytes, the
// wavefront 1 KiB, landing contiguously at a wavefront-uniform LDS address), so no registers
// carry them: kStages LDS stages of 16 KiB, the loads of tile kt + kStages - 1 issued while
// tile kt feeds the MFMAs, one barrier per tile.  Chunk c of row r sits at slot
// c ^ ((r >> 2) & 3), so that the lanes that read one chunk of consecutive rows hit different
// groups of four banks; a lane's global address picks the chunk that belongs at its LDS
// slot.  Rows past M or N read row M - 1 or N - 1 (their results are never stored).
constexpr int kStages = 3;
constexpr int kCPR = TBK / 8;                 // 16-byte chunks per tile row
constexpr int kLPW = TBM * kCPR / 256;        // 1 KiB loads per wavefront, operand and tile
__device__ __forceinline__ int lds_slot(int row, int c) { return c ^ ((row >> 2) & 3); }

// EPI_F32:  C32[m][n] = alpha * acc + (bias ? bias[n] : 0)
// EPI_GELU: Z = acc + bias[n]; C32 = Z; Cbf = bf16(gelu(Z))
// EPI_PARTIAL (split K): workgroup z of gridDim.z sums the k tiles
//           [z nk / Z, (z + 1) nk / Z) and writes its raw sums to C32 + z M ldc;
//           k_splitk_reduce then adds the Z slices in order and applies the epilogue.
template <int EPI>
__global__ void __launch_bounds__(256) k_gemm_nt(int M, int N, int K, const unsigned short *__restrict__ A, int lda,
                                                 const unsigned short *__restrict__ B, int ldb, float alpha,
                                                 const float *__restrict__ bias, float *__restrict__ C32, int ldc,
                                                 unsigned short *__restrict__ Cbf, int ldcb) {
    // [stage][A, B][128 rows x 4 chunks of 16 bytes], 48 KiB
    __shared__ __attribute__((aligned(16))) uint4 lds[kStages][2][TBM * kCPR];
    typedef __attribute__((address_space(3))) char lds_char;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int wm = wave >> 1, wn = wave & 1;
    int tm, tn, tz;
    gemm_tile(M, N, tm, tn, tz);
    const int m0 = tm * TBM, n0 = tn * TBN;
    const int nk_all = K / TBK;
    const int kt0 = (int)((long long)nk_all * tz / gridDim.z);
    const int nk = (int)((long long)nk_all * (tz + 1) / gridDim.z);
    // this lane's chunk of each of the wavefront's 1 KiB loads per operand: LDS chunk
    // p = (kLPW wave + i) 64 + lane of a tile, row p / kCPR, slot p % kCPR
    const unsigned short *ga[kLPW], *gb[kLPW];
#pragma unroll
    for (int i = 0; i < kLPW; ++i) {
        const int p = (kLPW * wave + i) * 64 + lane, row = p / kCPR, c = lds_slot(row, p % kCPR);
        ga[i] = A + (size_t)min(m0 + row, M - 1) * lda + c * 8;
        gb[i] = B + (size_t)min(n0 + row, N - 1) * ldb + c * 8;
    }
    lds_char *const base = (lds_char *)&lds[0][0][0];
    auto issue = [&](int kt, int st) {
        lds_char *da = base + (size_t)(st * 2 + 0) * (TBM * kCPR * 16) + (size_t)(kLPW * wave) * 1024;
        lds_char *db = base + (size_t)(st * 2 + 1) * (TBM * kCPR * 16) + (size_t)(kLPW * wave) * 1024;
        const int ko = kt * TBK;
#pragma unroll
        for (int i = 0; i < kLPW; ++i) {
            __builtin_amdgcn_global_load_lds((const void *)(ga[i] + ko), (void __attribute__((address_space(3))) *)(da + i * 1024),
                                             16, 0, 0);
            __builtin_amdgcn_global_load_lds((const void *)(gb[i] + ko), (void __attribute__((address_space(3))) *)(db + i * 1024),
                                             16, 0, 0);
        }
    };
    f32x4 acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int st = 0; st < kStages - 1; ++st)
        if (kt0 + st < nk) issue(kt0 + st, st);
    for (int kt = kt0; kt < nk; ++kt) {
        const int st = (kt - kt0) % kStages;
        // this wavefront's loads of tile kt have landed once at most those of the tiles after
        // it are outstanding (loads complete in issue order)
        if (kt + kStages - 2 < nk) {
            constexpr int n = (kStages - 2) * 2 * kLPW;
            static_assert(n < 64, "vmcnt field");
            __builtin_amdgcn_s_waitcnt((n & 0xF) | ((n >> 4) << 14) | (0x7 << 4) | (0xF << 8));
        } else {
            __builtin_amdgcn_s_waitcnt(0x0 | (0x7 << 4) | (0xF << 8));
        }
        // every wavefront's part of tile kt is in LDS, and every wavefront is done with tile
        // kt - 1, whose stage the next loads overwrite.  A bare s_barrier: __syncthreads()
        // adds a release fence, which waits for every outstanding load, the later tiles' too.
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        if (kt + kStages - 1 < nk) issue(kt + kStages - 1, (kt - kt0 + kStages - 1) % kStages);
        bf16x8 af[4], bfr[4];
        const int ch = lane >> 4;   // this lane's k chunk of the tile
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = wm * 64 + i * 16 + (lane & 15);
            af[i] = *(const bf16x8 *)&lds[st][0][row * kCPR + lds_slot(row, ch)];
            const int col = wn * 64 + i * 16 + (lane & 15);
            bfr[i] = *(const bf16x8 *)&lds[st][1][col * kCPR + lds_slot(col, ch)];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    }
    gemm_epilogue<EPI>(acc, M, N, m0, n0, tz, wm, wn, lane, alpha, bias, C32, ldc, Cbf, ldcb);
}

// Sum of the Z split-K slices P[z][M][N] in order z = 0, 1, ..., then the epilogue of EPI.
template <int EPI>
__global__ void __launch_bounds__(256) k_splitk_reduce(int M, int N, int Z, const float *__restrict__ P, float alpha,
                                                       const float *__restrict__ bias, float *__restrict__ C32,
                                                       int ldc, unsigned short *__restrict__ Cbf, int ldcb) {
    const size_t MN = (size_t)M * N;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < MN; i += (size_t)gridDim.x * blockDim.x) {
        const int row = (int)(i / N), col = (int)(i - (size_t)row * N);
        float acc = 0.f;
        for (int z = 0; z < Z; ++z) acc += P[z * MN + i];
        const float v = alpha * acc + (bias ? bias[col] : 0.f);
        C32[(size_t)row * ldc + col] = v;
        if (EPI == EPI_GELU) Cbf[(size_t)row * ldcb + col] = f2bf(gelu(v));
    }
}

// out[c][r] = in[r][c] for an R x C BF16 matrix, R and C multiples of 8, 16-byte aligned
// rows.  Each wavefront moves a 64 x 64 tile and each lane an 8 x 8 block of it through its
// registers: lane l takes block row l / 8 and block column l % 8, so that 8 lanes read 128
// contiguous bytes of an input row and write 128 contiguous bytes of an output row.
__global__ void __launch_bounds__(256) k_transpose_bf16(int R, int C, const unsigned short *__restrict__ in,
                                                        unsigned short *__restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int tile = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int tiles_c = (C + 63) / 64;
    const int tr = tile / tiles_c, tc = tile - tr * tiles_c;
    const int r = tr * 64 + (lane >> 3) * 8, c = tc * 64 + (lane & 7) * 8;
    if (r >= R || c >= C) return;
    unsigned a[8][4];   // rows r .. r + 7, columns c .. c + 7, two per word
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const uint4 u = *(const uint4 *)(in + (size_t)(r + i) * C + c);
        a[i][0] = u.x;
        a[i][1] = u.y;
        a[i][2] = u.z;
        a[i][3] = u.w;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        // column c + j: element j of each row, i.e. half j % 2 of word j / 2
        unsigned w[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned lo = (a[2 * k][j / 2] >> (16 * (j % 2))) & 0xFFFFu;
            const unsigned hi = (a[2 * k + 1][j / 2] >> (16 * (j % 2))) & 0xFFFFu;
            w[k] = lo | (hi << 16);
        }
        *(uint4 *)(out + (size_t)(c + j) * R + r) = make_uint4(w[0], w[1], w[2], w[3]);
    }
}

// The same for any R, C and alignment: 32 x 32 tiles through LDS, one element per access.
__global__ void __launch_bounds__(256) k_transpose_bf16_any(int R, int C, const unsigned short *__restrict__ in,
                                                            unsigned short *__restrict__ out) {
    __shared__ unsigned short t[32][33];
    const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int y = ty; y < 32; y += 8) {
        const int r = r0 + y, c = c0 + tx;
        t[y][tx] = (r < R && c < C) ? in[(size_t)r * C + c] : 0;
    }
    __syncthreads();
    for (int y = ty; y < 32; y += 8) {
        const int c = c0 + y, r = r0 + tx;
        if (c < C && r < R) out[(size_t)c * R + r] = t[tx][y];
    }
}

__global__ void k_f32_to_bf16(size_t n, const float *__restrict__ in, unsigned short *__restrict__ out) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        out[i] = f2bf(in[i]);
}

// dY = bf16(scale (Y - T)); per-block partial sums of (Y - T)^2 into part[blockIdx.x]
__global__ void __launch_bounds__(256) k_mse_grad(size_t n, const float *__restrict__ Y, const float *__restrict__ T,
                                                  float scale, unsigned short *__restrict__ dY,
                                                  double *__restrict__ part) {
    __shared__ double red[4];
    double s = 0.0;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const float d = Y[i] - T[i];
        dY[i] = f2bf(scale * d);
        s += (double)d * d;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// loss = inv_n * sum of the n block partials (one 256-thread block, fixed order)
__global__ void __launch_bounds__(256) k_sum_parts(int n, const double *__restrict__ part, double inv_n,
                                                   float *__restrict__ loss) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) loss[0] = (float)((red[0] + red[1] + red[2] + red[3]) * inv_n);
}

// dZ = bf16(dA * gelu'(Z))
__global__ void k_gelu_bwd(size_t n, const float *__restrict__ dA, const float *__restrict__ Z,
                           unsigned short *__restrict__ dZ) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dZ[i] = f2bf(dA[i] * gelu_prime(Z[i]));
}

// db[n] = alpha * sum_m bf2f(D[m][n])  (D is rows x cols BF16).  A block of 64 x 16
// threads owns 64 columns; thread (c, t) sums the rows r = t (mod 16) of its column,
// then the 16 partial sums are added in order.
// db[c] = alpha * sum over rows of D[r][c] (BF16 [rows][cols], cols a multiple of 8, 16-byte
// aligned rows).  A block of 128 threads sums 64 columns: thread (tr, q) adds columns
// 8q .. 8q + 7 of the rows tr, tr + 16, ... (one 16-byte load per row; 8 threads read 128
// contiguous bytes of a row), then the 16 row-group partials are added in order.
__global__ void __launch_bounds__(128) k_col_sums(int rows, int cols, const unsigned short *__restrict__ D,
                                                  float alpha, float *__restrict__ db) {
    __shared__ float part[16][64];
    const int tc = (threadIdx.x & 7) * 8, tr = threadIdx.x >> 3;
    const int c = blockIdx.x * 64 + tc;
    float s[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (c < cols)
        for (int r = tr; r < rows; r += 16) {
            const uint4 u = *(const uint4 *)(D + (size_t)r * cols + c);
            const unsigned w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                s[2 * k] += bf2f((unsigned short)(w[k] & 0xFFFFu));
                s[2 * k + 1] += bf2f((unsigned short)(w[k] >> 16));
            }
        }
#pragma unroll
    for (int k = 0; k < 8; ++k) part[tr][tc + k] = s[k];
    __syncthreads();
    const int cc = blockIdx.x * 64 + threadIdx.x;
    if (threadIdx.x < 64 && cc < cols) {
        float t = 0.f;
#pragma unroll
        for (int i = 0; i < 16; ++i) t += part[i][threadIdx.x];
        db[cc] = alpha * t;
    }
}

// The three weight matrices' BF16 copies: master entries [off[k], off[k] + len[k]) go to
// dst[k][i - off[k]].
struct Bf16Copies {
    size_t off[3], len[3];
    unsigned short *dst[3];
};

// One Adam step over all parameters, which also writes the BF16 copy of every updated weight
// (the same rounding as k_f32_to_bf16), so the copies need no second pass over the masters.
// The first 4 n4 parameters four per thread and access (16-byte loads and stores; the matrices
// start and end at multiples of four, so a group of four lies inside one matrix or outside all
// three), the rest one at a time (n4 = 0 when a buffer is not 16-byte aligned).
__device__ __forceinline__ float adam_one(float &w, float &m, float &v, float g, float lr, float b1, float b2,
                                          float eps, float c1, float c2) {
    m = b1 * m + (1.f - b1) * g;
    v = b2 * v + (1.f - b2) * g * g;
    w = w - lr * (m * c1) / (sqrtf(v * c2) + eps);
    return w;
}
__global__ void k_adam(size_t n, size_t n4, float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2,
                       Bf16Copies bc) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < n4; q += stride) {
        float4 wq = ((float4 *)w)[q], mq = ((float4 *)m)[q], vq = ((float4 *)v)[q];
        const float4 gq = ((const float4 *)g)[q];
        adam_one(wq.x, mq.x, vq.x, gq.x, lr, b1, b2, eps, c1, c2);
        adam_one(wq.y, mq.y, vq.y, gq.y, lr, b1, b2, eps, c1, c2);
        adam_one(wq.z, mq.z, vq.z, gq.z, lr, b1, b2, eps, c1, c2);
        adam_one(wq.w, mq.w, vq.w, gq.w, lr, b1, b2, eps, c1, c2);
        ((float4 *)w)[q] = wq;
        ((float4 *)m)[q] = mq;
        ((float4 *)v)[q] = vq;
        const size_t i = 4 * q;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (i - bc.off[k] < bc.len[k])
                *(uint2 *)(bc.dst[k] + (i - bc.off[k])) =
                    make_uint2(f2bf(wq.x) | ((unsigned)f2bf(wq.y) << 16), f2bf(wq.z) | ((unsigned)f2bf(wq.w) << 16));
    }
    for (size_t i = 4 * n4 + blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        float wi = w[i], mi = m[i], vi = v[i];
        adam_one(wi, mi, vi, g[i], lr, b1, b2, eps, c1, c2);
        w[i] = wi;
        m[i] = mi;
        v[i] = vi;
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (i - bc.off[k] < bc.len[k]) bc.dst[k][i - bc.off[k]] = f2bf(wi);
    }
}

__global__ void k_fill_f32(size_t n, float *__restrict__ p, float v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

inline unsigned grid1(size_t n) {
    size_t b = (n + 255) / 256;
    return (unsigned)(b > 16384 ? 16384 : (b < 1 ? 1 : b));
}

}  // namespace

// ---------------------------------------------------------------------------
// Buffer layouts.
//   params (caller-owned, bz_mlp_param_bytes): FP32 master [W1 b1 W2 b2 W3 b3],
//     Adam m and v (same layout), then BF16 W1, W2, W3 ([out][in]) and BF16
//     transposed W2^T, W3^T ([in][out]).
//   workspace (bz_mlp_workspace_bytes(batch)): activations and gradients.
// ---------------------------------------------------------------------------
struct ParamView {
    float *master, *m, *v;
    unsigned short *W1, *W2, *W3, *W2t, *W3t;
};

static size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

static ParamView param_view(const bz_mlp_s *n, void *p) {
    char *c = (char *)p;
    ParamView v;
    const size_t fb = a256(n->n_params * 4);
    v.master = (float *)c;
    v.m = (float *)(c + fb);
    v.v = (float *)(c + 2 * fb);
    char *b = c + 3 * fb;
    v.W1 = (unsigned short *)b;
    b += a256((size_t)n->n_hid * n->n_in * 2);
    v.W2 = (unsigned short *)b;
    b += a256((size_t)n->n_hid * n->n_hid * 2);
    v.W3 = (unsigned short *)b;
    b += a256((size_t)n->n_out * n->n_hid * 2);
    v.W2t = (unsigned short *)b;
    b += a256((size_t)n->n_hid * n->n_hid * 2);
    v.W3t = (unsigned short *)b;
    return v;
}

static size_t param_bytes(const bz_mlp_s *n) {
    return 3 * a256(n->n_params * 4) + a256((size_t)n->n_hid * n->n_in * 2) + 2 * a256((size_t)n->n_hid * n->n_hid * 2) +
           2 * a256((size_t)n->n_out * n->n_hid * 2);
}

// split-K slices: up to kMaxSplit x batch x n_hid FP32 values
constexpr int kMaxSplit = 16;

struct WorkView {
    float *split;                // split-K slices
    size_t split_floats;
    float *Z1, *Z2, *Y, *dA;     // FP32
    unsigned short *A1, *A2;     // BF16 activations
    unsigned short *dY, *dZ;     // BF16 gradients (dZ reused for layers 2 and 1)
    unsigned short *tA, *tB;     // transposes
    double *part;
    float *loss;
};

static WorkView work_view(const bz_mlp_s *n, int B, void *w) {
    char *c = (char *)w;
    WorkView v;
    auto take = [&c](size_t bytes) {
        char *p = c;
        c += a256(bytes);
        return p;
    };
    const size_t H = n->n_hid, O = n->n_out, I = n->n_in;
    v.split_floats = (size_t)kMaxSplit * B * H;
    v.split = (float *)take(v.split_floats * 4);
    v.Z1 = (float *)take((size_t)B * H * 4);
    v.Z2 = (float *)take((size_t)B * H * 4);
    v.Y = (float *)take((size_t)B * O * 4);
    v.dA = (float *)take((size_t)B * H * 4);
    v.A1 = (unsigned short *)take((size_t)B * H * 2);
    v.A2 = (unsigned short *)take((size_t)B * H * 2);
    v.dY = (unsigned short *)take((size_t)B * O * 2);
    v.dZ = (unsigned short *)take((size_t)B * H * 2);
    const size_t big = std::max(std::max(O, I), H) * (size_t)B * 2;
    v.tA = (unsigned short *)take(big);
    v.tB = (unsigned short *)take(big);
    v.part = (double *)take(16384 * 8);
    v.loss = (float *)take(256);
    return v;
}

static size_t work_bytes(const bz_mlp_s *n, int B) {
    const size_t H = n->n_hid, O = n->n_out, I = n->n_in;
    return a256((size_t)kMaxSplit * B * H * 4) + a256((size_t)B * H * 4) * 3 + a256((size_t)B * O * 4) +
           a256((size_t)B * H * 2) * 3 +
           a256((size_t)B * O * 2) + 2 * a256(std::max(std::max(O, I), H) * (size_t)B * 2) + a256(16384 * 8) + 256;
}

// C = alpha A B^T (+ bias, epilogue).  A product with fewer output tiles than
// there are compute units and a long K is split over K into up to kMaxSplit
// slices (at least 256 deep each) when the workspace slice buffer holds them.
static hipError_t gemm(int epi, int M, int N, int K, const unsigned short *A, int lda, const unsigned short *B, int ldb,
                       float alpha, const float *bias, float *C32, int ldc, unsigned short *Cbf, int ldcb,
                       const WorkView &wv, hipStream_t s) {
    dim3 grid((N + TBN - 1) / TBN, (M + TBM - 1) / TBM);
    const int tiles = (int)(grid.x * grid.y);
    int split = 1;
    if (tiles < 128) {
        split = std::min(std::min(kMaxSplit, K / 256), (256 + tiles - 1) / tiles);
        const size_t cap = wv.split_floats / ((size_t)M * N);
        if ((size_t)split > cap) split = (int)cap;
    }
    if (split >= 2) {
        grid.z = split;
        hipLaunchKernelGGL(k_gemm_nt<EPI_PARTIAL>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, 1.f, nullptr,
                           wv.split, N, nullptr, 0);
        const size_t mn = (size_t)M * N;
        const unsigned rg = (unsigned)std::min<size_t>((mn + 255) / 256, 4096);
        if (epi == EPI_GELU)
            hipLaunchKernelGGL(k_splitk_reduce<EPI_GELU>, dim3(rg), dim3(256), 0, s, M, N, split, wv.split, alpha, bias,
                               C32, ldc, Cbf, ldcb);
        else
            hipLaunchKernelGGL(k_splitk_reduce<EPI_F32>, dim3(rg), dim3(256), 0, s, M, N, split, wv.split, alpha, bias,
                               C32, ldc, Cbf, ldcb);
        return hipGetLastError();
    }
    if (epi == EPI_GELU)
        hipLaunchKernelGGL(k_gemm_nt<EPI_GELU>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, alpha, bias, C32, ldc,
                           Cbf, ldcb);
    else
        hipLaunchKernelGGL(k_gemm_nt<EPI_F32>, grid, dim3(256), 0, s, M, N, K, A, lda, B, ldb, alpha, bias, C32, ldc,
                           Cbf, ldcb);
    return hipGetLastError();
}

static hipError_t transpose(int R, int C, const unsigned short *in, unsigned short *out, hipStream_t s) {
    if (R % 8 || C % 8 || ((uintptr_t)in | (uintptr_t)out) % 16) {
        hipLaunchKernelGGL(k_transpose_bf16_any, dim3((C + 31) / 32, (R + 31) / 32), dim3(256), 0, s, R, C, in, out);
        return hipGetLastError();
    }
    const long long tiles = (long long)((R + 63) / 64) * ((C + 63) / 64);
    hipLaunchKernelGGL(k_transpose_bf16, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, R, C, in, out);
    return hipGetLastError();
}

static hipError_t col_sums(int rows, int cols, const unsigned short *D, float alpha, float *db, hipStream_t s) {
    if (cols % 8 || (uintptr_t)D % 16) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_col_sums, dim3((cols + 63) / 64), dim3(128), 0, s, rows, cols, D, alpha, db);
    return hipGetLastError();
}

// W2^T and W3^T from the BF16 copies of W2 and W3
static hipError_t refresh_transposes(const bz_mlp_s *n, const ParamView &pv, hipStream_t s) {
    const size_t H = n->n_hid, O = n->n_out;
    hipError_t e = transpose((int)H, (int)H, pv.W2, pv.W2t, s);
    if (e == hipSuccess) e = transpose((int)O, (int)H, pv.W3, pv.W3t, s);
    return e == hipSuccess ? hipGetLastError() : e;
}

static hipError_t refresh_bf16(const bz_mlp_s *n, const ParamView &pv, hipStream_t s) {
    const size_t H = n->n_hid, O = n->n_out, I = n->n_in;
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1(H * I)), dim3(256), 0, s, H * I, pv.master + n->oW1, pv.W1);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1(H * H)), dim3(256), 0, s, H * H, pv.master + n->oW2, pv.W2);
    hipLaunchKernelGGL(k_f32_to_bf16, dim3(grid1(O * H)), dim3(256), 0, s, O * H, pv.master + n->oW3, pv.W3);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? refresh_transposes(n, pv, s) : e;
}

static hipError_t forward(const bz_mlp_s *n, const ParamView &pv, const unsigned short *X, int B, const WorkView &wv,
                          float *Y, hipStream_t s) {
    const int H = n->n_hid, O = n->n_out, I = n->n_in;
    hipError_t e = gemm(EPI_GELU, B, H, I, X, I, pv.W1, I, 1.f, pv.master + n->ob1, wv.Z1, H, wv.A1, H, wv, s);
    if (e == hipSuccess) e = gemm(EPI_GELU, B, H, H, wv.A1, H, pv.W2, H, 1.f, pv.master + n->ob2, wv.Z2, H, wv.A2, H, wv, s);
    if (e == hipSuccess) e = gemm(EPI_F32, B, O, H, wv.A2, H, pv.W3, H, 1.f, pv.master + n->ob3, Y, O, nullptr, 0, wv, s);
    return e;
}

// gradients of mean((Y - T)^2) into g (FP32, master layout); dY is kept as bf16(Y - T),
// the factor 2 / (B n_out) is applied in the weight-gradient GEMMs and bias sums.
static hipError_t backward(const bz_mlp_s *n, const ParamView &pv, const unsigned short *X, const float *T, int B,
                           const WorkView &wv, float *g, hipStream_t s) {
    const int H = n->n_hid, O = n->n_out, I = n->n_in;
    const size_t nY = (size_t)B * O;
    const float gs = 2.0f / (float)nY;
    hipLaunchKernelGGL(k_mse_grad, dim3(grid1(nY) > 4096 ? 4096 : grid1(nY)), dim3(256), 0, s, nY, wv.Y, T, 1.0f,
                       wv.dY, wv.part);
    const int nparts = grid1(nY) > 4096 ? 4096 : (int)grid1(nY);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, nparts, wv.part, 1.0 / (double)nY, wv.loss);
    // layer 3: dW3 = gs dY^T A2 ([O x B] x [H x B]^T), db3 = gs colsum(dY), dA2 = dY W3 (via W3t [H x O])
    hipError_t e = transpose(B, O, wv.dY, wv.tA, s);
    if (e == hipSuccess) e = transpose(B, H, wv.A2, wv.tB, s);
    if (e == hipSuccess) e = gemm(EPI_F32, O, H, B, wv.tA, B, wv.tB, B, gs, nullptr, g + n->oW3, H, nullptr, 0, wv, s);
    if (e == hipSuccess) e = col_sums(B, O, wv.dY, gs, g + n->ob3, s);
    if (e == hipSuccess) e = gemm(EPI_F32, B, H, O, wv.dY, O, pv.W3t, O, gs, nullptr, wv.dA, H, nullptr, 0, wv, s);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(grid1((size_t)B * H)), dim3(256), 0, s, (size_t)B * H, wv.dA, wv.Z2, wv.dZ);
    // layer 2 (dZ holds the true gradient dL/dZ2)
    if (e == hipSuccess) e = transpose(B, H, wv.dZ, wv.tA, s);
    if (e == hipSuccess) e = transpose(B, H, wv.A1, wv.tB, s);
    if (e == hipSuccess) e = gemm(EPI_F32, H, H, B, wv.tA, B, wv.tB, B, 1.f, nullptr, g + n->oW2, H, nullptr, 0, wv, s);
    if (e == hipSuccess) e = col_sums(B, H, wv.dZ, 1.f, g + n->ob2, s);
    if (e == hipSuccess) e = gemm(EPI_F32, B, H, H, wv.dZ, H, pv.W2t, H, 1.f, nullptr, wv.dA, H, nullptr, 0, wv, s);
    hipLaunchKernelGGL(k_gelu_bwd, dim3(grid1((size_t)B * H)), dim3(256), 0, s, (size_t)B * H, wv.dA, wv.Z1, wv.dZ);
    // layer 1
    if (e == hipSuccess) e = transpose(B, H, wv.dZ, wv.tA, s);
    if (e == hipSuccess) e = transpose(B, I, X, wv.tB, s);
    if (e == hipSuccess) e = gemm(EPI_F32, H, I, B, wv.tA, B, wv.tB, B, 1.f, nullptr, g + n->oW1, I, nullptr, 0, wv, s);
    if (e == hipSuccess) e = col_sums(B, H, wv.dZ, 1.f, g + n->ob1, s);
    return e == hipSuccess ? hipGetLastError() : e;
}

}  // namespace bz

using namespace bz;

extern "C" {

bz_status bz_mlp_create(int n_in, int n_hidden, int n_out, bz_mlp *out) {
    if (!out) return fail(BZ_EINVAL, "bz_mlp_create: out is NULL");
    *out = nullptr;
    if (n_in < 32 || n_hidden < 32 || n_out < 32 || n_in % 32 || n_hidden % 32 || n_out % 32)
        return fail(BZ_EINVAL, "bz_mlp_create: n_in, n_hidden and n_out must be multiples of 32");
    bz_mlp_s *n = new (std::nothrow) bz_mlp_s();
    if (!n) return fail(BZ_ENOMEM, "bz_mlp_create: allocation failed");
    n->n_in = n_in;
    n->n_hid = n_hidden;
    n->n_out = n_out;
    size_t o = 0;
    n->oW1 = o; o += (size_t)n_hidden * n_in;
    n->ob1 = o; o += n_hidden;
    n->oW2 = o; o += (size_t)n_hidden * n_hidden;
    n->ob2 = o; o += n_hidden;
    n->oW3 = o; o += (size_t)n_out * n_hidden;
    n->ob3 = o; o += n_out;
    n->n_params = o;
    *out = n;
    return BZ_OK;
}

void bz_mlp_free(bz_mlp n) { delete n; }
size_t bz_mlp_param_count(bz_mlp n) { return n ? n->n_params : 0; }
size_t bz_mlp_param_bytes(bz_mlp n) { return n ? param_bytes(n) : 0; }
size_t bz_mlp_workspace_bytes(bz_mlp n, int batch) { return (n && batch > 0) ? work_bytes(n, batch) : 0; }

bz_status bz_mlp_set_params(bz_mlp n, void *d_params, const float *master, void *stream) {
    if (!n || !d_params || !master) return fail(BZ_EINVAL, "bz_mlp_set_params: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ParamView pv = param_view(n, d_params);
    BZ_HIP(hipMemcpyAsync(pv.master, master, n->n_params * 4, hipMemcpyHostToDevice, s), "upload weights");
    hipLaunchKernelGGL(k_fill_f32, dim3(grid1(n->n_params)), dim3(256), 0, s, n->n_params, pv.m, 0.f);
    hipLaunchKernelGGL(k_fill_f32, dim3(grid1(n->n_params)), dim3(256), 0, s, n->n_params, pv.v, 0.f);
    BZ_HIP(hipGetLastError(), "zero Adam moments");
    BZ_HIP(refresh_bf16(n, pv, s), "bf16 copies");
    BZ_HIP(hipStreamSynchronize(s), "bz_mlp_set_params sync");
    return BZ_OK;
}

bz_status bz_mlp_get_params(bz_mlp n, const void *d_params, float *master, void *stream) {
    if (!n || !d_params || !master) return fail(BZ_EINVAL, "bz_mlp_get_params: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BZ_HIP(hipMemcpyAsync(master, d_params, n->n_params * 4, hipMemcpyDeviceToHost, s), "download weights");
    BZ_HIP(hipStreamSynchronize(s), "bz_mlp_get_params sync");
    return BZ_OK;
}

bz_status bz_mlp_forward(bz_mlp n, const void *d_params, const uint16_t *d_x, int batch, float *d_y, void *d_work,
                         size_t work_bytes_, void *stream) {
    if (!n || !d_params || !d_x || !d_y || !d_work) return fail(BZ_EINVAL, "bz_mlp_forward: NULL argument");
    if (batch < 1) return fail(BZ_EINVAL, "bz_mlp_forward: batch must be >= 1");
    if (work_bytes_ < work_bytes(n, batch)) return fail(BZ_EINVAL, "bz_mlp_forward: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    ParamView pv = param_view(n, (void *)d_params);
    WorkView wv = work_view(n, batch, d_work);
    BZ_HIP(forward(n, pv, (const unsigned short *)d_x, batch, wv, d_y, s), "bz_mlp_forward");
    return BZ_OK;
}

bz_status bz_mlp_backward(bz_mlp n, const void *d_params, const uint16_t *d_x, const float *d_target, int batch,
                          float *d_grad, float *d_loss, void *d_work, size_t work_bytes_, void *stream) {
    if (!n || !d_params || !d_x || !d_target || !d_grad || !d_work)
        return fail(BZ_EINVAL, "bz_mlp_backward: NULL argument");
    if (batch < 32 || batch % 32) return fail(BZ_EINVAL, "bz_mlp_backward: batch must be a multiple of 32");
    if (work_bytes_ < work_bytes(n, batch)) return fail(BZ_EINVAL, "bz_mlp_backward: workspace too small");
    hipStream_t s = (hipStream_t)stream;
    ParamView pv = param_view(n, (void *)d_params);
    WorkView wv = work_view(n, batch, d_work);
    const unsigned short *X = (const unsigned short *)d_x;
    BZ_HIP(forward(n, pv, X, batch, wv, wv.Y, s), "bz_mlp_backward: forward");
    BZ_HIP(backward(n, pv, X, d_target, batch, wv, d_grad, s), "bz_mlp_backward");
    if (d_loss) BZ_HIP(hipMemcpyAsync(d_loss, wv.loss, 4, hipMemcpyDeviceToDevice, s), "copy loss");
    return BZ_OK;
}

bz_status bz_mlp_adam(bz_mlp n, void *d_params, const float *d_grad, int step, float lr, void *stream) {
    if (!n || !d_params || !d_grad) return fail(BZ_EINVAL, "bz_mlp_adam: NULL argument");
    if (step < 1 || !(lr >= 0)) return fail(BZ_EINVAL, "bz_mlp_adam: step >= 1 and lr >= 0 required");
    hipStream_t s = (hipStream_t)stream;
    ParamView pv = param_view(n, d_params);
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f / (1.0f - std::pow(b1, (float)step)), c2 = 1.0f / (1.0f - std::pow(b2, (float)step));
    const size_t H = n->n_hid, O = n->n_out, I = n->n_in;
    const Bf16Copies bc{{n->oW1, n->oW2, n->oW3}, {H * I, H * H, O * H}, {pv.W1, pv.W2, pv.W3}};
    const bool al = ((uintptr_t)d_grad | (uintptr_t)d_params) % 16 == 0;
    const size_t n4 = al ? n->n_params / 4 : 0;
    hipLaunchKernelGGL(k_adam, dim3(grid1(al ? n4 : n->n_params)), dim3(256), 0, s, n->n_params, n4, pv.master, pv.m,
                       pv.v, d_grad, lr, b1, b2, 1e-8f, c1, c2, bc);
    BZ_HIP(hipGetLastError(), "bz_mlp_adam");
    BZ_HIP(refresh_transposes(n, pv, s), "bz_mlp_adam: transposed bf16 copies");
    return BZ_OK;
}

}  // extern "C"
