// 1-D-in-space transport (Sec. 3.4, eq. upwind) with a diffuse Maxwell wall
// (Sec. 2.1, eq. BC) and far-field ghost cells, advanced with Heun's RK2, and
// the Strang-split step T(dt/2) C(dt) T(dt/2) of Sec. 3.1.
//
// Layout: f[j][k], cell j = 0..nx-1 along x, of width dx_j (Sec. 3.4: cells
// "not necessarily uniform"), k the flat velocity index of the cell's N^3 mesh;
// v1 = dv (k1 - N/2) is the transport velocity.
// Fluxes at face j-1/2:  v1 (f_{j-1} + dx_{j-1}/2 s_{j-1})  if v1 >= 0,
//                        v1 (f_j     - dx_j/2 s_j)          otherwise,
// s_j = minmod((f_j - f_{j-1})/d_{j-1/2}, (f_{j+1} - f_j)/d_{j+1/2}) with the
// centre distances d_{j+1/2} = (dx_j + dx_{j+1})/2, and the update divides by
// dx_j (on a uniform mesh, the printed formula).  Left end: two ghost cells of
// width dx_0 copy cell 0 (slope 0 there); the wall face flux is v1 sigma_w M_w for
// v1 > 0 and v1 f_0 for v1 < 0 with sigma_w = sum_{v1<0}|v1| f_0 / sum_{v1>0} v1 M_w,
// so the net wall mass flux is zero.  Right end: ghosts of width dx_{nx-1} hold M_far.
// Memory-bound (a window of 12 stencil reads per 8 cells of one velocity, the base term and
// one write of 8 bytes per (cell, velocity)); small next to the collision step.
#include <cmath>
#include <new>
#include <vector>

#include "bz_internal.h"

struct bz_transport_s {
    int N = 0, nx = 0;
    double L = 0, T_wall = 0, in_norm = 0;
    double *d_tab = nullptr;  // [2][N^3]: M_wall, M_far; then the nx cell widths
    const double *d_dx = nullptr;
};

namespace bz {
namespace {

__device__ inline double minmod(double a, double b) {
    return a * b > 0.0 ? (a > 0.0 ? fmin(a, b) : fmax(a, b)) : 0.0;
}

// sigma_w = sum_{v1 < 0} |v1| f_0 dv^3 / in_norm, one block of 1024 threads over the half of the
// wall cell with v1 < 0, fixed reduction order.  N is a template parameter so that the loop has
// a fixed trip count and its loads are issued together
template <int N>
__global__ void __launch_bounds__(1024) k_wall_sigma(double dv, const double *__restrict__ f0, double in_norm,
                                                     double *__restrict__ sigma) {
    __shared__ double red[16];
    // v1 < 0 exactly on the first half of the cell (k1 < N/2)
    constexpr int H = N * N * N / 2;
    double s = 0.0;
#pragma unroll 4
    for (int k = threadIdx.x; k < H; k += 1024) {
        const double v1 = dv * (k / (N * N) - N / 2);
        s = fma(-v1, f0[k], s);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        sigma[0] = t * dv * dv * dv / in_norm;
    }
}

__device__ inline double cellv(const double *__restrict__ f, const double *__restrict__ mfar, int nx, int M, int j,
                               int k) {
    if (j < 0) return f[k];
    if (j >= nx) return mfar[k];
    return f[(size_t)j * M + k];
}

// width of cell j, ghosts taking the width of the cell they border
__device__ inline double cellw(const double *__restrict__ dx, int nx, int j) {
    return dx[j < 0 ? 0 : (j >= nx ? nx - 1 : j)];
}

// out = alpha * base + beta * (fin + dt * rhs(fin)) at every (cell, velocity).  Thread (b, k)
// takes velocity k of the cells kTrCells b .. kTrCells b + kTrCells - 1 with a window over the
// stencil, so each value of fin it needs is loaded once (kTrCells + 4 loads for kTrCells
// outputs instead of 5 per output); every output takes the same arithmetic as with a
// one-point stencil.  N is a template parameter so that the index splits are divisions by
// constants.
constexpr int kTrCells = 8;
template <int N>
__global__ void __launch_bounds__(256) k_transport_stage(int nx, double dv, const double *__restrict__ dx, double dt,
                                                         const double *__restrict__ fin,
                                                         const double *__restrict__ base, double alpha, double beta,
                                                         const double *__restrict__ tab,
                                                         const double *__restrict__ sigma, double *__restrict__ out) {
    constexpr int M = N * N * N;
    const size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    const int nb = (nx + kTrCells - 1) / kTrCells;
    if (idx >= (size_t)nb * M) return;
    const int jb = (int)(idx / M), k = (int)(idx - (size_t)jb * M), j0 = jb * kTrCells;
    const double *mwall = tab, *mfar = tab + M;
    const double v1 = dv * (k / (N * N) - N / 2);
    double fv[kTrCells + 4], wv[kTrCells + 4];   // cells j0 - 2 .. j0 + kTrCells + 1
#pragma unroll
    for (int t = 0; t < kTrCells + 4; ++t) {
        fv[t] = cellv(fin, mfar, nx, M, j0 - 2 + t, k);
        wv[t] = cellw(dx, nx, j0 - 2 + t);
    }
#pragma unroll
    for (int t = 0; t < kTrCells; ++t) {
        const int j = j0 + t;
        if (j >= nx) break;
        const double a = fv[t], b = fv[t + 1], c = fv[t + 2], d = fv[t + 3], e = fv[t + 4];
        const double wa = wv[t], wb = wv[t + 1], wc = wv[t + 2], wd = wv[t + 3], we = wv[t + 4];
        // centre distances
        const double dab = 0.5 * (wa + wb), dbc = 0.5 * (wb + wc), dcd = 0.5 * (wc + wd), dde = 0.5 * (wd + we);
        const double sb = minmod((b - a) / dab, (c - b) / dbc);
        const double sc = minmod((c - b) / dbc, (d - c) / dcd);
        const double sd = minmod((d - c) / dcd, (e - d) / dde);
        // face j-1/2
        double Fl;
        if (j == 0)
            Fl = v1 > 0.0 ? v1 * sigma[0] * mwall[k] : v1 * c;
        else
            Fl = v1 >= 0.0 ? v1 * (b + 0.5 * wb * sb) : v1 * (c - 0.5 * wc * sc);
        // face j+1/2
        const double Fr = v1 >= 0.0 ? v1 * (c + 0.5 * wc * sc) : v1 * (d - 0.5 * wd * sd);
        const double y = c + dt * (-(Fr - Fl) / wc);
        const size_t o = (size_t)j * M + k;
        out[o] = (alpha != 0.0 ? alpha * base[o] : 0.0) + beta * y;
    }
}

}  // namespace

template <int N>
static hipError_t transport_rk2_n(const bz_transport_s *t, double *f, double dt, double *fs, double *sigma,
                                  hipStream_t s) {
    constexpr int M = N * N * N;
    const double dv = 2.0 * t->L / N;
    const size_t n = (size_t)((t->nx + kTrCells - 1) / kTrCells) * M;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_wall_sigma<N>, dim3(1), dim3(1024), 0, s, dv, f, t->in_norm, sigma);
    hipLaunchKernelGGL(k_transport_stage<N>, dim3(blocks), dim3(256), 0, s, t->nx, dv, t->d_dx, dt, f, f, 0.0, 1.0,
                       t->d_tab, sigma, fs);
    hipLaunchKernelGGL(k_wall_sigma<N>, dim3(1), dim3(1024), 0, s, dv, fs, t->in_norm, sigma);
    // a thread reads f only at the indices it writes (the base term), so f may be the output
    hipLaunchKernelGGL(k_transport_stage<N>, dim3(blocks), dim3(256), 0, s, t->nx, dv, t->d_dx, dt, fs, f, 0.5, 0.5,
                       t->d_tab, sigma, f);
    return hipGetLastError();
}

static hipError_t transport_rk2(const bz_transport_s *t, double *f, double dt, double *fs, double *sigma,
                                hipStream_t s) {
    switch (t->N) {
    case 8: return transport_rk2_n<8>(t, f, dt, fs, sigma, s);
    case 12: return transport_rk2_n<12>(t, f, dt, fs, sigma, s);
    case 16: return transport_rk2_n<16>(t, f, dt, fs, sigma, s);
    case 20: return transport_rk2_n<20>(t, f, dt, fs, sigma, s);
    case 24: return transport_rk2_n<24>(t, f, dt, fs, sigma, s);
    case 28: return transport_rk2_n<28>(t, f, dt, fs, sigma, s);
    case 32: return transport_rk2_n<32>(t, f, dt, fs, sigma, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace bz

using namespace bz;

extern "C" {

bz_status bz_transport_create(bz_grid g, int nx, double x_length, double T_wall, double far_rho, double far_u1,
                              double far_T, bz_transport *out) {
    if (!out) return fail(BZ_EINVAL, "bz_transport_create: out is NULL");
    *out = nullptr;
    if (nx < 1) return fail(BZ_EINVAL, "bz_transport_create: nx must be >= 1");
    if (!(x_length > 0) || !std::isfinite(x_length)) return fail(BZ_EINVAL, "bz_transport_create: bad length");
    std::vector<double> w((size_t)nx, x_length / nx);
    return bz_transport_create_ex(g, nx, w.data(), T_wall, far_rho, far_u1, far_T, out);
}

bz_status bz_transport_create_ex(bz_grid g, int nx, const double *dx, double T_wall, double far_rho, double far_u1,
                                 double far_T, bz_transport *out) {
    if (!out) return fail(BZ_EINVAL, "bz_transport_create: out is NULL");
    *out = nullptr;
    if (!g || !dx) return fail(BZ_EINVAL, "bz_transport_create: NULL grid or widths");
    if (nx < 1) return fail(BZ_EINVAL, "bz_transport_create: nx must be >= 1");
    for (int j = 0; j < nx; ++j)
        if (!(dx[j] > 0) || !std::isfinite(dx[j])) return fail(BZ_EINVAL, "bz_transport_create: bad cell width");
    if (!(T_wall > 0) || !(far_T > 0) || !(far_rho >= 0) || !std::isfinite(far_u1))
        return fail(BZ_EINVAL, "bz_transport_create: bad wall or far-field state");
    bz_transport_s *t = new (std::nothrow) bz_transport_s();
    if (!t) return fail(BZ_ENOMEM, "bz_transport_create: allocation failed");
    const int N = g->N, M = N * N * N;
    t->N = N;
    t->L = g->L;
    t->nx = nx;
    t->T_wall = T_wall;
    std::vector<double> tab(2 * (size_t)M + nx);
    for (int j = 0; j < nx; ++j) tab[2 * (size_t)M + j] = dx[j];
    const double dv = g->dv;
    double in_norm = 0.0;
    for (int k = 0; k < M; ++k) {
        const double v1 = dv * (k / (N * N) - N / 2), v2 = dv * ((k / N) % N - N / 2), v3 = dv * (k % N - N / 2);
        const double r2 = v1 * v1 + v2 * v2 + v3 * v3;
        tab[k] = std::pow(2.0 * M_PI * T_wall, -1.5) * std::exp(-r2 / (2.0 * T_wall));
        const double q2 = (v1 - far_u1) * (v1 - far_u1) + v2 * v2 + v3 * v3;
        tab[M + k] = far_rho * std::pow(2.0 * M_PI * far_T, -1.5) * std::exp(-q2 / (2.0 * far_T));
        if (v1 > 0.0) in_norm += v1 * tab[k];
    }
    t->in_norm = in_norm * dv * dv * dv;
    hipError_t e = hipMalloc(&t->d_tab, tab.size() * sizeof(double));
    if (e == hipSuccess) e = hipMemcpy(t->d_tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice);
    t->d_dx = t->d_tab + 2 * (size_t)M;
    if (e != hipSuccess) {
        if (t->d_tab) (void)hipFree(t->d_tab);
        delete t;
        return hip_fail(e, "bz_transport_create: upload wall and far-field tables");
    }
    *out = t;
    return BZ_OK;
}

void bz_transport_free(bz_transport t) {
    if (!t) return;
    if (t->d_tab) (void)hipFree(t->d_tab);
    delete t;
}

size_t bz_transport_workspace_bytes(bz_transport t) {
    if (!t) return 0;
    return ((size_t)t->nx * t->N * t->N * t->N * 8 + 255) / 256 * 256 + 256;
}

bz_status bz_transport_step(bz_transport t, double *d_f, double dt, void *d_work, size_t work_bytes, void *stream) {
    if (!t || !d_f || !d_work) return fail(BZ_EINVAL, "bz_transport_step: NULL argument");
    if (work_bytes < bz_transport_workspace_bytes(t)) return fail(BZ_EINVAL, "bz_transport_step: workspace too small");
    if (!std::isfinite(dt)) return fail(BZ_EINVAL, "bz_transport_step: dt must be finite");
    const size_t arr = ((size_t)t->nx * t->N * t->N * t->N * 8 + 255) / 256 * 256;
    double *fs = (double *)d_work;
    double *sigma = (double *)((char *)d_work + arr);
    hipError_t e = transport_rk2(t, d_f, dt, fs, sigma, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "bz_transport_step");
    return BZ_OK;
}

size_t bz_strang_workspace_bytes(bz_batch b, bz_transport t) {
    if (!b || !t) return 0;
    return (bz_step_workspace_bytes(b) + 255) / 256 * 256 + bz_transport_workspace_bytes(t);
}

bz_status bz_strang_step(bz_batch b, bz_transport t, double *d_f, double dt, double eps, void *d_work,
                         size_t work_bytes, void *stream) {
    if (!b || !t || !d_f || !d_work) return fail(BZ_EINVAL, "bz_strang_step: NULL argument");
    if (!(eps > 0) || !std::isfinite(dt)) return fail(BZ_EINVAL, "bz_strang_step: need finite dt and eps > 0");
    if (work_bytes < bz_strang_workspace_bytes(b, t)) return fail(BZ_EINVAL, "bz_strang_step: workspace too small");
    if (bz_batch_elems(b) != (size_t)t->nx * t->N * t->N * t->N)
        return fail(BZ_EINVAL, "bz_strang_step: the batch must hold the nx cells of the transport mesh");
    // the transport scratch follows the collision-step workspace (whose flag word must survive)
    const size_t a = (bz_step_workspace_bytes(b) + 255) / 256 * 256;
    char *tw = (char *)d_work + a;
    bz_status st = bz_transport_step(t, d_f, 0.5 * dt, tw, work_bytes - a, stream);
    if (st != BZ_OK) return st;
    if ((st = bz_step(b, d_f, dt / eps, d_work, a, stream)) != BZ_OK) return st;
    return bz_transport_step(t, d_f, 0.5 * dt, tw, work_bytes - a, stream);
}

bz_status bz_closure_strang_step(bz_batch b, bz_transport t, const bz_closure *c, double *d_f, double dt,
                                 double eps, void *d_work, size_t work_bytes, void *stream) {
    if (!b || !t || !c || !d_f || !d_work) return fail(BZ_EINVAL, "bz_closure_strang_step: NULL argument");
    if (!(eps > 0) || !std::isfinite(dt)) return fail(BZ_EINVAL, "bz_closure_strang_step: need finite dt and eps > 0");
    const size_t a = (bz_closure_workspace_bytes(b, c) + 255) / 256 * 256;
    if (a == 0) return fail(BZ_EINVAL, "bz_closure_strang_step: bad closure description");
    if (work_bytes < a + bz_transport_workspace_bytes(t))
        return fail(BZ_EINVAL, "bz_closure_strang_step: workspace too small");
    if (bz_batch_elems(b) != (size_t)t->nx * t->N * t->N * t->N)
        return fail(BZ_EINVAL, "bz_closure_strang_step: the batch must hold the nx cells of the transport mesh");
    char *tw = (char *)d_work + a;
    bz_status st = bz_transport_step(t, d_f, 0.5 * dt, tw, work_bytes - a, stream);
    if (st != BZ_OK) return st;
    if ((st = bz_closure_step(b, c, d_f, dt / eps, d_work, a, stream)) != BZ_OK) return st;
    return bz_transport_step(t, d_f, 0.5 * dt, tw, work_bytes - a, stream);
}

// ---------------------------------------------------------------------------
// HIP graphs of one step.
// ---------------------------------------------------------------------------
}  // extern "C"

struct bz_graph_s {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

template <typename F>
static bz_status capture(void *stream, F &&enqueue, bz_graph *out) {
    if (!out) return fail(BZ_EINVAL, "bz_graph_capture: out is NULL");
    *out = nullptr;
    if (!stream) return fail(BZ_EINVAL, "bz_graph_capture: cannot capture the NULL stream");
    hipStream_t s = (hipStream_t)stream;
    BZ_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed), "bz_graph_capture: begin");
    bz_status st = enqueue();
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(s, &g);
    if (st != BZ_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return hip_fail(e, "bz_graph_capture: end");
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return hip_fail(e, "bz_graph_capture: instantiate");
    }
    bz_graph_s *h = new (std::nothrow) bz_graph_s();
    if (!h) {
        (void)hipGraphExecDestroy(x);
        (void)hipGraphDestroy(g);
        return fail(BZ_ENOMEM, "bz_graph_capture: allocation failed");
    }
    h->graph = g;
    h->exec = x;
    *out = h;
    return BZ_OK;
}

extern "C" {

bz_status bz_graph_capture_step(bz_batch b, double *d_f, double dt_over_eps, void *d_work, size_t work_bytes,
                                void *stream, bz_graph *out) {
    return capture(stream, [&]() { return bz_step(b, d_f, dt_over_eps, d_work, work_bytes, stream); }, out);
}

bz_status bz_graph_capture_strang(bz_batch b, bz_transport t, double *d_f, double dt, double eps, void *d_work,
                                  size_t work_bytes, void *stream, bz_graph *out) {
    return capture(stream, [&]() { return bz_strang_step(b, t, d_f, dt, eps, d_work, work_bytes, stream); }, out);
}

bz_status bz_graph_launch(bz_graph g, void *stream) {
    if (!g) return fail(BZ_EINVAL, "bz_graph_launch: NULL graph");
    BZ_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream), "bz_graph_launch");
    return BZ_OK;
}

void bz_graph_free(bz_graph g) {
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

}  // extern "C"
