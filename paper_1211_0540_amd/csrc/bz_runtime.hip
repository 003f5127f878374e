// Host runtime of libbz: mesh handles, the universal weight table, batch
// planning (groups of 64 cells, longest-first work lists) and the C ABI
// declared in include/bz.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <thread>

#include "bz_internal.h"

namespace bz {

static thread_local std::string g_err;

bz_status fail(bz_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

bz_status hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipErrorOutOfMemory ? BZ_ENOMEM : BZ_EDEVICE;
}

constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------------------
// Universal table (Sec. 2.2 eq. GHat_calc with r = L s and dzeta L = pi):
//   T_lambda(p, q) = int_0^1 s^{lambda+2} sinc(a s) sinc(b s) ds,
//   a = pi sqrt(p) / 2, b = pi sqrt(q) / 2,
// in closed form for lambda = 0, 1:
//   lambda = 0:  [S(a-b) - S(a+b)] / (2ab),          S(x) = sin x / x
//   lambda = 1:  [U(a-b) - U(a+b)] / (2ab),          U(x) = int_0^1 s cos(xs) ds
//                                                         = sin x/x - 2 sin^2(x/2)/x^2
// with the one-sided limits for a or b = 0.  Non-zero a, b are >= pi/2 and a
// non-zero |a - b| is >= pi/(4 sqrt(3) N), so no series expansions are needed;
// the half-angle form of cos x - 1 removes the only cancellation.
// ---------------------------------------------------------------------------
static double S0(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }
static double U1(double x) {
    if (x == 0.0) return 0.5;
    const double hs = std::sin(0.5 * x);
    return std::sin(x) / x - 2.0 * hs * hs / (x * x);
}

static double T_closed(int lam, double a, double b) {
    if (a == 0.0 && b == 0.0) return 1.0 / (lam + 3);
    if (a == 0.0 || b == 0.0) {
        const double c = a + b, sc = std::sin(c), cc = std::cos(c), hs = std::sin(0.5 * c);
        if (lam == 0) return (sc - c * cc) / (c * c * c);
        // int_0^1 s^2 sin(c s) ds / c
        return (-cc / c + 2.0 * sc / (c * c) - 4.0 * hs * hs / (c * c * c)) / c;
    }
    if (lam == 0) return (S0(a - b) - S0(a + b)) / (2.0 * a * b);
    return (U1(a - b) - U1(a + b)) / (2.0 * a * b);
}

// ---------------------------------------------------------------------------
// Other lambda > -3 (the text after eq. GHat_calc: a one-dimensional integral
// evaluated by quadrature).  T_lambda(p, q) = int_0^1 s^alpha g(s) ds with
// alpha = lambda + 2 > -1 and g(s) = sinc(a s) sinc(b s) entire, g(0) = 1:
//   [0, s_K]            g = 1 to O(s_K^2):  s_K^{alpha+1} / (alpha+1)
//   [s_{k+1}, s_k]      geometric panels s_k = sigma^k / P (k < K), which
//                       resolve the endpoint behaviour of s^alpha
//   [i/P, (i+1)/P]      P - 1 uniform panels (i >= 1) for the oscillation
// each panel with an m-point Gauss-Legendre rule.  On a graded panel the
// singular point s = 0 lies sigma / (1 - sigma) panel widths away, which bounds
// the rule's convergence factor; sigma = 0.3 gives about 1e-17 per panel with
// m = 16.  With K = 40 and P = 16 the rule is exact to rounding for the
// |a| + |b| <= 130 of the meshes here (checked against arbitrary-precision
// quadrature).
// ---------------------------------------------------------------------------
// Gauss-Legendre nodes and weights on [-1, 1]: Newton's method on P_n, evaluated
// by its three-term recurrence, from the Chebyshev-like first guesses.
static void gauss_legendre_rule(int n, std::vector<double> &x, std::vector<double> &w) {
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

// nodes s_i in (0, 1], weights W_i holding s_i^alpha, and the head term of [0, s_K]
static void radial_rule(double alpha, std::vector<double> &s, std::vector<double> &W, double &head) {
    constexpr int m = 16, P = 16, K = 40;
    constexpr double sigma = 0.3;
    std::vector<double> gx, gw;
    gauss_legendre_rule(m, gx, gw);
    s.clear();
    W.clear();
    auto panel = [&](double a, double b) {
        for (int i = 0; i < m; ++i) {
            const double t = 0.5 * (a + b) + 0.5 * (b - a) * gx[i];
            s.push_back(t);
            W.push_back(0.5 * (b - a) * gw[i] * std::pow(t, alpha));
        }
    };
    double hi = 1.0 / P;
    for (int k = 0; k < K; ++k) {
        panel(hi * sigma, hi);
        hi *= sigma;
    }
    head = std::pow(hi, alpha + 1.0) / (alpha + 1.0);
    for (int i = 1; i < P; ++i) panel((double)i / P, (double)(i + 1) / P);
}

static double sinc_of(double x) { return x == 0.0 ? 1.0 : std::sin(x) / x; }

// p in [0, 3N^2/4], q in [0, 3N^2] (q = 4 nc reaches 3N^2 on the loss row).
static void build_table(int N, double lam, std::vector<double> &T, int &qs) {
    const int pmax = 3 * N * N / 4, qmax = 3 * N * N;
    qs = qmax + 1;
    T.assign((size_t)(pmax + 1) * qs, 0.0);
    std::vector<double> sq(qs);
    for (int q = 0; q < qs; ++q) sq[q] = 0.5 * kPi * std::sqrt((double)q);
    if (lam == 0.0 || lam == 1.0) {
        for (int p = 0; p <= pmax; ++p) {
            const double a = sq[p];
            double *row = T.data() + (size_t)p * qs;
            for (int q = 0; q < qs; ++q) row[q] = T_closed((int)lam, a, sq[q]);
        }
        return;
    }
    std::vector<double> s, W;
    double head = 0.0;
    radial_rule(lam + 2.0, s, W, head);
    const size_t n = s.size();
    // S[q][i] = sinc(sq[q] s_i); T[p][q] = head + sum_i W_i S[p][i] S[q][i]
    std::vector<double> S((size_t)qs * n);
    for (int q = 0; q < qs; ++q)
        for (size_t i = 0; i < n; ++i) S[(size_t)q * n + i] = sinc_of(sq[q] * s[i]);
    const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (unsigned t = 0; t < nt; ++t)
        pool.emplace_back([&, t]() {
            std::vector<double> aw(n);
            for (int p = (int)t; p <= pmax; p += (int)nt) {
                for (size_t i = 0; i < n; ++i) aw[i] = W[i] * S[(size_t)p * n + i];
                double *row = T.data() + (size_t)p * qs;
                for (int q = 0; q < qs; ++q) {
                    const double *b = S.data() + (size_t)q * n;
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                    size_t i = 0;
                    for (; i + 4 <= n; i += 4) {
                        a0 += aw[i] * b[i];
                        a1 += aw[i + 1] * b[i + 1];
                        a2 += aw[i + 2] * b[i + 2];
                        a3 += aw[i + 3] * b[i + 3];
                    }
                    for (; i < n; ++i) a0 += aw[i] * b[i];
                    row[q] = head + ((a0 + a1) + (a2 + a3));
                }
            }
        });
    for (auto &th : pool) th.join();
}

static double weight_scale(const bz_grid_s *g) {
    // 4pi (2pi)^{-3/2} L^{lambda+3} dzeta^3
    return 4.0 * kPi * std::pow(2.0 * kPi, -1.5) * std::pow(g->L, g->lambda + 3.0) * g->dzeta * g->dzeta * g->dzeta;
}

// Cholesky of the Gram matrix C C^T of the constraint rows dv^3 {1, v1, v2, v3, |v|^2}.
static bool constraint_linv(int N, double dv, double linv[25]) {
    std::vector<double> v(N);
    for (int k = 0; k < N; ++k) v[k] = dv * (k - N / 2);
    double s[5] = {0, 0, 0, 0, 0};  // 1-D power sums sum_k v^p, p = 0..4
    for (int k = 0; k < N; ++k) {
        double t = 1.0;
        for (int p = 0; p < 5; ++p) {
            s[p] += t;
            t *= v[k];
        }
    }
    const double w2 = std::pow(dv, 6);
    // moments of the 3-D mesh via separability
    auto m = [&](int a, int b, int c) { return s[a] * s[b] * s[c]; };
    double G[5][5];
    const int e[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            G[i][j] = m(e[i][0] + e[j][0], e[i][1] + e[j][1], e[i][2] + e[j][2]);
    for (int i = 0; i < 4; ++i) {
        double t = 0;
        for (int d = 0; d < 3; ++d) {
            int x[3] = {e[i][0], e[i][1], e[i][2]};
            x[d] += 2;
            t += m(x[0], x[1], x[2]);
        }
        G[i][4] = G[4][i] = t;
    }
    {
        double t = 0;
        for (int d1 = 0; d1 < 3; ++d1)
            for (int d2 = 0; d2 < 3; ++d2) {
                int x[3] = {0, 0, 0};
                x[d1] += 2;
                x[d2] += 2;
                t += m(x[0], x[1], x[2]);
            }
        G[4][4] = t;
    }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) G[i][j] *= w2;
    double Lc[5][5] = {{0}};
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j <= i; ++j) {
            double t = G[i][j];
            for (int k = 0; k < j; ++k) t -= Lc[i][k] * Lc[j][k];
            if (i == j) {
                if (!(t > 0)) return false;
                Lc[i][i] = std::sqrt(t);
            } else {
                Lc[i][j] = t / Lc[j][j];
            }
        }
    // invert the lower-triangular factor
    double Li[5][5] = {{0}};
    for (int j = 0; j < 5; ++j) {
        Li[j][j] = 1.0 / Lc[j][j];
        for (int i = j + 1; i < 5; ++i) {
            double t = 0;
            for (int k = j; k < i; ++k) t -= Lc[i][k] * Li[k][j];
            Li[i][j] = t / Lc[i][i];
        }
    }
    for (int i = 0; i < 5; ++i)
        for (int j = 0; j < 5; ++j) linv[i * 5 + j] = Li[i][j];
    return true;
}

static void build_schedules(bz_grid_s *g) {
    const int N = g->N;
    Schedule &s = g->sched;
    s.row_woff.resize(N * N);
    s.row_steps.resize(N * N);
    long long off = 0;
    for (int r = 0; r < N * N; ++r) {
        s.row_woff[r] = off;
        s.row_steps[r] = cells_steps(N, r / N, r % N);
        off += (long long)s.row_steps[r] * pairs_per_step(N);
    }
    s.cells_weights = off;
    // pass E3 of the conjugate-symmetric schedule: the m1 = 0 block of rows (a < N/2, b)
    s.e3_woff.assign(N * N, 0);
    off = 0;
    for (int r = 0; r < N / 2 * N; ++r) {
        s.e3_woff[r] = off;
        off += (long long)axis_cnt(N, r % N) * pairs_per_step(N);
    }
    s.e3_weights = off;
    const int R = plain_rows(N), NB = N / R, LN = R * N;
    s.blk_woff.resize(N * NB);
    off = 0;
    for (int b = 0; b < N * NB; ++b) {
        s.blk_woff[b] = off;
        off += plain_block_iters(N, b / NB, b % NB) * LN;
    }
    s.plain_weights = off;
}

// Core items of the one-launch queue are spread over the first 3/5 of its FP32 items.
constexpr size_t kCoreSpreadNum = 3, kCoreSpreadDen = 5;

// Low-frequency core (CoreSched): the disk rows, and for every output row its
// core steps, pairs of disk rows (m1, m2) <= (j1, j2) with j = k + N/2 - m.
static void build_core(bz_grid_s *g, int r2) {
    bz::CoreSched &c = g->sched.core;
    c = bz::CoreSched();
    if (r2 < 1) return;
    const int N = g->N, h = N / 2;
    c.r2 = r2;
    while ((c.r + 1) * (c.r + 1) <= r2) ++c.r;
    c.disk_idx.assign(N * N, -1);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            if ((a - h) * (a - h) + (b - h) * (b - h) <= r2) {
                c.disk_idx[a * N + b] = c.nD++;
                int e = 0;
                while ((e + 1) * (e + 1) <= r2 - (a - h) * (a - h) - (b - h) * (b - h)) ++e;
                c.disk_ext.push_back(e);
            }
    c.row_steps.assign(N * N, 0);
    c.row_soff.assign(N * N, 0);
    for (int k1 = 0; k1 < N; ++k1)
        for (int k2 = 0; k2 < N; ++k2) {
            const int row = k1 * N + k2;
            c.row_soff[row] = (long long)c.steps.size();
            for (int m1 = 0; m1 < N; ++m1)
                for (int m2 = 0; m2 < N; ++m2) {
                    const int dm = c.disk_idx[m1 * N + m2];
                    const int j1 = k1 + h - m1, j2 = k2 + h - m2;
                    if (dm < 0 || j1 < 0 || j1 >= N || j2 < 0 || j2 >= N) continue;
                    const int dj = c.disk_idx[j1 * N + j2];
                    if (dj < 0 || m1 > j1 || (m1 == j1 && m2 > j2)) continue;
                    c.steps.push_back(dm | (dj << 16));
                }
            c.row_steps[row] = (int)((long long)c.steps.size() - c.row_soff[row]);
        }
    c.nsteps = (long long)c.steps.size();
}

static size_t kind_elem(int kind) {
    return (kind == BZ_W_BATCHED_F64 || kind == BZ_W_PLAIN_F64) ? 8 : 4;
}
static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }
// byte offset of the pass-E3 stream in a batched weight buffer (after the main stream and its pad)
static size_t e3_base_bytes(const bz_grid_s *g, size_t elem) {
    return align256((size_t)g->sched.cells_weights * elem + kWeightPadBytes);
}
// byte offset of the FP64 core stream in a batched FP32 weight buffer (after the E3 stream and its pad)
static size_t core_base_bytes(const bz_grid_s *g) {
    return align256(e3_base_bytes(g, 4) + (size_t)g->sched.e3_weights * 4 + kWeightPadBytes);
}
static size_t core_stream_bytes(const bz_grid_s *g) {
    const CoreSched &c = g->sched.core;
    return c.r2 < 1 ? 0 : (size_t)c.nsteps * core_wstride(c.r) * sizeof(double);
}

// Weights of the core steps in stream order (CoreSched), FP64, dzeta^3 folded in.
static void core_weights(const bz_grid_s *g, const std::vector<double> &T, int qs, double scale,
                         std::vector<double> &out) {
    const CoreSched &c = g->sched.core;
    const int N = g->N, h = N / 2, r = c.r, S = 2 * r + 1, WS = core_wstride(r);
    out.assign((size_t)c.nsteps * WS, 0.0);
    std::vector<int> da(c.nD), db(c.nD);
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b)
            if (c.disk_idx[a * N + b] >= 0) {
                da[c.disk_idx[a * N + b]] = a;
                db[c.disk_idx[a * N + b]] = b;
            }
    auto sq = [](int x, int y, int z) { return x * x + y * y + z * z; };
    for (int k1 = 0; k1 < N; ++k1)
        for (int k2 = 0; k2 < N; ++k2) {
            const int row = k1 * N + k2;
            for (long long st = c.row_soff[row]; st < c.row_soff[row] + c.row_steps[row]; ++st) {
                const int dm = c.steps[st] & 0xffff, dj = c.steps[st] >> 16;
                const int m1 = da[dm], m2 = db[dm], j1 = da[dj], j2 = db[dj];
                const bool diag = dm == dj;
                for (int tm = 0; tm < S; ++tm)
                    for (int tj = 0; tj < S; ++tj) {
                        const int m3 = h - r + tm, j3 = h - r + tj, k3 = m3 + j3 - h;
                        if (k3 < 0 || k3 >= N || (diag && tm > tj)) continue;
                        const int ncm = sq(m1 - h, m2 - h, m3 - h), ncj = sq(j1 - h, j2 - h, j3 - h);
                        if (ncm > c.r2 || ncj > c.r2) continue;
                        const int na = sq(k1 - h, k2 - h, k3 - h), nb = sq(m1 - j1, m2 - j2, m3 - j3);
                        double v;
                        if (g->beta != 1.0) {
                            const int lam = (int)g->lambda;
                            const double gm = gain_beta(lam, g->beta, h, k1, k2, k3, m1, m2, m3);
                            v = (diag && tm == tj) ? gm - T[4 * ncm]
                                                   : gm + gain_beta(lam, g->beta, h, k1, k2, k3, j1, j2, j3) -
                                                         T[4 * ncm] - T[4 * ncj];
                        } else {
                            v = (diag && tm == tj) ? T[(size_t)na * qs] - T[4 * ncm]
                                                   : 2.0 * T[(size_t)na * qs + nb] - T[4 * ncm] - T[4 * ncj];
                        }
                        out[(size_t)st * WS + tm * S + tj] = scale * v;
                    }
            }
        }
}

// ---------------------------------------------------------------------------
// Batch.
// ---------------------------------------------------------------------------
struct Part {
    bz_grid g = nullptr;
    int gi = 0;
    std::vector<int> cells;  // batch cell indices
    int groups = 0;
    const void *w = nullptr;
    int wkind = 0;
    // device tables (offsets into the batch's device buffer)
    long long *d_f_off = nullptr;    // per cell: offset of f (doubles)
    long long *d_fh_base = nullptr;  // per cell: base of fhat/qhat (complex units)
    long long *d_row_woff = nullptr;
    long long *d_blk_woff = nullptr;
    long long *d_zero = nullptr;     // single 0 (plain: base of the one cell)
    long long *d_e3_woff = nullptr;  // pass-E3 row offsets (conjugate-symmetric schedule)
    int4 *d_items = nullptr;
    int n_items = 0;
    bool herm = false;               // conjugate-symmetric (halved) batched schedule
    int parts = 1;                   // partial-sum buffers of pass A (and of pass Z) of the batched schedule
    int variant = 0;                 // convolution kernel variant
    std::vector<long long> f_off;    // host copy
    std::vector<int4> h_items;       // host copy of the work items
    std::vector<int4> h_core_items;  // host copy of the FP64 core items
    // FP64 low-frequency core (batched FP32 mode with a core on the mesh)
    bool core = false;
    int4 *d_core_items = nullptr;
    int n_core_items = 0;
    int core_parts = 1;              // step pieces per core row, each with its own partial sum
    int *d_core_steps = nullptr;
    int *d_disk_idx = nullptr;
    int *d_disk_ext = nullptr;
    // workspace offsets (bytes)
    size_t ws_fh = 0, ws_qh = 0, ws_counter = 0;
    size_t ws_cf = 0, ws_cq = 0, ws_ccounter = 0;
};

}  // namespace bz

struct bz_batch_s {
    int mode = 0;
    int n_cells = 0;
    std::vector<bz_grid> grids;
    std::vector<int> grid_of_cell;
    std::vector<long long> cell_off;
    size_t elems = 0;
    std::vector<bz::Part> parts;   // one per mesh used, largest N first
    void *d_tables = nullptr;
    // per cell, in batch order (device, inside d_tables): f offset, N, dv
    long long *d_cell_off = nullptr;
    int *d_cell_N = nullptr;
    double *d_cell_dv = nullptr;
    size_t ws_scratch = 0, ws_flag = 0, ws_total = 0;
    int plain_split = 4;
    // convolution timing
    bool timing = false;
    double core_ms = 0.0;            // FP64 core launches timed at the last bz_batch_timer_read
    int core_launches = 0;
    // batched FP32 mode with several meshes: one convolution launch for all of them (NULL: one per mesh)
    int4 *d_multi_items = nullptr;
    int n_multi_items = 0;
    bz::MeshConvDesc *d_desc = nullptr;   // per mesh, uploaded by bz_batch_set_weights
    size_t ws_mcounter = 0;
    bool per_mesh_now = false;       // one launch per mesh in place of the one-launch queue (autotuner)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_used, ev_free, ev_core_used;
    int closure_phase = 0;
    // closure: the network runs on a second stream of default priority, forked from and joined to
    // the caller's stream by events (created on the first closure call)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // FP64 cores of the per-mesh form: their own stream of default priority, forked from and
    // joined to the caller's stream around the FP32 convolution; persistent grid (wavefronts,
    // 0: the default)
    hipStream_t core_stream = nullptr;
    hipEvent_t ev_cfork = nullptr, ev_cjoin = nullptr;
    int core_waves = 0;
};

namespace bz {

static bool batched(int mode) { return mode == BZ_MODE_BATCHED_F32 || mode == BZ_MODE_BATCHED_F64; }
static bool mode_f64(int mode) { return mode == BZ_MODE_PLAIN_F64 || mode == BZ_MODE_BATCHED_F64; }
static int mode_wkind(int mode) {
    switch (mode) {
    case BZ_MODE_BATCHED_F32: return BZ_W_BATCHED_F32;
    case BZ_MODE_BATCHED_F64: return BZ_W_BATCHED_F64;
    case BZ_MODE_PLAIN_F32: return BZ_W_PLAIN_F32;
    default: return BZ_W_PLAIN_F64;
    }
}
static int plain_split_for(int N) {
    // enough partial sums to give >= ~2048 single-wave blocks, bounded by the m1 band
    const int nb = N * (N / plain_rows(N));
    int s = (2048 + nb - 1) / nb;
    const int cmin = N / 2;
    if (s > cmin) s = cmin;
    if (s < 1) s = 1;
    if (s > 8) s = 8;
    return s;
}

static bool timer_pair(bz_batch_s *b, std::pair<hipEvent_t, hipEvent_t> &ev, bool core = false) {
    if (b->ev_free.empty()) {
        hipEvent_t a, c;
        if (hipEventCreate(&a) != hipSuccess) return false;
        if (hipEventCreate(&c) != hipSuccess) {
            (void)hipEventDestroy(a);
            return false;
        }
        b->ev_free.emplace_back(a, c);
    }
    ev = b->ev_free.back();
    b->ev_free.pop_back();
    (core ? b->ev_core_used : b->ev_used).push_back(ev);
    return true;
}

// variant chosen per (N, groups, mode) by bz_batch_autotune in this process (or loaded by
// bz_tuning_load), guarded by g_tuned_mu
static std::vector<std::pair<long long, int>> g_tuned;
static std::mutex g_tuned_mu;
static long long tune_key(int N, int groups, int mode) { return ((long long)N << 40) | ((long long)groups << 8) | mode; }
static void remember_variant(long long key, int v) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    for (auto &kv : g_tuned)
        if (kv.first == key) {
            kv.second = v;
            return;
        }
    g_tuned.emplace_back(key, v);
}
static int recalled_variant(long long key, int fallback) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    for (auto &kv : g_tuned)
        if (kv.first == key) return kv.second;
    return fallback;
}

}  // namespace bz

using namespace bz;

extern "C" {

int bz_api_version(void) { return BZ_API_VERSION; }

const char *bz_status_string(bz_status s) {
    switch (s) {
    case BZ_OK: return "ok";
    case BZ_EINVAL: return "invalid argument";
    case BZ_EUNSUPPORTED: return "unsupported";
    case BZ_EDEVICE: return "device error";
    case BZ_ENOMEM: return "out of memory";
    case BZ_ENONFINITE: return "non-finite value";
    case BZ_ESTATE: return "invalid state";
    }
    return "unknown status";
}

const char *bz_status_str(bz_status s) { return bz_status_string(s); }

const char *bz_last_error(void) { return g_err.c_str(); }

bz_status bz_grid_init(int N, double L, double lambda, bz_grid *out) {
    return bz_grid_init_ex(N, L, lambda, BZ_CORE_DEFAULT, out);
}

bz_status bz_grid_init_ex(int N, double L, double lambda, int core_r2, bz_grid *out) {
    const bz_grid_params p{N, L, lambda, core_r2, 1.0};
    return bz_grid_create(&p, out);
}

bz_status bz_grid_create(const bz_grid_params *prm, bz_grid *out) {
    if (!out) return fail(BZ_EINVAL, "bz_grid_init: out is NULL");
    if (!prm) return fail(BZ_EINVAL, "bz_grid_init: NULL parameters");
    const int N = prm->N, core_r2 = prm->core_r2;
    const double L = prm->L, lambda = prm->lambda, beta = prm->beta;
    *out = nullptr;
    if (N < kMinN || N > kMaxN || (N % 4) != 0)
        return fail(BZ_EINVAL, "bz_grid_init: N must be a multiple of 4 in [8, 32]");
    if (!(L > 0) || !std::isfinite(L)) return fail(BZ_EINVAL, "bz_grid_init: L must be positive and finite");
    if (!(lambda > -3.0 && lambda <= 1.0))
        return fail(BZ_EUNSUPPORTED, "bz_grid_init: lambda must lie in (-3, 1]");
    if (!(beta >= 0.5 && beta <= 1.0))
        return fail(BZ_EINVAL, "bz_grid_init: beta must lie in [1/2, 1] (restitution 2 beta - 1 in [0, 1])");
    if (beta != 1.0 && !(lambda == 0.0 || lambda == 1.0))
        return fail(BZ_EUNSUPPORTED, "bz_grid_init: inelastic collisions need lambda = 0 or 1");
    bz_grid_s *g = new (std::nothrow) bz_grid_s();
    if (!g) return fail(BZ_ENOMEM, "bz_grid_init: allocation failed");
    g->N = N;
    g->L = L;
    g->lambda = lambda;
    g->beta = beta;
    g->dv = 2.0 * L / N;
    g->dzeta = kPi / L;
    const long long a = 3LL * N * N / 4;
    g->pairs = a * a * a;
    if (!constraint_linv(N, g->dv, g->linv)) {
        delete g;
        return fail(BZ_EINVAL, "bz_grid_init: constraint Gram matrix not positive definite");
    }
    // inelastic collisions do not preserve energy (Sec. 3.3): the leading 4 x 4 block of the
    // Cholesky factor is that of the mass and momentum rows alone, so zeroing the energy row of
    // L^{-1} leaves the projection onto those four constraints
    if (beta != 1.0)
        for (int j = 0; j < 5; ++j) g->linv[4 * 5 + j] = 0.0;
    build_schedules(g);
    // core ball: the default is |zeta| < pi sqrt(min(1, N/32)), i.e. nc < L^2 sqrt(N/32) in index
    // units, kept inside the interior of the mesh (r <= N/2 - 1) and within the kernel's largest
    // half-width.  A coarser mesh sums fewer FP32 terms per output, so a smaller ball leaves the
    // same error: an emulation of the kernel's FP32 arithmetic on the cells of largest
    // cancellation gives at most 3.7e-6, 5.0e-6 and 4.3e-6 at N = 16, 24, 32 (L = 6, 7, 8)
    const int h = N / 2, cmax = std::min(h * h - 1, (kCoreMaxR + 1) * (kCoreMaxR + 1) - 1);
    int r2 = core_r2;
    if (core_r2 == BZ_CORE_DEFAULT)
        r2 = std::min(cmax, (int)std::ceil(L * L * std::sqrt(std::min(1.0, N / 32.0))) - 1);
    else if (core_r2 != BZ_CORE_OFF && (core_r2 < 1 || core_r2 > cmax)) {
        delete g;
        return fail(BZ_EINVAL, "bz_grid_init: core_r2 must be in [1, min(N^2/4, 81) - 1], BZ_CORE_DEFAULT or BZ_CORE_OFF");
    }
    build_core(g, core_r2 == BZ_CORE_OFF ? 0 : r2);
    *out = g;
    return BZ_OK;
}

void bz_grid_free(bz_grid g) { delete g; }

bz_status bz_grid_query(bz_grid g, bz_grid_info *info) {
    if (!g || !info) return fail(BZ_EINVAL, "bz_grid_query: NULL argument");
    info->N = g->N;
    info->L = g->L;
    info->lambda = g->lambda;
    info->dv = g->dv;
    info->dzeta = g->dzeta;
    info->pairs = g->pairs;
    info->core_r2 = g->sched.core.r2 < 1 ? 0 : g->sched.core.r2;
    info->beta = g->beta;
    info->core_steps = g->sched.core.nsteps;
    return BZ_OK;
}

bz_status bz_grid_coords(bz_grid g, double *v, double *zeta) {
    if (!g) return fail(BZ_EINVAL, "bz_grid_coords: NULL grid");
    for (int k = 0; k < g->N; ++k) {
        if (v) v[k] = g->dv * (k - g->N / 2);
        if (zeta) zeta[k] = g->dzeta * (k - g->N / 2);
    }
    return BZ_OK;
}

size_t bz_weight_table_size(int N) {
    if (N < kMinN || N > kMaxN || (N % 4) != 0) return 0;
    return (size_t)(3 * N * N / 4 + 1) * (3 * N * N + 1);
}

bz_status bz_weight_table(int N, double lambda, double *out) {
    if (!out) return fail(BZ_EINVAL, "bz_weight_table: NULL argument");
    if (bz_weight_table_size(N) == 0) return fail(BZ_EINVAL, "bz_weight_table: N must be a multiple of 4 in [8, 32]");
    if (!(lambda > -3.0 && lambda <= 1.0)) return fail(BZ_EUNSUPPORTED, "bz_weight_table: lambda must lie in (-3, 1]");
    std::vector<double> T;
    int qs = 0;
    build_table(N, lambda, T, qs);
    std::memcpy(out, T.data(), T.size() * sizeof(double));
    return BZ_OK;
}

size_t bz_weights_bytes(bz_grid g, int kind) {
    if (!g) return 0;
    switch (kind) {
    case BZ_W_BATCHED_F32:
        if (core_stream_bytes(g)) return core_base_bytes(g) + core_stream_bytes(g) + kWeightPadBytes;
        return e3_base_bytes(g, 4) + (size_t)g->sched.e3_weights * 4 + kWeightPadBytes;
    case BZ_W_BATCHED_F64:
        return e3_base_bytes(g, kind_elem(kind)) + (size_t)g->sched.e3_weights * kind_elem(kind) + kWeightPadBytes;
    case BZ_W_PLAIN_F32:
    case BZ_W_PLAIN_F64: return (size_t)g->sched.plain_weights * kind_elem(kind);
    default: return 0;
    }
}

bz_status bz_weights(bz_grid g, int kind, void *d_w, size_t bytes, void *stream) {
    if (!g || !d_w) return fail(BZ_EINVAL, "bz_weights: NULL argument");
    const size_t need = bz_weights_bytes(g, kind);
    if (need == 0) return fail(BZ_EINVAL, "bz_weights: unknown weight kind");
    if (bytes < need) return fail(BZ_EINVAL, "bz_weights: buffer too small");
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> T;
    int qs = 0;
    build_table(g->N, g->lambda, T, qs);
    const bool cells = kind == BZ_W_BATCHED_F32 || kind == BZ_W_BATCHED_F64;
    const std::vector<long long> &off = cells ? g->sched.row_woff : g->sched.blk_woff;
    double *dT = nullptr;
    long long *dOff = nullptr;
    const size_t noff = off.size() + (cells ? g->sched.e3_woff.size() : 0);
    BZ_HIP(hipMalloc(&dT, T.size() * sizeof(double)), "bz_weights: hipMalloc table");
    hipError_t e = hipMalloc(&dOff, noff * sizeof(long long));
    if (e != hipSuccess) {
        (void)hipFree(dT);
        return hip_fail(e, "bz_weights: hipMalloc offsets");
    }
    e = hipMemcpyAsync(dT, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(dOff, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice, s);
    if (e == hipSuccess && cells)
        e = hipMemcpyAsync(dOff + off.size(), g->sched.e3_woff.data(), g->sched.e3_woff.size() * sizeof(long long),
                           hipMemcpyHostToDevice, s);
    const bool f64 = kind_elem(kind) == 8;
    // the FP32 stream leaves the pairs of the low-frequency core to the FP64 core stream
    const bool core = kind == BZ_W_BATCHED_F32 && core_stream_bytes(g) > 0;
    if (e == hipSuccess)
        e = cells ? launch_expand_cells(g->N, dT, qs, weight_scale(g), dOff, d_w, f64, core ? g->sched.core.r2 : -1,
                                        (int)g->lambda, g->beta, s)
                  : launch_expand_plain(g->N, dT, qs, weight_scale(g), dOff, d_w, f64, (int)g->lambda, g->beta, s);
    std::vector<double> cw;
    if (e == hipSuccess && core) {
        core_weights(g, T, qs, weight_scale(g), cw);
        e = hipMemcpyAsync((char *)d_w + core_base_bytes(g), cw.data(), cw.size() * sizeof(double),
                           hipMemcpyHostToDevice, s);
    }
    // the pass-E3 stream is derived from the main stream
    if (e == hipSuccess && cells)
        e = launch_build_e3(g->N, dOff, dOff + off.size(), d_w, (char *)d_w + e3_base_bytes(g, kind_elem(kind)), f64,
                            s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(dT);
    (void)hipFree(dOff);
    if (e != hipSuccess) return hip_fail(e, "bz_weights");
    return BZ_OK;
}

bz_status bz_batch_create(int n_cells, const int32_t *grid_of_cell, int n_grids, const bz_grid *grids, int mode,
                          bz_batch *out) {
    return bz_batch_create_ex(n_cells, grid_of_cell, n_grids, grids, mode, 0, out);
}

bz_status bz_batch_create_ex(int n_cells, const int32_t *grid_of_cell, int n_grids, const bz_grid *grids, int mode,
                             int flags, bz_batch *out) {
    if (!out) return fail(BZ_EINVAL, "bz_batch_create: out is NULL");
    if (flags & ~(BZ_BATCH_FULL_SUM | BZ_BATCH_FINE_SPLIT | BZ_BATCH_PER_MESH))
        return fail(BZ_EINVAL, "bz_batch_create: unknown flags");
    *out = nullptr;
    if (n_cells < 1 || !grid_of_cell || n_grids < 1 || !grids)
        return fail(BZ_EINVAL, "bz_batch_create: empty batch or NULL argument");
    if (mode < BZ_MODE_PLAIN_F64 || mode > BZ_MODE_PLAIN_F32) return fail(BZ_EINVAL, "bz_batch_create: bad mode");
    for (int i = 0; i < n_grids; ++i)
        if (!grids[i]) return fail(BZ_EINVAL, "bz_batch_create: NULL grid handle");
    for (int c = 0; c < n_cells; ++c)
        if (grid_of_cell[c] < 0 || grid_of_cell[c] >= n_grids)
            return fail(BZ_EINVAL, "bz_batch_create: grid index out of range");
    std::unique_ptr<bz_batch_s> b(new (std::nothrow) bz_batch_s());
    if (!b) return fail(BZ_ENOMEM, "bz_batch_create: allocation failed");
    b->mode = mode;
    b->n_cells = n_cells;
    b->grids.assign(grids, grids + n_grids);
    b->grid_of_cell.assign(grid_of_cell, grid_of_cell + n_cells);
    b->cell_off.resize(n_cells);
    size_t off = 0;
    for (int c = 0; c < n_cells; ++c) {
        b->cell_off[c] = (long long)off;
        const int N = grids[grid_of_cell[c]]->N;
        off += (size_t)N * N * N;
    }
    b->elems = off;
    // parts, largest mesh first (longest-processing-time order)
    std::vector<int> order(n_grids);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return grids[x]->N > grids[y]->N; });
    for (int gi : order) {
        Part p;
        p.g = grids[gi];
        p.gi = gi;
        for (int c = 0; c < n_cells; ++c)
            if (grid_of_cell[c] == gi) p.cells.push_back(c);
        if (p.cells.empty()) continue;
        p.groups = (int)((p.cells.size() + kWave - 1) / kWave);
        // untuned default: the output-slot variant with interleaved partials from N = 24 on,
        // the in-register FP64 total with interleaved partials below (measured on MI355X)
        p.variant = recalled_variant(tune_key(p.g->N, p.groups, mode), p.g->N >= 24 ? 10 : 13);
        b->parts.push_back(std::move(p));
    }
    // host tables, then one device buffer for all of them
    const bool bat = batched(mode);
    const bool f64 = mode_f64(mode);
    std::vector<char> host;
    auto put = [&host](const void *src, size_t bytes) {
        size_t o = align256(host.size());
        host.resize(o + bytes);
        std::memcpy(host.data() + o, src, bytes);
        return o;
    };
    struct Offs { size_t f_off, fh_base, row, blk, zero, items, e3, core_items, core_steps, disk, disk_ext; };
    std::vector<Offs> offs;
    size_t ws = 0, scratch = 0;
    for (Part &p : b->parts) {
        const int N = p.g->N;
        const long long M = (long long)N * N * N;
        Offs o{};
        p.f_off.resize(p.cells.size());
        std::vector<long long> base(p.cells.size());
        for (size_t i = 0; i < p.cells.size(); ++i) {
            p.f_off[i] = b->cell_off[p.cells[i]];
            base[i] = bat ? (long long)(i / kWave) * M * kWave + (long long)(i % kWave) : 0;
        }
        o.f_off = put(p.f_off.data(), p.f_off.size() * sizeof(long long));
        o.fh_base = put(base.data(), base.size() * sizeof(long long));
        long long zero = 0;
        o.zero = put(&zero, sizeof zero);
        o.row = put(p.g->sched.row_woff.data(), p.g->sched.row_woff.size() * sizeof(long long));
        o.blk = put(p.g->sched.blk_woff.data(), p.g->sched.blk_woff.size() * sizeof(long long));
        if (bat) {
            // split every row's steps into `parts` contiguous ranges so that there are
            // enough work items to fill the chip (with BZ_BATCH_FINE_SPLIT: from the rows of
            // one group alone); order longest first
            const int h = N / 2;
            p.herm = !(flags & BZ_BATCH_FULL_SUM);
            long long rows = 0;
            for (int r = 0; r < N * N; ++r)
                if (!p.herm || !herm_derived_row(N, r / N, r % N)) ++rows;
            if (!(flags & BZ_BATCH_FINE_SPLIT)) rows *= p.groups;
            int parts = (int)(((p.herm ? 4096 : 8192) + rows - 1) / rows);
            // at most 8 partial sums (6 with the fine split: measured best for one convolved group)
            parts = std::max(1, std::min(parts, (flags & BZ_BATCH_FINE_SPLIT) ? 6 : 8));
            p.parts = parts;
            std::vector<int4> items;
            const std::vector<int> &st = p.g->sched.row_steps;
            // every item writes its whole output slot, so an empty step range still
            // leaves zeros where the assembly reads
            auto item = [&](int gq, int r, int q, int pass, int a, int e) {
                items.push_back(make_int4(gq, r | (q << 16) | (pass << 20), a, e));
            };
            // steps [s0, st[r]) of row r in `parts` contiguous ranges
            auto split = [&](int gq, int r, int pass, int s0) {
                const long long n = st[r] - s0;
                for (int q = 0; q < parts; ++q)
                    item(gq, r, q, pass, s0 + (int)(n * q / parts), s0 + (int)(n * (q + 1) / parts));
            };
            for (int gq = 0; gq < p.groups; ++gq) {
                // pass A runs on fhat with its k_d = 0 planes zeroed, so the steps with
                // m1 = 0 (the first axis_cnt(k2) steps of rows k1 < N/2) add nothing
                for (int r = 0; r < N * N; ++r) {
                    const int k1 = r / N, k2 = r % N;
                    if (!p.herm) split(gq, r, kPassA, 0);
                    else if (!herm_derived_row(N, k1, k2)) split(gq, r, kPassA, k1 < h ? axis_cnt(N, k2) : 0);
                }
                if (!p.herm) continue;
                for (int a = 0; a < h; ++a)
                    for (int b = 0; b < N; ++b) {
                        // the m1 = 0 block of row (a, b) is its first axis_cnt(b) steps
                        const int c = axis_cnt(N, b), cut = b < h ? 1 : 0;
                        item(gq, a * N + b, 0, kPassE1, 0, c);
                        item(gq, a * N + b, 0, kPassE2, cut, c - cut);
                        item(gq, a * N + b, 0, kPassE3, cut, c - cut);
                    }
                for (int b = h; b < N; ++b) split(gq, b, kPassZ, 0);
            }
            std::stable_sort(items.begin(), items.end(),
                             [](const int4 &x, const int4 &y) { return x.w - x.z > y.w - y.z; });
            p.n_items = (int)items.size();
            p.h_items = items;
            o.items = put(items.data(), items.size() * sizeof(int4));
            o.e3 = put(p.g->sched.e3_woff.data(), p.g->sched.e3_woff.size() * sizeof(long long));
            const CoreSched &cs = p.g->sched.core;
            p.core = mode == BZ_MODE_BATCHED_F32 && cs.r2 >= 1;
            if (p.core) {
                // one item per (group, output row within 2r of the centre), every such row written
                // (rows without core steps write zeros), longest first.  The derived rows of the
                // conjugate-symmetric schedule are conjugates of their mirrors except at k3 = 0, which
                // the outputs k3 <= N/2 (item kind 0) reach when 2r >= N/2; other rows take all their
                // outputs (kind 2).
                // A row's steps are cut into core_parts pieces, each summed into its own partial
                // buffer, so that no core item runs longer than the longest FP32 item of the mesh
                // (a core step, up to (2r+1)^2 FP64 products and two row loads, is counted as twice
                // (2r+1)^2 FP32 pairs).  That matters when few groups are convolved, as under the
                // gated closure: a central core row of one group would otherwise outlast them.
                int max_core = 0;
                long long max_conv = 1;
                for (int row = 0; row < N * N; ++row) max_core = std::max(max_core, cs.row_steps[row]);
                for (const int4 &it : items)
                    max_conv = std::max(max_conv, (long long)(it.w - it.z) * pairs_per_step(N));
                const long long S2 = (long long)(2 * cs.r + 1) * (2 * cs.r + 1);
                p.core_parts = (int)std::min<long long>(
                    kCoreMaxParts, std::max<long long>(1, (2 * S2 * max_core + max_conv - 1) / max_conv));
                std::vector<int4> ci;
                for (int gq = 0; gq < p.groups; ++gq)
                    for (int k1 = std::max(0, h - 2 * cs.r); k1 <= std::min(N - 1, h + 2 * cs.r); ++k1)
                        for (int k2 = std::max(0, h - 2 * cs.r); k2 <= std::min(N - 1, h + 2 * cs.r); ++k2) {
                            const int row = k1 * N + k2;
                            const int a = (int)cs.row_soff[row], n = cs.row_steps[row];
                            const bool derived = herm_derived_row(N, k1, k2);
                            if (derived && 2 * cs.r < h) continue;
                            // every piece is an item (an empty one writes zeros to its partial sum)
                            for (int q = 0; q < p.core_parts; ++q)
                                ci.push_back(make_int4(gq, row | ((derived ? 0 : 2) << 16) | (q << 20),
                                                       a + (n * q) / p.core_parts, a + (n * (q + 1)) / p.core_parts));
                        }
                std::stable_sort(ci.begin(), ci.end(), [](const int4 &x, const int4 &y) { return x.w - x.z > y.w - y.z; });
                p.n_core_items = (int)ci.size();
                p.h_core_items = ci;
                o.core_items = put(ci.data(), ci.size() * sizeof(int4));
                o.core_steps = put(cs.steps.data(), cs.steps.size() * sizeof(int));
                o.disk = put(cs.disk_idx.data(), cs.disk_idx.size() * sizeof(int));
                o.disk_ext = put(cs.disk_ext.data(), cs.disk_ext.size() * sizeof(int));
            }
        }
        offs.push_back(o);
        // workspace: fhat, qhat, counter
        const size_t cs = f64 ? 16 : 8;
        if (bat) {
            p.ws_fh = ws;
            ws = align256(ws + (size_t)(p.herm ? 4 : 1) * p.groups * M * kWave * cs);
            // qhat buffers, in units of B = one full output buffer: pass A's partial sums (B
            // each), then E1, E2, E3 (rows k_a < N/2: B/2 each) and Z's partial sums (the
            // rows N/2..N-1 of one plane: B/(2N) each)
            const size_t B = (size_t)p.groups * M * kWave;
            p.ws_qh = ws;
            ws = align256(ws + (p.parts * B + (p.herm ? 3 * (B / 2) + p.parts * (B / (2 * N)) : 0)) * 16);
        } else {
            const int sp = plain_split_for(N);
            p.ws_fh = ws;
            ws = align256(ws + (size_t)M * cs);
            p.ws_qh = ws;
            ws = align256(ws + (size_t)sp * M * 16);
        }
        p.ws_counter = ws;
        ws = align256(ws + 256);
        if (p.core) {
            // FP64 core rows [G][nD][2r+1][64] and the core sum [G][N^3][64]
            const CoreSched &cs = p.g->sched.core;
            p.ws_cf = ws;
            ws = align256(ws + (size_t)p.groups * cs.nD * (2 * cs.r + 1) * kWave * 16);
            p.ws_cq = ws;
            ws = align256(ws + (size_t)p.core_parts * p.groups * M * kWave * 16);
            p.ws_ccounter = ws;
            ws = align256(ws + 256);
        }
        const size_t sc = (bat ? (size_t)p.groups * kWave : 1) * (size_t)M * 16;
        scratch = std::max(scratch, sc);
    }
    // one convolution launch for the items of every mesh: the mesh's index in bits 24..27, the
    // FP32 items ordered by cost (steps x pairs per step), longest first, and the FP64 core items
    // (kCoreItemBit) spread evenly through the first part of that order, so that at any time a
    // few wavefronts load core rows while the others do FP32 arithmetic.  A one-mesh batch with
    // a core takes the same launch.
    size_t o_multi = 0, o_desc = 0;
    bool has_core = false;
    for (const Part &p : b->parts) has_core = has_core || p.core;
    const bool multi = mode == BZ_MODE_BATCHED_F32 && (b->parts.size() >= 2 || has_core) &&
                       b->parts.size() <= (size_t)kMaxMultiMeshes && !(flags & BZ_BATCH_PER_MESH);
    std::vector<int4> mitems;
    if (multi) {
        std::vector<int4> conv, core;
        for (size_t mi = 0; mi < b->parts.size(); ++mi) {
            for (int4 it : b->parts[mi].h_items) {
                it.y |= (int)mi << 24;
                conv.push_back(it);
            }
            for (int4 it : b->parts[mi].h_core_items) {
                it.y |= ((int)mi << 24) | kCoreItemBit;
                core.push_back(it);
            }
        }
        auto cost = [&](const int4 &x) {
            const int N = b->parts[(x.y >> 24) & 0xf].g->N;
            return (long long)(x.w - x.z) * pairs_per_step(N);
        };
        std::stable_sort(conv.begin(), conv.end(), [&](const int4 &x, const int4 &y) { return cost(x) > cost(y); });
        std::stable_sort(core.begin(), core.end(), [](const int4 &x, const int4 &y) { return x.w - x.z > y.w - y.z; });
        const size_t span = (conv.size() * kCoreSpreadNum) / kCoreSpreadDen;
        size_t ci = 0;
        for (size_t i = 0; i < conv.size(); ++i) {
            // core items due before FP32 item i: ceil(i * ncore / span)
            while (ci < core.size() && (span == 0 || ci * span < i * core.size())) mitems.push_back(core[ci++]);
            mitems.push_back(conv[i]);
        }
        while (ci < core.size()) mitems.push_back(core[ci++]);
        o_multi = put(mitems.data(), mitems.size() * sizeof(int4));
        std::vector<MeshConvDesc> zero(b->parts.size());
        o_desc = put(zero.data(), zero.size() * sizeof(MeshConvDesc));
        b->ws_mcounter = ws;
        ws = align256(ws + 256);
    }
    // per-cell tables of the diagnostics
    std::vector<int> cn(n_cells);
    std::vector<double> cdv(n_cells);
    for (int c = 0; c < n_cells; ++c) {
        cn[c] = grids[grid_of_cell[c]]->N;
        cdv[c] = grids[grid_of_cell[c]]->dv;
    }
    const size_t o_coff = put(b->cell_off.data(), n_cells * sizeof(long long));
    const size_t o_cn = put(cn.data(), n_cells * sizeof(int));
    const size_t o_cdv = put(cdv.data(), n_cells * sizeof(double));
    b->ws_scratch = ws;
    ws = align256(ws + scratch);
    b->ws_flag = ws;
    ws = align256(ws + 256);
    b->ws_total = ws;
    if (!host.empty()) {
        hipError_t e = hipMalloc(&b->d_tables, host.size());
        if (e != hipSuccess) return hip_fail(e, "bz_batch_create: hipMalloc tables");
        e = hipMemcpy(b->d_tables, host.data(), host.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            (void)hipFree(b->d_tables);
            return hip_fail(e, "bz_batch_create: upload tables");
        }
    }
    bool any_core = false;
    for (const Part &p : b->parts) any_core = any_core || p.core;
    if (any_core) {
        if (hipStreamCreateWithFlags(&b->core_stream, hipStreamNonBlocking) != hipSuccess) {
            b->core_stream = nullptr;
            if (b->d_tables) (void)hipFree(b->d_tables);
            return fail(BZ_EDEVICE, "bz_batch_create: hipStreamCreateWithFlags failed");
        }
        if (hipEventCreateWithFlags(&b->ev_cfork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&b->ev_cjoin, hipEventDisableTiming) != hipSuccess) {
            bz_batch_free(b.release());
            return fail(BZ_EDEVICE, "bz_batch_create: hipEventCreateWithFlags failed");
        }
    }
    char *base = (char *)b->d_tables;
    if (multi) {
        b->d_multi_items = (int4 *)(base + o_multi);
        b->n_multi_items = (int)mitems.size();
        b->d_desc = (MeshConvDesc *)(base + o_desc);
    }
    b->d_cell_off = (long long *)(base + o_coff);
    b->d_cell_N = (int *)(base + o_cn);
    b->d_cell_dv = (double *)(base + o_cdv);
    for (size_t i = 0; i < b->parts.size(); ++i) {
        Part &p = b->parts[i];
        p.d_f_off = (long long *)(base + offs[i].f_off);
        p.d_fh_base = (long long *)(base + offs[i].fh_base);
        p.d_zero = (long long *)(base + offs[i].zero);
        p.d_row_woff = (long long *)(base + offs[i].row);
        p.d_blk_woff = (long long *)(base + offs[i].blk);
        p.d_items = bat ? (int4 *)(base + offs[i].items) : nullptr;
        p.d_e3_woff = bat ? (long long *)(base + offs[i].e3) : nullptr;
        if (p.core) {
            p.d_core_items = (int4 *)(base + offs[i].core_items);
            p.d_core_steps = (int *)(base + offs[i].core_steps);
            p.d_disk_idx = (int *)(base + offs[i].disk);
            p.d_disk_ext = (int *)(base + offs[i].disk_ext);
        }
    }
    *out = b.release();
    return BZ_OK;
}

void bz_batch_free(bz_batch b) {
    if (!b) return;
    if (b->d_tables) (void)hipFree(b->d_tables);
    for (auto &e : b->ev_used) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto &e : b->ev_core_used) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto &e : b->ev_free) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    if (b->ev_join) (void)hipEventDestroy(b->ev_join);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->ev_cfork) (void)hipEventDestroy(b->ev_cfork);
    if (b->ev_cjoin) (void)hipEventDestroy(b->ev_cjoin);
    if (b->core_stream) (void)hipStreamDestroy(b->core_stream);
    delete b;
}

static ConvPasses conv_passes(const Part &p, bool f64);

bz_status bz_batch_set_weights(bz_batch b, int grid_index, int kind, const void *d_w) {
    if (!b || !d_w) return fail(BZ_EINVAL, "bz_batch_set_weights: NULL argument");
    if (grid_index < 0 || grid_index >= (int)b->grids.size())
        return fail(BZ_EINVAL, "bz_batch_set_weights: grid index out of range");
    if (kind != mode_wkind(b->mode))
        return fail(BZ_EINVAL, "bz_batch_set_weights: weight kind does not match the batch mode");
    for (Part &p : b->parts)
        if (p.gi == grid_index) {
            p.w = d_w;
            p.wkind = kind;
        }
    // the descriptors of the one-launch convolution, once every mesh has its weights
    if (b->d_desc) {
        std::vector<MeshConvDesc> d(b->parts.size());
        for (size_t i = 0; i < b->parts.size(); ++i) {
            const Part &p = b->parts[i];
            if (!p.w) return BZ_OK;
            d[i].fh_bytes = (long long)p.ws_fh;
            d[i].qh_bytes = (long long)p.ws_qh;
            d[i].N = p.g->N;
            d[i].ps = conv_passes(p, false);
            if (p.core) {
                const CoreSched &cs = p.g->sched.core;
                d[i].cf_bytes = (long long)p.ws_cf;
                d[i].cq_bytes = (long long)p.ws_cq;
                d[i].cq_pstride = (long long)p.groups * p.g->N * p.g->N * p.g->N * kWave;
                d[i].core_steps = p.d_core_steps;
                d[i].core_ext = p.d_disk_ext;
                d[i].core_w = (const double *)((const char *)p.w + core_base_bytes(p.g));
                d[i].nD = cs.nD;
                d[i].core_r = cs.r;
            }
        }
        BZ_HIP(hipMemcpy(b->d_desc, d.data(), d.size() * sizeof(MeshConvDesc), hipMemcpyHostToDevice),
               "bz_batch_set_weights: upload descriptors");
    }
    return BZ_OK;
}

int bz_variant_count(void) { return conv_variant_count(); }

bz_status bz_batch_set_variant(bz_batch b, int grid_index, int variant) {
    if (!b) return fail(BZ_EINVAL, "bz_batch_set_variant: NULL batch");
    if (variant < 0 || variant >= bz_variant_count()) return fail(BZ_EINVAL, "bz_batch_set_variant: bad variant");
    if (grid_index < 0 || grid_index >= (int)b->grids.size())
        return fail(BZ_EINVAL, "bz_batch_set_variant: grid index out of range");
    for (Part &p : b->parts)
        if (p.gi == grid_index) p.variant = variant;
    return BZ_OK;
}

int bz_batch_get_variant(bz_batch b, int grid_index) {
    if (!b) return -1;
    for (Part &p : b->parts)
        if (p.gi == grid_index) return p.variant;
    return -1;
}

bz_status bz_batch_timer(bz_batch b, int enable) {
    if (!b) return fail(BZ_EINVAL, "bz_batch_timer: NULL batch");
    b->timing = enable != 0;
    return BZ_OK;
}

bz_status bz_batch_timer_read(bz_batch b, double *conv_ms, int *launches) {
    if (!b) return fail(BZ_EINVAL, "bz_batch_timer_read: NULL batch");
    double tot = 0.0;
    for (auto &e : b->ev_used) {
        BZ_HIP(hipEventSynchronize(e.second), "bz_batch_timer_read: sync");
        float ms = 0.f;
        BZ_HIP(hipEventElapsedTime(&ms, e.first, e.second), "bz_batch_timer_read: elapsed");
        tot += ms;
    }
    if (conv_ms) *conv_ms = tot;
    if (launches) *launches = (int)b->ev_used.size();
    b->ev_free.insert(b->ev_free.end(), b->ev_used.begin(), b->ev_used.end());
    b->ev_used.clear();
    double ctot = 0.0;
    for (auto &e : b->ev_core_used) {
        BZ_HIP(hipEventSynchronize(e.second), "bz_batch_timer_read: sync");
        float ms = 0.f;
        BZ_HIP(hipEventElapsedTime(&ms, e.first, e.second), "bz_batch_timer_read: elapsed");
        ctot += ms;
    }
    b->core_ms = ctot;
    b->core_launches = (int)b->ev_core_used.size();
    b->ev_free.insert(b->ev_free.end(), b->ev_core_used.begin(), b->ev_core_used.end());
    b->ev_core_used.clear();
    return BZ_OK;
}

bz_status bz_batch_set_core_waves(bz_batch b, int waves) {
    if (!b) return fail(BZ_EINVAL, "bz_batch_set_core_waves: NULL batch");
    if (waves < 0) return fail(BZ_EINVAL, "bz_batch_set_core_waves: negative count");
    b->core_waves = waves;
    return BZ_OK;
}

bz_status bz_batch_core_timer(bz_batch b, double *core_ms, int *launches) {
    if (!b) return fail(BZ_EINVAL, "bz_batch_core_timer: NULL batch");
    if (core_ms) *core_ms = b->core_ms;
    if (launches) *launches = b->core_launches;
    return BZ_OK;
}

bz_status bz_batch_autotune(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes, int reps,
                            void *stream) {
    if (!b || !d_f || !d_Qt || !d_work) return fail(BZ_EINVAL, "bz_batch_autotune: NULL argument");
    if (reps < 1) reps = 1;
    if (!batched(b->mode)) return BZ_OK;  // the plain schedule has no variants
    const bool was = b->timing;
    b->per_mesh_now = true;   // each mesh's own launch is timed
    std::vector<int> saved;
    for (Part &p : b->parts) saved.push_back(p.variant);
    // time every variant for all parts at once (each part's launch is timed separately)
    const int nv = bz_variant_count();
    std::vector<std::vector<double>> t(b->parts.size(), std::vector<double>(nv, 0.0));
    b->timing = true;
    bz_status st = BZ_OK;
    for (int v = 0; v < nv && st == BZ_OK; ++v) {
        if (mode_f64(b->mode) && v > 0) break;  // the FP64 kernel has one variant
        for (Part &p : b->parts) p.variant = v;
        st = bz_collide_batch(b, d_f, d_Qt, d_work, work_bytes, stream);  // warm-up
        double junk;
        if (st == BZ_OK) st = bz_batch_timer_read(b, &junk, nullptr);
        for (int r = 0; r < reps && st == BZ_OK; ++r) st = bz_collide_batch(b, d_f, d_Qt, d_work, work_bytes, stream);
        if (st != BZ_OK) break;
        // events are recorded in part order, reps times
        const size_t np = b->parts.size();
        for (size_t i = 0; i < b->ev_used.size(); ++i) {
            auto &e = b->ev_used[i];
            BZ_HIP(hipEventSynchronize(e.second), "autotune sync");
            float ms = 0.f;
            BZ_HIP(hipEventElapsedTime(&ms, e.first, e.second), "autotune elapsed");
            t[i % np][v] += ms;
        }
        b->ev_free.insert(b->ev_free.end(), b->ev_used.begin(), b->ev_used.end());
        b->ev_used.clear();
        b->ev_free.insert(b->ev_free.end(), b->ev_core_used.begin(), b->ev_core_used.end());
        b->ev_core_used.clear();
    }
    b->timing = false;
    b->per_mesh_now = false;
    if (st != BZ_OK) {
        b->timing = was;
        for (size_t i = 0; i < b->parts.size(); ++i) b->parts[i].variant = saved[i];
        return st;
    }
    for (size_t i = 0; i < b->parts.size(); ++i) {
        Part &p = b->parts[i];
        int fastest = 0;
        const int nvv = mode_f64(b->mode) ? 1 : nv;
        for (int v = 1; v < nvv; ++v)
            if (t[i][v] < t[i][fastest]) fastest = v;
        // within 3% of the fastest, prefer the more accurate accumulation
        int best = fastest;
        for (int v = 0; v < nvv; ++v) {
            if (t[i][v] > 1.03 * t[i][fastest]) continue;
            const int rv = conv_variant_accuracy_rank(v), rb = conv_variant_accuracy_rank(best);
            if (rv > rb || (rv == rb && t[i][v] < t[i][best])) best = v;
        }
        p.variant = best;
        remember_variant(tune_key(p.g->N, p.groups, b->mode), best);
    }
    // one launch for every mesh (and the cores) or one launch per mesh with the variants just
    // chosen: the whole evaluation is timed both ways and the faster kept
    if (b->d_multi_items) {
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
            if (e0) (void)hipEventDestroy(e0);
            b->timing = was;
            return fail(BZ_EDEVICE, "bz_batch_autotune: hipEventCreate failed");
        }
        double t[2] = {0.0, 0.0};
        for (int per = 0; per < 2 && st == BZ_OK; ++per) {
            b->per_mesh_now = per != 0;
            st = bz_collide_batch(b, d_f, d_Qt, d_work, work_bytes, stream);   // warm-up
            if (st != BZ_OK) break;
            if (hipEventRecord(e0, (hipStream_t)stream) != hipSuccess) st = fail(BZ_EDEVICE, "bz_batch_autotune: event");
            for (int r = 0; r < reps && st == BZ_OK; ++r) st = bz_collide_batch(b, d_f, d_Qt, d_work, work_bytes, stream);
            float ms = 0.f;
            if (st == BZ_OK && (hipEventRecord(e1, (hipStream_t)stream) != hipSuccess ||
                                hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                st = fail(BZ_EDEVICE, "bz_batch_autotune: event timing");
            t[per] = ms;
        }
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        b->per_mesh_now = st == BZ_OK && t[1] < t[0];
    }
    b->timing = was;
    return st;
}

int bz_batch_one_launch(bz_batch b) { return b && b->d_multi_items && !b->per_mesh_now ? 1 : 0; }

bz_status bz_tuning_save(const char *path) {
    if (!path) return fail(BZ_EINVAL, "bz_tuning_save: NULL path");
    std::FILE *fp = std::fopen(path, "w");
    if (!fp) return fail(BZ_EINVAL, "bz_tuning_save: cannot open the file for writing");
    std::fprintf(fp, "# bz tuning: N groups mode variant\n");
    {
        std::lock_guard<std::mutex> lock(g_tuned_mu);
        for (const auto &kv : g_tuned)
            std::fprintf(fp, "%lld %lld %lld %d\n", kv.first >> 40, (kv.first >> 8) & 0xffffffffLL, kv.first & 0xff,
                         kv.second);
    }
    const bool ok = std::fclose(fp) == 0;
    return ok ? BZ_OK : fail(BZ_EINVAL, "bz_tuning_save: write failed");
}

bz_status bz_tuning_load(const char *path) {
    if (!path) return fail(BZ_EINVAL, "bz_tuning_load: NULL path");
    std::FILE *fp = std::fopen(path, "r");
    if (!fp) return fail(BZ_EINVAL, "bz_tuning_load: cannot open the file");
    std::vector<std::pair<long long, int>> got;
    char line[256];
    bool bad = false;
    while (std::fgets(line, sizeof line, fp)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        long long N, groups, mode;
        int v;
        if (std::sscanf(line, "%lld %lld %lld %d", &N, &groups, &mode, &v) != 4 || N < kMinN || N > kMaxN ||
            groups < 1 || groups > 0xffffffffLL || mode < 0 || mode > 0xff || v < 0 || v >= bz_variant_count()) {
            bad = true;
            break;
        }
        got.emplace_back(tune_key((int)N, (int)groups, (int)mode), v);
    }
    std::fclose(fp);
    if (bad) return fail(BZ_EINVAL, "bz_tuning_load: malformed line (N groups mode variant)");
    for (const auto &kv : got) remember_variant(kv.first, kv.second);   // the whole file or nothing
    return BZ_OK;
}

size_t bz_batch_elems(bz_batch b) { return b ? b->elems : 0; }
size_t bz_batch_cell_offset(bz_batch b, int cell) {
    if (!b || cell < 0 || cell >= b->n_cells) return 0;
    return (size_t)b->cell_off[cell];
}
size_t bz_workspace_bytes(bz_batch b) { return b ? b->ws_total : 0; }
size_t bz_step_workspace_bytes(bz_batch b) { return b ? align256(b->ws_total) + 2 * align256(b->elems * 8) : 0; }

static bz_status collide_impl(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes,
                              void *stream, const unsigned char *skip, const long long *slot_off);

bz_status bz_collide_batch(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes,
                           void *stream) {
    return collide_impl(b, d_f, d_Qt, d_work, work_bytes, stream, nullptr, nullptr);
}

}  // extern "C"

// Workspace of bz_collide_batch_static: one array per GPU, resident for the life of the process.
// Host code never uses the array's own name as a device address: the address on each device
// comes from hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) char scratch[BZ_STATIC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::vector<void *> g_scratch_ptr;   // per device id; nullptr until looked up

static bz_status static_scratch(void **out) {
    int dev = 0;
    BZ_HIP(hipGetDevice(&dev), "bz_collide_batch_static: hipGetDevice");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if ((int)g_scratch_ptr.size() <= dev) g_scratch_ptr.resize(dev + 1, nullptr);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        BZ_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)), "bz_collide_batch_static: hipGetSymbolAddress");
        if (!ptr) return fail(BZ_EDEVICE, "bz_collide_batch_static: no device address for the static scratch");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return BZ_OK;
}

extern "C" {

bz_status bz_collide_batch_static(bz_batch b, const double *d_f, double *d_Qt, void *stream) {
    if (!b || !d_f || !d_Qt) return fail(BZ_EINVAL, "bz_collide_batch_static: NULL argument");
    if (b->ws_total > (size_t)BZ_STATIC_SCRATCH_BYTES) {
        char msg[200];
        std::snprintf(msg, sizeof msg,
                      "bz_collide_batch_static: the batch needs %zu bytes of workspace, the static scratch holds %zu",
                      b->ws_total, (size_t)BZ_STATIC_SCRATCH_BYTES);
        return fail(BZ_EINVAL, msg);
    }
    // the convolution timer would create HIP events on demand
    if (b->timing) return fail(BZ_ESTATE, "bz_collide_batch_static: switch the batch's timer off first");
    void *ws = nullptr;
    const bz_status st = static_scratch(&ws);
    if (st != BZ_OK) return st;
    return collide_impl(b, d_f, d_Qt, ws, (size_t)BZ_STATIC_SCRATCH_BYTES, stream, nullptr, nullptr);
}

// The five passes of a mesh's batched convolution (HermAssembly layout; the full-sum schedule
// uses pass A only): offsets relative to the mesh's fhat copies and output buffers.
static ConvPasses conv_passes(const Part &p, bool f64) {
    const int N = p.g->N;
    const long long M = (long long)N * N * N;
    const long long pstride = (long long)p.groups * M * kWave;  // one copy of fhat, one output buffer
    const void *w_e3 = (const char *)p.w + e3_base_bytes(p.g, f64 ? 8 : 4);
    const long long P = p.parts, gM = M * kWave, gE = gM / 2, gZ = (long long)(N / 2) * N * kWave;
    const long long e0 = P * pstride, z0 = e0 + 3 * (pstride / 2);
    ConvPasses ps{};
    ps.p[kPassA] = ConvPass{p.herm ? 3 * pstride : 0, 0, p.w, p.d_row_woff, p.herm ? 1 : 0, 0, gM, pstride};
    ps.p[kPassE1] = ConvPass{0, e0, p.w, p.d_row_woff, 0, 0, gE, 0};
    ps.p[kPassE2] = ConvPass{pstride, e0 + pstride / 2, p.w, p.d_row_woff, 0, 0, gE, 0};
    ps.p[kPassE3] = ConvPass{2 * pstride, e0 + pstride, w_e3, p.d_e3_woff, 0, 0, gE, 0};
    ps.p[kPassZ] = ConvPass{2 * pstride, z0, p.w, p.d_row_woff, 0, N / 2, gZ, pstride / (2 * N)};
    return ps;
}

// Batched modes: forward transforms of every mesh, the convolution (one launch for all meshes
// and their FP64 cores, or one per mesh with the cores on their own stream), then the inverse
// transforms.
static bz_status collide_batched(bz_batch b, const double *d_f, double *d_Qt, char *ws, hipStream_t s,
                                 const unsigned char *skip, const long long *slot_off) {
    double2 *scratch = (double2 *)(ws + b->ws_scratch);
    const bool f64 = mode_f64(b->mode);
    // skip and slot_off come with one-mesh batches (the gated closure); the group index of an
    // item is then the skip index
    const bool merged = b->d_multi_items && !b->per_mesh_now;
    for (const Part &p : b->parts) {
        const CoreSched &cs = p.g->sched.core;
        const long long *f_off = slot_off ? slot_off : p.d_f_off;
        // the first output buffer of the mesh serves as the second scratch buffer of the transforms
        const CoreFill cfill{p.core ? (double2 *)(ws + p.ws_cf) : nullptr, p.d_disk_idx, cs.nD, cs.r, cs.r2};
        BZ_HIP(launch_dft_forward_grouped(p.g->N, p.g->L, (int)p.cells.size(), d_f, f_off, scratch,
                                          (double2 *)(ws + p.ws_qh), ws + p.ws_fh, !f64, p.herm ? 4 : 1, cfill, skip,
                                          s),
               "forward transform");
    }
    // the FP64 cores: in the one-launch queue, or else on their own stream after the forward
    // transforms
    bool cores = false;
    for (const Part &p : b->parts) {
        if (!p.core || merged) continue;   // the one-launch queue holds the core items
        hipStream_t cst = b->core_stream;
        if (!cores) {
            BZ_HIP(hipEventRecord(b->ev_cfork, s), "core fork");
            BZ_HIP(hipStreamWaitEvent(cst, b->ev_cfork, 0), "core fork");
            cores = true;
        }
        const CoreSched &cs = p.g->sched.core;
        const CoreLaunch co{p.g->N, cs.r, cs.nD, (const double2 *)(ws + p.ws_cf), p.d_core_items, p.n_core_items,
                            (unsigned *)(ws + p.ws_ccounter), p.d_core_steps, p.d_disk_ext,
                            (const double *)((const char *)p.w + core_base_bytes(p.g)), (double2 *)(ws + p.ws_cq),
                            (long long)p.groups * p.g->N * p.g->N * p.g->N * kWave, skip, b->core_waves};
        std::pair<hipEvent_t, hipEvent_t> ce{};
        if (b->timing) {
            if (!timer_pair(b, ce, true)) return fail(BZ_EDEVICE, "bz_collide_batch: hipEventCreate failed");
            BZ_HIP(hipEventRecord(ce.first, cst), "core timer start");
        }
        BZ_HIP(launch_conv_core(co, cst), "FP64 core convolution");
        if (b->timing) BZ_HIP(hipEventRecord(ce.second, cst), "core timer stop");
    }
    if (cores) BZ_HIP(hipEventRecord(b->ev_cjoin, b->core_stream), "core join");
    if (merged) {
        const MultiLaunch ml{b->d_multi_items, b->n_multi_items, (unsigned *)(ws + b->ws_mcounter), b->d_desc, ws,
                             skip};
        std::pair<hipEvent_t, hipEvent_t> ev{};
        if (b->timing) {
            if (!timer_pair(b, ev)) return fail(BZ_EDEVICE, "bz_collide_batch: hipEventCreate failed");
            BZ_HIP(hipEventRecord(ev.first, s), "timer start");
        }
        BZ_HIP(launch_conv_cells_multi(ml, s), "batched convolution (all meshes)");
        if (b->timing) BZ_HIP(hipEventRecord(ev.second, s), "timer stop");
    } else {
        for (const Part &p : b->parts) {
            CellsLaunch cl{p.g->N, ws + p.ws_fh, p.d_items, p.n_items, (unsigned *)(ws + p.ws_counter),
                           (double2 *)(ws + p.ws_qh), p.variant, skip, conv_passes(p, f64)};
            std::pair<hipEvent_t, hipEvent_t> ev{};
            if (b->timing) {
                if (!timer_pair(b, ev)) return fail(BZ_EDEVICE, "bz_collide_batch: hipEventCreate failed");
                BZ_HIP(hipEventRecord(ev.first, s), "timer start");
            }
            BZ_HIP(launch_conv_cells(cl, f64, s), "batched convolution");
            if (b->timing) BZ_HIP(hipEventRecord(ev.second, s), "timer stop");
        }
    }
    if (cores) BZ_HIP(hipStreamWaitEvent(s, b->ev_cjoin, 0), "core join");
    for (const Part &p : b->parts) {
        const CoreSched &cs = p.g->sched.core;
        const long long *f_off = slot_off ? slot_off : p.d_f_off;
        const long long pstride = (long long)p.groups * p.g->N * p.g->N * p.g->N * kWave;
        const CoreAdd cadd{p.core ? (const double2 *)(ws + p.ws_cq) : nullptr, cs.r, p.core_parts, pstride};
        const HermAssembly herm{p.herm, p.parts};
        double2 *qh = (double2 *)(ws + p.ws_qh);
        // groups whose cells are all served by the closure (skip) need no transforms: the
        // closure writes their outputs
        BZ_HIP(launch_dft_inverse_grouped(p.g->N, p.g->L, (int)p.cells.size(), qh, p.parts, pstride, herm, cadd,
                                          scratch, qh, d_Qt, f_off, skip, s),
               "inverse transform");
    }
    return BZ_OK;
}

// skip (device, per group of the batched modes, may be NULL): groups whose outputs are not needed.
// slot_off (device, may be NULL): offsets of f and Qt of the cell in each slot of a one-mesh batch,
// in place of the batch's own cell order.
static bz_status collide_impl(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes,
                              void *stream, const unsigned char *skip, const long long *slot_off) {
    if (!b || !d_f || !d_Qt || !d_work) return fail(BZ_EINVAL, "bz_collide_batch: NULL argument");
    if (work_bytes < b->ws_total) return fail(BZ_EINVAL, "bz_collide_batch: workspace too small");
    if ((const void *)d_f == (const void *)d_Qt) return fail(BZ_EINVAL, "bz_collide_batch: f and Qt alias");
    for (const Part &p : b->parts)
        if (!p.w) return fail(BZ_ESTATE, "bz_collide_batch: no weights bound for a mesh of the batch");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_work;
    if (batched(b->mode)) return collide_batched(b, d_f, d_Qt, ws, s, skip, slot_off);
    double2 *scratch = (double2 *)(ws + b->ws_scratch);
    const bool f64 = mode_f64(b->mode);
    for (const Part &p : b->parts) {
        const int N = p.g->N;
        const long long M = (long long)N * N * N;
        void *fh = ws + p.ws_fh;
        double2 *qh = (double2 *)(ws + p.ws_qh);
        const int sp = plain_split_for(N);
        for (size_t i = 0; i < p.cells.size(); ++i) {
            BZ_HIP(launch_dft_forward(N, p.g->L, 1, d_f, p.d_f_off + i, scratch, fh, !f64, p.d_zero, 1, s),
                   "forward transform");
            PlainLaunch pl{N, fh, p.w, p.d_blk_woff, sp, qh};
            std::pair<hipEvent_t, hipEvent_t> ev{};
            if (b->timing) {
                if (!timer_pair(b, ev)) return fail(BZ_EDEVICE, "bz_collide_batch: hipEventCreate failed");
                BZ_HIP(hipEventRecord(ev.first, s), "timer start");
            }
            BZ_HIP(launch_conv_plain(pl, f64, s), "plain convolution");
            if (b->timing) BZ_HIP(hipEventRecord(ev.second, s), "timer stop");
            BZ_HIP(launch_dft_inverse(N, p.g->L, 1, qh, p.d_zero, 1, sp, M, scratch, d_Qt, p.d_f_off + i, s),
                   "inverse transform");
        }
    }
    return BZ_OK;
}

bz_status bz_project(bz_batch b, double *d_Q, void *stream) {
    if (!b || !d_Q) return fail(BZ_EINVAL, "bz_project: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    for (const Part &p : b->parts)
        BZ_HIP(launch_project(p.g->N, p.g->dv, p.g->linv, (int)p.cells.size(), d_Q, p.d_f_off, s), "projection");
    return BZ_OK;
}

bz_status bz_cell_moments(bz_batch b, const double *d_f, double *d_mom, void *stream) {
    if (!b || !d_f || !d_mom) return fail(BZ_EINVAL, "bz_cell_moments: NULL argument");
    BZ_HIP(launch_cell_moments(b->n_cells, d_f, b->d_cell_off, b->d_cell_N, b->d_cell_dv, d_mom, (hipStream_t)stream),
           "bz_cell_moments");
    return BZ_OK;
}

bz_status bz_marginal_v1(bz_batch b, const double *d_f, int cell, double *d_out, void *stream) {
    if (!b || !d_f || !d_out) return fail(BZ_EINVAL, "bz_marginal_v1: NULL argument");
    if (cell < 0 || cell >= b->n_cells) return fail(BZ_EINVAL, "bz_marginal_v1: cell index out of range");
    const bz_grid g = b->grids[b->grid_of_cell[cell]];
    BZ_HIP(launch_marginal_v1(g->N, g->dv, d_f + b->cell_off[cell], d_out, (hipStream_t)stream), "bz_marginal_v1");
    return BZ_OK;
}

bz_status bz_step(bz_batch b, double *d_f, double dt_over_eps, void *d_work, size_t work_bytes, void *stream) {
    if (!b || !d_f || !d_work) return fail(BZ_EINVAL, "bz_step: NULL argument");
    if (work_bytes < bz_step_workspace_bytes(b)) return fail(BZ_EINVAL, "bz_step: workspace too small");
    if (!std::isfinite(dt_over_eps)) return fail(BZ_EINVAL, "bz_step: dt/eps must be finite");
    for (const Part &p : b->parts)
        if (!p.w) return fail(BZ_ESTATE, "bz_step: no weights bound for a mesh of the batch");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_work;
    double *q = (double *)(ws + align256(b->ws_total));
    double *fs = (double *)(ws + align256(b->ws_total) + align256(b->elems * 8));
    unsigned *flag = (unsigned *)(ws + b->ws_flag);
    bz_status st = bz_collide_batch(b, d_f, q, d_work, b->ws_total, stream);
    if (st != BZ_OK) return st;
    if ((st = bz_project(b, q, stream)) != BZ_OK) return st;
    BZ_HIP(launch_axpy(b->elems, d_f, q, dt_over_eps, fs, flag, s), "heun stage 1");
    if ((st = bz_collide_batch(b, fs, q, d_work, b->ws_total, stream)) != BZ_OK) return st;
    if ((st = bz_project(b, q, stream)) != BZ_OK) return st;
    BZ_HIP(launch_heun_final(b->elems, d_f, fs, q, dt_over_eps, d_f, flag, s), "heun stage 2");
    return BZ_OK;
}

bz_status bz_step_check(bz_batch b, void *d_work, void *stream) {
    if (!b || !d_work) return fail(BZ_EINVAL, "bz_step_check: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    unsigned *flag = (unsigned *)((char *)d_work + b->ws_flag);
    unsigned h = 0;
    BZ_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s), "bz_step_check: read flag");
    BZ_HIP(hipStreamSynchronize(s), "bz_step_check: sync");
    if (h) BZ_HIP(launch_fill_u32(flag, 1, 0u, s), "bz_step_check: clear flag");
    if (h & BZ_FLAG_NONFINITE) return fail(BZ_ENONFINITE, "bz_step: a non-finite value was produced");
    return BZ_OK;
}

bz_status bz_step_flags(bz_batch b, void *d_work, unsigned *flags, void *stream) {
    if (!b || !d_work || !flags) return fail(BZ_EINVAL, "bz_step_flags: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    unsigned *flag = (unsigned *)((char *)d_work + b->ws_flag);
    unsigned h = 0;
    BZ_HIP(hipMemcpyAsync(&h, flag, sizeof h, hipMemcpyDeviceToHost, s), "bz_step_flags: read flag");
    BZ_HIP(hipStreamSynchronize(s), "bz_step_flags: sync");
    if (h) BZ_HIP(launch_fill_u32(flag, 1, 0u, s), "bz_step_flags: clear flag");
    *flags = h;
    return BZ_OK;
}

// ---------------------------------------------------------------------------
// Gated closure.  Workspace: [step workspace][state n*10 doubles][skip groups][slot offsets n]
// [x n*M bf16][y n*M float][stats 4 uint][network workspace for batch n].
// ---------------------------------------------------------------------------
struct ClosureView {
    double *state;
    unsigned char *skip;
    long long *slot_off;
    unsigned short *x;
    float *y;
    unsigned *stats;
    char *mlp_work;
    size_t mlp_bytes;
    size_t total;
};

static ClosureView closure_view(bz_batch b, const bz_closure *c, void *d_work) {
    ClosureView v{};
    const Part &p = b->parts[0];
    const size_t n = p.cells.size(), M = (size_t)p.g->N * p.g->N * p.g->N;
    size_t o = align256(bz_step_workspace_bytes(b));
    char *w = (char *)d_work;
    auto take = [&](size_t bytes) {
        char *q = w ? w + o : nullptr;
        o = align256(o + bytes);
        return q;
    };
    v.state = (double *)take(n * 10 * sizeof(double));
    v.skip = (unsigned char *)take((size_t)p.groups);
    v.slot_off = (long long *)take(n * sizeof(long long));
    v.x = (unsigned short *)take(n * M * 2);
    v.y = (float *)take(n * M * 4);
    v.stats = (unsigned *)take(256);
    v.mlp_bytes = bz_mlp_workspace_bytes(c->net, (int)n);
    v.mlp_work = take(v.mlp_bytes);
    v.total = o;
    return v;
}

static bz_status closure_check(bz_batch b, const bz_closure *c, const char *who) {
    if (!b || !c || !c->net || !c->d_params) return fail(BZ_EINVAL, std::string(who) + ": NULL argument");
    if (b->parts.size() != 1) return fail(BZ_EUNSUPPORTED, std::string(who) + ": the closure needs a one-mesh batch");
    const size_t M = (size_t)b->parts[0].g->N * b->parts[0].g->N * b->parts[0].g->N;
    if (bz_mlp_param_count(c->net) == 0) return fail(BZ_EINVAL, std::string(who) + ": bad network");
    // n_in and n_out must both be N^3: check through the parameter count of a square-ended net
    size_t hid = 0;
    {
        // count = h*M + h + h*h + h + M*h + M  ->  solve h^2 + (2M + 2) h + M - count = 0
        const double cnt = (double)bz_mlp_param_count(c->net), A = 2.0 * M + 2.0;
        const double hh = (-A + std::sqrt(A * A + 4.0 * (cnt - (double)M))) / 2.0;
        hid = (size_t)std::llround(hh);
        if (hid * M + hid + hid * hid + hid + M * hid + M != (size_t)cnt)
            return fail(BZ_EINVAL, std::string(who) + ": network input and output must be N^3 wide");
    }
    if (!(c->gate >= 0) || !(c->s_in > 0) || !(c->s_out > 0) || c->judge_every < 0)
        return fail(BZ_EINVAL, std::string(who) + ": bad gate, scales or judge rate");
    return BZ_OK;
}

static bz_status closure_side(bz_batch b) {
    if (b->side) return BZ_OK;
    if (hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking) != hipSuccess) {
        b->side = nullptr;
        return fail(BZ_EDEVICE, "closure: hipStreamCreateWithFlags failed");
    }
    if (hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_join, hipEventDisableTiming) != hipSuccess)
        return fail(BZ_EDEVICE, "closure: hipEventCreateWithFlags failed");
    return BZ_OK;
}

static bz_status closure_collide_impl(bz_batch b, const bz_closure *c, const double *d_f, double *d_Qt, void *d_work,
                                      hipStream_t s) {
    const Part &p = b->parts[0];
    const int n = (int)p.cells.size(), N = p.g->N;
    ClosureView v = closure_view(b, c, d_work);
    bz_status st = closure_side(b);
    if (st != BZ_OK) return st;
    BZ_HIP(launch_sur_prepare(N, p.g->dv, n, d_f, p.d_f_off, c->gate, c->s_in, c->judge_every, b->closure_phase++,
                              v.stats, v.state, v.x, s),
           "closure prepare");
    const unsigned char *skip = nullptr;
    const long long *slot_off = nullptr;
    if (batched(b->mode)) {
        // the cells that need the convolution go to the first groups; the rest are skipped
        BZ_HIP(launch_pack_slots(n, v.state, p.d_f_off, v.slot_off, v.skip, s), "closure slot packing");
        skip = v.skip;
        slot_off = v.slot_off;
    }
    // the network (its own input, output and workspace) overlaps the transforms and the convolution
    BZ_HIP(hipEventRecord(b->ev_fork, s), "closure fork");
    BZ_HIP(hipStreamWaitEvent(b->side, b->ev_fork, 0), "closure fork");
    st = bz_mlp_forward(c->net, c->d_params, v.x, n, v.y, v.mlp_work, v.mlp_bytes, b->side);
    if (st != BZ_OK) return st;
    BZ_HIP(hipEventRecord(b->ev_join, b->side), "closure join");
    st = collide_impl(b, d_f, d_Qt, d_work, b->ws_total, s, skip, slot_off);
    BZ_HIP(hipStreamWaitEvent(s, b->ev_join, 0), "closure join");
    if (st != BZ_OK) return st;
    BZ_HIP(launch_sur_finish(N, p.g->dv, p.g->linv, n, v.state, v.y, c->s_out, c->judge_floor, c->judge_tol,
                             p.d_f_off, d_Qt, v.stats, s),
           "closure finish");
    return BZ_OK;
}

size_t bz_closure_workspace_bytes(bz_batch b, const bz_closure *c) {
    if (closure_check(b, c, "bz_closure_workspace_bytes") != BZ_OK) return 0;
    return closure_view(b, c, nullptr).total;
}

bz_status bz_closure_prepare(bz_batch b, const double *d_f, double gate, double s_in, double *d_state, uint16_t *d_x,
                             void *stream) {
    if (!b || !d_f || !d_state || !d_x) return fail(BZ_EINVAL, "bz_closure_prepare: NULL argument");
    if (b->parts.size() != 1) return fail(BZ_EUNSUPPORTED, "bz_closure_prepare: needs a one-mesh batch");
    if (!(s_in > 0)) return fail(BZ_EINVAL, "bz_closure_prepare: s_in must be positive");
    const Part &p = b->parts[0];
    BZ_HIP(launch_sur_prepare(p.g->N, p.g->dv, (int)p.cells.size(), d_f, p.d_f_off, gate, s_in, 0, 0, nullptr, d_state,
                              (unsigned short *)d_x, (hipStream_t)stream),
           "bz_closure_prepare");
    return BZ_OK;
}

bz_status bz_closure_targets(bz_batch b, const double *d_state, const double *d_Q, double s_out, float *d_y,
                             void *stream) {
    if (!b || !d_state || !d_Q || !d_y) return fail(BZ_EINVAL, "bz_closure_targets: NULL argument");
    if (b->parts.size() != 1) return fail(BZ_EUNSUPPORTED, "bz_closure_targets: needs a one-mesh batch");
    if (!(s_out > 0)) return fail(BZ_EINVAL, "bz_closure_targets: s_out must be positive");
    const Part &p = b->parts[0];
    BZ_HIP(launch_sur_targets(p.g->N, (int)p.cells.size(), d_state, d_Q, p.d_f_off, s_out, d_y, (hipStream_t)stream),
           "bz_closure_targets");
    return BZ_OK;
}

bz_status bz_closure_collide(bz_batch b, const bz_closure *c, const double *d_f, double *d_Qt, void *d_work,
                             size_t work_bytes, void *stream) {
    bz_status st = closure_check(b, c, "bz_closure_collide");
    if (st != BZ_OK) return st;
    if (!d_f || !d_Qt || !d_work) return fail(BZ_EINVAL, "bz_closure_collide: NULL argument");
    if (work_bytes < closure_view(b, c, nullptr).total) return fail(BZ_EINVAL, "bz_closure_collide: workspace too small");
    for (const Part &p : b->parts)
        if (!p.w) return fail(BZ_ESTATE, "bz_closure_collide: no weights bound");
    return closure_collide_impl(b, c, d_f, d_Qt, d_work, (hipStream_t)stream);
}

bz_status bz_closure_step(bz_batch b, const bz_closure *c, double *d_f, double dt_over_eps, void *d_work,
                          size_t work_bytes, void *stream) {
    bz_status st = closure_check(b, c, "bz_closure_step");
    if (st != BZ_OK) return st;
    if (!d_f || !d_work) return fail(BZ_EINVAL, "bz_closure_step: NULL argument");
    if (work_bytes < closure_view(b, c, nullptr).total) return fail(BZ_EINVAL, "bz_closure_step: workspace too small");
    if (!std::isfinite(dt_over_eps)) return fail(BZ_EINVAL, "bz_closure_step: dt/eps must be finite");
    for (const Part &p : b->parts)
        if (!p.w) return fail(BZ_ESTATE, "bz_closure_step: no weights bound");
    hipStream_t s = (hipStream_t)stream;
    char *ws = (char *)d_work;
    double *q = (double *)(ws + align256(b->ws_total));
    double *fs = (double *)(ws + align256(b->ws_total) + align256(b->elems * 8));
    unsigned *flag = (unsigned *)(ws + b->ws_flag);
    if ((st = closure_collide_impl(b, c, d_f, q, d_work, s)) != BZ_OK) return st;
    if ((st = bz_project(b, q, stream)) != BZ_OK) return st;
    BZ_HIP(launch_axpy(b->elems, d_f, q, dt_over_eps, fs, flag, s), "closure heun stage 1");
    if ((st = closure_collide_impl(b, c, fs, q, d_work, s)) != BZ_OK) return st;
    if ((st = bz_project(b, q, stream)) != BZ_OK) return st;
    BZ_HIP(launch_heun_final(b->elems, d_f, fs, q, dt_over_eps, d_f, flag, s), "closure heun stage 2");
    return BZ_OK;
}

bz_status bz_closure_read_stats(bz_batch b, const bz_closure *c, void *d_work, bz_closure_stats *out, void *stream) {
    bz_status st = closure_check(b, c, "bz_closure_read_stats");
    if (st != BZ_OK) return st;
    if (!d_work || !out) return fail(BZ_EINVAL, "bz_closure_read_stats: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    ClosureView v = closure_view(b, c, d_work);
    unsigned h[10] = {};
    BZ_HIP(hipMemcpyAsync(h, v.stats, sizeof h, hipMemcpyDeviceToHost, s), "read closure stats");
    BZ_HIP(hipStreamSynchronize(s), "read closure stats sync");
    out->served = h[0];
    out->judged = h[1];
    float e;
    std::memcpy(&e, &h[2], sizeof e);
    out->max_err = e;
    out->failed = h[3];
    out->unbounded = h[6];
    unsigned long long cap;
    std::memcpy(&cap, &h[8], sizeof cap);
    cap = ~cap;
    double g = 0.0;
    if (~cap) std::memcpy(&g, &cap, sizeof g);   // a stored 0 (no cap) reads as 0
    out->gate_cap = g;
    // the counters restart; the gate cap persists (zero the workspace to lift it)
    BZ_HIP(launch_fill_u32(v.stats, 7, 0u, s), "clear closure stats");
    return BZ_OK;
}

}  // extern "C"
