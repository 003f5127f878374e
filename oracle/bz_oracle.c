/*
 * FP64 CPU oracle for the conservative spectral collision operator of
 * Gamba-Tharkabhushanam as used by Haack & Gamba (arXiv:1211.0540).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  The product path
 * (the HIP library) shares no code, header, table or constant with it.
 *
 * Every routine is written from the paper's definitions, in FP64, with no
 * blocking, fusion or reordering beyond what the definition states:
 *   - mesh                      : Sec. 3.1, eq. (meshpoints)
 *   - Fourier transform         : Sec. 2.2 (the choice of test function
 *                                 phi = exp(-i zeta.v)/(2 pi)^{3/2}), sampled
 *                                 with the uniform trapezoid rule (Sec. 3.2)
 *   - convolution weights       : Sec. 2.2 eq. (GHat_calc), cut off at r0 = L
 *                                 (Sec. 3.1), by Gauss-Legendre quadrature
 *   - weighted convolution      : Sec. 3.2, trapezoid sum with fhat = 0
 *                                 outside the Fourier box
 *   - conservation projection   : Sec. 3.3, solved by Lagrange multipliers
 *                                 with a 5x5 Gaussian elimination
 *   - time integration          : Sec. 3.1 (Heun second-order Runge-Kutta)
 *   - transport / wall          : Sec. 3.4 eq. (upwind), Sec. 2.1 eq. (BC)
 *
 * Readings where the paper is silent or garbled (beta = 1, the sign of the
 * projection, uniform quadrature weights, the real part of the inverse
 * transform, Heun for RK2, T(dt/2) C(dt) T(dt/2) for Strang) are the ones
 * stated in the design notes; each is repeated at the routine it affects.
 *
 * Complex arrays are interleaved (re, im) doubles.  Cell layout is the flat
 * index (k1*N + k2)*N + k3 with v_k = dv*(k - N/2).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define BZO_PI 3.14159265358979323846264338327950288

/* Planted-mistake switch for the pin tests (always 0 outside them):
 *   1 drop the loss term of Ghat        2 swap the roles of xi and zeta in Ghat
 *   3 wrong partner index j = k + m - N/2  4 drop dv^3 from the forward transform
 *   5 flip the sign of the projection   6 conjugate the partner fhat
 *   7 inelastic weights: drop beta from the first sinc                          */
int bzo_mutation = 0;
void bzo_set_mutation(int m) { bzo_mutation = m; }

/* ------------------------------------------------------------------ */
/* Mesh: Sec. 3.1 eq. (meshpoints).  dv = 2L/N, dzeta = pi/L,         */
/* v_k = dv (k - N/2), zeta_k = dzeta (k - N/2), k = 0..N-1.          */
/* ------------------------------------------------------------------ */
int bzo_grid(int N, double L, double *v, double *zeta, double *dv, double *dzeta)
{
    if (N < 2 || (N & 1) || !(L > 0)) return -1;
    double h = 2.0 * L / N, hz = BZO_PI / L;
    for (int k = 0; k < N; ++k) {
        if (v) v[k] = h * (k - N / 2);
        if (zeta) zeta[k] = hz * (k - N / 2);
    }
    if (dv) *dv = h;
    if (dzeta) *dzeta = hz;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Gauss-Legendre nodes/weights on [-1, 1] by Newton iteration on the */
/* three-term recurrence of the Legendre polynomials.                  */
/* ------------------------------------------------------------------ */
static void legendre_eval(int n, double z, double *pn, double *dpn)
{
    /* P_n(z) and P_n'(z) by the recurrence (k) P_k = (2k-1) z P_{k-1} - (k-1) P_{k-2} */
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    *pn = p1;
    *dpn = n * (z * p1 - p0) / (z * z - 1.0);
}

int bzo_gauss_legendre(int n, double *x, double *w)
{
    if (n < 1) return -1;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = cos(BZO_PI * (i + 0.75) / (n + 0.5));
        double p0, p1, dp;
        for (int it = 0; it < 100; ++it) {
            legendre_eval(n, z, &p1, &dp);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) <= 1e-15) break;
        }
        legendre_eval(n, z, &p0, &dp);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
    return 0;
}

static double sinc(double x) { return x == 0.0 ? 1.0 : sin(x) / x; }

/* ------------------------------------------------------------------ */
/* Convolution weights, Sec. 2.2 eq. (GHat_calc), isotropic b = 1/4pi, */
/* for any lambda > -3 (the text after the equation: a one-dimensional   */
/* integral for other values of lambda, evaluated by quadrature).  The   */
/* default rule is Gauss-Legendre with the factor r^{lambda+2} folded    */
/* into the weights, exact enough for the integer lambda = 0, 1; for other */
/* lambda the Python side passes a Gauss-Jacobi rule whose weight is     */
/* r^{lambda+2} itself (bzo_ctx_create_q, bzo_ghat_q).                   */
/* beta = 1 (elastic law of eq. (velocity_interact)), integral cut off */
/* at r0 = L (Sec. 3.1).  The two pieces are returned separately:       */
/*   gain(|zeta|, |xi - zeta/2|) = int_0^L r^{l+2} sinc(r|zeta|/2)      */
/*                                          sinc(r|xi - zeta/2|) dr     */
/*   loss(|xi|)                  = int_0^L r^{l+2} sinc(r|xi|) dr       */
/* and Ghat = 4 pi / (2 pi)^{3/2} (gain - loss).                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int n;
    double *x, *w; /* nodes and weights mapped to [0, L], weight includes r^{l+2} */
} quad_t;

static int quad_init(quad_t *q, int n, double L, double lambda)
{
    q->n = n;
    q->x = (double *)malloc(sizeof(double) * n);
    q->w = (double *)malloc(sizeof(double) * n);
    if (!q->x || !q->w) return -1;
    bzo_gauss_legendre(n, q->x, q->w);
    for (int i = 0; i < n; ++i) {
        double r = 0.5 * L * (q->x[i] + 1.0);
        q->x[i] = r;
        q->w[i] = 0.5 * L * q->w[i] * pow(r, lambda + 2.0);
    }
    return 0;
}

/* Explicit radial rule: n nodes r_i in [0, L] and weights that already hold
 * the factor r^{lambda+2} (for a weight the nodes integrate exactly). */
static int quad_init_explicit(quad_t *q, int n, const double *r, const double *w)
{
    q->n = n;
    q->x = (double *)malloc(sizeof(double) * n);
    q->w = (double *)malloc(sizeof(double) * n);
    if (!q->x || !q->w) return -1;
    memcpy(q->x, r, sizeof(double) * n);
    memcpy(q->w, w, sizeof(double) * n);
    return 0;
}

static void quad_free(quad_t *q) { free(q->x); free(q->w); }

static double quad_gain(const quad_t *q, double zeta_abs, double xh_abs)
{
    double s = 0.0;
    for (int i = 0; i < q->n; ++i) {
        double r = q->x[i];
        s += q->w[i] * sinc(0.5 * r * zeta_abs) * sinc(r * xh_abs);
    }
    return s;
}

static double quad_loss(const quad_t *q, double xi_abs)
{
    double s = 0.0;
    for (int i = 0; i < q->n; ++i) s += q->w[i] * sinc(q->x[i] * xi_abs);
    return s;
}

static double ghat_with(const quad_t *q, const double *xi, const double *zeta);

/* Ghat(xi, zeta) for explicit vectors, by quadrature with nq nodes. */
double bzo_ghat(const double *xi, const double *zeta, double lambda, double L, int nq)
{
    quad_t q;
    if (quad_init(&q, nq, L, lambda)) return NAN;
    double g = ghat_with(&q, xi, zeta);
    quad_free(&q);
    return g;
}

/* Same with an explicit radial rule (nodes in [0, L], weights holding r^{lambda+2}). */
double bzo_ghat_q(const double *xi, const double *zeta, int n, const double *r, const double *w)
{
    quad_t q;
    if (quad_init_explicit(&q, n, r, w)) return NAN;
    double g = ghat_with(&q, xi, zeta);
    quad_free(&q);
    return g;
}

static double ghat_with(const quad_t *q, const double *xi, const double *zeta)
{
    double za = 0, xh = 0, xa = 0;
    for (int d = 0; d < 3; ++d) {
        za += zeta[d] * zeta[d];
        double t = xi[d] - 0.5 * zeta[d];
        xh += t * t;
        xa += xi[d] * xi[d];
    }
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
    return c0 * (quad_gain(q, sqrt(za), sqrt(xh)) - quad_loss(q, sqrt(xa)));
}

/* The integrand depends on (xi, zeta) only through |zeta|, |xi - zeta/2| and
 * |xi|.  On the mesh these are dzeta*sqrt(na), (dzeta/2)*sqrt(nb) and
 * dzeta*sqrt(nc) for the integers
 *   na = sum (k_d - N/2)^2, nb = sum (2 m_d - k_d - N/2)^2, nc = sum (m_d - N/2)^2,
 * so the quadrature values are memoised by those integers (an exact cache,
 * not an approximation). */
typedef struct {
    int N, na_max, nb_max, nc_max;
    double *gain; /* [(na_max+1) * (nb_max+1)] */
    double *loss; /* [nc_max+1] */
} ghat_cache_t;

static int ghat_cache_fill(ghat_cache_t *c, int N, double L, const quad_t *q);

static int ghat_cache_build(ghat_cache_t *c, int N, double L, double lambda, int nq)
{
    quad_t q;
    if (quad_init(&q, nq, L, lambda)) return -1;
    int rc = ghat_cache_fill(c, N, L, &q);
    quad_free(&q);
    return rc;
}

static int ghat_cache_fill(ghat_cache_t *c, int N, double L, const quad_t *qp)
{
    double dz = BZO_PI / L;
    c->N = N;
    c->na_max = 3 * (N / 2) * (N / 2);
    c->nb_max = 3 * (N - 1) * (N - 1);
    c->nc_max = 3 * (N / 2) * (N / 2);
    size_t ng = (size_t)(c->na_max + 1) * (c->nb_max + 1);
    c->gain = (double *)malloc(sizeof(double) * ng);
    c->loss = (double *)malloc(sizeof(double) * (c->nc_max + 1));
    if (!c->gain || !c->loss) return -1;
#pragma omp parallel for schedule(dynamic, 4)
    for (int na = 0; na <= c->na_max; ++na) {
        double za = dz * sqrt((double)na);
        for (int nb = 0; nb <= c->nb_max; ++nb)
            c->gain[(size_t)na * (c->nb_max + 1) + nb] = quad_gain(qp, za, 0.5 * dz * sqrt((double)nb));
    }
    for (int nc = 0; nc <= c->nc_max; ++nc) c->loss[nc] = quad_loss(qp, dz * sqrt((double)nc));
    return 0;
}

static void ghat_cache_free(ghat_cache_t *c) { free(c->gain); free(c->loss); }

/* ------------------------------------------------------------------ */
/* Fourier transform sampled on the mesh (Sec. 2.2 / Sec. 3.2):        */
/*   fhat_k = (2pi)^{-3/2} dv^3 sum_j f_j exp(-i zeta_k . v_j)          */
/* computed as a naive sum, factorised over the three axes (the        */
/* exponential of a sum is the product of exponentials).              */
/* ------------------------------------------------------------------ */
static void dft_axis(int N, const double *in, double *out, const double *cs, const double *sn, int axis, int sign)
{
    /* out[..k..] = sum_j in[..j..] * (cs[k*N+j] + i*sign*sn[k*N+j]) along `axis` */
    int s[3] = {N * N, N, 1};
    int st = s[axis];
    int oa = (axis + 1) % 3, ob = (axis + 2) % 3;
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            size_t base = (size_t)a * s[oa] + (size_t)b * s[ob];
            for (int k = 0; k < N; ++k) {
                double re = 0.0, im = 0.0;
                for (int j = 0; j < N; ++j) {
                    double xr = in[2 * (base + (size_t)j * st)], xi = in[2 * (base + (size_t)j * st) + 1];
                    double c = cs[k * N + j], sgn = sign * sn[k * N + j];
                    re += xr * c - xi * sgn;
                    im += xr * sgn + xi * c;
                }
                out[2 * (base + (size_t)k * st)] = re;
                out[2 * (base + (size_t)k * st) + 1] = im;
            }
        }
}

static void phase_tables(int N, double L, double **cs, double **sn)
{
    double v[64], z[64], dv, dz;
    bzo_grid(N, L, v, z, &dv, &dz);
    *cs = (double *)malloc(sizeof(double) * N * N);
    *sn = (double *)malloc(sizeof(double) * N * N);
    for (int k = 0; k < N; ++k)
        for (int j = 0; j < N; ++j) {
            double a = z[k] * v[j];
            (*cs)[k * N + j] = cos(a);
            (*sn)[k * N + j] = sin(a);
        }
}

/* f: M real values -> fhat: M complex (interleaved). */
int bzo_dft_forward(int N, double L, const double *f, double *fhat)
{
    if (N < 2 || N > 64 || (N & 1)) return -1;
    size_t M = (size_t)N * N * N;
    double *a = (double *)calloc(2 * M, sizeof(double));
    double *b = (double *)calloc(2 * M, sizeof(double));
    double *cs, *sn;
    phase_tables(N, L, &cs, &sn);
    for (size_t i = 0; i < M; ++i) a[2 * i] = f[i];
    dft_axis(N, a, b, cs, sn, 2, -1);
    dft_axis(N, b, a, cs, sn, 1, -1);
    dft_axis(N, a, b, cs, sn, 0, -1);
    double dv = 2.0 * L / N;
    double c = pow(2.0 * BZO_PI, -1.5) * dv * dv * dv;
    if (bzo_mutation == 4) c = pow(2.0 * BZO_PI, -1.5);
    for (size_t i = 0; i < 2 * M; ++i) fhat[i] = c * b[i];
    free(a); free(b); free(cs); free(sn);
    return 0;
}

/* Inverse transform (Sec. 3.2):
 *   Qt_j = Re[ (2pi)^{-3/2} dzeta^3 sum_k Qhat_k exp(+i zeta_k . v_j) ]
 * The asymmetric mesh (k - N/2 in [-N/2, N/2-1]) breaks Hermitian symmetry
 * at the Nyquist planes, so the sum is not exactly real; the real part is
 * kept and the largest |imaginary part| is reported in *max_imag. */
int bzo_dft_inverse(int N, double L, const double *qhat, double *qt, double *max_imag)
{
    if (N < 2 || N > 64 || (N & 1)) return -1;
    size_t M = (size_t)N * N * N;
    double *a = (double *)malloc(sizeof(double) * 2 * M);
    double *b = (double *)malloc(sizeof(double) * 2 * M);
    double *cs, *sn;
    phase_tables(N, L, &cs, &sn);
    memcpy(a, qhat, sizeof(double) * 2 * M);
    dft_axis(N, a, b, cs, sn, 2, +1);
    dft_axis(N, b, a, cs, sn, 1, +1);
    dft_axis(N, a, b, cs, sn, 0, +1);
    double dz = BZO_PI / L;
    double c = pow(2.0 * BZO_PI, -1.5) * dz * dz * dz;
    double mi = 0.0;
    for (size_t i = 0; i < M; ++i) {
        qt[i] = c * b[2 * i];
        double im = fabs(c * b[2 * i + 1]);
        if (im > mi) mi = im;
    }
    if (max_imag) *max_imag = mi;
    free(a); free(b); free(cs); free(sn);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Weighted convolution, Sec. 3.2:                                      */
/*   Qhat(zeta_k) = sum_m Ghat(xi_m, zeta_k) fhat(xi_m) fhat(zeta_k - xi_m) w_m */
/* with the uniform trapezoid weight w_m = dzeta^3 and fhat(zeta_k - xi_m) */
/* = 0 when zeta_k - xi_m leaves the Fourier box.  On the mesh           */
/* zeta_k - xi_m = dzeta ((k - m + N/2) - N/2), i.e. the mesh point with  */
/* index j = k - m + N/2, which must lie in [0, N-1] on every axis.       */
/* Parallel over zeta (one output per OpenMP iteration, as in Sec. 4).    */
/* ------------------------------------------------------------------ */
typedef struct bzo_ctx_s {
    int N;
    double L, lambda;
    int nq;
    ghat_cache_t cache;
} bzo_ctx;

bzo_ctx *bzo_ctx_create(int N, double L, double lambda, int nq)
{
    if (N < 2 || N > 64 || (N & 1) || !(L > 0)) return NULL;
    bzo_ctx *c = (bzo_ctx *)calloc(1, sizeof(bzo_ctx));
    c->N = N; c->L = L; c->lambda = lambda; c->nq = nq > 0 ? nq : 400;
    if (ghat_cache_build(&c->cache, N, L, lambda, c->nq)) { free(c); return NULL; }
    return c;
}

/* Context whose weight cache comes from an explicit radial rule (see bzo_ghat_q). */
bzo_ctx *bzo_ctx_create_q(int N, double L, double lambda, int n, const double *r, const double *w)
{
    if (N < 2 || N > 64 || (N & 1) || !(L > 0) || n < 1) return NULL;
    bzo_ctx *c = (bzo_ctx *)calloc(1, sizeof(bzo_ctx));
    c->N = N; c->L = L; c->lambda = lambda; c->nq = n;
    quad_t q;
    if (quad_init_explicit(&q, n, r, w)) { free(c); return NULL; }
    int rc = ghat_cache_fill(&c->cache, N, L, &q);
    quad_free(&q);
    if (rc) { free(c); return NULL; }
    return c;
}

void bzo_ctx_free(bzo_ctx *c)
{
    if (!c) return;
    ghat_cache_free(&c->cache);
    free(c);
}

/* Ghat for mesh indices k (zeta) and m (xi), from the memoised quadrature. */
double bzo_ctx_ghat(const bzo_ctx *c, const int *k, const int *m)
{
    int N = c->N, h = N / 2;
    long na = 0, nb = 0, nc = 0;
    for (int d = 0; d < 3; ++d) {
        long a = k[d] - h, b = 2 * m[d] - k[d] - h, e = m[d] - h;
        na += a * a; nb += b * b; nc += e * e;
        int j = k[d] - m[d] + h;
        if (k[d] < 0 || k[d] >= N || m[d] < 0 || m[d] >= N || j < 0 || j >= N) return NAN;
    }
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
    return c0 * (c->cache.gain[(size_t)na * (c->cache.nb_max + 1) + nb] - c->cache.loss[nc]);
}

static double mutated_weight(const bzo_ctx *c, const int *k, const int *m)
{
    int N = c->N, h = N / 2;
    long na = 0, nb = 0, nc = 0;
    for (int d = 0; d < 3; ++d) {
        long a = k[d] - h, b = 2 * m[d] - k[d] - h, e = m[d] - h;
        if (bzo_mutation == 2) { a = m[d] - h; b = 2 * k[d] - m[d] - h; e = k[d] - h; }
        na += a * a; nb += b * b; nc += e * e;
    }
    if (na > c->cache.na_max || nb > c->cache.nb_max || nc > c->cache.nc_max) return 0.0;
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
    double loss = bzo_mutation == 1 ? 0.0 : c->cache.loss[nc];
    return c0 * (c->cache.gain[(size_t)na * (c->cache.nb_max + 1) + nb] - loss);
}

int bzo_collide_hat(const bzo_ctx *c, const double *fhat, double *qhat, long long *pairs)
{
    int N = c->N, h = N / 2;
    size_t M = (size_t)N * N * N;
    double dz = BZO_PI / c->L;
    double w = dz * dz * dz;
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
    int nbs = c->cache.nb_max + 1;
    long long npairs = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : npairs)
    for (long kk = 0; kk < (long)M; ++kk) {
        int k1 = (int)(kk / (N * N)), k2 = (int)((kk / N) % N), k3 = (int)(kk % N);
        long na = (long)(k1 - h) * (k1 - h) + (long)(k2 - h) * (k2 - h) + (long)(k3 - h) * (k3 - h);
        const double *grow = c->cache.gain + (size_t)na * nbs;
        double re = 0.0, im = 0.0;
        for (int m1 = 0; m1 < N; ++m1) {
            int j1 = k1 - m1 + h;
            if (j1 < 0 || j1 >= N) continue;
            for (int m2 = 0; m2 < N; ++m2) {
                int j2 = k2 - m2 + h;
                if (j2 < 0 || j2 >= N) continue;
                for (int m3 = 0; m3 < N; ++m3) {
                    int j3 = k3 - m3 + h;
                    if (j3 < 0 || j3 >= N) continue;
                    long b1 = 2 * m1 - k1 - h, b2 = 2 * m2 - k2 - h, b3 = 2 * m3 - k3 - h;
                    long e1 = m1 - h, e2 = m2 - h, e3 = m3 - h;
                    double G = c0 * (grow[b1 * b1 + b2 * b2 + b3 * b3] - c->cache.loss[e1 * e1 + e2 * e2 + e3 * e3]);
                    size_t im_ = ((size_t)m1 * N + m2) * N + m3;
                    size_t ij_ = ((size_t)j1 * N + j2) * N + j3;
                    if (bzo_mutation) {
                        int kk3[3] = {k1, k2, k3}, mm3[3] = {m1, m2, m3};
                        G = mutated_weight(c, kk3, mm3);
                        if (bzo_mutation == 3) {
                            int q1 = k1 + m1 - h, q2 = k2 + m2 - h, q3 = k3 + m3 - h;
                            if (q1 < 0 || q1 >= N || q2 < 0 || q2 >= N || q3 < 0 || q3 >= N) continue;
                            ij_ = ((size_t)q1 * N + q2) * N + q3;
                        }
                    }
                    double ar = fhat[2 * im_], ai = fhat[2 * im_ + 1];
                    double br = fhat[2 * ij_], bi = fhat[2 * ij_ + 1];
                    if (bzo_mutation == 6) bi = -bi;
                    re += G * (ar * br - ai * bi);
                    im += G * (ar * bi + ai * br);
                    ++npairs;
                }
            }
        }
        qhat[2 * kk] = w * re;
        qhat[2 * kk + 1] = w * im;
    }
    if (pairs) *pairs = npairs;
    return 0;
}

/* Diagnostic for floating-point tolerances: out[k] = dzeta^3 sum_m |Ghat| |fhat_m| |fhat_j|,
 * the sum of the magnitudes of the terms of the convolution at zeta_k.  The ratio of its
 * norm to the norm of Qhat measures how much the terms cancel. */
int bzo_collide_hat_abs(const bzo_ctx *c, const double *fhat, double *out)
{
    int N = c->N, h = N / 2;
    size_t M = (size_t)N * N * N;
    double dz = BZO_PI / c->L;
    double w = dz * dz * dz;
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
    int nbs = c->cache.nb_max + 1;
#pragma omp parallel for schedule(dynamic, 16)
    for (long kk = 0; kk < (long)M; ++kk) {
        int k1 = (int)(kk / (N * N)), k2 = (int)((kk / N) % N), k3 = (int)(kk % N);
        long na = (long)(k1 - h) * (k1 - h) + (long)(k2 - h) * (k2 - h) + (long)(k3 - h) * (k3 - h);
        const double *grow = c->cache.gain + (size_t)na * nbs;
        double s = 0.0;
        for (int m1 = 0; m1 < N; ++m1) {
            int j1 = k1 - m1 + h;
            if (j1 < 0 || j1 >= N) continue;
            for (int m2 = 0; m2 < N; ++m2) {
                int j2 = k2 - m2 + h;
                if (j2 < 0 || j2 >= N) continue;
                for (int m3 = 0; m3 < N; ++m3) {
                    int j3 = k3 - m3 + h;
                    if (j3 < 0 || j3 >= N) continue;
                    long b1 = 2 * m1 - k1 - h, b2 = 2 * m2 - k2 - h, b3 = 2 * m3 - k3 - h;
                    long e1 = m1 - h, e2 = m2 - h, e3 = m3 - h;
                    double G = c0 * (grow[b1 * b1 + b2 * b2 + b3 * b3] - c->cache.loss[e1 * e1 + e2 * e2 + e3 * e3]);
                    size_t im_ = ((size_t)m1 * N + m2) * N + m3;
                    size_t ij_ = ((size_t)j1 * N + j2) * N + j3;
                    s += fabs(G) * hypot(fhat[2 * im_], fhat[2 * im_ + 1]) * hypot(fhat[2 * ij_], fhat[2 * ij_ + 1]);
                }
            }
        }
        out[kk] = w * s;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Conservation, Sec. 3.3.  C (5 x M) has rows w_j, v^i_j w_j, |v_j|^2 w_j */
/* with w_j = dv^3.  The minimiser of |Qt - Q|^2 / 2 subject to CQ = 0 is   */
/* Q = Qt - C^T (C C^T)^{-1} C Qt (Lagrange multipliers; the printed       */
/* formula has the opposite sign and a transposed C).  The 5x5 system is   */
/* solved by Gaussian elimination with partial pivoting plus one step of   */
/* iterative refinement.                                                    */
/* ------------------------------------------------------------------ */
static void constraint_row(int N, double L, size_t j, double *row)
{
    double v[64], dv;
    bzo_grid(N, L, v, NULL, &dv, NULL);
    int j1 = (int)(j / ((size_t)N * N)), j2 = (int)((j / N) % N), j3 = (int)(j % N);
    double w = dv * dv * dv;
    row[0] = w;
    row[1] = v[j1] * w;
    row[2] = v[j2] * w;
    row[3] = v[j3] * w;
    row[4] = (v[j1] * v[j1] + v[j2] * v[j2] + v[j3] * v[j3]) * w;
}

/* n x n system (n <= 5), Gaussian elimination with partial pivoting. */
static int gauss_solve(int n, const double *A_in, const double *b_in, double *x)
{
    double A[5][6];
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j < n; ++j) A[i][j] = A_in[i * n + j];
        A[i][n] = b_in[i];
    }
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(A[r][col]) > fabs(A[p][col])) p = r;
        if (A[p][col] == 0.0) return -1;
        if (p != col)
            for (int j = 0; j <= n; ++j) { double t = A[col][j]; A[col][j] = A[p][j]; A[p][j] = t; }
        for (int r = col + 1; r < n; ++r) {
            double f = A[r][col] / A[col][col];
            for (int j = col; j <= n; ++j) A[r][j] -= f * A[col][j];
        }
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = A[i][n];
        for (int j = i + 1; j < n; ++j) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
    return 0;
}

/* Projection onto the first `nrows` constraints: 5 (mass, momentum, energy) for
 * elastic collisions, 4 (mass, momentum) for inelastic ones, which do not
 * preserve energy (Sec. 3.3). */
int bzo_project_rows(int N, double L, int nrows, const double *qt, double *q, double *lambda_out)
{
    if (nrows < 1 || nrows > 5) return -1;
    size_t M = (size_t)N * N * N;
    const int n = nrows;
    double G[25] = {0}, mu[5] = {0};
    for (size_t j = 0; j < M; ++j) {
        double r[5];
        constraint_row(N, L, j, r);
        for (int a = 0; a < n; ++a) {
            mu[a] += r[a] * qt[j];
            for (int b = 0; b < n; ++b) G[a * n + b] += r[a] * r[b];
        }
    }
    double lam[5] = {0}, res[5], dl[5];
    if (gauss_solve(n, G, mu, lam)) return -1;
    for (int a = 0; a < n; ++a) {
        res[a] = mu[a];
        for (int b = 0; b < n; ++b) res[a] -= G[a * n + b] * lam[b];
    }
    if (gauss_solve(n, G, res, dl)) return -1;
    for (int a = 0; a < n; ++a) lam[a] += dl[a];
    for (size_t j = 0; j < M; ++j) {
        double r[5];
        constraint_row(N, L, j, r);
        double s = 0.0;
        for (int a = 0; a < n; ++a) s += r[a] * lam[a];
        q[j] = bzo_mutation == 5 ? qt[j] + s : qt[j] - s;
    }
    if (lambda_out) memcpy(lambda_out, lam, sizeof(double) * n);
    return 0;
}

int bzo_project(int N, double L, const double *qt, double *q, double *lambda_out)
{
    return bzo_project_rows(N, L, 5, qt, q, lambda_out);
}

/* ------------------------------------------------------------------ */
/* Inelastic collisions: eq. (GHat_calc) with the factor beta of eq.    */
/* (G_eqn) kept (beta = 1 is the elastic law; beta < 1 loses energy):   */
/*   Ghat = 4pi (2pi)^{-3/2} int_0^L r^{lambda+2} [sinc(beta r|zeta|/2)   */
/*          sinc(r |xi - beta zeta/2|) - sinc(r |xi|)] dr.                 */
/* On the mesh |zeta|^2 = dzeta^2 na, |xi|^2 = dzeta^2 nc and            */
/* |xi - beta zeta/2|^2 = dzeta^2 (nc - beta d + beta^2 na / 4) with the  */
/* integer d = (m - N/2).(k - N/2): the gain integrals are memoised by    */
/* (na, nc, d), computed for the triples the sum meets.                  */
/* ------------------------------------------------------------------ */
typedef struct bzo_inel_s {
    int N;
    double L, beta;
    int nmax, dmax;
    double *gain;   /* [(nmax+1)][(nmax+1)][2 dmax + 1], NaN where unused */
    double *loss;   /* [nmax+1] */
} bzo_inel;

static size_t inel_idx(const bzo_inel *c, long na, long nc, long d)
{
    return ((size_t)na * (c->nmax + 1) + (size_t)nc) * (2 * c->dmax + 1) + (size_t)(d + c->dmax);
}

bzo_inel *bzo_inel_create(int N, double L, double beta, int n, const double *r, const double *w)
{
    if (N < 2 || N > 32 || (N & 1) || !(L > 0) || !(beta > 0) || n < 1) return NULL;
    bzo_inel *c = (bzo_inel *)calloc(1, sizeof(bzo_inel));
    int h = N / 2;
    c->N = N; c->L = L; c->beta = beta;
    c->nmax = 3 * h * h;
    c->dmax = 3 * h * h;
    size_t ng = (size_t)(c->nmax + 1) * (c->nmax + 1) * (2 * c->dmax + 1);
    c->gain = (double *)malloc(sizeof(double) * ng);
    c->loss = (double *)malloc(sizeof(double) * (c->nmax + 1));
    unsigned char *used = (unsigned char *)calloc(ng, 1);
    quad_t q;
    if (!c->gain || !c->loss || !used || quad_init_explicit(&q, n, r, w)) return NULL;
    /* mark the (na, nc, d) the sum meets */
    for (int k1 = 0; k1 < N; ++k1) for (int k2 = 0; k2 < N; ++k2) for (int k3 = 0; k3 < N; ++k3) {
        int k[3] = {k1, k2, k3};
        long na = 0;
        for (int e = 0; e < 3; ++e) na += (long)(k[e] - h) * (k[e] - h);
        for (int m1 = 0; m1 < N; ++m1) for (int m2 = 0; m2 < N; ++m2) for (int m3 = 0; m3 < N; ++m3) {
            int m[3] = {m1, m2, m3};
            long nc = 0, d = 0;
            int ok = 1;
            for (int e = 0; e < 3; ++e) {
                int j = k[e] - m[e] + h;
                if (j < 0 || j >= N) ok = 0;
                nc += (long)(m[e] - h) * (m[e] - h);
                d += (long)(m[e] - h) * (k[e] - h);
            }
            if (ok) used[inel_idx(c, na, nc, d)] = 1;
        }
    }
    double dz = BZO_PI / L;
#pragma omp parallel for schedule(dynamic, 1)
    for (long na = 0; na <= c->nmax; ++na)
        for (long nc = 0; nc <= c->nmax; ++nc)
            for (long d = -c->dmax; d <= c->dmax; ++d) {
                size_t i = inel_idx(c, na, nc, d);
                if (!used[i]) { c->gain[i] = NAN; continue; }
                double xh2 = (double)nc - beta * (double)d + 0.25 * beta * beta * (double)na;
                double xh = dz * sqrt(xh2 > 0.0 ? xh2 : 0.0);
                double za = beta * dz * sqrt((double)na);   /* quad_gain halves it: sinc(beta r |zeta| / 2) */
                c->gain[i] = bzo_mutation == 7 ? quad_gain(&q, dz * sqrt((double)na), xh) : quad_gain(&q, za, xh);
            }
    for (long nc = 0; nc <= c->nmax; ++nc) c->loss[nc] = quad_loss(&q, dz * sqrt((double)nc));
    quad_free(&q);
    free(used);
    return c;
}

void bzo_inel_free(bzo_inel *c)
{
    if (!c) return;
    free(c->gain); free(c->loss); free(c);
}

/* Qhat of Sec. 3.2 with the inelastic weights (same trapezoid sum as bzo_collide_hat). */
int bzo_inel_collide_hat(const bzo_inel *c, const double *fhat, double *qhat)
{
    int N = c->N, h = N / 2;
    size_t M = (size_t)N * N * N;
    double dz = BZO_PI / c->L;
    double w = dz * dz * dz;
    double c0 = 4.0 * BZO_PI / pow(2.0 * BZO_PI, 1.5);
#pragma omp parallel for schedule(dynamic, 16)
    for (long kk = 0; kk < (long)M; ++kk) {
        int k[3] = {(int)(kk / (N * N)), (int)((kk / N) % N), (int)(kk % N)};
        long na = 0;
        for (int e = 0; e < 3; ++e) na += (long)(k[e] - h) * (k[e] - h);
        double re = 0.0, im = 0.0;
        for (int m1 = 0; m1 < N; ++m1) for (int m2 = 0; m2 < N; ++m2) for (int m3 = 0; m3 < N; ++m3) {
            int m[3] = {m1, m2, m3}, j[3];
            long nc = 0, d = 0;
            int ok = 1;
            for (int e = 0; e < 3; ++e) {
                j[e] = k[e] - m[e] + h;
                if (j[e] < 0 || j[e] >= N) ok = 0;
                nc += (long)(m[e] - h) * (m[e] - h);
                d += (long)(m[e] - h) * (k[e] - h);
            }
            if (!ok) continue;
            double G = c0 * (c->gain[inel_idx(c, na, nc, d)] - c->loss[nc]);
            size_t im_ = ((size_t)m1 * N + m2) * N + m3;
            size_t ij_ = ((size_t)j[0] * N + j[1]) * N + j[2];
            double ar = fhat[2 * im_], ai = fhat[2 * im_ + 1];
            double br = fhat[2 * ij_], bi = fhat[2 * ij_ + 1];
            re += G * (ar * br - ai * bi);
            im += G * (ar * bi + ai * br);
        }
        qhat[2 * kk] = w * re;
        qhat[2 * kk + 1] = w * im;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Whole collision step for one cell: f -> Qt (unprojected) and Q.      */
/* ------------------------------------------------------------------ */
int bzo_collide(const bzo_ctx *c, const double *f, double *qt, double *q, double *max_imag, long long *pairs)
{
    int N = c->N;
    size_t M = (size_t)N * N * N;
    double *fh = (double *)malloc(sizeof(double) * 2 * M);
    double *qh = (double *)malloc(sizeof(double) * 2 * M);
    double *tmp = qt ? qt : (double *)malloc(sizeof(double) * M);
    int rc = bzo_dft_forward(N, c->L, f, fh);
    if (!rc) rc = bzo_collide_hat(c, fh, qh, pairs);
    if (!rc) rc = bzo_dft_inverse(N, c->L, qh, tmp, max_imag);
    if (!rc && q) rc = bzo_project(N, c->L, tmp, q, NULL);
    if (!qt) free(tmp);
    free(fh); free(qh);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Space-homogeneous time integration df/dt = Q(f,f)/eps with Heun's     */
/* second-order Runge-Kutta (Sec. 3.1 names "second-order Runge-Kutta";  */
/* Heun is the reading used):                                            */
/*   f*      = f + (dt/eps) Q(f)                                         */
/*   f^{n+1} = (f + f* + (dt/eps) Q(f*)) / 2                              */
/* Q is the projected operator.  `cells` independent cells of the same  */
/* mesh are advanced `steps` times in place.                             */
/* ------------------------------------------------------------------ */
int bzo_rk2_homogeneous(const bzo_ctx *c, double *f, int cells, double dt, double eps, int steps)
{
    size_t M = (size_t)c->N * c->N * c->N;
    double *q = (double *)malloc(sizeof(double) * M);
    double *fs = (double *)malloc(sizeof(double) * M);
    int rc = 0;
    for (int s = 0; s < steps && !rc; ++s)
        for (int cc = 0; cc < cells && !rc; ++cc) {
            double *fc = f + (size_t)cc * M;
            rc = bzo_collide(c, fc, NULL, q, NULL, NULL);
            for (size_t i = 0; i < M && !rc; ++i) fs[i] = fc[i] + dt / eps * q[i];
            if (!rc) rc = bzo_collide(c, fs, NULL, q, NULL, NULL);
            for (size_t i = 0; i < M && !rc; ++i) fc[i] = 0.5 * (fc[i] + fs[i] + dt / eps * q[i]);
        }
    free(q); free(fs);
    return rc;
}

int bzo_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
