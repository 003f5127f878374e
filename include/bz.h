/*
 * bz.h - C ABI of the MI355X (gfx950) conservative spectral collision library.
 *
 * The library computes, for every spatial cell of a batch, the collision
 * operator of the conservative spectral method of Gamba and Tharkabhushanam
 * as extended by Haack & Gamba (arXiv:1211.0540):
 *
 *   fhat   = F[f]                        Fourier transform on the mesh (Sec. 2.2, 3.2)
 *   Qhat_k = sum_m Ghat(xi_m, zeta_k) fhat_m fhat_{k-m+N/2} dzeta^3
 *                                         trapezoid-rule weighted convolution (Sec. 3.2)
 *   Qt     = Re F^{-1}[Qhat]              inverse transform (Sec. 3.2)
 *   Q      = Qt - C^T (C C^T)^{-1} C Qt   conservation projection (Sec. 3.3)
 *
 * with the weights Ghat of eq. (GHat_calc) (isotropic scattering, b = 1/4pi,
 * elastic collisions beta = 1, radial cut-off r0 = L).
 *
 * Conventions for every entry point:
 *   - Mesh (Sec. 3.1): N a multiple of 4, 8 <= N <= 32, half-width L > 0;
 *     v_k = (2L/N)(k - N/2), zeta_k = (pi/L)(k - N/2), k = 0..N-1.
 *   - A cell is N^3 FP64 values, C-contiguous, flat index (k1*N + k2)*N + k3;
 *     axis 1 is the transport direction v1.  The cells of a batch are stored
 *     back to back in the order given at batch creation.
 *   - Pointers named d_* are device pointers (HIP device memory, 256-byte
 *     aligned is sufficient); everything else is host memory.
 *   - The caller owns every device buffer (distribution functions, results,
 *     weights, workspace).  The library owns only its opaque handles and a
 *     few kilobytes of device index tables per batch, released by *_free.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default
 *     stream.  Calls enqueue work and return without synchronising unless
 *     stated otherwise.
 *   - Arguments are validated on the host before anything is enqueued: a
 *     call that returns an error has no side effect.  No C++ exception
 *     crosses this interface.  bz_last_error() returns a thread-local message
 *     for the last failing call of the calling thread.
 *   - Threads: a mesh handle is immutable after bz_grid_init and may be
 *     shared.  A batch handle carries per-call state (chosen kernel variants,
 *     timing events, the closure's judge rotation and its second stream), so
 *     the calls on one batch must not overlap in time from several host
 *     threads; distinct batches are independent.  Calls that enqueue on one
 *     batch with the same workspace on different streams race on the
 *     workspace, as any two kernels writing one buffer would.
 */
#ifndef BZ_H
#define BZ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BZ_API_VERSION 3

typedef enum {
    BZ_OK = 0,
    BZ_EINVAL = -1,        /* invalid argument (message in bz_last_error) */
    BZ_EUNSUPPORTED = -2,  /* valid request this build does not implement */
    BZ_EDEVICE = -3,       /* a HIP runtime call failed */
    BZ_ENOMEM = -4,        /* host or device allocation failed */
    BZ_ENONFINITE = -5,    /* a non-finite value was produced */
    BZ_ESTATE = -6         /* call out of order (e.g. weights not bound) */
} bz_status;

/* Weight buffer kinds: arithmetic type and the schedule the buffer is laid out for. */
enum {
    BZ_W_BATCHED_F32 = 1,  /* symmetric pair weights, wave-uniform order, FP32 */
    BZ_W_BATCHED_F64 = 2,  /* same, FP64 */
    BZ_W_PLAIN_F32 = 3,    /* per-output weights, one cell at a time, FP32 */
    BZ_W_PLAIN_F64 = 4     /* same, FP64 */
};

/* Collision modes. */
enum {
    BZ_MODE_PLAIN_F64 = 1,    /* FP64, one cell per launch: the plain baseline */
    BZ_MODE_BATCHED_F32 = 2,  /* FP32 products with compensated accumulation,
                                 all cells of a mesh in one persistent launch */
    BZ_MODE_BATCHED_F64 = 3,  /* FP64, all cells of a mesh in one launch */
    BZ_MODE_PLAIN_F32 = 4     /* FP32 + compensated accumulation, one cell per launch */
};

/* ------------------------------------------------------------------ */
/* Mesh (Sec. 3.1 eq. meshpoints; Sec. 3.3 constraint matrix C)         */
/* ------------------------------------------------------------------ */
typedef struct bz_grid_s *bz_grid;

typedef struct {
    int N;               /* points per axis */
    double L;            /* half-width of the velocity cube [-L, L)^3 */
    double lambda;       /* exponent of |u| in B = |u|^lambda b, in (-3, 1] (0: Maxwell molecules, 1: hard spheres) */
    double dv;           /* 2L/N */
    double dzeta;        /* pi/L */
    long long pairs;     /* valid (zeta_k, xi_m) pairs of the convolution: (3N^2/4)^3 */
    int core_r2;         /* radius^2 of the FP64 core ball in index units (0: no core) */
    long long core_steps;/* steps of the core schedule (row pairs; 0 without a core) */
    double beta;         /* 1: elastic; < 1: inelastic (bz_grid_create) */
} bz_grid_info;

/* Parameters of bz_grid_create.  beta is the factor of eq. (G_eqn) and
 * (GHat_calc): 1 for the elastic interaction law of eq. (velocity_interact),
 * beta in [1/2, 1) for inelastic collisions with restitution coefficient
 * 2 beta - 1 (post-collisional velocities v' = v + (beta/2)(|u| sigma - u)).
 * Inelastic collisions do not preserve energy (Sec. 3.3): the conservation
 * projection of such a mesh keeps mass and momentum only. */
typedef struct {
    int N;
    double L;
    double lambda;
    int core_r2;         /* as for bz_grid_init_ex */
    double beta;
} bz_grid_params;

/* Low-frequency FP64 core of the batched FP32 mode.
 *
 * The terms of the sum of Sec. 3.2 are largest where both partners lie near
 * zeta = 0 (the transform of a distribution is concentrated there).  Rounding
 * fhat and the weights to FP32 perturbs each term by about 6e-8 of itself; on
 * near-equilibrium cells, whose terms cancel to a Qhat hundreds to thousands of
 * times smaller than their magnitudes, that leaves a relative error above
 * 1e-5 however the sum is accumulated.  With a core, the pairs whose two
 * partners both lie in the ball nc = |m - N/2|^2 <= core_r2 (index units) are
 * summed by a separate FP64 kernel from FP64 fhat and FP64 weights, and their
 * weights in the FP32 stream are zero: the same sum, split by frequency, each
 * term evaluated once.  The core costs a few percent of the FP32 work.  It
 * applies to BZ_MODE_BATCHED_F32 only (the FP64 modes are exact already, the
 * plain FP32 mode keeps its single stream). */
#define BZ_CORE_DEFAULT (-1)  /* nc <= ceil(L^2 sqrt(min(1, N/32))) - 1, capped as below */
#define BZ_CORE_OFF (-2)      /* no core: every pair in FP32 */

/* Create a mesh handle.  Host only, no device work.  lambda is the exponent
 * of |u| in the collision kernel (Sec. 2): -3 < lambda <= 1, i.e. soft
 * potentials (< 0), Maxwell molecules (0), variable hard potentials (0..1) and
 * hard spheres (1).  For lambda = 0 and 1 the weight integral of eq.
 * (GHat_calc) is evaluated in closed form, otherwise by quadrature (see
 * bz_weight_table).  Errors: BZ_EINVAL for N not a multiple of 4, N outside
 * [8, 32], L <= 0 or non-finite; BZ_EUNSUPPORTED for lambda outside (-3, 1]. */
bz_status bz_grid_init(int N, double L, double lambda, bz_grid *out);
/* As bz_grid_init with an explicit core: core_r2 in [1, min(N^2/4, 81) - 1]
 * (the ball stays off the k_d = 0 planes and within the kernel's half-width of
 * 8), BZ_CORE_DEFAULT (what bz_grid_init uses) or BZ_CORE_OFF.  The core is a
 * property of the mesh: it fixes the layout of its BZ_W_BATCHED_F32 weights.
 * Errors: as bz_grid_init, and BZ_EINVAL for a core_r2 out of range. */
bz_status bz_grid_init_ex(int N, double L, double lambda, int core_r2, bz_grid *out);
/* The general form: bz_grid_init_ex with beta.  With beta < 1 the gain part
 * of every weight, sinc(beta r |zeta|/2) sinc(r |xi - beta zeta/2|), no longer
 * factors through integer norms: it is evaluated per weight slot in closed
 * form, so beta < 1 needs lambda = 0 or 1 (BZ_EUNSUPPORTED otherwise).
 * Errors: as bz_grid_init_ex, BZ_EINVAL for beta outside [1/2, 1] or NULL. */
bz_status bz_grid_create(const bz_grid_params *p, bz_grid *out);
void bz_grid_free(bz_grid g);
bz_status bz_grid_query(bz_grid g, bz_grid_info *info);
/* Host copies of the 1-D velocity and frequency nodes (N doubles each, either may be NULL). */
bz_status bz_grid_coords(bz_grid g, double *v, double *zeta);

/* ------------------------------------------------------------------ */
/* Convolution weights (Sec. 2.2 eq. GHat_calc; "precomputed once and    */
/* stored", Sec. 2.2).  The weights of a mesh factor through the integer */
/* norms na = |k - N/2|^2, nb = |2m - k - N/2|^2, nc = |m - N/2|^2 as     */
/*   Ghat = 4pi (2pi)^{-3/2} L^{lambda+3} [T(na, nb) - T(0, 4 nc)],       */
/*   T(p, q) = int_0^1 s^{lambda+2} sinc(pi s sqrt(p)/2) sinc(pi s sqrt(q)/2) ds, */
/* and are expanded into the caller's buffer in the order the chosen      */
/* schedule reads them (dzeta^3 folded in).                               */
/* ------------------------------------------------------------------ */
/* The universal table T_lambda(p, q), p = 0..3N^2/4, q = 0..3N^2, row-major
 * (bz_weight_table_size(N) doubles, 0 for a bad N), into host memory `out`.
 * For lambda = 0, 1 in closed form; otherwise
 *   T = int_0^1 s^{lambda+2} sinc(a s) sinc(b s) ds
 * by composite Gauss-Legendre quadrature: 16 nodes on each of 15 uniform
 * panels of [1/16, 1], on 40 panels [0.3^{k+1}, 0.3^k]/16 graded towards
 * s = 0 (which resolve the endpoint behaviour of s^{lambda+2}), and the exact
 * integral of s^{lambda+2} on the remaining [0, 0.3^40/16].  Host only,
 * threaded.  Errors: BZ_EINVAL for a bad N or NULL, BZ_EUNSUPPORTED for
 * lambda outside (-3, 1]. */
size_t bz_weight_table_size(int N);
bz_status bz_weight_table(int N, double lambda, double *out);

/* Bytes needed for a weight buffer of the given kind (0 for an unknown kind).
 * A batched buffer holds the weight stream of every output row in schedule
 * order and, after it, the stream of the edge pass of the conjugate-symmetric
 * schedule (bz_batch_create_ex); a BZ_W_BATCHED_F32 buffer of a mesh with a
 * core then holds the FP64 weights of the core steps. */
size_t bz_weights_bytes(bz_grid g, int kind);
/* Fill d_w (bytes >= bz_weights_bytes) on `stream`.  Synchronises the stream
 * before returning (it uploads a host-built table).  Errors: BZ_EINVAL for a
 * bad kind, NULL pointer or short buffer; BZ_EDEVICE / BZ_ENOMEM from HIP. */
bz_status bz_weights(bz_grid g, int kind, void *d_w, size_t bytes, void *stream);

/* ------------------------------------------------------------------ */
/* Batches: a fixed list of cells, each on one of a few meshes.          */
/* ------------------------------------------------------------------ */
typedef struct bz_batch_s *bz_batch;

/* grid_of_cell[c] (host, n_cells entries) indexes grids[] (host, n_grids
 * handles that must outlive the batch).  `mode` is one of BZ_MODE_*.  The
 * batch groups the cells of each mesh 64 to a wavefront (batched modes),
 * orders the work longest-first and uploads its index tables (synchronous).
 * Errors: BZ_EINVAL for n_cells < 1, a bad index or mode. */
bz_status bz_batch_create(int n_cells, const int32_t *grid_of_cell, int n_grids, const bz_grid *grids,
                          int mode, bz_batch *out);
/* As bz_batch_create, with schedule flags for the batched modes (ignored by
 * the plain modes):
 *   0                  the conjugate-symmetric schedule (the default of
 *                      bz_batch_create).  f is real (Sec. 2), so its transform
 *                      satisfies fhat(-zeta) = conj fhat(zeta) wherever -zeta is
 *                      a mesh node, i.e. off the planes k_d = 0; the weights of
 *                      eq. (GHat_calc) are even in (xi, zeta).  The sum of Sec. 3.2
 *                      is evaluated over about half of the output rows, plus the
 *                      pairs with a coordinate on a k_d = 0 plane and the outputs
 *                      with no mirror; the other outputs are the conjugates of
 *                      their mirrors corrected by those edge sums.  Same result
 *                      up to rounding as the full sum; about 0.61 / 0.65 / 0.71
 *                      of its work at N = 32 / 24 / 16.
 *   BZ_BATCH_FULL_SUM  every output row is summed directly.
 *   BZ_BATCH_PER_MESH  (BZ_MODE_BATCHED_F32) one convolution launch per mesh
 *                      with its autotuned variant, and the FP64 cores on a
 *                      second stream of the batch.  By default a batch of up
 *                      to four meshes, or of one mesh with an FP64 core, runs
 *                      the work items of all meshes and all cores in one
 *                      persistent launch from one queue: the FP32 items
 *                      ordered by cost, each naming its mesh (the variant
 *                      with FOLD 16 and two interleaved partials for every
 *                      mesh), and the FP64 core items spread through the
 *                      first 3/5 of it; the transforms stay one launch per
 *                      mesh and pass.  bz_batch_autotune may switch a batch
 *                      to the per-mesh launches when they are faster.
 *   BZ_BATCH_FINE_SPLIT  cut the rows into work items small enough for the
 *                      rows of a single 64-cell group to fill the device (by
 *                      default the whole batch is counted; at most 6 pieces
 *                      per row).  For batches of which only a few groups are
 *                      usually convolved, as with the gated closure; a full
 *                      batch takes somewhat longer.  The same sum in more
 *                      partial sums: results agree with the default split to
 *                      rounding.
 * Errors: as bz_batch_create, and BZ_EINVAL for unknown flags. */
#define BZ_BATCH_FULL_SUM 1
#define BZ_BATCH_FINE_SPLIT 2
#define BZ_BATCH_PER_MESH 4
bz_status bz_batch_create_ex(int n_cells, const int32_t *grid_of_cell, int n_grids, const bz_grid *grids,
                             int mode, int flags, bz_batch *out);
void bz_batch_free(bz_batch b);
/* Bind the weight buffer of grids[grid_index] (built by bz_weights with the
 * kind the mode reads: BZ_W_BATCHED_* for batched modes, BZ_W_PLAIN_* for
 * plain modes).  `kind` must match the buffer.  The buffer must outlive the
 * batch's use. */
bz_status bz_batch_set_weights(bz_batch b, int grid_index, int kind, const void *d_w);
/* Number of doubles of a batch's f (sum of N_c^3), and the offset (in
 * doubles) of cell c's data. */
size_t bz_batch_elems(bz_batch b);
size_t bz_batch_cell_offset(bz_batch b, int cell);
/* Workspace bytes bz_collide_batch / bz_step need for this batch. */
size_t bz_workspace_bytes(bz_batch b);

/* Qt = Re F^{-1}[ weighted convolution of F[f] ] for every cell (Sec. 3.2),
 * unprojected.  d_f and d_Qt hold bz_batch_elems doubles; they may not alias.
 * d_work holds work_bytes >= bz_workspace_bytes.  Errors: BZ_ESTATE when a
 * mesh of the batch has no weights bound, BZ_EINVAL for NULL pointers or a
 * short workspace. */
bz_status bz_collide_batch(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes,
                           void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * bz_collide_batch with the library's own workspace, a static device array
 * of BZ_STATIC_SCRATCH_BYTES (256 MiB) per GPU, held from the library's
 * load until the process ends; the call itself allocates nothing.  The
 * caller passes the inputs and outputs as for bz_collide_batch.  Every call
 * on one GPU shares that GPU's array and leaves its contents behind, so
 * calls that overlap on one GPU (on different streams, or from different
 * threads) race; calls ordered on one stream do not.  Errors: BZ_EINVAL for
 * NULL pointers or a batch whose bz_workspace_bytes exceeds
 * BZ_STATIC_SCRATCH_BYTES, BZ_ESTATE when the batch's timer is on (it
 * creates events) or a mesh has no weights bound. */
#define BZ_STATIC_SCRATCH_BYTES (256u * 1024u * 1024u)
bz_status bz_collide_batch_static(bz_batch b, const double *d_f, double *d_Qt, void *stream);

/* In place, per cell: Q <- Q - C^T (C C^T)^{-1} C Q (Sec. 3.3; the sign and
 * transposition are those of the Lagrange solution of the stated problem).
 * FP64 throughout; the moments are reduced twice (one refinement pass). */
bz_status bz_project(bz_batch b, double *d_Q, void *stream);

/* One Heun (second-order Runge-Kutta, Sec. 3.1) step of the space-
 * homogeneous equation df/dt = Q(f,f)/eps for every cell, in place:
 *   f* = f + h P Q(f),  f <- (f + f* + h P Q(f*)) / 2,  h = dt/eps,
 * with P the projection.  d_work as for bz_collide_batch plus 2 batch
 * arrays (bz_step_workspace_bytes).  If any produced value is non-finite
 * the step still completes and bz_step_check later reports BZ_ENONFINITE. */
size_t bz_step_workspace_bytes(bz_batch b);
bz_status bz_step(bz_batch b, double *d_f, double dt_over_eps, void *d_work, size_t work_bytes, void *stream);
/* Synchronises `stream` and returns BZ_ENONFINITE if any bz_step enqueued
 * with this workspace since the last check produced a non-finite value,
 * BZ_OK otherwise; clears the flags of bz_step_flags. */
bz_status bz_step_check(bz_batch b, void *d_work, void *stream);
/* Flags of the bz_step calls enqueued with this workspace since the last
 * check: BZ_FLAG_NONFINITE when a value of the new f was not finite,
 * BZ_FLAG_NEGATIVE when one was below zero (the projection of Sec. 3.3
 * restores the moments, not the sign of f; a diagnostic, not an error).
 * Synchronises `stream`, writes the flags to *flags and clears them. */
#define BZ_FLAG_NONFINITE 1u
#define BZ_FLAG_NEGATIVE 2u
bz_status bz_step_flags(bz_batch b, void *d_work, unsigned *flags, void *stream);

/* ------------------------------------------------------------------ */
/* 1-D transport (Sec. 3.4, eq. upwind) with a diffuse wall (Sec. 2.1,    */
/* eq. BC) and the Strang-split step (Sec. 3.1).                          */
/* ------------------------------------------------------------------ */
typedef struct bz_transport_s *bz_transport;

/* nx uniform cells of width x_length/nx along x (axis 1 of the velocity
 * mesh of `g` is the transport direction).  Left end: diffuse Maxwell wall
 * at rest with temperature T_wall; two ghost cells copy the first cell (its
 * minmod slope is 0) and the wall face emits sigma_w M_wall for v1 > 0 with
 * sigma_w = sum_{v1<0}|v1| f_0 / sum_{v1>0} v1 M_wall (discrete, so the net
 * wall mass flux is zero).  Right end: two ghost cells hold the far-field
 * Maxwellian M(far_rho, (far_u1, 0, 0), far_T).  Uploads two N^3 tables
 * (owned by the handle).  Errors: BZ_EINVAL for nx < 1, non-positive
 * length or temperatures, negative density. */
bz_status bz_transport_create(bz_grid g, int nx, double x_length, double T_wall, double far_rho, double far_u1,
                              double far_T, bz_transport *out);
/* As bz_transport_create on cells of the given widths (Sec. 3.4: cells of
 * size dx_j, "not necessarily uniform"): dx (host, nx positive values,
 * copied) lists cell 0 at the wall first.  The minmod slope of cell j uses
 * the distances between cell centres, (dx_{j-1} + dx_j)/2 and
 * (dx_j + dx_{j+1})/2; the cell is reconstructed to its faces with dx_j/2
 * and updated with the flux difference over dx_j; ghost cells take the width
 * of the cell they border.  Equal widths give bitwise the uniform scheme.
 * Errors: as bz_transport_create, and BZ_EINVAL for a NULL, non-positive or
 * non-finite width. */
bz_status bz_transport_create_ex(bz_grid g, int nx, const double *dx, double T_wall, double far_rho, double far_u1,
                                 double far_T, bz_transport *out);
void bz_transport_free(bz_transport t);
size_t bz_transport_workspace_bytes(bz_transport t);
/* Heun RK2 over dt of df/dt + v1 df/dx = 0 for the nx cells of d_f (layout
 * [cell][velocity], nx * N^3 doubles), in place, second-order upwind fluxes
 * with minmod slopes. */
bz_status bz_transport_step(bz_transport t, double *d_f, double dt, void *d_work, size_t work_bytes, void *stream);
/* Strang step T(dt/2) C(dt) T(dt/2): transport half steps around one Heun
 * collision step (bz_step with dt/eps) of the batch `b`, which must hold the
 * nx cells of the transport mesh in x order. */
size_t bz_strang_workspace_bytes(bz_batch b, bz_transport t);
bz_status bz_strang_step(bz_batch b, bz_transport t, double *d_f, double dt, double eps, void *d_work,
                         size_t work_bytes, void *stream);

/* Diagnostics of the sudden-heating run (Sec. 5: evolution of the bulk
 * velocity and of the marginal distribution near the wall), FP64.
 * bz_cell_moments writes for every cell c of the batch, at d_mom[5 c ..],
 * the density rho = sum f dv^3, the bulk velocity u_d = sum v_d f dv^3 / rho
 * (d = 1..3) and the temperature T = sum |v - u|^2 f dv^3 / (3 rho).
 * bz_marginal_v1 writes the N values sum_{k2,k3} f(k1, k2, k3) dv^2 of cell
 * `cell` to d_out.  Errors: BZ_EINVAL for NULL pointers or a cell index out
 * of range. */
bz_status bz_cell_moments(bz_batch b, const double *d_f, double *d_mom, void *stream);
bz_status bz_marginal_v1(bz_batch b, const double *d_f, int cell, double *d_out, void *stream);

/* ------------------------------------------------------------------ */
/* Learned closure: network kernels.  A 3-layer perceptron                */
/*   n_in -> n_hidden -> n_hidden -> n_out, exact-erf GELU after the two  */
/* hidden layers, BF16 weights and activations on the matrix cores with   */
/* FP32 accumulation, FP32 master weights and Adam (beta 0.9 / 0.999,     */
/* eps 1e-8), loss = mean squared error.  Weights are stored [out][in].   */
/* ------------------------------------------------------------------ */
typedef struct bz_mlp_s *bz_mlp;

/* Host handle (sizes only).  n_in, n_hidden and n_out must be multiples of 32
 * (the GEMM's k-tile); BZ_EINVAL otherwise. */
bz_status bz_mlp_create(int n_in, int n_hidden, int n_out, bz_mlp *out);
void bz_mlp_free(bz_mlp n);
/* FP32 master parameter count, laid out [W1 b1 W2 b2 W3 b3]. */
size_t bz_mlp_param_count(bz_mlp n);
/* Bytes of the caller's parameter buffer (master, Adam moments, BF16 copies). */
size_t bz_mlp_param_bytes(bz_mlp n);
/* Bytes of the caller's workspace for a batch of `batch` samples. */
size_t bz_mlp_workspace_bytes(bz_mlp n, int batch);
/* Upload host FP32 master weights (param_count floats), zero the Adam moments,
 * derive the BF16 copies.  Synchronous. */
bz_status bz_mlp_set_params(bz_mlp n, void *d_params, const float *master, void *stream);
/* Download the FP32 master weights.  Synchronous. */
bz_status bz_mlp_get_params(bz_mlp n, const void *d_params, float *master, void *stream);
/* d_y[batch][n_out] (FP32) = network(d_x[batch][n_in] (BF16 bit patterns)). */
bz_status bz_mlp_forward(bz_mlp n, const void *d_params, const uint16_t *d_x, int batch, float *d_y, void *d_work,
                         size_t work_bytes, void *stream);
/* Gradients of the loss against d_target[batch][n_out] (FP32) into d_grad
 * (param_count floats, master layout); d_loss (may be NULL) receives the
 * loss as one float.  batch must be a multiple of 32. */
bz_status bz_mlp_backward(bz_mlp n, const void *d_params, const uint16_t *d_x, const float *d_target, int batch,
                          float *d_grad, float *d_loss, void *d_work, size_t work_bytes, void *stream);
/* One Adam step (step number >= 1) with learning rate lr, then refresh the BF16 copies. */
bz_status bz_mlp_adam(bz_mlp n, void *d_params, const float *d_grad, int step, float lr, void *stream);

/* ------------------------------------------------------------------ */
/* Gated learned closure around the collision step.                      */
/* ------------------------------------------------------------------ */
/* Per cell: rho, u, T (FP64 moments), the local Maxwellian M, the deviation
 * d = |f - M|_2 / |M|_2.  Cells with d < gate are served by the network.  Its
 * BF16 input x is the direction of f - M scaled to unit RMS,
 *   x_j = (f_j - M_j) sqrt(N^3) / |f - M|_2   (j > 0),
 * with the amplitude x_0 = d / s_in in the corner entry v = (-L, -L, -L),
 * where f - M is negligible; the closure is Q_s = rho |f - M|_2 s_out net(x)
 * (near equilibrium Q is linear in f - M with a coefficient proportional to
 * rho, so the network sees the direction and a bounded amplitude, and Q_s
 * vanishes with f - M).  The others take the weighted convolution.  The gated cells of the 64-cell groups g with
 * g mod judge_every = (evaluation count) mod judge_every are also convolved
 * ("judged"), compared after projection,
 *   err = |P(Q_s - Q_c)|_2 / (|P Q_c|_2 + judge_floor rho |M|_2)
 * (the floor is on the scale of the loss term, so that cells at equilibrium,
 * whose Q is only the discretisation residual, are judged against the
 * collision rate),
 * counted as failed if err > judge_tol, and keeps the convolution result.
 * A failed judge also caps the gate of every later evaluation with this
 * workspace at that cell's deviation d, so no cell at least as far from
 * equilibrium is served again (the cap lives in the workspace's closure
 * counters: zeroing the workspace lifts it), and the cells served in an
 * evaluation whose judge failed are counted as unbounded.
 * The FP64 projection of Sec. 3.3 is always applied.  In the batched modes
 * the cells that need the convolution (not gated, or judged) are packed into
 * the first 64-cell groups of the launch, and only those groups are
 * transformed and convolved; every cell's result is the same as in the
 * batch's own order.  The network runs on a second stream that the batch
 * owns (default priority, created on the first closure call), ordered after
 * the preparation and before the selection by events on `stream`, so that it
 * overlaps the transforms and the convolution; the calls still only enqueue.
 * Requires a batch on one mesh with n_in = n_out = N^3. */
typedef struct {
    bz_mlp net;
    const void *d_params;   /* network parameters (bz_mlp_set_params / training) */
    double gate;
    double s_in, s_out;
    int judge_every;        /* 0: no judged cells */
    double judge_tol;
    double judge_floor;
} bz_closure;

typedef struct {
    unsigned served;        /* cells that took the network's result */
    unsigned judged;        /* gated cells also convolved and compared */
    unsigned failed;        /* judged cells with err > judge_tol */
    float max_err;          /* largest judged err */
    unsigned unbounded;     /* served cells of evaluations in which a judge failed */
    double gate_cap;        /* the gate cap set by failed judges (0: none) */
} bz_closure_stats;

/* Workspace of the closure calls: bz_step_workspace_bytes plus the closure's
 * per-cell state, network input and output, its counters and gate cap, and
 * the network workspace.  Zero it before the first closure call with it (the
 * counters and the cap start from its contents). */
size_t bz_closure_workspace_bytes(bz_batch b, const bz_closure *c);
/* Gate and network input for every cell (used to harvest training data):
 * d_state[n_cells][10] = (rho, u1, u2, u3, T, d, gated, 0, |M|_2, 0),
 * d_x[n_cells][N^3] BF16. */
bz_status bz_closure_prepare(bz_batch b, const double *d_f, double gate, double s_in, double *d_state,
                             uint16_t *d_x, void *stream);
/* Training targets d_y[n_cells][N^3] = Q / (rho |f - M|_2 s_out) from a
 * projected Q (0 for a cell with f = M). */
bz_status bz_closure_targets(bz_batch b, const double *d_state, const double *d_Q, double s_out, float *d_y,
                             void *stream);
/* Qt of every cell with the gate applied (unprojected, like bz_collide_batch). */
bz_status bz_closure_collide(bz_batch b, const bz_closure *c, const double *d_f, double *d_Qt, void *d_work,
                             size_t work_bytes, void *stream);
/* bz_step and bz_strang_step with the closure in every collision evaluation. */
bz_status bz_closure_step(bz_batch b, const bz_closure *c, double *d_f, double dt_over_eps, void *d_work,
                          size_t work_bytes, void *stream);
bz_status bz_closure_strang_step(bz_batch b, bz_transport t, const bz_closure *c, double *d_f, double dt,
                                 double eps, void *d_work, size_t work_bytes, void *stream);
/* Counters accumulated since the last read (synchronises `stream`, then clears
 * them; the gate cap persists). */
bz_status bz_closure_read_stats(bz_batch b, const bz_closure *c, void *d_work, bz_closure_stats *out, void *stream);

/* ------------------------------------------------------------------ */
/* HIP graphs of a whole step.                                           */
/* ------------------------------------------------------------------ */
/* Capture one bz_step (resp. bz_strang_step) with the given arguments on
 * `stream` (which must not be the NULL stream) and instantiate it; replaying
 * the graph re-runs the step on the same buffers.  The steps enqueue no
 * memset nodes (counters are cleared by fill kernels) and no host
 * synchronisation.  The convolution timer must be off while capturing. */
typedef struct bz_graph_s *bz_graph;
bz_status bz_graph_capture_step(bz_batch b, double *d_f, double dt_over_eps, void *d_work, size_t work_bytes,
                                void *stream, bz_graph *out);
bz_status bz_graph_capture_strang(bz_batch b, bz_transport t, double *d_f, double dt, double eps, void *d_work,
                                  size_t work_bytes, void *stream, bz_graph *out);
bz_status bz_graph_launch(bz_graph g, void *stream);
void bz_graph_free(bz_graph g);

/* ------------------------------------------------------------------ */
/* Tuning and measurement.                                               */
/* ------------------------------------------------------------------ */
/* Select the convolution kernel variant for the cells of grids[grid_index]
 * (batched modes; 0 is the default, bz_variant_count() variants exist).
 * Every variant computes the same sums; they differ in compensation, fold
 * interval and how weights reach the arithmetic units. */
int bz_variant_count(void);
bz_status bz_batch_set_variant(bz_batch b, int grid_index, int variant);
int bz_batch_get_variant(bz_batch b, int grid_index);
/* Time every variant on this batch's data (d_f, d_work as for
 * bz_collide_batch; d_Qt receives a result), `reps` launches each, with HIP
 * events on `stream`, and keep per mesh, among the variants within 3% of the
 * fastest, the one with the most accurate accumulation (more interleaved
 * partials, then the shorter fold interval).  Then, for a batch that has the
 * one-launch queue (BZ_BATCH_PER_MESH), time `reps` whole evaluations with
 * it and with the per-mesh launches and keep the faster.  Synchronous.  The
 * variants are also remembered per (N, number of wavefront groups, mode) for
 * the rest of the process. */
bz_status bz_batch_autotune(bz_batch b, const double *d_f, double *d_Qt, void *d_work, size_t work_bytes,
                            int reps, void *stream);
/* 1 if the batch's convolution currently runs as the one persistent launch
 * for all its meshes and cores (see BZ_BATCH_PER_MESH), else 0 (also for
 * NULL). */
int bz_batch_one_launch(bz_batch b);
/* The variants remembered per (N, number of wavefront groups, mode) — by
 * bz_batch_autotune or a load — as a text file of lines "N groups mode
 * variant" (host only; a batch created later starts from a remembered
 * variant).  bz_tuning_load merges a file into the process's memory, all of
 * it or, on a malformed line, nothing.  Errors: BZ_EINVAL for a NULL path, a
 * file that cannot be opened, written or parsed, or a variant out of range. */
bz_status bz_tuning_save(const char *path);
bz_status bz_tuning_load(const char *path);
/* enable = 1: record a HIP event pair around every convolution launch of
 * this batch (on the stream the launch uses); enable = 0: stop recording.
 * bz_batch_timer_read synchronises on the recorded events, returns the
 * summed kernel time in milliseconds and the number of launches, and clears
 * the record. */
bz_status bz_batch_timer(bz_batch b, int enable);
bz_status bz_batch_timer_read(bz_batch b, double *conv_ms, int *launches);
/* The separate FP64 core launches of the per-mesh form (BZ_BATCH_PER_MESH)
 * are timed by the same switch: their summed time and count as of the last
 * bz_batch_timer_read (none when the cores run inside the one launch). */
bz_status bz_batch_core_timer(bz_batch b, double *core_ms, int *launches);
/* Size of the separate FP64 core kernel's persistent grid in wavefronts (0,
 * the default: eight per compute unit), for the per-mesh form, where the
 * cores run on a stream of the batch (default priority), forked from and
 * joined to the caller's stream.  Results do not depend on it.  Errors:
 * BZ_EINVAL for a negative count. */
bz_status bz_batch_set_core_waves(bz_batch b, int waves);

const char *bz_status_string(bz_status s);
const char *bz_status_str(bz_status s);   /* the same text */
const char *bz_last_error(void);
int bz_api_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BZ_H */
