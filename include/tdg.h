/*
 * libtdg: tent-pitched space-time Trefftz-DG for the first-order acoustic
 * wave system on MI355X (gfx950).
 *
 * The problem statement follows Sec. 2.1 of Perugia, Schoeberl, Stocker,
 * Wintersteiger, "Tent pitching and Trefftz-DG method for the acoustic wave
 * equation" (eq. 2.1):
 *     div sigma + c^-2 dv/dt = 0,   grad v + dsigma/dt = 0   in Omega x (0,T),
 *     v(.,0) = v0, sigma(.,0) = sigma0,  v = g_D on the Dirichlet boundary,
 *     sigma.n = g_N on the Neumann boundary,
 * with a wave speed c > 0 that is constant on each spatial element.  With
 * v = dU/dt and sigma = -grad U this is the scalar wave equation (eq. 2.2).
 *
 * The library pitches tents over the vertex patches of a simplicial mesh of
 * Omega (Sec. 2.2), then solves the tents layer by layer: all tents of a
 * layer are independent and run in one launch.  Each tent solves the dense
 * local Trefftz-DG system of eq. 4.1 (plus the interface terms of Sec. 4.2
 * where the speed jumps inside the tent, and one recovery row per speed group
 * for the constant of U, Sec. 5) and overwrites the values stored at the
 * spatial quadrature points under it with its top values (Sec. 4.1).
 *
 * Conventions
 *  - Degree p is the degree of the scalar Trefftz space U^p (Sec. 3); a tent
 *    with one speed has N = dim U^p = C(p+n,n) + C(p-1+n,n) unknowns; the
 *    first-order fields (v, sigma) have degree p - 1.
 *  - Every call returns 0 (TDG_OK) or a negative TDG_E* code; no exception
 *    crosses the interface.  tdg_last_error() gives a message for the
 *    calling thread.
 *  - Host arrays passed in are borrowed for the duration of the call and
 *    copied.  tdg_tents and tdg_ctx are owned by the library and released by
 *    tent_free / trefftz_destroy.
 *  - The library allocates no device memory: the caller allocates the
 *    buffers listed by trefftz_buffer_sizes (for instance as PyTorch tensors)
 *    and hands them over with trefftz_bind; they must outlive the context.
 *  - Device work is queued on the HIP stream passed in (NULL = the default
 *    stream) and is asynchronous, except in calls that return host scalars,
 *    which synchronise that stream.
 *  - Double precision throughout unless the context is created with
 *    precision = 1 (FP32 matrix-core assembly, FP64 solve and refinement).
 */
#ifndef TDG_H
#define TDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  TDG_OK = 0,
  TDG_EINVAL = -1,      /* invalid argument (sizes, degenerate element, c <= 0, p out of range) */
  TDG_ENONCAUSAL = -2,  /* a pitched front would not be space-like: c |grad phi| >= 1 (Sec. 2.2) */
  TDG_ESINGULAR = -3,   /* a local system had a zero pivot */
  TDG_ENOCONV = -4,     /* iterative refinement of the mixed-precision solve did not converge */
  TDG_ENAN = -5,        /* NaN or Inf in data or results */
  TDG_EHIP = -6,        /* a HIP runtime call failed */
  TDG_ENOMEM = -7,      /* host allocation failed or a bound buffer is too small */
  TDG_ESTATE = -8       /* call out of order (e.g. solve before bind) */
};

/* Spatial simplicial mesh.  coords: nv*dim doubles, vertex-major.
 * elems: ne*(dim+1) vertex indices, element-major.  bface_kind: the kind of
 * every boundary facet, 0 = Dirichlet, 1 = Neumann (eq. 4.1, T^D and T^N), in
 * ascending (element, local index of the opposite vertex) order, the order
 * tdg_boundary_facets lists; NULL = every boundary facet Dirichlet.  Other
 * values: TDG_EINVAL.  The pitcher ignores it. */
typedef struct {
  int32_t dim, nv, ne;
  const double* coords;
  const int32_t* elems;
  const int8_t* bface_kind;
} tdg_mesh;

typedef struct tdg_tents tdg_tents;
typedef struct tdg_ctx tdg_ctx;
typedef void* tdg_stream; /* a hipStream_t */

/* ---- tent pitching (host only, Sec. 2.2) -------------------------------------
 * Advancing front from t = 0 to T.  Edge limit kappa_VW = gamma |X_W - X_V| /
 * c_VW with c_VW the largest speed on the edge.  Each layer takes the local
 * minima of the front in (tau, vertex) order, greedily skipping neighbours of
 * vertices already taken, and raises each to min(T, min_W tau_W + kappa_VW).
 * Fails with TDG_ENONCAUSAL if a front element would become c|grad phi| >= 1.
 * c: ne speeds.  Requires dim in {1,2,3}, T > 0, gamma > 0. */
int tent_pitch(const tdg_mesh* mesh, const double* c, double T, double gamma, tdg_tents** out);
/* The boundary facets of a mesh in the order of tdg_mesh.bface_kind: nbf and
 * (facets may be NULL) facets[2 i], facets[2 i + 1] = element, local index of
 * the vertex opposite the facet.  Validates the mesh like tent_pitch. */
int tdg_boundary_facets(const tdg_mesh* mesh, int64_t* nbf, int32_t* facets);
/* Layer and tent counts and the largest c|grad phi| over all pitched fronts. */
int tent_info(const tdg_tents* tents, int32_t* n_layers, int64_t* n_tents, double* max_face_slope);
/* Copies the tent list: vertex[n_tents], t_bot[n_tents], t_top[n_tents] and
 * layer_ptr[n_layers+1] (tents of layer l are layer_ptr[l] .. layer_ptr[l+1]-1).
 * Any pointer may be NULL to skip it. */
int tent_export(const tdg_tents* tents, int32_t* vertex, double* t_bot, double* t_top, int64_t* layer_ptr);
void tent_free(tdg_tents* tents);

/* ---- solver context ------------------------------------------------------------ */
typedef struct {
  int32_t p_max;     /* highest degree of U^p used by any tent, 1..10; in 3+1D at most 9 (at
                        p = 10 a tent's working set does not fit in LDS: TDG_EINVAL) */
  int32_t q;         /* Gauss points per direction of the simplex rule; 0 -> p_max (exact to 2q-1) */
  double alpha;      /* penalty on Dirichlet and interface faces (Sec. 2.4), e.g. 0.5 */
  double beta;       /* interface penalty (Sec. 2.4), e.g. 0.5 */
  int32_t precision; /* 0 = FP64; 1 = FP32 matrix-core Gram + FP64 LU + FP64 refinement */
  int32_t layout;    /* must be 1: values stored at spatial quadrature points (Sec. 4.1) */
  int32_t recover_U; /* recovery of U, the solution of the second-order equation (Sec. 5):
                        1: one row per speed group matching the mean of U over the tent's
                           bottom facets with the incoming U ((v, sigma) are exactly eq. 4.1);
                        2: the paper's terms int_bot U V = int_bot U_bot V added for every
                           test function V of U^p, the constants solved with the functions
                           (quadrature Gram only: trefftz_set_gram_mode(1) and precision = 1
                           are rejected);
                        0: off; other values: TDG_EINVAL */
  int32_t seed_basis;/* spatial basis that seeds the recursion of eq. 3.1 at t = t_K (Sec. 3;
                        the three choices compared in Sec. 6.3), in the scaled coordinates of
                        Remark 3.1: 0 = monomials x^beta (the default; the best conditioned),
                        1 = products of Legendre polynomials P_(beta_m)(x_m), 2 = products of
                        Chebyshev polynomials T_(beta_m)(x_m); all span the same U^p, so the
                        solution differs by round-off only, as far as the conditioning of the
                        tent systems allows: the seeded bases are worse conditioned, and at
                        3+1D p = 8 Chebyshev-seeded tent systems are singular to working
                        precision (condition numbers up to 1.7e20).  Other values: TDG_EINVAL */
} tdg_opts;

enum {
  TDG_BUF_F64 = 0,   /* static mesh/quadrature/basis tables, doubles */
  TDG_BUF_I32 = 1,   /* static topology and tent tables, 32-bit ints */
  TDG_BUF_STATE = 2, /* (v, sigma_1..sigma_n, U) at every quadrature point */
  TDG_BUF_STATE0 = 3,/* copy of the initial values (trefftz_reset) */
  TDG_BUF_TAU = 4,   /* advancing front, one time per vertex */
  TDG_BUF_GD = 5,    /* boundary data (g_D or g_N) at the boundary points */
  TDG_BUF_WORK = 6,  /* scratch: reductions, error data, device status word */
  TDG_BUF_TENT = 7,  /* per-tent outputs: dissipation, refinement steps */
  TDG_NBUF = 8
};

/* Builds the context for a pitched mesh: topology, the simplex rule and the
 * exact Trefftz tables for p = 1..p_max.  c: ne speeds (the same as pitched). */
int trefftz_create(const tdg_mesh* mesh, const double* c, const tdg_tents* tents, const tdg_opts* opts,
                   tdg_ctx** out);
/* Spatial quadrature points, element-major: nq = ne * Q points of dim
 * coordinates.  Pass xq = NULL to query nq.  w (nullable) gets the weights. */
int trefftz_quad_points(const tdg_ctx* ctx, int64_t* nq, double* xq, double* w);
/* Space-time points (dim+1 coordinates, time last) of the boundary faces of
 * every tent, in tent order, per tent the Dirichlet faces then the Neumann
 * faces; the caller evaluates g_D or g_N there (trefftz_boundary_kinds).  xt
 * may be NULL. */
int trefftz_boundary_points(const tdg_ctx* ctx, int64_t* nb, double* xt);
/* kind[nb]: 0 where the boundary point lies on a Dirichlet face (g_D), 1 on a
 * Neumann face (g_N, the prescribed sigma.n). */
int trefftz_boundary_kinds(const tdg_ctx* ctx, int8_t* kind);
/* Sizes in bytes of the TDG_NBUF device buffers the caller must provide. */
int trefftz_buffer_sizes(const tdg_ctx* ctx, int64_t sizes[TDG_NBUF]);
/* Hands over the device buffers (each at least the queried size, 256-byte
 * aligned) and uploads the static tables on the stream. */
int trefftz_bind(tdg_ctx* ctx, void* const dev_ptrs[TDG_NBUF], tdg_stream stream);
/* Initial data at the quadrature points (host arrays): v0[nq], sigma0[nq*dim]
 * (point-major), U0[nq] (nullable = 0).  Also resets the front to t = 0. */
int trefftz_set_initial(tdg_ctx* ctx, const double* v0, const double* sigma0, const double* U0,
                        tdg_stream stream);
/* Boundary data at the points of trefftz_boundary_points (host array, nb):
 * g_D at points of Dirichlet faces, g_N at points of Neumann faces. */
int trefftz_set_boundary(tdg_ctx* ctx, const double* gD, tdg_stream stream);
/* Restores the initial values and the flat front t = 0 (device-to-device). */
int trefftz_reset(tdg_ctx* ctx, tdg_stream stream);
/* Solves the tents of layers [layer_begin, layer_end) in order, one launch
 * per layer.  p_per_tent: device array of n_tents degrees (int8, 1..p_max) or
 * NULL for p_max everywhere. */
int trefftz_layer_solve(tdg_ctx* ctx, int32_t layer_begin, int32_t layer_end, const int8_t* p_per_tent,
                        tdg_stream stream);
/* Error e of Sec. 6 on the flat front t = T against host arrays of exact
 * values at the quadrature points: v_ex[nq], sigma_ex[nq*dim].  e_rel divides
 * by the same norm of the exact values.  Synchronises; also reports device
 * errors raised by earlier solves. */
int trefftz_eval_error(tdg_ctx* ctx, const double* v_ex, const double* sigma_ex, double* e_abs, double* e_rel,
                       tdg_stream stream);
/* L2 error of U on the flat front t = T (the error Sec. 6.6 reports) against
 * exact values U_ex[nq] at the quadrature points: e_abs = ||U - U_ex||,
 * e_rel = e_abs / ||U_ex||.  Synchronises. */
int trefftz_eval_u_error(tdg_ctx* ctx, const double* U_ex, double* e_abs, double* e_rel, tdg_stream stream);
/* Energy on the current front, E = 1/2 int c^-2 v^2 + |sigma|^2 - 2 v sigma.grad phi
 * (the energy of Sec. 6.5 where the front is flat), and the sum over tents of
 * the per-tent indicator eta_T (see trefftz_set_indicator; 0 for tents solved
 * with the indicator off since the last bind).  Synchronises. */
int trefftz_energy(tdg_ctx* ctx, double* E_front, double* dissipated, tdg_stream stream);
/* Synchronises the stream and returns the first error a kernel reported. */
int trefftz_status(tdg_ctx* ctx, tdg_stream stream);
/* Copies the stored values to host memory in the layout of the inputs:
 * v[nq], sigma[nq*dim], U[nq] (any may be NULL).  Synchronises. */
int trefftz_read_state(tdg_ctx* ctx, double* v, double* sigma, double* U, tdg_stream stream);
/* Sizes of the degree-p basis tables: N = dim U^p, nnz_fields = stored
 * coefficients of the first-order fields (v, sigma) of functions 1..N-1,
 * n_mono = monomials t^k x^alpha with k + |alpha| <= p, and the points per
 * element Q.  For operation counts; any output pointer may be NULL. */
int trefftz_table_info(const tdg_ctx* ctx, int32_t p, int32_t* N, int32_t* nnz_fields, int32_t* n_mono, int32_t* Q);
/* Execution shape of the tent kernel (all tents of a layer in one launch):
 * pts_per_chunk = quadrature points staged per chunk (0 = largest that fits in
 * LDS, else 4, 8, 16, 32 or 64 if it fits); persistent = 1: a grid of resident
 * workgroups takes the layer's tents from a device counter (balances tents of
 * uneven size and degree), 0: one workgroup per tent.  Results do not depend
 * on the shape.  TDG_EINVAL if the shape does not fit.  A sweep recorded by
 * trefftz_capture_sweep is released (it holds the old shape): replay then
 * returns TDG_ESTATE until the next capture. */
int trefftz_set_tuning(tdg_ctx* ctx, int32_t pts_per_chunk, int32_t persistent);
/* How the top Gram, the bottom right-hand side, the recovery row and the
 * Dirichlet terms of eq. 4.1 are formed (FP64 contexts):
 *   mode 0 (default): the fields of the basis at every quadrature point, Gram
 *     on the matrix cores (work ~ points x N^2);
 *   mode 1: moments of the monomials of degree <= 2p-2 over the points, then
 *     the sparse field tables (work ~ points x (monomials of degree <= 2p-2)
 *     + the table terms), far less at high degree.
 * Both give the same system up to rounding.  TDG_EINVAL for mode 1 in a
 * mixed-precision context or if it does not fit in LDS.  Like
 * trefftz_set_tuning, a successful call releases a recorded sweep. */
int trefftz_set_gram_mode(tdg_ctx* ctx, int32_t mode);
int trefftz_get_gram_mode(const tdg_ctx* ctx, int32_t* mode);
int trefftz_get_tuning(const tdg_ctx* ctx, int32_t* pts_per_chunk, int32_t* persistent, int32_t* lds_bytes);
/* Records layers [layer_begin, layer_end) (as trefftz_layer_solve, preceded by
 * trefftz_reset if with_reset) into a HIP graph owned by the context, captured
 * on `stream` (which must not be the default stream).  trefftz_replay_sweep
 * launches the recorded graph on a stream: same buffers, same degrees.  A new
 * capture replaces the previous graph. */
int trefftz_capture_sweep(tdg_ctx* ctx, int32_t layer_begin, int32_t layer_end, const int8_t* p_per_tent,
                          int32_t with_reset, tdg_stream stream);
int trefftz_replay_sweep(tdg_ctx* ctx, tdg_stream stream);
/* Per-tent outputs of the last solve of tents [first_tent, first_tent+count):
 * ir_steps = refinement steps of the mixed-precision solve (+1000 where the
 * tent fell back to the FP64 Gram; 0 in FP64 contexts), dissipation = the
 * indicator eta_T of trefftz_set_indicator (0 where it was not computed).
 * Either pointer may be NULL.  Synchronises. */
int trefftz_tent_stats(tdg_ctx* ctx, int64_t first_tent, int64_t count, int32_t* ir_steps, double* dissipation,
                       tdg_stream stream);

/* ---- per-tent degree (learned degree selection) -------------------------------
 * Indicator of a tent (a term of its energy balance, from eq. 4.1 with w = u):
 *   eta_T = 1/2 int_{bottom} c^-2 dv^2 + |dsigma|^2 - 2 dv dsigma.grad phi_old,
 * (dv, dsigma) = tent solution minus the incoming values at the bottom points,
 * i.e. the energy of the jump the tent's Trefftz space cannot match; it
 * shrinks with the degree where the solution is smooth.  All arrays below are
 * device arrays indexed by the global tent number (n_tents entries; a call
 * writes the entries of its layers only). */

/* on = 1: trefftz_layer_solve also computes eta_T (into the per-tent outputs
 * of trefftz_tent_stats); 0 (the default) skips it. */
int trefftz_set_indicator(tdg_ctx* ctx, int32_t on);
/* Features of the tents of `layer` from the current front and stored values
 * (call after the layers below it are solved): feats[tent*8 + k],
 *   0 log(dt c_max / h_V)  1 log h_V  2 |patch| / 16  3 log c_max
 *   4 log(c_max / c_min)  5 log(incoming energy / patch volume)
 *   6 log(relative spread of the incoming values inside the patch elements)
 *   7 1 if V lies on the Dirichlet boundary,
 * with h_V the largest distance from X_V to a patch vertex and dt the tent
 * height. */
int trefftz_tent_features(tdg_ctx* ctx, int32_t layer, float* feats, tdg_stream stream);
/* eta_T of every tent of `layer` solved at degree p (1..p_max), written to
 * eta[tent]; stored values and front are left untouched (a probe). */
int trefftz_layer_indicator(tdg_ctx* ctx, int32_t layer, int32_t p, double* eta, tdg_stream stream);
/* Solves layers [layer_begin, layer_end) with a degree per tent.  With a
 * network (w_bf16, tdg_mlp_nparam() BF16 values): per layer, features ->
 * feats, the network's predicted log eta_T(p) for p = 2..8 -> p_sel[tent] =
 * the smallest p <= p_max whose prediction is <= log_eta_tol (else p_max); a
 * tent whose realised eta_T exceeds eta_tol (if > 0) is solved again one
 * degree higher, up to p_max (accepted there), before anything is written.
 * With a network the layer's tents are then drawn in decreasing chosen degree
 * (index order inside a degree), so that the costliest start first and the
 * cheap ones fill the end of the layer; the results do not depend on the
 * order (the tents of a layer are independent).  w_bf16 = NULL: fixed p_max
 * everywhere (the fallback; p_sel is filled with p_max), index order.  p_used
 * (nullable) gets the degree each tent was finally solved with, eta (nullable)
 * its eta_T. */
int trefftz_layer_solve_adaptive(tdg_ctx* ctx, int32_t layer_begin, int32_t layer_end, const uint16_t* w_bf16,
                                 float log_eta_tol, double eta_tol, float* feats, int8_t* p_sel, int8_t* p_used,
                                 double* eta, tdg_stream stream);

/* ---- degree network: 3 dense layers 8 -> 64 -> 64 -> 7, tanh, BF16 weights,
 * FP32 arithmetic.  Parameter vector (tdg_mlp_nparam() values): W1[64][8],
 * b1[64], W2[64][64], b2[64], W3[7][64], b3[7] (row-major, out x in).  Every
 * pointer is a device pointer; the calls only enqueue work on the stream. */
int tdg_mlp_nparam(void);
/* y[n][7] = network(x[n][8]) with the BF16 weights w_bf16. */
int tdg_mlp_forward(const uint16_t* w_bf16, const float* x, int64_t n, float* y, tdg_stream stream);
/* Gradient of L = sum_s sum_o mask[s][o] (y[s][o] - target[s][o])^2 / norm
 * with respect to the parameters (at the BF16 weights) into grad[0..nparam-1]
 * and L into grad[nparam] (nparam+1 floats); n >= 1, norm > 0.  partial:
 * scratch of ceil(n/32) * (nparam+1) floats.  Blocks of 32 samples are summed
 * in block order (deterministic). */
int tdg_mlp_backward(const uint16_t* w_bf16, const float* x, const float* target, const float* mask, int64_t n,
                     float norm, float* partial, float* grad, tdg_stream stream);
/* The same gradient for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * per-block partial gradients live in a fixed device array of the library
 * (one per GPU, 256 blocks x (nparam+1) floats = 5.3 MB, held until the
 * process ends) instead of a caller scratch, and the call allocates nothing.
 * Same kernels and summation order as tdg_mlp_backward, so the same result.
 * 1 <= n <= 8192 samples (TDG_EINVAL beyond, with a message).  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (streams
 * running concurrently) race and must be ordered by the caller. */
int tdg_mlp_backward_noalloc(const uint16_t* w_bf16, const float* x, const float* target, const float* mask,
                             int64_t n, float norm, float* grad, tdg_stream stream);
/* One Adam step (Kingma and Ba) on the FP32 master weights w32 with moments
 * m, v (step >= 1 counts from 1), then w_bf16 = round-to-nearest-even(w32). */
int tdg_mlp_adam(float* w32, uint16_t* w_bf16, const float* grad, float* m, float* v, int32_t step, float lr,
                 float b1, float b2, float eps, tdg_stream stream);
/* w_bf16 = round-to-nearest-even(w32). */
int tdg_mlp_round(const float* w32, uint16_t* w_bf16, tdg_stream stream);

void trefftz_destroy(tdg_ctx* ctx);
const char* tdg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TDG_H */
