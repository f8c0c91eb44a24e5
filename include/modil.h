/*
 * modil.h -- C ABI of the multiresolution ODIL (mODIL) iteration on gfx950.
 *
 * The method (Karnakov, Litvinov & Koumoutsakos, arXiv 2303.04679) solves a
 * PDE-constrained reconstruction problem by minimising a discrete loss
 * (Section 2.1): squared residuals of the discretised equations on the inner
 * points, squared misfits at measured points, and regularisation / initial /
 * boundary terms.  The unknown fields are represented by the multigrid
 * decomposition u = M_L(u_1..u_L) = u_1 + T_1(u_2 + T_2(... + T_{L-1} u_L))
 * (Section 2.2, Horner form), with T the cell-based linear interpolation whose
 * 1-D matrices the paper prints.  One optimiser iteration prolongs all
 * levels, evaluates residuals and the loss, forms the exact adjoint (the
 * transposed stencils, then M_L^T back to every level) and applies Adam to
 * every level.
 *
 * Conventions
 *   - Every pointer is a device pointer unless its name ends in _host.
 *   - The caller owns all device memory (parameter packs, gradients, Adam
 *     moments, the workspace).  The library keeps non-owning pointers and
 *     performs no device allocation.  All work is enqueued on the stream
 *     given at creation (or by modil_set_stream) and is asynchronous unless a
 *     function says otherwise.  A context is not thread safe.
 *   - No C++ exception crosses this interface.  Every function returns a
 *     MODIL_* status; on failure modil_last_error(ctx) (or
 *     modil_last_error(NULL) for failures without a context) describes it.
 *   - Floating-point arrays have the problem's dtype (float or double);
 *     loss terms are always double.
 *
 * Parameter pack layout (one flat array of the problem dtype)
 *   [level][instance][field][slowest axis]...[fastest axis]
 *   Levels run from the finest (l = 0) to the coarsest; level l has
 *   dims[a] / 2^l cells along every axis the field spans.  modil_layout()
 *   returns every offset.  Gradient packs and the Adam moments m, v use the
 *   same layout, so Adam is one flat sweep.
 *
 * Fine-field layout (modil_prolong / modil_restrict_adjoint)
 *   [instance][field][cells of that field on the finest grid].
 */
#ifndef MODIL_H
#define MODIL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MODIL_ABI_VERSION 1

/* ---- status codes ---------------------------------------------------- */
#define MODIL_OK 0
#define MODIL_ERR_INVALID_ARG (-1) /* null pointer, bad enum, bad value   */
#define MODIL_ERR_SHAPE (-2)       /* grid / level / index out of range   */
#define MODIL_ERR_DTYPE (-3)       /* unsupported dtype or centering      */
#define MODIL_ERR_HIP (-4)         /* HIP runtime error (message has it)  */
#define MODIL_ERR_NONFINITE (-5)   /* a loss term became NaN or Inf       */
#define MODIL_ERR_STATE (-6)       /* call out of order / missing input   */

/* ---- enumerations ---------------------------------------------------- */
#define MODIL_F32 0
#define MODIL_F64 1

#define MODIL_CELL 0 /* values at cell centres                           */
#define MODIL_NODE 1 /* values at grid nodes: POISSON, CAVITY, NS3D    */

/* Residual operators (the discretised PDEs of Sections 3.1-3.5).
 *   POISSON   d = 1,2,3; Laplacian u = f, Dirichlet u = 0 by quadratic
 *             extrapolation (Section 3.1).  1 field, 1 equation.
 *   BURGERS   space-time [t][x]; implicit first-order upwind
 *             finite-volume residual on inner points (Section 3.2) plus
 *             w_reg * (gradient-squared smoothing in x and t).  1 field.
 *   HEAT_KX   space-time [t][x]; implicit heat residual with conductivity
 *             k(x) = softplus(q(x)) (Section 3.4 scheme with k depending on
 *             x), plus w_bc * wall terms.  Fields: u [t][x], q [x].
 *   NS3D      steady Navier-Stokes with Brinkman penalisation in a channel
 *             [z][y][x] (Section 3.5): fields u, v, w, p, chihat with
 *             chi = sigmoid(chihat - chi_shift); with MODIL_FLAG_CHI_FIXED
 *             the fields are u, v, w, p and chi is a given array.
 *   CAVITY    steady 2-D Navier-Stokes, lid-driven cavity [y][x]
 *             (Section 3.3): fields u, v, p.                              */
#define MODIL_OP_POISSON 0
#define MODIL_OP_BURGERS 1
#define MODIL_OP_HEAT_KX 2
#define MODIL_OP_NS3D 3
#define MODIL_OP_CAVITY 4

#define MODIL_FLAG_CHI_FIXED 1
/* MODIL_FLAG_FUSED_RESTRICT: where the fused finest-level kernel runs (FP32
 * cell-based NS3D with coarse levels), it also sums the finest gradient over
 * the fine planes of every level-1 plane (the z part of M_L^T) and stores
 * those sums in place of the finest gradient; an assembly kernel applies
 * T^T in y and x, adds the sums at z-chunk ends and updates level 1.  The
 * workspace then holds the sums (fine cells / 2 x (1 + 4 / chunk planes)
 * values per field).  Same gradient up to the order of the sums; measured
 * slower than the default (finest gradient written, marching restriction)
 * on 128^3 and even on 256^3, so off by default.                          */
#define MODIL_FLAG_FUSED_RESTRICT 2

/* Loss terms, in the order of every terms array. */
#define MODIL_TERM_PDE 0
#define MODIL_TERM_DATA 1
#define MODIL_TERM_REG 2
#define MODIL_TERM_IC 3
#define MODIL_TERM_BC 4
#define MODIL_N_TERMS 5

/* Device arrays attached with modil_set_field. */
#define MODIL_FIELD_FORCING0 0 /* forcing of equation 0..3 (fine grid,  */
#define MODIL_FIELD_FORCING1 1 /* [instance][cells]); subtracted from   */
#define MODIL_FIELD_FORCING2 2 /* the residual of that equation         */
#define MODIL_FIELD_FORCING3 3
#define MODIL_FIELD_CHI 4      /* fixed body fraction, [instance][cells] */

/* Per-instance scalars (modil_set_instance_scalar). */
#define MODIL_SCALAR_RE 0

#define MODIL_MAX_LEVELS 8
#define MODIL_MAX_FIELDS 5

/* ---- problem description ---------------------------------------------
 * dims / lengths list the grid axes slowest first (ndim entries used):
 *   POISSON [z][y][x] (last ndim), BURGERS/HEAT [t][x], NS3D [z][y][x],
 *   CAVITY [y][x].  For space-time grids lengths[0] is the time horizon.
 * Validation: ndim matches the operator, dims[a] divisible by
 * 2^(n_levels-1) with at least 2 coarsest cells per axis (cell-based
 * extrapolation needs two), lengths > 0, batch >= 1, 1 <= n_levels <= 8.
 * MODIL_NODE (POISSON, CAVITY, NS3D; Sections 2.2, 3.1, 3.3, 3.5): dims are cells
 * per axis and a field holds (dims[a] >> l) + 1 nodes per axis on level l,
 * boundary nodes included; T is the node-based interpolation of Section 2.2
 * (even fine nodes copy the coarse node, odd ones average two).  Boundary
 * nodes carry no equation and get a zero gradient; forcing arrays and
 * measurement indices address nodes; the forcing enters interior rows only.
 *   POISSON: interior nodes carry the finite-difference Laplacian (weight
 *   w_pde h^d); the zero Dirichlet value is imposed on the boundary nodes,
 *   which enter their neighbours' stencils as zero whatever the prolonged
 *   field holds there.
 *   CAVITY: interior nodes carry the three cell-based cavity equations
 *   (central differences, stabilised continuity); on the wall nodes the
 *   velocity is imposed (zero, u = u_ref on the lid row y = 1 without its
 *   corners) and the pressure is that of the interior neighbour across the
 *   wall (zero normal derivative), whatever the prolonged fields hold there.
 *   NS3D: interior nodes carry the four cell-based channel equations; on the
 *   boundary nodes the inlet imposes u = (u_ref, 0, 0) and copies p from the
 *   interior node next to it, the outlet imposes p = 0 and copies the
 *   velocity, the free-slip walls impose a zero normal velocity and copy the
 *   other components and p, whatever the prolonged fields hold there.  The
 *   fused FP32 kernel is cell-based; node values run on the generic engine. */
typedef struct {
  int32_t ndim;
  int32_t dims[3];
  double lengths[3];
  int32_t n_levels;
  int32_t centering; /* MODIL_CELL, or MODIL_NODE (see below)               */
  int32_t dtype;     /* MODIL_F32 / MODIL_F64 */
  int32_t op;        /* MODIL_OP_* */
  int32_t flags;     /* MODIL_FLAG_* */
  int32_t batch;     /* independent instances of the same shape */
  int32_t max_meas;  /* capacity: measurement entries over all lists */
  double re;         /* Reynolds number (default for every instance) */
  double diam;       /* characteristic length D (viscosity D / Re) */
  double lambda_;    /* Brinkman penalisation coefficient */
  double chi_shift;  /* chi = sigmoid(chihat - chi_shift) */
  double tau_coef;   /* pressure stabilisation: tau_a = tau_coef * h_a */
  double u_ref;      /* inlet / lid velocity */
  double w_pde;      /* weight of the integrated squared residuals */
  double w_reg;      /* weight of the smoothing terms (BURGERS) */
  double w_bc;       /* weight of the wall terms (HEAT_KX) */
} modil_problem;

typedef struct {
  int32_t n_fields;
  int32_t n_levels;
  int64_t total;                                  /* elements of one pack  */
  int64_t level_offset[MODIL_MAX_LEVELS];         /* start of level l      */
  int64_t level_stride[MODIL_MAX_LEVELS];         /* elements per instance */
  int64_t field_offset[MODIL_MAX_LEVELS][MODIL_MAX_FIELDS]; /* in instance */
  int32_t field_dims[MODIL_MAX_LEVELS][MODIL_MAX_FIELDS][3]; /* z,y,x, 1s  */
  int64_t fine_total;      /* elements of one fine-field array (all inst.) */
  int64_t fine_cells;      /* cells of the finest grid (one instance)      */
  size_t workspace_bytes;  /* device workspace modil_create needs          */
} modil_pack_layout;

typedef struct {
  double lr, beta1, beta2, eps;
} modil_adam_hp;

typedef struct modil_ctx modil_ctx;

/* ---- version and errors ---------------------------------------------- */
int modil_abi_version(void);
const char *modil_status_str(int status);
/* Message of the last failure on ctx (NULL: last failure of a call that
 * had no context, e.g. modil_layout / modil_create). Never NULL. */
const char *modil_last_error(const modil_ctx *ctx);

/* ---- layout and lifetime ----------------------------------------------
 * modil_layout validates the problem and fills the pack layout and the
 * workspace size.  Host only; needs no GPU.
 * modil_create validates again, binds the caller's workspace (device, at
 * least layout.workspace_bytes, 256-byte aligned) and the stream
 * (hipStream_t, NULL = default stream) and the current HIP device.
 * modil_destroy releases host-side state only (the caller frees memory).  */
int modil_layout(const modil_problem *problem, modil_pack_layout *out);
int modil_create(const modil_problem *problem, void *workspace, size_t workspace_bytes,
                 void *hip_stream, modil_ctx **out);
int modil_destroy(modil_ctx *ctx);
int modil_set_stream(modil_ctx *ctx, void *hip_stream);

/* ---- problem data -------------------------------------------------------
 * Measurements {(x_k, u_k)} (Sections 3.2, 3.4, 3.5): a list of n cells of
 * one field of one instance, given as flat C-order indices into that
 * field's finest grid, with values; the loss gains
 *     weight * sum_k (u(cell_k) - value_k)^2
 * in term `term` (MODIL_TERM_DATA, or MODIL_TERM_IC for an initial
 * condition).  Host arrays are copied (synchronously) into the workspace;
 * values are kept in double.  Indices must be in range and unique within
 * the list (MODIL_ERR_SHAPE / MODIL_ERR_INVALID_ARG), the total over all
 * lists must not exceed max_meas.  With node-based values an index on a
 * boundary node is rejected (MODIL_ERR_SHAPE): the boundary nodes hold
 * imposed values that no equation reads from the unknowns, so a measurement
 * there would fit a free value.  Lists accumulate until
 * modil_clear_measurements.                                              */
int modil_set_measurements(modil_ctx *ctx, int32_t instance, int32_t field, int32_t term,
                           int32_t n, const int32_t *cell_idx_host,
                           const double *values_host, double weight);
int modil_clear_measurements(modil_ctx *ctx);

/* Attach (or detach with NULL) a fine-grid device array of the problem dtype,
 * layout [instance][cells]: forcing subtracted from residual equation e
 * (manufactured solutions, Section 3.1), or the fixed body fraction chi of
 * NS3D with MODIL_FLAG_CHI_FIXED.  The array must stay valid while used. */
int modil_set_field(modil_ctx *ctx, int32_t which, const void *dev_ptr);

/* Per-instance scalar (MODIL_SCALAR_RE): Reynolds number of one instance. */
int modil_set_instance_scalar(modil_ctx *ctx, int32_t instance, int32_t which, double value);

/* ---- the iteration -------------------------------------------------------
 * modil_prolong: fine = M_L(theta) for every field (Section 2.2).
 * modil_restrict_adjoint: grad = M_L^T fine, the exact transpose.
 * modil_loss: terms[instance][MODIL_N_TERMS] (double, device) of the loss
 *   at theta.
 * modil_loss_grad: terms and grad = dL/dtheta on every level (exact
 *   adjoint: transposed stencils, then M_L^T).  Nothing of the fine field
 *   is kept between calls.
 * modil_adam: elementwise Adam over the whole pack (Kingma & Ba, cited in
 *   Section 2.1): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 *   theta_out <- theta_in - lr/(1-b1^t) * m / (sqrt(v/(1-b2^t)) + eps).
 *   step t >= 1.  theta_out may equal theta_in.
 * modil_step: one full iteration -- loss terms at theta_in (written to terms
 *   if not NULL), gradient, and Adam into theta_out.  theta_out must differ
 *   from theta_in (tiles read neighbours of theta_in while theta_out is
 *   written) -> MODIL_ERR_INVALID_ARG.
 * modil_run: n_steps >= 1 iterations of modil_step with steps
 *   step0 .. step0 + n_steps - 1, theta alternating between the two packs:
 *   step step0 + k reads theta_a and writes theta_b for even k, the reverse
 *   for odd k, so the result is in theta_b if n_steps is odd, else theta_a.
 *   Loss terms of the last iteration go to terms (if not NULL).  The same
 *   arithmetic as calling modil_step n_steps times, without a host round
 *   trip per iteration.  theta_a must differ from theta_b.
 * modil_residual_metric: r[instance] = RMS over the points carrying the PDE
 *   equations and over the equations of the cell-integrated residual,
 *   sqrt(sum (V R)^2 / (n_eq * n_points)), evaluated in double from the PDE
 *   term.  The points are every cell (cell-based values), the interior nodes
 *   (node-based values) or the inner points n >= 1, 1 <= i <= N_x - 2 of the
 *   space-time grids (BURGERS, HEAT_KX).                                  */
int modil_prolong(modil_ctx *ctx, const void *theta_pack, void *fine_out);
int modil_restrict_adjoint(modil_ctx *ctx, const void *fine_in, void *grad_pack_out);
int modil_loss(modil_ctx *ctx, const void *theta_pack, double *terms);
int modil_loss_grad(modil_ctx *ctx, const void *theta_pack, void *grad_pack, double *terms);
int modil_adam(modil_ctx *ctx, const void *theta_in, void *theta_out, void *m, void *v,
               const void *grad, const modil_adam_hp *hp, int64_t step);
int modil_step(modil_ctx *ctx, const void *theta_in, void *theta_out, void *m, void *v,
               const modil_adam_hp *hp, int64_t step, double *terms);
int modil_run(modil_ctx *ctx, void *theta_a, void *theta_b, void *m, void *v,
              const modil_adam_hp *hp, int64_t step0, int32_t n_steps, double *terms);
int modil_residual_metric(modil_ctx *ctx, const void *theta_pack, double *r);

/* ---- allocation-free prolongation -------------------------------------------
 * For callers that cannot allocate device memory or provide a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): modil_prolong_noalloc computes fine = M_L(theta) like
 * modil_prolong, for a problem given directly (no context), on `hip_stream`
 * of the current device.  The intermediate Horner levels go to a device
 * array of MODIL_NOALLOC_SCRATCH_BYTES that the library holds on every GPU
 * it runs on until the process ends; the call allocates nothing, host or
 * device, on success.  theta_pack and fine_out are device arrays in the
 * layouts above (caller-owned).  A problem whose intermediate levels need
 * more scratch than that (bytes of the pack up to the coarsest level) fails
 * with MODIL_ERR_SHAPE before any launch; an invalid problem as in
 * modil_layout.  Every call on one GPU uses that GPU's one array: calls
 * whose work overlaps on one GPU (other streams, other threads) race, and
 * must be ordered by the caller.  Nothing in the array needs clearing: each
 * call writes every value it reads.                                       */
#define MODIL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int modil_prolong_noalloc(const modil_problem *problem, const void *theta_pack, void *fine_out,
                          void *hip_stream);

/* ---- options --------------------------------------------------------------
 * MODIL_OPT_FUSED (default 1): use the fused finest-level kernel where one
 * exists (NS3D in FP32, one Reynolds number for the batch, measurements on
 * velocity / pressure only); 0 selects the generic stencil engine.  Both
 * compute the same iteration.                                             */
#define MODIL_OPT_FUSED 0
/* MODIL_OPT_MARCH (default 1): transfer levels whose fields span every axis
 * they have with the lane-shift kernels -- the marching restriction (each
 * fine value loaded once per wave, Adam fused; node-based levels with lanes
 * over the flattened coarse plane) and the block prolongation (one coarse
 * cell per thread writing its 2^d fine cells); 0 selects the per-cell
 * kernels.  Same results up to the order of the sums.
 * MODIL_OPT_MARCH_TILE (default 0 = automatic): coarse rows and planes per
 * wave of the marching kernel as 64 * rows + planes: rows 2 with planes 1,
 * 2, 4 or 8; rows 4 with planes 1, 2, 4, 8 or 16; rows 8 with planes 4 or 8.
 * A tile that does not divide a level's grid leaves that level to the
 * gather kernel.                                                          */
#define MODIL_OPT_MARCH 1
#define MODIL_OPT_MARCH_TILE 2
/* MODIL_OPT_TAIL (default 1): the small coarse levels of each instance (from
 * the first level that fits in one block's LDS together with the next one)
 * are prolonged, and restricted with Adam, by one launch with one block per
 * instance working in LDS; 0 launches one kernel per level instead.       */
#define MODIL_OPT_TAIL 3
/* MODIL_OPT_TILE (default 1): the generic engine on 2-D problems stages tiles
 * of the fine fields in LDS and forms every cell's residuals once; 0 selects
 * the per-cell kernel, which forms the residuals of each cell's neighbours
 * again.  Same results up to the order of the sums.                       */
#define MODIL_OPT_TILE 4
/* MODIL_OPT_TWO_PASS (default 1): the generic engine on 3-D problems forms
 * every cell's residuals once and writes the face sensitivities of its star
 * to workspace scratch, then gathers them per cell; 0 selects the per-cell
 * kernel, which forms the residuals of each cell's neighbours again.  The
 * scratch (6 x fields coupled through neighbours x cells) is part of the
 * workspace only where the two-pass form can run: 3-D problems except FP32
 * cell-based NS3D, whose generic engine (when the fused kernel does not
 * apply) is always the per-cell kernel.  Same results up to the order of
 * the sums.                                                               */
#define MODIL_OPT_TWO_PASS 5
int modil_set_option(modil_ctx *ctx, int32_t option, int64_t value);
/* modil_fused_active: 1 if the next loss / gradient / step of this context
 * runs the fused finest-level kernel (option on and the problem, its
 * measurements and Reynolds numbers admit it), 0 if the generic engine, or a
 * negative status for a NULL context.                                      */
int modil_fused_active(const modil_ctx *ctx);

/* ---- health and timing ---------------------------------------------------
 * modil_check: synchronises the stream; returns MODIL_ERR_NONFINITE if a
 * loss term computed since the last check was NaN or Inf (and clears the
 * flag), MODIL_ERR_HIP on an asynchronous runtime error, else MODIL_OK.
 * modil_profile: enable (1) / disable (0) HIP-event timing of every kernel
 * launch class; modil_profile_read returns the accumulated milliseconds and
 * launch count of one class (synchronises), then resets it.
 * Classes: 0 fine-level kernel, 1 Horner (coarse prolongation),
 * 2 restriction, 3 Adam, 4 reductions / data terms, 5 L-BFGS dot products,
 * 6 L-BFGS vector updates (direction, trial point, new pair, accepted point). */
int modil_check(modil_ctx *ctx);
int modil_profile(modil_ctx *ctx, int32_t enable);
int modil_profile_read(modil_ctx *ctx, int32_t kernel_class, double *total_ms, int64_t *count);

/* ---- learned warm start: a small convolutional network --------------------
 * Not part of the paper: a network that maps measurements of a lid-driven
 * cavity instance to the coarse multigrid levels of its solution, used as
 * the starting point of the iteration (cold-start mODIL stays the fallback).
 *
 * Input image [batch][4][size][size] (float): channels u_obs, v_obs, mask of
 * observed cells, (Re - re_center) / re_scale.  Fixed topology, parameters
 * in bf16 (rounded to nearest even from float masters), float accumulation:
 *   trunk 1: 4 -> width1, 4x4 kernel, stride 4          -> size/4
 *   trunk 2: width1 -> width2, 3x3, stride 2, pad 1     -> size/8
 *   trunk 3: width2 -> width3, 3x3, stride 2, pad 1     -> size/16
 *   head k (k = 1, 2, 3): trunk k -> out_ch, 3x3, stride 1, pad 1
 * ReLU after the trunk layers, none after the heads.  Output: the three head
 * maps concatenated, [batch][out_ch][size/4]^2, then size/8, then size/16.
 * Parameter pack (float / bf16, same layout): for the layers in the order
 * trunk 1..3, head 1..3, the weights [co][ci][k][k] then the biases [co].
 * Loss: mean squared error over all outputs, accumulated in double.       */
typedef struct {
  int32_t batch;   /* maximum images per call */
  int32_t size;    /* image side, a multiple of 16 */
  int32_t n_obs;   /* observed cells per image */
  int32_t width1, width2, width3, out_ch;
  double re_center, re_scale;
} modil_cnn_desc;

typedef struct {
  int64_t n_params;        /* parameters (weights and biases)            */
  int64_t w_offset[6];     /* offsets of the layers' weights in the pack */
  int64_t b_offset[6];     /* offsets of the layers' biases              */
  int64_t img_size;        /* floats of one input image                  */
  int64_t act_size;        /* floats of the trunk activations, one image */
  int64_t out_size;        /* floats of the three head maps, one image   */
  size_t workspace_bytes;
} modil_cnn_layout_t;

typedef struct modil_cnn modil_cnn;

int modil_cnn_layout(const modil_cnn_desc *desc, modil_cnn_layout_t *out);
int modil_cnn_create(const modil_cnn_desc *desc, void *workspace, size_t workspace_bytes,
                     void *hip_stream, modil_cnn **out);
int modil_cnn_destroy(modil_cnn *net);
/* img[b] from obs_idx[b][n_obs] (flat cell indices, unique per image),
 * obs_u, obs_v [b][n_obs] and re[b] (all device arrays). */
int modil_cnn_rasterize(modil_cnn *net, int32_t batch, const int32_t *obs_idx, const float *obs_u,
                        const float *obs_v, const float *re, float *img);
/* acts [batch][act_size] (trunk activations), out [batch][out_size]. */
int modil_cnn_forward(modil_cnn *net, int32_t batch, const uint16_t *params_bf16, const float *img,
                      float *acts, float *out);
/* loss (device double) = mean over all outputs of (out - target)^2 and the
 * gradient of the loss with respect to every parameter (float pack), for
 * the acts / out of the preceding forward call on the same input. */
int modil_cnn_loss_backward(modil_cnn *net, int32_t batch, const uint16_t *params_bf16,
                            const float *img, const float *acts, const float *out,
                            const float *target, double *loss, float *grad);
/* Adam on the float masters, then params_bf16 = round-to-nearest-even(master). */
int modil_cnn_adam(modil_cnn *net, float *master, uint16_t *params_bf16, float *m, float *v,
                   const float *grad, const modil_adam_hp *hp, int64_t step);
/* params_bf16 = round-to-nearest-even(master) */
int modil_cnn_to_bf16(modil_cnn *net, const float *master, uint16_t *params_bf16);

/* ---- L-BFGS ----------------------------------------------------------------
 * Limited-memory BFGS on the loss and gradient of a context: the optimiser of
 * most results of the paper (SciPy's L-BFGS-B without bounds, Section 2.1; a
 * history of 50 pairs in Section 3.1).
 *   direction  d = -H g, H the L-BFGS matrix of the stored pairs with
 *              H0 = gamma I, gamma = s^T y / y^T y of the newest pair, applied
 *              through its compact representation (Byrd, Nocedal & Schnabel
 *              1994): two passes over the stored pairs per iteration;
 *              d = -g while no pair is stored
 *   step       a line search that brackets a step satisfying the strong Wolfe
 *              conditions and zooms in (Nocedal & Wright, Algorithms 3.5 and
 *              3.6) with safeguarded cubic trial steps; first trial step
 *              min(1, 1/||d||) without pairs, else 1; the bracketing phase
 *              doubles the step; after max_evals evaluations the best point
 *              with sufficient decrease is taken (status 1), if there is one
 *   memory     the pair s = alpha d, y = g_new - g is stored when
 *              s^T y > eps y^T y (FP64 unit roundoff); beyond `history` pairs
 *              the oldest is dropped; a non-descent direction clears it
 * The objective is the sum of all loss terms of all batch instances; the
 * instances are optimised as one vector.
 *
 * State: a caller-provided device workspace of modil_lbfgs_workspace bytes
 * (256-byte aligned): history + 1 pair slots and four more pack-sized
 * vectors in the problem dtype, and FP64 partial sums.  The small matrices S^T Y and Y^T Y
 * stay on the host in FP64.  Dot products accumulate in FP64 in a fixed order
 * (deterministic).  The object keeps pointers into the workspace and uses the
 * context's stream; it allocates pinned host memory for the scalars it
 * exchanges with the device.  Every line-search evaluation synchronises the
 * stream once.
 *
 * modil_lbfgs_step: one iteration on theta (device pack, updated in place to
 * the accepted point).  The first call after create / reset also evaluates
 * the loss and gradient at theta.  Between calls theta must not change; call
 * modil_lbfgs_reset after changing it.  On status 2 (no step found) theta is
 * unchanged and the memory is cleared.                                    */
typedef struct modil_lbfgs modil_lbfgs;

#define MODIL_LBFGS_MAX_HISTORY 64

typedef struct {
  int32_t history;    /* stored pairs m, 1..MODIL_LBFGS_MAX_HISTORY */
  int32_t max_evals;  /* loss-and-gradient evaluations per line search, >= 2 */
  double c1, c2;      /* Wolfe constants, 0 < c1 < c2 < 1 */
} modil_lbfgs_params;

typedef struct {
  double loss;        /* objective at theta after the call */
  double grad_norm;   /* ||gradient||_2 at theta after the call */
  double step;        /* accepted step length (0 if none) */
  int32_t evals;      /* evaluations made by the call */
  int32_t status;     /* 0 strong Wolfe step, 1 sufficient decrease only, 2 no step */
  int32_t pairs;      /* stored pairs after the call */
  int32_t iteration;  /* iterations since create / reset */
} modil_lbfgs_info;

int modil_lbfgs_workspace(const modil_ctx *ctx, int32_t history, size_t *bytes);
int modil_lbfgs_create(modil_ctx *ctx, const modil_lbfgs_params *params, void *workspace,
                       size_t workspace_bytes, modil_lbfgs **out);
int modil_lbfgs_destroy(modil_lbfgs *lb);
int modil_lbfgs_reset(modil_lbfgs *lb);
int modil_lbfgs_step(modil_lbfgs *lb, void *theta, modil_lbfgs_info *info);

#ifdef __cplusplus
}
#endif
#endif /* MODIL_H */
