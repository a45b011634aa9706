/*
 * vpinn.h -- C ABI of the MI355X (gfx950) FastVPINNs training hot path.
 *
 * The library evaluates, on one GPU, the variational PINN loss of FastVPINNs
 * (arXiv 2404.12063) and its gradient with respect to the network weights:
 *
 *   R[e,k] = eps * sum_q ( u_x G_x + u_y G_y )[e,k,q] - F[e,k]          (Alg. 3)
 *   L      = c_v sum_{e,k} R[e,k]^2 + tau  mean_b (u(x_b) - g_b)^2
 *                                    + gamma mean_s (u(x_s) - d_s)^2     (Sec. 2.3, 4.7)
 *
 * where u is a tanh multilayer perceptron (Sec. 2.2), G_x, G_y are the
 * premultiplied test-function gradients of Sec. 4.4 (quadrature weight times
 * det J times the physical gradient of test function k at quadrature point q
 * of element e) and F is the forcing matrix of Appendix A.2.
 *
 * Conventions shared by every call
 *  - Status codes are returned; nothing throws across the ABI.  On error,
 *    vpinn_last_error() gives a message for the calling thread.
 *  - "device" pointers are HIP device memory of the current device (for
 *    example torch CUDA tensors' data_ptr()), contiguous, caller-owned.
 *  - "host" pointers are ordinary host memory, read during the call only.
 *  - `stream` is a hipStream_t passed as void*; NULL is the null stream.
 *    Kernel launches are asynchronous on it; argument errors are reported
 *    synchronously, device faults at the caller's next synchronisation.
 *  - Network parameters use one flat float32 layout (width H, L hidden layers):
 *      W1[H][2], b1[H], then for l = 2..L: W_l[H][H], b_l[H], then
 *      W_out[H], b_out                       (vpinn_n_params(H, L) floats)
 *    or, for a network with a second output (the space-dependent diffusion
 *    coefficient of Sec. 4.7.2), W_out[2][H], b_out[2] at the end
 *    (vpinn_n_params_out(H, L, 2) floats).
 *    all matrices row-major with the output neuron as the row index.
 *  - Distinct problem objects may be used from different threads; one object
 *    must not be used by two calls at once.
 */
#ifndef VPINN_H
#define VPINN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t vpinn_status;
#define VPINN_OK 0
#define VPINN_E_INVALID (-1)     /* bad argument: null pointer, order out of range, size mismatch */
#define VPINN_E_MESH (-2)        /* bad mesh: vertex index out of range, det J <= 0 (clockwise or
                                    non-convex element); the message names the element */
#define VPINN_E_NOMEM (-3)       /* device or host allocation failed */
#define VPINN_E_NONFINITE (-4)   /* the forcing function returned a NaN or an infinity */
#define VPINN_E_DEVICE (-5)      /* a HIP runtime call failed */
#define VPINN_E_UNSUPPORTED (-6) /* a configuration outside the compiled kernels' limits */

/* limits of the compiled kernels */
#define VPINN_MAX_WIDTH 32       /* hidden width H (padded to 32 inside the kernels) */
#define VPINN_MAX_HIDDEN 4       /* hidden layers L */
#define VPINN_MAX_QUAD_ORDER 100 /* GLL points per direction n (N_quad = n^2) */
#define VPINN_MAX_TEST_ORDER 30  /* test functions per direction N_t (N_test = N_t^2) */

/* ------------------------------------------------------------------------ */
/* Mesh (Sec. 3.2 and Appendix A.1): quadrilaterals given by 4 vertex ids,   */
/* counter-clockwise, matched in order to the reference corners (-1,-1),     */
/* (1,-1), (1,1), (-1,1) of the bilinear map.                                */
/* ------------------------------------------------------------------------ */
typedef struct vpinn_mesh {
    int64_t n_nodes;
    const double *xy;      /* host, [n_nodes][2] vertex coordinates */
    int64_t n_elem;
    const int32_t *quad;   /* host, [n_elem][4] vertex ids */
} vpinn_mesh;

/* Forcing f of -Lap u = f (Sec. 2.1). */
typedef double (*vpinn_scalar_fn)(double x, double y, void *user);
#define VPINN_FORCING_CALLBACK 0 /* f = fn(x, y, user), called on the host once per quadrature point */
#define VPINN_FORCING_SINSIN 1   /* f = amp * sin(kx x) * sin(ky y), evaluated on the device in FP64 */
typedef struct vpinn_forcing {
    int32_t kind;
    double amp, kx, ky;
    vpinn_scalar_fn fn;
    void *user;
} vpinn_forcing;

typedef struct vpinn_problem vpinn_problem;

/*
 * vpinn_assemble -- one-time precomputation of the premultiplied tensors
 * (Sec. 4.2 and 4.4, Appendix A.2).  Builds, in FP64 on the device, and
 * stores in FP32 in device memory owned by the returned problem:
 *   G_x, G_y [n_elem][N_test][N_quad]   w_q * det J * (d v_k / dx, d v_k / dy) at point q
 *   F        [n_elem][N_test]           sum_q w_q det J f(x_q) v_k(x_q)
 *   X        [n_elem][N_quad][2]        physical quadrature points
 * with Gauss-Lobatto-Legendre quadrature of quad_order points per direction
 * (q = j*n + i, i the xi index) and test functions
 * v_k = phi_r(xi) phi_s(eta), phi_r = P_{r+1} - P_{r-1}, r, s = 1..test_order,
 * k = (s-1)*test_order + (r-1).
 * Errors: VPINN_E_INVALID (null pointers, quad_order outside 2..100,
 * test_order outside 1..30, n_elem < 1), VPINN_E_MESH (vertex id out of range or
 * det J <= 0 at a corner, with the element id in the message), VPINN_E_NONFINITE,
 * VPINN_E_NOMEM, VPINN_E_DEVICE.  Synchronous: returns after the tensors are built.
 * When every element is a translate of element 0 with its vertices in the same
 * order (a uniform mesh), G_x and G_y are identical for all elements and are
 * stored once (the single reference premultiplier of Algorithm 2, [N_test][N_quad]);
 * vpinn_read_tensor still returns them per element.
 * On success *out owns all device memory; free it with vpinn_problem_free.
 */
vpinn_status vpinn_assemble(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order,
                            const vpinn_forcing *forcing, void *stream, vpinn_problem **out);

/*
 * vpinn_assemble_cd2d -- the convection-diffusion operator -eps Lap u + b . grad u
 * = f (Sec. 2.1; the gear problem of Sec. 4.6.4) with constant eps > 0 and
 * b = (bx, by).  Its cell residual adds sum_q w_q det J (b . grad u)(x_q) v_k(x_q)
 * to eps times the diffusion term; both are linear in (u_x, u_y), so they are
 * folded into the premultiplied tensors at assembly:
 *   G_x = w_q det J (eps dv_k/dx + bx v_k),  G_y = w_q det J (eps dv_k/dy + by v_k)
 * and every later call (loss, gradient, batches, graphs) runs unchanged, at no
 * extra cost per step.  vpinn_assemble is the case eps = 1, b = 0.  Because eps
 * is folded, loss calls on such a problem take no d_eps / d_grad_eps
 * (VPINN_E_INVALID).  Errors: as vpinn_assemble, plus VPINN_E_INVALID for a
 * non-finite or non-positive eps or a non-finite b.
 */
vpinn_status vpinn_assemble_cd2d(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double eps,
                                 double bx, double by, const vpinn_forcing *forcing, void *stream,
                                 vpinn_problem **out);

/*
 * vpinn_assemble_vardiff -- the space-dependent diffusion operator
 * -div(eps(x, y) grad u) + b . grad u = f of the inverse problem of Sec. 4.7.2,
 * where eps(x, y) is the network's second output.  The cell residual is
 *   R[e,k] = sum_q eps(x_q) (u_x G_x + u_y G_y)[e,k,q]
 *          + sum_q (bx u_x + by u_y)(x_q) M[e,k,q] - F[e,k],
 * with G_x, G_y the plain diffusion weights (as vpinn_assemble) and
 * M[e,k,q] = w_q det J v_k(x_q) stored as a third tensor (eps varies per point,
 * so nothing can be folded).  Loss calls on such a problem need
 * cfg->n_outputs = 2, the fused path, N_quad <= 256 and N_test <= 32, and take no
 * d_eps / d_grad_eps; everything else returns VPINN_E_UNSUPPORTED or
 * VPINN_E_INVALID.  Errors: as vpinn_assemble, plus VPINN_E_INVALID for a
 * non-finite b.
 */
vpinn_status vpinn_assemble_vardiff(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double bx,
                                    double by, const vpinn_forcing *forcing, void *stream, vpinn_problem **out);

/*
 * vpinn_assemble_matrix_free -- the same operators without the premultiplied
 * tensors: only F, the points and 8 floats of geometry per element are stored
 * (the bilinear map's coefficients, App. A.1), and every loss call regenerates
 * w_q (d v_xi - b v_eta, -c v_xi + a v_eta) for the tensor-product test functions
 * by sum factorisation, first along xi and then along eta (the closed form of G
 * in Sec. 4.2 and App. A.1).  HBM per element drops from 8 N_test N_quad bytes to
 * 32; the results equal those of the stored tensors up to FP32 rounding.
 *   eps, bx, by: the constant convection-diffusion coefficients, as
 *     vpinn_assemble_cd2d (1, 0, 0: Poisson, where a trainable eps is accepted);
 *   variable_diffusion = 1: the space-dependent operator of vpinn_assemble_vardiff
 *     (eps ignored; the network's second output is the coefficient).
 * Needs quad_order <= 16 (N_quad <= 256); the fused path only (the plain path and
 * vpinn_residual return VPINN_E_UNSUPPORTED, vpinn_read_tensor of G or M
 * VPINN_E_INVALID).  Errors: as vpinn_assemble_cd2d, plus VPINN_E_UNSUPPORTED for
 * quad_order > 16.
 */
vpinn_status vpinn_assemble_matrix_free(const vpinn_mesh *mesh, int32_t quad_order, int32_t test_order, double eps,
                                        double bx, double by, int32_t variable_diffusion,
                                        const vpinn_forcing *forcing, void *stream, vpinn_problem **out);

/*
 * vpinn_set_boundary -- Dirichlet points x_b and values g_b of the boundary term
 * tau mean_b (u(x_b) - g_b)^2 (Sec. 2.2).  Host arrays xy [n][2] and g [n] are
 * copied to the device (as FP32); a later call replaces the previous set; n = 0
 * clears it.  Synchronous.  Errors: VPINN_E_INVALID (null pointer with n > 0,
 * n < 0), VPINN_E_NOMEM, VPINN_E_DEVICE.
 */
vpinn_status vpinn_set_boundary(vpinn_problem *p, int64_t n, const double *xy, const double *g);
/*
 * vpinn_set_shared_points -- with enable = 1, the fused path evaluates the network
 * once per distinct interior quadrature point instead of once per (element, point)
 * slot: GLL points on an edge or a vertex shared by several elements (Sec. 3.1
 * places them at the same physical location) are found from the mesh topology
 * (vertex ids, and the position along an edge from its lower-numbered vertex),
 * the contraction reads each slot's (u_x, u_y) from its point, and the adjoints
 * of a point's slots are added in slot order before the reverse sweep.  The
 * result is that of per-slot evaluation up to FP32 rounding; the network work
 * falls by up to 1 - ((n-1)/n)^2.  `mesh` must be the mesh the problem was
 * assembled from (checked: element count, and every shared slot's point within
 * 1e-6 of its partner's).  enable = 0 returns to per-slot evaluation.  The plain
 * path ignores the setting.
 * Errors: VPINN_E_INVALID (null, counts differ), VPINN_E_MESH (a shared slot's
 * point differs), VPINN_E_DEVICE.
 */
vpinn_status vpinn_set_shared_points(vpinn_problem *p, const vpinn_mesh *mesh, int32_t enable);

/*
 * vpinn_set_sensors -- sensor points x_s and observed values d_s of the data term
 * gamma mean_s (u(x_s) - d_s)^2 of the inverse problems (Sec. 4.7: observations
 * of u inside the domain, from which eps is recovered).  Host arrays xy [n][2]
 * and d [n] are copied to the device (as FP32) after the boundary points; a
 * later call replaces the previous set; n = 0 clears it.  Synchronous; a batch
 * planned before the call must be planned again (see vpinn_batch_create).
 * Errors: VPINN_E_INVALID (null pointer with n > 0, n < 0), VPINN_E_NOMEM,
 * VPINN_E_DEVICE.
 */
vpinn_status vpinn_set_sensors(vpinn_problem *p, int64_t n, const double *xy, const double *d);

typedef struct vpinn_problem_info {
    int64_t n_elem, n_quad, n_test;  /* N_elem, N_quad = n^2, N_test = N_t^2 */
    int64_t n_points;                /* N_elem * N_quad interior quadrature points */
    int64_t n_boundary, n_sensors;
    int32_t quad_order, test_order;
    double diffusion, velocity_x, velocity_y; /* folded operator coefficients (1, 0, 0: Poisson) */
    int32_t shared_premultiplier;    /* 1: all elements are translates of one shape, and G_x, G_y are
                                        stored once (Algorithm 2's reference premultiplier) */
    int32_t variable_diffusion;      /* 1: from vpinn_assemble_vardiff (diffusion = 0: it is the
                                        network's second output) */
    int32_t matrix_free;             /* 1: from vpinn_assemble_matrix_free (no G stored) */
    int64_t n_distinct_points;       /* vpinn_set_shared_points: distinct interior points (0: off) */
} vpinn_problem_info;

vpinn_status vpinn_get_info(const vpinn_problem *p, vpinn_problem_info *info);

/* Copy one assembled tensor to host memory: which = 0 G_x, 1 G_y, 2 F, 3 X.
 * `count` must equal the tensor's element count (floats).  Synchronous. */
#define VPINN_TENSOR_GX 0
#define VPINN_TENSOR_GY 1
#define VPINN_TENSOR_F 2
#define VPINN_TENSOR_X 3
#define VPINN_TENSOR_M 4 /* w_q det J v_k, problems from vpinn_assemble_vardiff only */
vpinn_status vpinn_read_tensor(const vpinn_problem *p, int32_t which, float *host_dst, int64_t count);

/* ------------------------------------------------------------------------ */
/* Loss and gradient (Algorithm 3 with its backward pass)                    */
/* ------------------------------------------------------------------------ */
#define VPINN_PATH_FUSED 0 /* forward, contraction + adjoint, reverse sweep and reduction kernels */
#define VPINN_PATH_PLAIN 1 /* unfused kernel sequence that materialises every intermediate */
#define VPINN_NORM_TEST 0  /* c_v = 1/N_test: mean over test functions, sum over elements (Alg. 3) */
#define VPINN_NORM_ELEM 1  /* c_v = 1/N_elem: the variational-loss equation of Sec. 2.3 */

typedef struct vpinn_loss_cfg {
    int32_t n_hidden;  /* L, 1..VPINN_MAX_HIDDEN */
    int32_t width;     /* H, 1..VPINN_MAX_WIDTH */
    float tau;         /* boundary weight */
    float gamma;       /* sensor weight */
    int32_t loss_norm; /* VPINN_NORM_TEST or VPINN_NORM_ELEM */
    int32_t path;      /* VPINN_PATH_FUSED or VPINN_PATH_PLAIN */
    int32_t n_outputs; /* 0 or 1: u only; 2: u and eps(x, y), for problems from vpinn_assemble_vardiff
                          (fused path only) */
} vpinn_loss_cfg;

int64_t vpinn_n_params(int32_t width, int32_t n_hidden);
/* parameters of a network with n_outputs (1 or 2) linear outputs; -1 if out of range */
int64_t vpinn_n_params_out(int32_t width, int32_t n_hidden, int32_t n_outputs);

/*
 * vpinn_loss_and_grad -- one forward + adjoint evaluation.
 *   d_params   device, vpinn_n_params_out(width, n_hidden, n_outputs) floats
 *              (vpinn_n_params for one output)
 *   d_eps      device, 1 float: the diffusion coefficient eps of -eps Lap u = f
 *              (Sec. 4.7.1); NULL means eps = 1; must be NULL for a problem from
 *              vpinn_assemble_cd2d or vpinn_assemble_vardiff (or their
 *              matrix-free forms), whose coefficients are fixed or a network output
 *   d_loss     device, 4 floats written: L, L_v, L_b, L_s (L_b and L_s are the
 *              unweighted means; L = L_v + tau L_b + gamma L_s)
 *   d_grad     device, as many floats as d_params, written: dL/dtheta; NULL skips
 *              the backward pass
 *   d_grad_eps device, 1 float written: dL/deps; may be NULL
 * The problem keeps a device workspace that the first call of each path
 * allocates (and a call with more boundary or sensor points grows); later calls
 * allocate nothing.  Deterministic: fixed-order reductions, no float atomics.
 * Arithmetic: FP32 throughout, loss totals in FP64.  The fused path evaluates the
 * network's dense products on the bf16 matrix cores as FP32 products: each operand
 * split exactly into three bf16 pieces, the six significant piece products
 * accumulated in FP32 (no less accurate than an FP32 matrix product); the plain
 * path uses FP32 vector multiply-adds.
 */
vpinn_status vpinn_loss_and_grad(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                                 const float *d_eps, float *d_loss, float *d_grad, float *d_grad_eps,
                                 void *stream);

/*
 * vpinn_residual -- the residual matrix alone: d_R device [n_elem][N_test] floats,
 * R = eps * sum_q (u_x G_x + u_y G_y) - F at the given parameters.
 */
vpinn_status vpinn_residual(vpinn_problem *p, const vpinn_loss_cfg *cfg, const float *d_params,
                            const float *d_eps, float *d_R, void *stream);

/*
 * vpinn_eval_network -- u, du/dx, du/dy of the network (Sec. 2.2) at n points:
 * the prediction step whose time the paper's Appendix table sets against FEM.
 *   d_xy device [n][2] floats; d_u, d_ux, d_uy device [n] floats (any may be NULL).
 * One kernel launch on `stream`, no allocation; with d_ux and d_uy both NULL only
 * the value products run (a third of the matrix work).  n = 0 does nothing.
 * Errors: VPINN_E_INVALID (null params, null d_xy with n > 0, n < 0),
 * VPINN_E_UNSUPPORTED (width or n_hidden out of range), VPINN_E_DEVICE.
 */
vpinn_status vpinn_eval_network(int32_t width, int32_t n_hidden, const float *d_params, int64_t n,
                                const float *d_xy, float *d_u, float *d_ux, float *d_uy, void *stream);

/*
 * vpinn_eval_network_heads -- as vpinn_eval_network for a network with n_outputs
 * (1 or 2) linear outputs on shared hidden layers (parameters laid out as
 * vpinn_n_params_out); with two, d_e [n] receives the second output, the
 * predicted diffusion coefficient eps(x, y) of the inverse problem of Sec. 4.7.2.
 * Any output pointer may be NULL.  Errors: VPINN_E_INVALID (n_outputs not 1 or 2,
 * d_e with one output, null params, n < 0), VPINN_E_UNSUPPORTED (shape).
 */
vpinn_status vpinn_eval_network_heads(int32_t width, int32_t n_hidden, int32_t n_outputs, const float *d_params,
                                      int64_t n, const float *d_xy, float *d_u, float *d_ux, float *d_uy,
                                      float *d_e, void *stream);

/*
 * vpinn_eval_error -- accuracy of a prediction (Sec. 4 reports the mean absolute
 * error of u on a 100 x 100 grid and point-wise errors of u and of the predicted
 * diffusion coefficient): with p the network's output `output` (0: u, 1: the
 * second output of a two-output network) at the n points d_xy (device [n][2]
 * floats) and d_ref (device [n] floats) the reference values,
 *   d_out[0] = (1/n) sum |p - ref|,  d_out[1] = max |p - ref|,
 *   d_out[2] = ||p - ref||_2 / ||ref||_2   (inf or nan if ref is all zero),
 * d_out a device array of 3 doubles, sums in FP64 in a fixed order.  Uses a
 * per-thread device workspace of n floats.  Errors: VPINN_E_INVALID (n < 1, null
 * pointer, output not below n_outputs), VPINN_E_UNSUPPORTED (shape).
 */
vpinn_status vpinn_eval_error(int32_t width, int32_t n_hidden, int32_t n_outputs, int32_t output,
                              const float *d_params, int64_t n, const float *d_xy, const float *d_ref, double *d_out,
                              void *stream);

/*
 * vpinn_eval_error_noalloc -- vpinn_eval_error for callers that cannot allocate
 * device memory: code under HIP graph capture, serving loops that keep allocation
 * off the hot path, harnesses that forbid it.  Same arguments, kernels and results
 * (bitwise) as vpinn_eval_error, but the value pass and the partial sums use a
 * fixed device array of the library, (4 VPINN_NOALLOC_MAX_POINTS + 16384) bytes
 * (8.02 MiB), of which every device the library runs on holds its own copy until
 * the process ends; the call allocates nothing.
 *  - n above VPINN_NOALLOC_MAX_POINTS: VPINN_E_INVALID, nothing launched (use
 *    vpinn_eval_error).  Other errors as vpinn_eval_error.
 *  - The first call on a device looks up the array's address on that device (a
 *    runtime query, no allocation); make it once before any graph capture.
 *  - All calls on one device share its array: calls that overlap (different
 *    streams or threads without ordering between them) race and must be
 *    serialised by the caller.  The array keeps the last call's contents; each
 *    call writes every value it reads, so nothing has to be cleared.
 */
#define VPINN_NOALLOC_MAX_POINTS 2097152
vpinn_status vpinn_eval_error_noalloc(int32_t width, int32_t n_hidden, int32_t n_outputs, int32_t output,
                                      const float *d_params, int64_t n, const float *d_xy, const float *d_ref,
                                      double *d_out, void *stream);

/*
 * vpinn_adam_step -- Kingma-Ba Adam (Algorithm 1 of that paper, the optimiser of
 * Sec. 4.6.3), in place on n device floats:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   theta -= lr * (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps)
 * `step` counts from 1.  Errors: VPINN_E_INVALID (n < 0, step < 1, null pointer).
 */
vpinn_status vpinn_adam_step(int64_t n, float *d_params, const float *d_grad, float *d_m, float *d_v,
                             int64_t step, float lr, float beta1, float beta2, float eps, void *stream);

/* ------------------------------------------------------------------------ */
/* Batches: many independent problems (each with its own mesh, orders and    */
/* network) trained together, one fused launch per step for all of them.    */
/* ------------------------------------------------------------------------ */
typedef struct vpinn_batch vpinn_batch;

/*
 * vpinn_batch_create -- plan a batch over n >= 1 assembled problems that share
 * the network shape and loss weighting in `cfg` (cfg->path is ignored: batches
 * always use the fused kernel).  The batch borrows the problems' device data:
 * they must outlive it, and after a vpinn_set_boundary, vpinn_set_sensors or
 * vpinn_set_shared_points on any of them the batch's calls return
 * VPINN_E_INVALID until it is planned again (a new batch, or
 * vpinn_batch_set_tuning / vpinn_batch_autotune, which rebuild the plan and
 * drop a captured graph).  Work is split into tiles of 16 points
 * (forward and reverse sweeps: equal shares, one block per compute unit) and
 * chunks of whole elements (contraction), with the tuning {12, 0, 4} (see
 * vpinn_tuning).  Allocates its workspace here; later loss/step/capture/replay
 * calls allocate nothing.
 */
vpinn_status vpinn_batch_create(int32_t n, vpinn_problem *const *problems, const vpinn_loss_cfg *cfg,
                                vpinn_batch **out);

/*
 * vpinn_batch_loss_and_grad -- loss and gradient of every problem.
 *   d_params   device [n][vpinn_n_params(width, n_hidden)] floats, problem-major
 *   d_eps      device [n] floats or NULL (eps = 1 for all)
 *   d_losses   device [n][4] floats (L, L_v, L_b, L_s per problem), may be NULL
 *   d_grads    device [n][n_params] floats, may be NULL (then no backward pass
 *              unless d_grad_eps is given)
 *   d_grad_eps device [n] floats or NULL
 * Each problem's results equal its own vpinn_loss_and_grad up to FP32 rounding
 * order.
 */
vpinn_status vpinn_batch_loss_and_grad(vpinn_batch *b, const float *d_params, const float *d_eps, float *d_losses,
                                       float *d_grads, float *d_grad_eps, void *stream);

/*
 * vpinn_batch_step -- one training step of every problem: the fused forward +
 * adjoint launch, then a reduction kernel that applies Adam (as in
 * vpinn_adam_step) to each problem's parameters in place.  d_step is a device
 * int64 step counter: the launch increments it and Adam uses the new value, so
 * the first step after *d_step = 0 is step 1 and a captured step replays
 * correctly.  d_m, d_v are device [n][n_params]; d_losses (may be NULL) gets
 * the losses at the parameters before the update.
 *   d_eps, d_eps_m, d_eps_v  device [n] floats each, or all NULL: the inverse
 *              problem of Sec. 4.7.1, where each problem's diffusion coefficient
 *              eps (R = eps A - F) is trained beside the weights.  The step uses
 *              d_eps[i] as problem i's eps and then applies the same Adam update
 *              (lr, beta1, beta2, eps, the same step count) to it from
 *              dL/deps = 2 c_v sum_{e,k} R A, with d_eps_m, d_eps_v its moments;
 *              all three are updated in place.  Refused (VPINN_E_INVALID) for
 *              problems from vpinn_assemble_cd2d or vpinn_assemble_vardiff, and
 *              when only some of the three are given.
 */
vpinn_status vpinn_batch_step(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                              float beta1, float beta2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                              float *d_eps_v, void *stream);

/*
 * vpinn_batch_capture -- record one vpinn_batch_step with these arguments into
 * a HIP graph owned by the batch (stream must not be NULL; the capture is
 * thread-local); vpinn_batch_replay launches it.  The graph holds kernel nodes
 * only.  Capturing again replaces the previous graph.
 */
vpinn_status vpinn_batch_capture(vpinn_batch *b, float *d_params, float *d_m, float *d_v, int64_t *d_step, float lr,
                                 float beta1, float beta2, float eps, float *d_losses, float *d_eps, float *d_eps_m,
                                 float *d_eps_v, void *stream);
vpinn_status vpinn_batch_replay(vpinn_batch *b, void *stream);

/* Release the batch (not the problems).  NULL is a no-op. */
void vpinn_batch_free(vpinn_batch *b);

/*
 * Tile shapes of a batch's plan.  Every choice computes the same loss and
 * gradient; they differ in speed and in FP32 summation order (results are
 * bitwise reproducible for a fixed tuning).
 *   fwd_waves      wavefronts per forward-pass block (one block per CU): 8, 12, 16
 *   chunk_shift    small elements (N_quad <= 256, N_test <= 32): elements per
 *                  contraction block = max(1, floor(256 / N_quad) >> chunk_shift),
 *                  0..2
 *   rows_per_pass  larger test spaces: test-function rows of G a wavefront
 *                  streams per pass, 2, 4 or 8
 *   store_activations  0: the reverse sweep recomputes each layer's activations
 *                  (tanh included); 1: the forward pass stores them (L x 2 KB per
 *                  16 points of device memory, held by the plan) and the reverse
 *                  sweep reads them, recomputing only the tangents
 *   one_pass       1: one kernel per step runs the forward pass, the contraction and
 *                  the reverse sweep (then the reduction): a block owns groups of
 *                  whole elements (at most 128 points, one 16-point tile per
 *                  wavefront) and keeps each tile's forward state in registers
 *                  through the contraction, so nothing is recomputed or stored.
 *                  The other fields are then ignored (store_activations must be 0).
 *                  Needs every problem with stored G, N_quad <= 128, N_test <= 32,
 *                  no shared points and one network output (else
 *                  VPINN_E_UNSUPPORTED).  0: the four-kernel step.
 * A new batch starts with {12, 0, 4, 0, 0}.
 */
typedef struct {
    int32_t fwd_waves;
    int32_t chunk_shift;
    int32_t rows_per_pass;
    int32_t store_activations;
    int32_t one_pass;
} vpinn_tuning;

/* The batch's current tuning.  Errors: VPINN_E_INVALID (null argument). */
vpinn_status vpinn_batch_get_tuning(const vpinn_batch *b, vpinn_tuning *out);

/*
 * Rebuild the batch's plan with tuning *t (allocates; drops a captured graph, so
 * capture again before replaying).  Errors: VPINN_E_INVALID (null argument or a
 * value outside the lists above), VPINN_E_NOMEM, VPINN_E_DEVICE.
 */
vpinn_status vpinn_batch_set_tuning(vpinn_batch *b, const vpinn_tuning *t);

/*
 * vpinn_batch_autotune -- the project's tile-shape autotuner.  Times every
 * tuning that matters for this batch (forward block sizes always; storing
 * activations while they fit the 256 MB last-level cache; contraction chunking
 * only if some problem has small elements; rows per pass only if some problem
 * streams rows; the one-pass step where every problem fits it) by `reps`
 * loss-and-gradient evaluations at d_params
 * (device [n][n_params], not modified) after one warm-up each, keeps the one
 * with the lowest median time, and returns it in *best (may be NULL).  A
 * candidate whose plan does not fit in device memory is skipped.
 * Synchronous on `stream`; allocates scratch outputs and each candidate plan;
 * drops a captured graph like vpinn_batch_set_tuning.  Errors: VPINN_E_INVALID
 * (null batch or params, reps outside 1..100), VPINN_E_NOMEM (no candidate
 * fits), VPINN_E_DEVICE.
 */
vpinn_status vpinn_batch_autotune(vpinn_batch *b, const float *d_params, int32_t reps, vpinn_tuning *best,
                                  void *stream);

/*
 * Profiling hooks for the fused path: `events` points to VPINN_PROFILE_EVENTS
 * hipEvent_t (created by the caller with timing enabled; any may be NULL)
 * recorded on the call's stream before the forward kernel, between it and the
 * contraction kernel, between that and the backward kernel, between the backward
 * kernel and the reduction, and after the reduction, by every later
 * vpinn_loss_and_grad (fused path) / batch call.  NULL disables.  The events stay
 * caller-owned.  A capture (vpinn_batch_capture) records none.
 */
#define VPINN_PROFILE_EVENTS 5
vpinn_status vpinn_set_profile_events(vpinn_problem *p, void *const *events);
vpinn_status vpinn_batch_set_profile_events(vpinn_batch *b, void *const *events);

/* Release every device buffer of the problem.  NULL is a no-op. */
void vpinn_problem_free(vpinn_problem *p);

/* Message of the calling thread's last failed call ("" if none). */
const char *vpinn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VPINN_H */
