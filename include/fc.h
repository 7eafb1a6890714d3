/*
 * fc.h -- C ABI of the MI355X finite cell Schwarz-PCG library (libfc).
 *
 * The library solves the symmetric positive (semi-)definite systems A x = b
 * that the finite cell method produces (Jomo et al., arXiv:1809.00828,
 * Sec. 2.1 Eq. 1 and Sec. 3.1 Eq. 2) by conjugate gradients preconditioned
 * with the paper's additive Schwarz preconditioner
 *
 *     S = sum_B R_B^T (R_B A R_B^T)^+ R_B          (Sec. 3.1, Eq. 6)
 *
 * built from element blocks, stabilised pseudo-inverses (Sec. 3.2, Eqs.
 * 9-11) and the diagonal-scaling fallback of Algorithm 1.
 *
 * Conventions shared by every entry point
 *   - Handles (fc_problem, fc_precond) own their device memory; the caller
 *     owns every vector buffer passed in.  Vector arguments named *_dev are
 *     device pointers (e.g. torch.Tensor.data_ptr()) of FP64 values; *_host
 *     arguments are host pointers.
 *   - stream is a hipStream_t (NULL = the default stream).  Calls enqueue
 *     their work on it and return without synchronising, except the set-up
 *     calls and fc_pcg_solve, which synchronise the stream once before they
 *     return.
 *   - Every call returns an fc_status; FC_OK is 0.  No exception or abort
 *     crosses the ABI.  fc_last_error() returns a thread-local message
 *     describing the last failure.
 *   - Unknowns are numbered on the tensor-product lattice: per direction
 *     g = p*e + L(a) with L(0) = 0, L(1) = p, L(j) = j-1 for local function
 *     a on cell e; node = g_0 + (pn+1)(g_1 + (pn+1) g_2); unknown =
 *     ncomp*node + component.  Element-local functions are ordered
 *     a_0 + (p+1)(a_1 + (p+1) a_2), components fastest.
 *   - Indices are int32: every supported system has fewer than 2^31
 *     unknowns and stored matrix blocks.
 */
#ifndef FC_H
#define FC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fc_problem_s* fc_problem;
typedef struct fc_precond_s* fc_precond;

typedef enum {
  FC_OK = 0,
  FC_E_ARG = 1,          /* invalid argument or inconsistent sizes        */
  FC_E_NOMEM = 2,        /* a device or host allocation failed            */
  FC_E_DEVICE = 3,       /* a HIP runtime call failed                     */
  FC_E_NOTCONV = 4,      /* PCG reached maxit; x holds the last iterate   */
  FC_E_BREAKDOWN = 5,    /* (p,Ap) <= 0 or (r,z) <= 0 during PCG          */
  FC_E_NAN = 6,          /* a non-finite value appeared                    */
  FC_E_UNSUPPORTED = 7   /* a size or option the library does not support */
} fc_status;

enum { FC_PDE_POISSON = 0, FC_PDE_ELASTICITY = 1 };
enum { FC_DOMAIN_VOIDS = 0, FC_DOMAIN_INCLUSIONS = 1 };

/*
 * Problem description (Sec. 2.1, Eq. 1 and Sec. 5.1 problem setup).
 * The embedding box is [0,1]^dim with n cells per direction and the full
 * tensor-product integrated Legendre basis of order p.  Shapes are axis-
 * aligned ellipsoids (centre, semi-axes, dim values each); a point is inside
 * one when sum(((x-c)/s)^2) <= 1.  The physical domain is the box minus the
 * shapes (FC_DOMAIN_VOIDS) or their union (FC_DOMAIN_INCLUSIONS); alpha is
 * the indicator value elsewhere.  Cut cells are integrated on a tree of
 * depth quad_depth with a (p+1)^dim Gauss rule on every leaf.
 *   POISSON:    a(u,v) = int alpha (grad u.grad v + u v),
 *               l(v)   = int alpha f v with
 *               f(x)   = sum_k mode_amp[k] cos(2 pi mode_k[k].x + mode_phase[k])
 *   ELASTICITY: a(u,v) = int alpha eps(v):C:eps(u) (E, nu), traction on the
 *               face x_{dim-1} = 1; clamp_zmin clamps (strongly: rows and
 *               columns zeroed, diagonal kept, load zeroed) every function
 *               that is nonzero on x_{dim-1} = 0.
 * discard_fictitious removes, in the same way, every function whose support
 * lies only in cells with eta_T = 0 (the paper's preprocessing of elements
 * completely outside the physical domain, Sec. 5.2; the unknowns keep their
 * lattice numbering).
 * All pointers are host pointers read during fc_setup only.
 */
typedef struct {
  int32_t dim, n, p, pde;
  double alpha;
  int32_t quad_depth, domain;
  int32_t n_shapes;
  const double* shape_centre;   /* [n_shapes*dim] */
  const double* shape_semi;     /* [n_shapes*dim] */
  int32_t n_modes;
  const double* mode_k;         /* [n_modes*dim]  */
  const double* mode_amp;       /* [n_modes]      */
  const double* mode_phase;     /* [n_modes]      */
  double E, nu;
  double traction[3];
  int32_t clamp_zmin;
  int32_t discard_fictitious;
} fc_problem_desc;

/* Assemble A (BSR, block = ncomp x ncomp), b, the per-cell volume fraction
 * eta_T (Sec. 3.2, Eq. 8) and the element blocks on the host, then upload
 * them.  Errors: FC_E_ARG (bad description), FC_E_UNSUPPORTED (block size
 * above the supported maximum), FC_E_NOMEM, FC_E_DEVICE. */
fc_status fc_setup(const fc_problem_desc* desc, void* stream, fc_problem* out);

/* Host-only assembly: run the assembler of fc_setup on the host without
 * touching a GPU, so the assembled system can be inspected or uploaded
 * later.  fc_host_system_export copies it out in the layout of
 * fc_setup_from_matrix (any pointer may be NULL): rowptr[n/bsr_dim+1],
 * col[nnzb], val[nnzb*bsr_dim^2] (row-major blocks), rhs[n],
 * elem_dofs[n_el*m], eta[n_el].  fc_setup_from_host uploads it (the host
 * system stays valid and must still be destroyed).
 * Errors: as fc_setup; fc_assemble never returns FC_E_DEVICE. */
typedef struct fc_host_system_s* fc_host_system;
fc_status fc_assemble(const fc_problem_desc* desc, fc_host_system* out);
fc_status fc_host_system_info(fc_host_system hs, int64_t* n_dofs, int64_t* nnzb,
                              int64_t* n_el, int32_t* m, int32_t* bsr_dim);
fc_status fc_host_system_export(fc_host_system hs, int32_t* rowptr, int32_t* col,
                                double* val, double* rhs, int32_t* elem_dofs,
                                double* eta);
fc_status fc_setup_from_host(fc_host_system hs, void* stream, fc_problem* out);
void fc_host_system_destroy(fc_host_system hs);
/* Wrap an assembled system given by the caller (host arrays, copied).
 * BSR with bsr_dim x bsr_dim blocks stored row-major per block:
 * rowptr[n/bsr_dim+1], col[nnzb] (sorted within each block row),
 * val[nnzb*bsr_dim^2]; rhs[n]; element blocks elem_dofs[n_el*m] in scalar
 * unknowns, which must list each node's bsr_dim components consecutively
 * (unknown = bsr_dim*node + c); eta[n_el] is each block's volume fraction.
 * Errors: FC_E_ARG, FC_E_UNSUPPORTED, FC_E_NOMEM, FC_E_DEVICE. */
fc_status fc_setup_from_matrix(int64_t n, int32_t bsr_dim,
                               const int32_t* rowptr, const int32_t* col,
                               const double* val, const double* rhs,
                               int64_t n_el, int32_t m,
                               const int32_t* elem_dofs, const double* eta,
                               void* stream, fc_problem* out);

/* Sizes of a problem: unknowns, stored BSR blocks, elements, block size m
 * (unknowns per element block), BSR block dimension. */
fc_status fc_problem_info(fc_problem pb, int64_t* n_dofs, int64_t* nnzb,
                          int64_t* n_el, int32_t* m, int32_t* bsr_dim);

/* Copy b to b_dev (device, n_dofs values) on the stream. */
fc_status fc_get_rhs(fc_problem pb, double* b_dev, void* stream);

/* Copy eta_T of every element to eta_host (n_el values, synchronous). */
fc_status fc_get_eta(fc_problem pb, double* eta_host);

/* Copy the matrix to host arrays in the layout of fc_setup_from_matrix
 * (rowptr[n/bsr_dim+1], col[nnzb], val[nnzb*bsr_dim^2]) and the element
 * blocks (elem_dofs[n_el*m]); any pointer may be NULL.  Synchronous. */
fc_status fc_export(fc_problem pb, int32_t* rowptr, int32_t* col, double* val,
                    int32_t* elem_dofs);

/* y = A x (Sec. 3.1, Eq. 2), x_dev and y_dev device buffers of n_dofs
 * FP64 values, must not alias. */
fc_status fc_apply_A(fc_problem pb, const double* x_dev, double* y_dev,
                     void* stream);

/* Preconditioner options (Algorithm 1 and Sec. 3.2).
 *   eta_bar    blocks only for elements with eta_T <= eta_bar (1.0: all);
 *              vertex patches: only patches with a cell of eta_T <= eta_bar
 *   eps        pseudo-inverse threshold: eigenvalues <= eps*max are dropped
 *   stabilize  1 = pseudo-inverse of Eqs. 10-11, 0 = plain inverse (S*)
 *   store_mask FC_STORE_* bits: extra low-precision copies of the block
 *              inverses (FP64 is always kept): FC_STORE_F32 the rounded
 *              scaled inverse with an FP64 list for blocks it would leave
 *              indefinite (fc_precond_lowprec_info), FC_STORE_BF16 the
 *              scaled Cholesky factor (positive semi-definite however
 *              rounded)
 *   block_kind FC_BLOCK_ELEMENT: one block per element, all functions
 *              supported on the cell (Sec. 3.1, the paper's blocks);
 *              FC_BLOCK_VERTEX_PATCH: one block per vertex of the cell grid,
 *              all functions supported on the (up to 2^dim) cells around it,
 *              so every element block lies inside a patch (problems set up
 *              from a description only; FP64 copy only; at most 192
 *              unknowns per patch, i.e. (2p+1)^dim * ncomp <= 192; patches
 *              at the boundary are padded to that size with rows and
 *              columns of zeros, whose eigenvalues the threshold drops and
 *              fc_precond_block_dropped does not count) */
enum { FC_STORE_F64 = 1, FC_STORE_F32 = 2, FC_STORE_BF16 = 4 };
enum { FC_BLOCK_ELEMENT = 0, FC_BLOCK_VERTEX_PATCH = 1 };
typedef struct {
  double eta_bar;
  double eps;
  int32_t stabilize;
  uint32_t store_mask;
  int32_t block_kind;
} fc_precond_opts;

/* Algorithm 1 on the device: select blocks, extract A_B = R_B A R_B^T,
 * compute the stabilised local inverses in FP64, then the diagonal
 * fallback 1/A_ll for every unknown whose diagonal in S is zero and
 * A_ll > 0.  opts NULL means {1.0, 1e-13, 1, FC_STORE_F64,
 * FC_BLOCK_ELEMENT}.
 * Errors: FC_E_ARG, FC_E_UNSUPPORTED, FC_E_NOMEM, FC_E_DEVICE. */
fc_status fc_precond_build(fc_problem pb, const fc_precond_opts* opts,
                           void* stream, fc_precond* out);

/* Statistics of a built preconditioner: number of blocks, unknowns that
 * received the diagonal fallback, blocks whose inverse needed the
 * eigen-decomposition (rather than the certified direct inverse), and
 * eigenvalues dropped by the threshold summed over all blocks. */
fc_status fc_precond_info(fc_precond pc, int64_t* n_blocks,
                          int64_t* n_fallback, int64_t* n_eig_blocks,
                          int64_t* n_dropped);
/* Launch shape the SpMV chose for this problem at set-up: lanes per block
 * row (fixed from the mean row length: the fewest of 8, 16, 32, 64 lanes
 * whose first pass covers the mean row, so the result of every product is
 * the same in every process), and whether the block columns are computed
 * from the lattice (1: the matrix came from a problem description and its
 * columns were verified to be each row's lattice box, so the column array
 * is not read; 2: as 1, and the scalar rows are also held in the sliced
 * layout, slices of 64 rows of one lattice line with equal boxes, which
 * the whole-matrix product reads) or read (0). */
fc_status fc_spmv_info(fc_problem pb, int32_t* group, int32_t* lattice);
/* FP32 copy (FC_STORE_F32): the diagonally scaled inverse D^1/2 P_B D^1/2
 * (D = diag(A) on the block) rounded to FP32, kept for the blocks where a
 * Cholesky factorisation of the rounded matrix shows it positive definite
 * (no pivot below 1e-10 of the largest diagonal entry); the other blocks
 * are applied from the FP64 copy.  Counts of both kinds. */
fc_status fc_precond_lowprec_info(fc_precond pc, int64_t* n_f32_blocks,
                                  int64_t* n_f32_from_f64);
/* Unknowns per block m (element blocks: the problem's m; vertex patches:
 * (2p+1)^dim * ncomp, the padded size) and the block kind (FC_BLOCK_*) of a
 * built preconditioner; either pointer may be NULL. */
fc_status fc_precond_shape(fc_precond pc, int32_t* m, int32_t* block_kind);

/* Eigenvalues dropped by the threshold of Eq. 11 (lambda <= eps * max
 * lambda, negative ones included) in every block, in block order
 * (dropped_host receives n_blocks values; 0 for a block whose certified
 * direct inverse showed that no eigenvalue lies at or below the threshold).
 * Errors: FC_E_ARG (NULL pc, or NULL dropped_host with blocks). */
fc_status fc_precond_block_dropped(fc_precond pc, int32_t* dropped_host);

/* Copy the FP64 local inverse of block k (m*m values, row-major) to host. */
fc_status fc_get_block_inverse(fc_precond pc, int64_t k, double* out_host);

/* z = S r (Sec. 3.1, Eq. 6 with the fallback of Algorithm 1); r_dev and
 * z_dev device buffers of n_dofs FP64 values, must not alias. */
fc_status fc_apply_M(fc_precond pc, const double* r_dev, double* z_dev,
                     void* stream);

/* PCG options.
 *   tol, maxit   stop when the criterion drops to tol (Sec. 5: 1e-10 and
 *                300000 in the paper's vertebra study) or after maxit
 *   stop         FC_STOP_PRECOND: ||S r_i|| / ||S b|| (Eq. 12, recurrence
 *                residual); FC_STOP_RESIDUAL: ||r_i|| / ||b||
 *   mode         FC_MODE_F64 plain FP64 PCG;
 *                FC_MODE_IR_F32 / FC_MODE_IR_BF16: iterative refinement --
 *                the FP64 residual b - A x is recomputed outside, and each
 *                correction comes from a PCG run with a row-mixed copy of A
 *                (the block rows of functions that touch a cell with
 *                eta_T < 1 in FP64, all other rows rounded to FP32; every
 *                row in FP32 for a problem set up from a bare matrix) and
 *                the FP32 / BF16 copy of the local inverses (built with
 *                FC_STORE_F32 / FC_STORE_BF16), FP32 accumulation in the
 *                FP32 rows and the block products, FP64 vectors and
 *                scalars, stopped at inner_tol (relative to its right-hand
 *                side) or at breakdown.  A correction that
 *                does not reduce the FP64 residual by 10 % is undone and the
 *                remaining inner runs use the FP64 matrix (counted in
 *                fc_solve_info.fallbacks).  tol then applies to
 *                ||b - A x|| / ||b|| whatever `stop` says;
 *                FC_MODE_S_F32 / FC_MODE_S_BF16: one PCG run with the FP64
 *                matrix and the FP32 / BF16 copy of the local inverses as the
 *                preconditioner (positive semi-definite however rounded);
 *                FC_MODE_LEARNED: flexible CG with z = S r + gamma P_c y,
 *                y the network attached with fc_learned_attach (see
 *                there); each new direction is z made A-orthogonal to the
 *                last fcg_m directions (fcg_m <= 1: the Polak-Ribiere form
 *                beta = -(z_new, A p)/(p, A p)); always the residual stop
 *                ||r_i|| / ||b||
 *   check_every  iterations between host checks of the device stop flag
 *   history_dev  optional device buffer of maxit+1 doubles receiving the
 *                relative stop criterion of every iteration, or NULL
 *   timing       k > 0: launch the steps directly (no captured graph) and
 *                bracket the SpMV and Schwarz block-product kernels of every
 *                k-th step with events on the solver stream;
 *                fc_solve_info.ms_spmv / ms_schwarz receive their summed
 *                times over the n_timed bracketed steps
 *   fcg_m        FC_MODE_LEARNED: directions kept by the flexible CG, 0 or
 *                1 (one) to 64; the solver holds 2 fcg_m vectors of n_dofs
 *                doubles for them.  A network is nonlinear in r, so the
 *                preconditioner changes from step to step, and one
 *                A-orthogonalisation no longer keeps the directions
 *                conjugate (FC_E_ARG above 64) */
enum { FC_STOP_PRECOND = 0, FC_STOP_RESIDUAL = 1 };
enum { FC_MODE_F64 = 0, FC_MODE_IR_F32 = 1, FC_MODE_IR_BF16 = 2, FC_MODE_S_F32 = 3,
       FC_MODE_S_BF16 = 4, FC_MODE_LEARNED = 5 };
typedef struct {
  double tol;
  int64_t maxit;
  int32_t stop;
  int32_t mode;
  int32_t check_every;
  double inner_tol;
  double* history_dev;
  int32_t timing;
  int32_t fcg_m;
} fc_solve_opts;

typedef struct {
  int64_t iters;          /* products with A inside the PCG iterations    */
  int64_t outer_iters;    /* refinement steps (1 for plain PCG)          */
  double rel_res_true;    /* ||b - A x|| / ||b|| recomputed at the end   */
  double rel_res_prec;    /* last ||S r_i|| / ||S b||                    */
  int32_t status;         /* fc_status of the solve                       */
  double ms_solve;        /* device time of the iteration, milliseconds   */
  double ms_spmv;         /* timing mode: summed SpMV kernel time          */
  double ms_schwarz;      /* timing mode: summed block-product kernel time */
  int64_t n_timed;        /* timing mode: iterations those sums cover      */
  int64_t fallbacks;      /* IR modes: switches to the FP64 matrix         */
} fc_solve_info;

/* Preconditioned CG (Sec. 5, with S of Eq. 6) from x = 0: b_dev and x_dev
 * are device buffers of n_dofs FP64 values (x_dev receives the solution).
 * Returns FC_OK, FC_E_NOTCONV (x = last iterate), FC_E_BREAKDOWN or
 * FC_E_NAN, and fills *info (may be NULL); FC_E_ARG or FC_E_UNSUPPORTED for
 * invalid arguments or options, FC_E_NOMEM or FC_E_DEVICE when a device or
 * host allocation or a launch fails.  Synchronises the stream. */
fc_status fc_pcg_solve(fc_problem pb, fc_precond pc, const double* b_dev,
                       double* x_dev, const fc_solve_opts* opts,
                       fc_solve_info* info, void* stream);

/* fc_pcg_solve for callers that cannot allocate device memory (code that
 * must not call hipMalloc, e.g. tight serving loops or harnesses that
 * forbid it): the same FP64 PCG with the same kernels and launch shapes,
 * launched directly on `stream` (no solver stream, events or graph), whose
 * CG vectors, dot partials and scalars live in one static device scratch
 * array of the library instead of a workspace allocated on first use.
 * The scratch holds at most 524,288 (2^19) unknowns, about 21 MB per GPU,
 * and stays resident on every GPU the library runs on until the process
 * ends; larger problems return FC_E_UNSUPPORTED.  The preconditioner's own
 * buffers (allocated by fc_precond_build) are used as in fc_pcg_solve.
 * Only opts->mode = FC_MODE_F64 with timing = 0 is accepted
 * (FC_E_UNSUPPORTED otherwise); history_dev is honoured.  The results
 * (x, iterations, info) equal those of fc_pcg_solve bit for bit.  Every
 * call on one GPU shares that GPU's scratch: calls that overlap on one GPU
 * (two host threads, two streams) race and must be serialised by the
 * caller.  The current device must be the problem's (FC_E_ARG otherwise).
 * Synchronises the stream after every check_every steps (it cannot be
 * captured into a graph).  Returns as fc_pcg_solve. */
fc_status fc_pcg_solve_noalloc(fc_problem pb, fc_precond pc, const double* b_dev,
                               double* x_dev, const fc_solve_opts* opts,
                               fc_solve_info* info, void* stream);

/* Batched solves (many independent problems, one set of launches).
 * fc_batch_create groups nprob problems with their preconditioners (built
 * by fc_precond_build, FP64) into one batch: shape classes, segmented work
 * lists of (problem, tile), per-problem CG scalars.  With autotune != 0 it
 * times the SpMV group widths and the block-product variants of every
 * shape class on the batch's own data and keeps the fastest (the choices
 * and timings are in the report of fc_batch_info).  The handles must
 * outlive the batch.  Errors: FC_E_ARG, FC_E_NOMEM, FC_E_DEVICE.
 * fc_pcg_solve_batch runs FP64 PCG (Sec. 5 with S of Eq. 6) on every
 * problem from x = 0; b_dev and x_dev are host arrays of nprob device
 * pointers (n_dofs of problem k each).  Every problem stops by its own
 * test (opts->stop, opts->tol, opts->maxit); converged problems drop out of
 * the work at once.  infos (may be NULL) receives one record per problem
 * (rel_res_true holds the recurrence residual ||r_i||/||b||; ms_solve is
 * the batch's time).  Returns FC_OK when every problem converged, else the
 * first failure's status.  Synchronises the stream. */
typedef struct fc_batch_s* fc_batch;
fc_status fc_batch_create(int32_t nprob, const fc_problem* problems,
                          const fc_precond* preconds, int32_t autotune,
                          void* stream, fc_batch* out);
fc_status fc_batch_info(fc_batch bt, int64_t* total_dofs, int32_t* n_spmv_classes,
                        int32_t* n_schwarz_classes, char* report, int64_t report_len);
fc_status fc_pcg_solve_batch(fc_batch bt, const double* const* b_dev,
                             double* const* x_dev, const fc_solve_opts* opts,
                             fc_solve_info* infos, void* stream);
void fc_batch_destroy(fc_batch bt);

/* Learned coarse correction (the coarse level the paper's outlook, Sec. 6,
 * names as the extension of the one-level Schwarz method).  A 4-level 3-D
 * U-Net on the coarse vertex grid: widths ch[0..3], in_ch input channels,
 * 'same' 3x3x3 convolutions, ReLU, average pooling over existing children,
 * nearest upsampling, additive skips, a 1-channel head.  Parameters are one
 * flat FP32 vector: per convolution W[co][ci][27] (tap dz*9+dy*3+dx) then
 * b[co], in the order enc0a enc0b enc1a enc1b enc2a enc2b bota botb up2a
 * up2b up1a up1b up0a up0b head.  Convolutions use a BF16 copy of the
 * weights with FP32 activations and accumulation.
 * Tensors are device buffers of FP32, layout [batch][channel][z][y][x]
 * with a cubic grid of `grid` points per direction. */
typedef struct fc_model_s* fc_model;
typedef struct {
  int32_t epochs;   /* passes over the samples                         */
  int32_t batch;    /* samples per Adam step (mini-batch)              */
  float lr;         /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
} fc_train_opts;
fc_status fc_model_param_count(const int32_t* ch, int32_t in_ch, int64_t* n);
/* params: host FP32 initial parameters (copied). */
fc_status fc_model_create(const int32_t* ch, int32_t in_ch, const float* params,
                          fc_model* out);
fc_status fc_model_get_params(fc_model m, float* params_host);
fc_status fc_model_set_params(fc_model m, const float* params_host);
/* y = network(x): x [batch][in_ch][grid^3], y [batch][1][grid^3]. */
fc_status fc_model_forward(fc_model m, int32_t batch, int32_t grid, const float* x_dev,
                           float* y_dev, void* stream);
/* Mean squared error against t and its gradient (FP32, copied to
 * grad_host if not NULL; loss to *loss).  Synchronises the stream. */
fc_status fc_model_loss_grad(fc_model m, int32_t batch, int32_t grid, const float* x_dev,
                             const float* t_dev, double* loss, float* grad_host,
                             void* stream);
/* Adam on mini-batches over n_samples pairs (x, t) held on the device;
 * mini-batch j of epoch e holds samples (j + i*steps + e) mod n.
 * history (may be NULL) receives the mean loss of every epoch. */
fc_status fc_model_train(fc_model m, int64_t n_samples, int32_t grid, const float* x_dev,
                         const float* t_dev, const fc_train_opts* opts, double* history,
                         void* stream);
void fc_model_destroy(fc_model m);

/* Coarse level of the learned correction, for a scalar 3-D lattice
 * problem with an even number n of cells per direction (else
 * FC_E_UNSUPPORTED).  The coarse grid has G = n/2 + 1 vertices per
 * direction, vertex (a, b, c) at fine vertex (2a, 2b, 2c), stored at
 * a + G (b + G c).  The vertex functions of the basis (Sec. 2) are the Q1
 * hats of the cells, so P_c, trilinear interpolation from the coarse
 * vertices written into the vertex unknowns (all other unknowns zero),
 * represents coarse trilinear functions exactly; restriction is P_c^T and
 * A_c = P_c^T A P_c (27-point, built once by 27 products with A).
 * The correction after z = S r is
 *   y = network(channel 0: P_c^T r at unit RMS, channel 1: eta of the
 *       coarse vertex = mean over the touching coarse cells of their fine
 *       cells' eta_T),
 *   gamma = (y . P_c^T r) / (y . A_c y), z += gamma P_c y,
 * with gamma = 0 (network term dropped) unless y . A_c y > 0 and the
 * quotient is finite, so (z, r) > 0 whenever (S r, r) > 0.
 * The coarse context lives with the preconditioner and is built on first
 * use by any of these calls. */

/* Attach model m (or detach with NULL) for FC_MODE_LEARNED.  The
 * preconditioner keeps a reference: m must outlive its use there. */
fc_status fc_learned_attach(fc_precond pc, fc_model m);
/* G, the coarse vertices per direction. */
fc_status fc_coarse_grid(fc_precond pc, int32_t* G);
/* Device FP32 copies of the eta channel and of the material mask (1 where
 * the vertex function touches a cell with eta_T > 0); either may be NULL. */
fc_status fc_coarse_channels(fc_precond pc, float* eta_dev, float* mask_dev);
/* rc = P_c^T r (FP64, G^3 values). */
fc_status fc_coarse_restrict(fc_precond pc, const double* r_dev, double* rc_dev,
                             void* stream);
/* z += gamma P_c y (y FP32 G^3 values, z FP64 n_dofs values).
 * Synchronises the stream. */
fc_status fc_coarse_prolong(fc_precond pc, const float* y_dev, double gamma, double* z_dev,
                            void* stream);
/* v = A_c y; *gamma receives (y . rc) / (y . A_c y) for the rc of the last
 * fc_coarse_restrict (0 unless y . A_c y > 0 and finite).  Synchronises. */
fc_status fc_coarse_apply(fc_precond pc, const float* y_dev, double* v_dev, double* gamma,
                          void* stream);
/* Plain Schwarz-PCG judges the network: solve A x = b to tol (relative
 * residual) once with FC_MODE_F64 and once with FC_MODE_LEARNED (fcg_m
 * kept directions, as in fc_solve_opts), keep the
 * network for later FC_MODE_LEARNED solves of this preconditioner only if
 * the learned run converges in less device time, else those solves run
 * plain PCG (fc_solve_info.fallbacks = 1).  *use_network receives the
 * decision; plain / learned (may be NULL) the two runs' infos.
 * fc_learned_attach resets the decision to "use". */
fc_status fc_learned_validate(fc_precond pc, const double* b_dev, double tol,
                              int32_t fcg_m, int32_t* use_network, fc_solve_info* plain,
                              fc_solve_info* learned, void* stream);
/* Corrections applied and dropped since fc_learned_attach. */
fc_status fc_learned_stats(fc_precond pc, int64_t* n_apply, int64_t* n_drop);
/* Training pairs from a running FP64 Schwarz-PCG solve of A x = b from
 * x = 0: at every iteration listed in iters (ascending; 0 is the start) the
 * network input of the residual r_k goes to xin_dev + i*2*G^3 and the
 * target to t_dev + i*G^3:
 *   kind 0: mask * (x_star - x_k - S r_k) at the coarse vertices,
 *   kind 1: mask * (x_star - x_k),
 *   kind 2: the coarse Galerkin projection of the error: y with
 *           A_c y = P_c^T r_k on the material vertices (mask 1), 0
 *           elsewhere, so that P_c y is the A-orthogonal projection of
 *           x_star - x_k onto those coarse vertex functions (solved by
 *           Jacobi-preconditioned CG on A_c to 1e-8; FC_E_NOTCONV or
 *           FC_E_BREAKDOWN if that fails; x_star is not read),
 * scaled to unit RMS (x_star: the converged solution, device).  Stops
 * early at convergence to tol (relative residual); *n_taken receives the
 * number of pairs written. */
fc_status fc_learned_snapshots(fc_precond pc, const double* b_dev, const double* x_star_dev,
                               int32_t n_snap, const int32_t* iters, int32_t kind,
                               double tol, float* xin_dev, float* t_dev, int32_t* n_taken,
                               void* stream);

void fc_problem_destroy(fc_problem pb);
void fc_precond_destroy(fc_precond pc);
const char* fc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FC_H */
