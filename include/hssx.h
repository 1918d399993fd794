/*
 * hssx.h - C ABI of the MI355X (gfx950) implementation of the hierarchical
 * nested-dissection + HSS preconditioner for 2D Galerkin wave problems
 * (Bonev & Hesthaven, "A hierarchical preconditioner for wave problems in
 * quasilinear complexity").
 *
 * Problem (Sec. 1, eq. 1.1; Sec. 4.2, eq. 4.2): A x = b with A the P1
 * Galerkin matrix of -lap u - (omega s(x))^2 u on the unit square with the
 * absorbing condition d_n u - i omega s u = 0 on its boundary,
 *     A = K - omega^2 M[s^2] - i omega G[s]         (complex symmetric),
 * on an N x N node grid (node (i,j) at (i h, j h), id j*N+i, h = 1/(N-1),
 * each cell split along its SW-NE diagonal).  The solve is preconditioned as
 * P^-1 A x = P^-1 b (eq. 1.2) with P = LDR (eq. 3.1) built by Algorithm 3.4
 * and applied by Algorithm 3.1.
 *
 * Conventions
 *   - Every function returns hssx_status; nothing throws across the ABI.
 *     Negative values are errors (outputs unspecified, handles still valid
 *     to destroy); HSSX_ENOCONV is a warning (x holds the last iterate).
 *     hssx_last_error() returns a thread-local message for the last failure.
 *   - Pointers documented as "device" are HIP device pointers (e.g. the
 *     data_ptr of a torch CUDA tensor).  Pointers documented as "host" are
 *     ordinary host memory.  The caller owns every buffer it passes; the
 *     library owns its handles and every internal buffer (allocated with
 *     hipMalloc on the handle's device) and frees them in *_destroy.
 *   - Complex vectors are complex128 (interleaved re, im doubles), column-
 *     major with leading dimension ld >= n.  Vectors use the natural node
 *     numbering.
 *   - stream is a hipStream_t passed as void* (NULL = default stream).  Work
 *     is stream-ordered; functions that must read results back (factor rank
 *     decisions, GMRES convergence tests) synchronise that stream and say so.
 *   - Arguments are validated before any launch; invalid ones give
 *     HSSX_EINVAL.
 */
#ifndef HSSX_H
#define HSSX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HSSX_OK = 0,
  HSSX_ENOCONV = 1,       /* GMRES hit maxit; x valid, stats filled */
  HSSX_EINVAL = -1,       /* invalid argument */
  HSSX_ENOMEM = -2,       /* device allocation failed */
  HSSX_ESINGULAR = -3,    /* zero pivot in a dense block; message names the node */
  HSSX_ERANKCAP = -4,     /* compression did not meet tol before its round limit */
  HSSX_EHIP = -5          /* HIP runtime error */
} hssx_status;

typedef enum { HSSX_C128 = 0, HSSX_C64 = 1 } hssx_dtype;

typedef struct hssx_op_ *hssx_op;      /* assembled operator A */
typedef struct hssx_fact_ *hssx_fact;  /* approximate factorization P */
typedef struct hssx_ctx_ *hssx_ctx;    /* caller-allocator context */

/* Device allocator of a context: alloc returns bytes of device memory on the
 * context's device (NULL: out of memory), usable by work queued on stream
 * (the hipStream_t of the library call, as void*; NULL outside a call);
 * free gives back a pointer alloc returned, with its size.  user is passed
 * through.  The callbacks may be called from any library call made on a
 * handle of the context, on that call's thread. */
typedef struct {
  void *(*alloc)(size_t bytes, void *stream, void *user);
  void (*free)(void *ptr, size_t bytes, void *stream, void *user);
  void *user;
} hssx_allocator;

/* Problem description (Sec. 4.2), with a first-order absorbing condition on
 * all four sides of the unit square. */
typedef struct {
  int N;          /* nodes per side, N >= 2 */
  double omega;   /* angular frequency; wavenumber k(x) = omega * s(x) */
} hssx_problem_desc;

/* Interior-penalty DG problem (Sec. 4.1-4.2, 4.6): N x N cells of the unit
 * square, polynomial degree p (1 or 2), boundary condition bc. */
enum { HSSX_BC_ABSORBING = 0, HSSX_BC_DIRICHLET = 1 };
typedef struct {
  int N;          /* cells per side, N >= 1 */
  int p;          /* polynomial degree: 1 or 2 */
  int bc;         /* HSSX_BC_ABSORBING (d_n u - i k u = 0) or HSSX_BC_DIRICHLET (u = 0) */
  double omega;   /* angular frequency; wavenumber k(x) = omega * s(x); 0 = Poisson */
} hssx_ipdg_desc;

/* Factorization options (Sec. 4 parameter choices; Algorithm 3.4, A.1). */
typedef struct {
  int beta;         /* HSS leaf size in DOFs (eq. 2.1); default 16 */
  int h_sw;         /* switching height: nodes higher than h_sw use HSS
                       arithmetic, their children compress S; < 0 = never
                       compress (exact sparse direct factorization) */
  int k0;           /* initial rank estimate of Algorithm A.1; default 32 */
  int r;            /* probe / rank step of Algorithm A.1; default 16 */
  int max_rounds;   /* rank-growth rounds per compression; default 32 */
  hssx_dtype dtype; /* factor storage / arithmetic: C128 or C64 */
  uint32_t seed;    /* key of the counter-based sketch generator */
  double id_rel_tol;/* relative pivot threshold of the interpolative
                       decomposition; <= 0 selects max(1e-2 * tol,
                       4 * unit roundoff of the factor dtype) */
  int apply_graph;  /* nonzero: the apply sweeps are captured once per
                       (right-hand-side count, transpose) and replayed as a
                       HIP graph; default 1 */
  int autotune;     /* nonzero: the apply tile shape of every tree depth is
                       measured on first use per (precision, sweep, size
                       bucket) and cached for the process; default 1 */
  int sample_bf16;  /* complex64 factors only: the sampling products
                       Y = S Omega run on bf16 matrix cores with fp32
                       accumulation; 1 = operands rounded to bf16, 2 = each
                       operand split into a bf16 head and tail (three
                       products, about 16 significant bits); 0 = fp32
                       vector arithmetic (default) */
  int switch_size;  /* > 0: switching by size instead of height: a node uses
                       HSS arithmetic when its interior |I| holds at least
                       switch_size DOFs or a child does (the paper's 3D rule
                       switches at four times beta); 0: the h_sw rule */
  int strict_tol;   /* nonzero: hssx_factor / hssx_refactor fail with
                       HSSX_ERANKCAP when any compression stops with its
                       error estimate above tol; 0 (default): such
                       compressions are accepted and counted in
                       hssx_factor_stats.n_above_tol */
  int wide_inverse; /* complex64 factors only, nonzero: the telescoping
                       inverses of the HSS blocks (Sec. 3.3) are computed in
                       complex128 from widened generators and stored in
                       complex64.  Lowers the disagreement between entries
                       and products of Schur complements whose interior
                       blocks are ill-conditioned (indefinite elastic
                       operators); 0 (default): complex64 throughout */
} hssx_factor_opts;

typedef struct {
  int m;            /* restart length; default 50 */
  double tol;       /* relative residual target; default 1e-8 */
  int maxit;        /* total Arnoldi steps; default 1000 */
  int flexible;     /* 0: left preconditioning (stop on ||P^-1 r||/||P^-1 b||,
                       then check ||r||/||b||); 1: flexible right
                       preconditioning (stop on ||r||/||b||) */
} hssx_gmres_opts;

typedef struct {
  int iters;            /* total Arnoldi steps (paper's "iters") */
  int converged;        /* 1 if true relative residual <= tol */
  double prec_res;      /* final preconditioned relative residual (left) */
  double true_res;      /* final ||b - A x|| / ||b|| */
} hssx_gmres_stats;

typedef struct {
  int n;                /* unknowns */
  int nodes;            /* elimination-tree nodes */
  int depth;            /* tree depth */
  int n_hss_nodes;      /* nodes using HSS arithmetic */
  int n_compressed;     /* Schur complements compressed (Algorithm A.1 calls on S) */
  int k_max;            /* largest rank among compressed blocks (Sec. 4.2) */
  int max_rounds_used;  /* most rank-growth rounds of any compression */
  double max_estimate;  /* largest accepted relative error estimate (eq. 2.7) */
  double factor_bytes;  /* bytes the apply reads: dense blocks (A_ii^-1, L, R)
                           of dense-class nodes; telescoping inverses and
                           Gauss-transform generators of HSS-class nodes */
  double factor_flops;  /* nominal flops of the numeric factorization
                           (products, eliminations, compressions) */
  double ms_symbolic;   /* host symbolic analysis (trees, orders) */
  double ms_numeric;    /* numeric factorization (device, hipEvents) */
  double ms_setup;      /* front descriptors, their upload and the front
                           pool allocation (host) */
  int rounds_total;     /* rank-growth rounds summed over all compressions */
  int n_above_tol;      /* compressions accepted with an estimate above tol
                           (round or capacity limit, or the complex64
                           rounding-noise floor) */
  double exact_factor_bytes;  /* the same counts for the exact multifrontal */
  double exact_factor_flops;  /* factorization of this tree (dense fronts,
                                 Gauss-Jordan), for comparison */
} hssx_factor_stats;

/* Contexts (the boundary's allocator injection; eq. 1.1 / eq. 3.1 calls made
 * with caller-owned device memory).  hssx_create makes a context on device
 * with a copy of *alloc.  hssx_bind(ctx) binds it to the calling thread
 * (NULL unbinds): operators and factors created by that thread while it is
 * bound (hssx_assemble*, hssx_op_batch, hssx_factor; also hssx_hss_eval)
 * belong to the context, and every device buffer the library takes for
 * them, in that call and in every later call on them (factor storage,
 * scratch arenas, staging areas, GMRES bases, apply workspaces and
 * programs), comes from its allocator and goes back through it when the
 * handle or the context is destroyed.  hssx_destroy synchronises the device,
 * frees the context's cached scratch and staging areas through the
 * allocator and deletes it: destroy the context's handles first.  Memory
 * HIP itself takes for graph instantiation and pinned host staging are not
 * device buffers of the library and do not pass through the allocator.
 * hssx_ctx_stats reports the bytes currently taken from the allocator and
 * the counts of alloc and free calls. */
hssx_status hssx_create(int device, const hssx_allocator *alloc,
                        hssx_ctx *ctx_out);
hssx_status hssx_bind(hssx_ctx ctx);
hssx_status hssx_ctx_stats(hssx_ctx ctx, long *live_bytes, long *allocs,
                           long *frees);
void hssx_destroy(hssx_ctx ctx);

/* Build A (CSR, natural numbering, 7-point P1 stencil, sorted columns) for
 * the slowness field s (device, float64[N*N], caller-owned, read during the
 * call).  Sec. 4.2 eq. 4.2 with the closed-form P1 integrals.  EINVAL for N
 * outside [2, 17000] (32-bit CSR offsets), a non-finite or negative omega or
 * null arguments. */
hssx_status hssx_assemble(int device, const hssx_problem_desc *desc,
                          const double *s_dev, void *stream, hssx_op *A_out);

/* Build the time-harmonic P1 elastic operator A = K[lam, mu] - omega^2
 * M[rho] - i omega C on the N x N grid (the elastic workload of Sec. 4):
 * displacement DOFs 2 * node + component, stiffness from the Lame fields
 * lam, mu (element means of their P1 interpolants), mass with density rho,
 * and the first-order absorbing traction rho (c_p u_n n + c_s u_t t) on all
 * four sides (c_p = sqrt((lam + 2 mu)/rho), c_s = sqrt(mu/rho)).  lam, mu,
 * rho: device float64[N*N], caller-owned, read during the call.  Pattern:
 * 2 x 2 blocks of the 7-point node stencil, columns sorted.  The operator
 * works with hssx_load (vector mass), hssx_matvec, hssx_factor, hssx_apply
 * and hssx_gmres_solve; not with hssx_dAds_contract or in batches.
 * EINVAL for N outside [2, 8500] (32-bit CSR offsets), a non-finite or
 * negative omega, or null fields. */
hssx_status hssx_assemble_elastic(int device, const hssx_problem_desc *desc,
                                  const double *lam_dev, const double *mu_dev,
                                  const double *rho_dev, void *stream,
                                  hssx_op *A_out);

/* Build the symmetric interior-penalty DG operator with P2 elements for the
 * Helmholtz problem (the IPDG discretization of Sec. 4.1-4.2) on desc->N x
 * desc->N cells of side h = 1/N, each split along its SW-NE diagonal into
 * the lower triangle (element 2 c) and the upper one (2 c + 1), c = j N + i;
 * DOF 6 e + a over the nodal P2 basis (vertices, then edge midpoints of
 * (v0,v1), (v1,v2), (v2,v0)).  Form: sum_T int grad u.grad v - k^2 u v, on
 * interior faces -{grad u.n}[v] - {grad v.n}[u] + 10 p^2/|F| [u][v], and
 * -i k u v on the absorbing boundary faces; k^2 = omega^2 times the P1
 * interpolant of s^2, k = omega times that of s.  s_dev: device float64
 * [(N+1)^2] slowness at the mesh vertices (vertex (i, j) at j (N+1) + i),
 * caller-owned, read during the call.  Pattern: 6 x 6 blocks of each
 * triangle with itself and its face neighbours, columns sorted.  Works with
 * hssx_load (block-diagonal P2 mass), hssx_matvec, hssx_factor, hssx_apply
 * and hssx_gmres_solve; not with hssx_dAds_contract or in batches.  EINVAL
 * for N outside [1, 2700] (32-bit CSR offsets), a non-finite or negative
 * omega, or null arguments. */
hssx_status hssx_assemble_dg(int device, const hssx_problem_desc *desc,
                             const double *s_dev, void *stream, hssx_op *A_out);

/* The symmetric interior-penalty DG operator of hssx_assemble_dg for either
 * polynomial degree and either boundary condition (the IPDG runs of Sec.
 * 4.1-4.2 and the p = 1 scaling study of Sec. 4.6 with u = 0 on the whole
 * boundary).  P1: DOF 3 e + a over the vertex functions (barycentric
 * coordinates), 3 x 3 blocks, tau_F = 10 / |F|; P2 as in hssx_assemble_dg.
 * Dirichlet faces add -int (grad u.n) v - int (grad v.n) u + tau_F int u v
 * with the outward normal (the interior face terms with zero outside); the
 * operator is then real (imaginary parts exactly zero) for real omega s.
 * hssx_load with f = 1 gives the load of the constant source f = 1.  s_dev,
 * ownership, uses and errors as for hssx_assemble_dg; EINVAL also for p or bc
 * out of range, and N above 5400 (P1) or 2700 (P2). */
hssx_status hssx_assemble_ipdg(int device, const hssx_ipdg_desc *desc,
                               const double *s_dev, void *stream, hssx_op *A_out);

/* Batch of independent problems as one block-diagonal operator (the
 * batching form: fronts of one tree depth, across all problems, are
 * eliminated and compressed in the same launches, and GMRES advances every
 * problem's Krylov basis together).  parts: count single-problem operators
 * (from hssx_assemble) on one device; their CSR, mass matrix and slowness
 * are copied, so the parts may be destroyed afterwards.  Part p owns rows
 * [off[p], off[p+1]) with off the running sum of the parts' n.  The batch
 * works with hssx_load, hssx_matvec, hssx_factor (a forest: one nested
 * dissection tree per part), hssx_apply, hssx_gmres_solve and
 * hssx_dAds_contract on vectors of the concatenated length.  EINVAL for an
 * empty list, a part that is itself a batch, mixed devices, or more than
 * 2^31 - 1 rows or nonzeros. */
hssx_status hssx_op_batch(int count, const hssx_op *parts, void *stream,
                          hssx_op *A_out);

/* Size of an operator: *n rows in total, *parts problems (1 unless built by
 * hssx_op_batch), and part_off (host int32[parts + 1], may be NULL) the row
 * offsets of the parts.  Host-only. */
hssx_status hssx_op_info(hssx_op A, int *n, int *parts, int32_t *part_off);

/* b = M f with M the plain P1 mass matrix: the load of nodal source samples
 * f (device, float64, n x nrhs, ld ldf) into b (device, complex128, ld ldb).*/
hssx_status hssx_load(hssx_op A, int nrhs, const double *f_dev, long ldf,
                      void *b_dev, long ldb, void *stream);

/* y = A x (trans = 0) or A^T x (trans = 1; equal to A x, A is symmetric).
 * x, y: device complex128, n x nrhs. */
hssx_status hssx_matvec(hssx_op A, int trans, int nrhs, const void *x_dev,
                        long ldx, void *y_dev, long ldy, void *stream);

/* Copy the CSR arrays of A to host buffers (sizes n+1, nnz, 2*nnz doubles);
 * any pointer may be NULL.  *nnz_out receives nnz.  Synchronises stream. */
hssx_status hssx_get_csr(hssx_op A, int32_t *rowptr, int32_t *col,
                         double *val, long *nnz_out, void *stream);

/* Approximate factorization P = LDR (Algorithm 3.4): box nested dissection
 * with leaf boxes of at most leaf_size DOFs (Sec. 4: ND until the leaf boxes
 * are small); dense fronts (Gauss-Jordan) up to the switching height h_sw
 * and at the roots; above it HSS arithmetic (Sec. 3.3-3.5): the children's
 * Schur complements stay in generator form, the interior block is inverted
 * by Algorithm 3.3 with telescoping HSS inverses of S_ii^mu and of the inner
 * Schur complement S~, the Gauss transforms are kept as low-rank generators
 * (eq. 3.7), and S(sigma) and S~ are compressed by adaptive randomized
 * sampling (Algorithm A.1, relative tolerance tol, eq. 2.7) from structured
 * products and entries without being formed.  With dtype HSSX_C64 every
 * factor is stored and computed in complex64 except the roots (top
 * separators), which stay complex128.  The rank of a compression grows by r
 * per round until its estimate meets tol; it also stops at max_rounds and
 * at the sample or local-block capacity (1024 columns; 2 (k + r) > 1024
 * rows), and, in complex64, when the estimate is within 10 tol and a round
 * no longer halves it (the rounding-noise floor of single precision) or
 * when a round keeps more than 0.7 of the previous estimate.  Compressions
 * that stop above tol are counted in n_above_tol (HSSX_ERANKCAP with
 * opts->strict_tol); max_estimate reports the largest accepted estimate.  A batch operator gets one
 * tree per problem, all processed depth by depth in the same launches.
 * Host-blocking: synchronises stream after every batch of compressions to
 * read the error estimates.  opts may be NULL (defaults). */
hssx_status hssx_factor(hssx_op A, double tol, int leaf_size,
                        const hssx_factor_opts *opts, void *stream,
                        hssx_fact *P_out);

/* Numeric refactorization (Algorithm 3.4 without the analysis): recompute
 * the factor P for operator A, which must have the pattern of the operator P
 * was built from (same kind and grid sides, e.g. new slowness or Lame fields
 * reassembled on the same grid, or a batch of the same grids).  The symbolic
 * analysis, front descriptors, front pool, sketch seeds, options and apply
 * graphs and tiles of P are kept; every numeric value is recomputed from A.
 * P refers to A afterwards.  Host-blocking like hssx_factor.  EINVAL for a
 * handle without a factorization or a different pattern; the factor is
 * unusable after a failed refactor (ESINGULAR, ENOMEM). */
hssx_status hssx_refactor(hssx_fact P, hssx_op A, void *stream);

/* y = P^-1 x (trans = 0) or P^-T x (trans = 1) by Algorithm 3.1
 * (bottom-up L sweep, block-diagonal solve, top-down R sweep).  x, y:
 * device complex128, n x nrhs; y may alias x. */
hssx_status hssx_apply(hssx_fact P, int trans, int nrhs, const void *x_dev,
                       long ldx, void *y_dev, long ldy, void *stream);

/* hssx_apply for callers that cannot allocate device memory (tight serving
 * loops, harnesses that forbid allocation): the same y = P^-1 x or P^-T x, with every device buffer it
 * needs (the elimination-order workspace, the HSS-class nodes' scratch and
 * their job arrays) taken from a 64 MiB array in the library's device image,
 * one per GPU, held until the process ends.  No hipMalloc, hipFree or
 * allocating library call; the dense nodes use the default tile shapes (no
 * autotuning) and no graph is captured.  HSSX_EINVAL when the workspace for
 * this factor and nrhs exceeds 64 MiB (about 2 n nrhs 16 bytes plus the HSS
 * nodes' share).  Every call on one GPU uses that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (other streams, other host
 * threads) race.  Synchronises stream before returning. */
hssx_status hssx_apply_noalloc(hssx_fact P, int trans, int nrhs,
                               const void *x_dev, long ldx, void *y_dev,
                               long ldy, void *stream);

/* Restarted GMRES on A x = b (eq. 1.2) with preconditioner P, all nrhs
 * right-hand sides advanced together; x0 = 0.  trans = 1 solves A^T x = b
 * with P^-T; trans = 2 solves the adjoint system A^H x = b, as
 * conj(A^-T conj(b)) with P^-T, the conjugations done in the library.  Each (right-hand side, problem) pair is its
 * own system with its own Krylov basis and stopping test; for a batch of np
 * problems, system r * np + p is part p of column r.  stats: host array of
 * nrhs * np entries in that order (may be NULL).  Host-blocking: reads
 * residual norms once per Arnoldi step. */
hssx_status hssx_gmres_solve(hssx_op A, hssx_fact P, int trans, int nrhs,
                             const void *b_dev, long ldb, void *x_dev,
                             long ldx, const hssx_gmres_opts *opts,
                             hssx_gmres_stats *stats, void *stream);

/* Adjoint contraction for a real functional J(x(s)), x = A(s)^-1 b:
 * grad_s[l] += -Re sum_rhs lambda^T (dA/ds_l) x, with lambda = A^-T dJ/dx
 * as solved by the caller.  lambda, x: device complex128 n x nrhs (ld n);
 * grad_s: device float64[n], accumulated.  dA/ds_l =
 * -2 omega^2 s_l M_l - i omega G_l with M_l, G_l the P1 triple-product
 * matrices of node l (of the node's own problem for a batch). */
hssx_status hssx_dAds_contract(hssx_op A, int nrhs, const void *lambda_dev,
                               const void *x_dev, double *grad_dev,
                               void *stream);

/* The same contraction with the adjoint state mu = A^-H dJ/dx (as returned
 * by hssx_gmres_solve with trans = 2): grad_s[l] += -Re sum_rhs
 * mu^H (dA/ds_l) x.  For J real, dJ/db = mu.  Same arguments and errors as
 * hssx_dAds_contract. */
hssx_status hssx_dAds_contract_adjoint(hssx_op A, int nrhs, const void *mu_dev,
                                       const void *x_dev, double *grad_dev,
                                       void *stream);

/* Symbolic analysis only (box nested dissection, elimination tree, cluster
 * trees; Sec. 3.1 Def. 3.1, Fig. 3, Fig. 4) for an N x N grid with dofs
 * unknowns per grid node (1: Helmholtz, 2: elastic, DOF dofs * node + c),
 * leaf boxes of at most leaf_size DOFs and HSS leaves of at most beta DOFs
 * (both >= dofs; a node's unknowns are never split).  Host-only:
 * makes no HIP call, so it runs without a GPU.  The handle supports
 * hssx_get_perm, hssx_get_tree and hssx_fact_destroy only. */
hssx_status hssx_analyze(int N, int dofs, int leaf_size, int beta, hssx_fact *P_out);

/* Symbolic analysis of the discontinuous mesh of hssx_assemble_dg (Nc x Nc
 * cells, whole triangles of 6 DOFs as units, Sec. 3.3 Fig. 5): boxes of cells,
 * adjacency across faces, cluster coordinates at the triangle centroids.
 * leaf_size and beta count DOFs (>= 6).  Host-only, as hssx_analyze. */
hssx_status hssx_analyze_dg(int Nc, int leaf_size, int beta, hssx_fact *P_out);

/* hssx_analyze_dg for either degree: units of 3 (p = 1) or 6 (p = 2) DOFs;
 * leaf_size and beta count DOFs (>= the unit).  Host-only. */
hssx_status hssx_analyze_ipdg(int Nc, int p, int leaf_size, int beta, hssx_fact *P_out);

/* Elimination permutation (host int32[n]): perm[k] = node id eliminated at
 * position k (concatenation of I(sigma) over the post-order). */
hssx_status hssx_get_perm(hssx_fact P, int32_t *perm_host, long n);

/* Elimination tree and cluster trees, flattened to host arrays for
 * bit-exact comparison.  Call once with NULL arrays to get the sizes in
 * *sizes_out (int64[4]: nodes, total |I|, total |B|, total clusters), then
 * with buffers: node_info int32[nodes*10] = (x0,x1,y0,y1,lo,hi,parent,
 * depth,height,p0); i_ids int32[total |I|] and i_ptr int32[nodes+1];
 * b_ids int32[total |B|] and b_ptr int32[nodes+1]; clusters int32[total*5] =
 * (start,size,left,right,level) per cluster, c_ptr int32[nodes+1]. */
hssx_status hssx_get_tree(hssx_fact P, int64_t *sizes_out,
                          int32_t *node_info, int32_t *i_ids, int32_t *i_ptr,
                          int32_t *b_ids, int32_t *b_ptr, int32_t *clusters,
                          int32_t *c_ptr);

hssx_status hssx_get_factor_stats(hssx_fact P, hssx_factor_stats *s);

/* Read a node's dense Schur complement S(sigma) as passed to its parent
 * (expanded from HSS when compressed), |B| x |B| column-major complex128 into
 * host memory.  For tests.  Synchronises. */
hssx_status hssx_get_schur(hssx_fact P, int node, double *S_host, long ld);

/* The HSS arithmetic the factorization runs on its compressed Schur
 * complements (Sec. 2.2, Sec. 3.3), applied to one complex symmetric HSS
 * matrix H given by the caller in generator form:
 *   op 0: Y = H X, the telescoping product (eqs. 2.5-2.6);
 *   op 1: Y = H^-1 X, the telescoping inverse (per level D^-1, the
 *         reduced blocks (U^T D^-1 U)^-1, and a dense inverse at the root)
 *         and its two-sweep solve;
 *   op 2: vals[e] = H(i, j), entry access through the full bases;
 *   op 3: vals[e] = H^-1(i, j), the same on the inverse's HSS form;
 *   op 4, op 5: op 1 and op 3 with the telescoping inverse computed in
 *         complex128 and stored in dtype (hssx_factor_opts.wide_inverse);
 * for (i, j) = (ij[2e], ij[2e+1]).  tree: host int32[ncl*5] (start, size,
 * left, right, level) per cluster in level order, root 0 = [0, m), each
 * internal cluster split into two consecutive children; rank: host
 * int32[ncl], rank[0] = 0.  gens: host float64 (re, im) pairs packed per
 * cluster c = 0, 1, ...: for c > 0 the basis U (rows x rank[c], rows = size
 * at a leaf, rank[left] + rank[right] otherwise), then D (size x size) at a
 * leaf, or B12 (rank[left] x rank[right]) and B21 (rank[right] x rank[left])
 * at an internal cluster; all column-major.  X, Y: device complex128
 * m x nrhs (ld m) for op 0/1/4; ij: host int32[2 nij], vals: host float64
 * [2 nij] for op 2/3/5.  dtype: arithmetic precision (C64 rounds the
 * generators and vectors).  ESINGULAR when a block of the inverse is
 * singular.  Synchronises stream. */
hssx_status hssx_hss_eval(int device, hssx_dtype dtype, int m, int ncl,
                          const int32_t *tree, const int32_t *rank,
                          const double *gens, int op, int nrhs,
                          const void *x_dev, void *y_dev, long nij,
                          const int32_t *ij, double *vals, void *stream);

/* Measurement support.  hssx_prof_enable(1) clears the records and starts
 * bracketing the main kernels with HIP events on their launch stream;
 * hssx_prof_query returns, for one kernel name, the summed event time (ms),
 * the number of launches and the summed algorithmic work of those launches:
 *   "front_eliminate"  flops (8 per complex multiply-add of Gauss-Jordan)
 *   "front_assemble"   bytes written
 *   "apply_up", "apply_down"  bytes of factor blocks and vectors moved
 *   "spmv"             bytes of CSR arrays and vectors moved
 *   "compress_level", "hss_matvec", "sample"  flops (nominal)
 * Unknown names report zero launches. */
hssx_status hssx_prof_enable(int on);
hssx_status hssx_prof_query(const char *kernel, double *ms, long *launches,
                            double *work);

void hssx_fact_destroy(hssx_fact P);
void hssx_op_destroy(hssx_op A);
const char *hssx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* HSSX_H */
