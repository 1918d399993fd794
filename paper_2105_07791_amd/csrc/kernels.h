// Host-side launchers of the device kernels, and the descriptor structs the
// batched kernels read.  Every launcher enqueues on the given stream and
// checks the launch.
#pragma once

#include "common.h"

namespace hssx {

// ------------------------------------------------------------ FEM / SpMV
void launch_assemble(int N, double omega, const double *s, const int *rowptr, const int *col,
                     c128 *val, double *mval, hipStream_t st);
// elastic operator on DOFs 2 v + c (pattern: 2 x 2 blocks of the 7-point node stencil)
void launch_assemble_elastic(int N, double omega, const double *lam, const double *mu,
                             const double *rho, const int *rowptr, const int *col, c128 *val,
                             double *mval, hipStream_t st);
// SIPG Helmholtz operator of degree deg (1 or 2) on Nc x Nc x 2 triangles
// (DOF nb e + a, nb = 3 or 6; pattern: nb x nb blocks of each triangle with
// itself and its face neighbours); dirichlet: 0 absorbing boundary, 1 u = 0
void launch_assemble_dg(int Nc, int deg, int dirichlet, double omega, const double *s_vertex,
                        const int *rowptr, const int *col, c128 *val, double *mval,
                        hipStream_t st);
void launch_load(int n, int nrhs, const int *rowptr, const int *col, const double *mval,
                 const double *f, long ldf, c128 *b, long ldb, hipStream_t st);
// row_max: longest row (7 scalar stencil, 14 for 2 x 2 blocks, 24 for P2 triangles)
void launch_spmv(int n, int nrhs, const int *rowptr, const int *col, const c128 *val,
                 const c128 *x, long ldx, c128 *y, long ldy, int row_max, hipStream_t st);
// grad[l] += -Re sum_rhs lam^T (dA/ds_l) x, with conj(lam) in place of lam
// when conj_lam is set
void launch_dads(int N, double omega, const double *s, int nrhs, const c128 *lam,
                 const c128 *x, long ld, double *grad, int conj_lam, hipStream_t st);

// ------------------------------------------------------------ dense fronts
// One elimination-tree node's augmented dense front
//   F = [[A_ii, A_ib, I], [A_bi, A_bb, 0]]      (f x (f + ni), f = ni + nb)
// column-major with leading dimension f, and where its inputs live.  After
// Gauss-Jordan elimination of the first ni columns it holds
//   F(0:ni, ni:f)  = R = -A_ii^-1 A_ib       (eq. 3.3b, negated in place)
//   F(0:ni, f:)    = A_ii^-1                  (block-diagonal factor D^-1)
//   F(ni:f, ni:f)  = S = A_bb - A_bi A_ii^-1 A_ib   (eq. 3.5)
//   F(ni:f, f:)    = L = -A_bi A_ii^-1        (eq. 3.3a)
struct FrontDesc {
  long foff;        // element offset of F in the front pool
  int f, ni, nb;    // front size, |I|, |B|
  int ioff;         // first position of I in the elimination order
  int bpos_off;     // offset of the nb positions of B in the B-position pool
  int src_off;      // offset of the f front-entry sources in the source pools
  int lo, hi;       // children (-1 for leaves)
};

// Assemble the augmented fronts of `count` nodes (ids in nodes[]): entries
// from the children's Schur blocks (same child, read from cpool) or from A
// (natural CSR, c128), and the identity block.  Each front is written to
// opool + foff (opool may differ from cpool: the roots of a complex64 factor
// are kept in complex128).
template <typename T, typename Tc>
void launch_front_assemble(int count, const int *nodes, const FrontDesc *desc,
                           const int *src_gid, const int *src_code,
                           const int *rowptr, const int *col, const c128 *val,
                           const cplx<Tc> *cpool, cplx<T> *opool, hipStream_t st, int max_f);

// Elimination job: Gauss-Jordan elimination of the first ne columns of the
// m x ncols matrix at ptr (leading dimension ld), partial pivoting among the
// first ne rows (pivot magnitude |re|+|im|, first row on ties), pivot rows
// normalised; every other row, including rows >= ne, is reduced.  Columns
// >= ne of rows >= ne end as the Schur complement.  With negate_r the block
// (0:ne, ne:m) is negated afterwards.
// The last ne columns of a job hold the identity on its pivot rows (and
// zeros below): they receive the inverse of the pivot block.
template <typename T> struct ElimJob {
  cplx<T> *ptr;
  int ld, m, ncols, ne, negate_r;
  int node;         // reported on a zero pivot
};
// lds_bytes > 0: every job's m x ncols block fits in that much LDS (at most
// 156 KiB) and runs staged there, as a persistent launch whose workgroups
// take jobs in list order from the device counter *queue (zero before the
// launch); 0: one workgroup per job from global memory
template <typename T>
void launch_eliminate(int count, const ElimJob<T> *jobs, int *err_node, hipStream_t st,
                      size_t lds_bytes = 0, int *queue = nullptr);
// Register-resident variant for jobs with m == ne <= 128, no negated R block
// and ncols - m <= eliminate_reg_max_cols<T>(m), persistent over the counter
// *queue (zero before the launch); it inverts in place and relies on the
// last ne columns holding the identity on input (every job of the
// factorization is laid out so).  Returns false (nothing launched) when the
// sizes do not fit
template <typename T> int eliminate_reg_max_cols(int max_m);
template <typename T>
bool launch_eliminate_reg(int count, const ElimJob<T> *jobs, int *err_node, hipStream_t st,
                          int max_m, int max_nc, int *queue);

// Blocked Gauss-Jordan, one column panel P = [p0, p0 + nb) of one job per
// entry (jobs of one launch may belong to different fronts):
//   panel:  pivots of P by partial-pivoted LU of rows [p0, ne) (scratch W),
//           G = (pivot block)^-1
//   swap:   apply the nb row interchanges to columns [p0, ncols)
//   gemm_a: Y = G F(P rows, J), J = [p0 + nb, ncols)
//   gemm_b: F(P rows, J) = Y;  F(other rows, J) -= F(other rows, P) Y
template <typename T> struct PanelJob {
  cplx<T> *F;
  int ld, m, ncols, ne, p0, nb;
  int *piv;        // nb pivot rows
  cplx<T> *G;      // nb x nb
  cplx<T> *Y;      // nb x (ncols - p0 - nb)
  cplx<T> *W;      // (ne - p0) x nb
  int node;
};
// C -= A B for a batch of jobs (complex, column-major, each job its own
// sizes and leading dimensions); K may be 0
template <typename T> struct GemmJob {
  const cplx<T> *A, *B;
  cplx<T> *C;
  int lda, ldb, ldc, M, N, K;
};
template <typename T>
void launch_gemm_sub(int count, const GemmJob<T> *jobs, int max_m, int max_n, hipStream_t st);

// max_prows = largest ne - p0, max_nb = largest nb of the launch; the panel
// runs register-resident when nb <= 32 (complex64) or 16 (complex128) and
// ne - p0 <= 1536, else from the scratch W.
template <typename T>
void launch_panel_step(int count, const PanelJob<T> *jobs, int max_m, int max_cols,
                       int max_prows, int max_nb, int *err_node, hipStream_t st);

// dst(i,j) += a * src1(i,j) + b * src2(i,j) for an m x n block (all column-major)
template <typename T> struct AxpbyJob {
  cplx<T> *dst;
  const cplx<T> *s1;
  const cplx<T> *s2;
  int ld_dst, ld1, ld2, m, n;
  T a, b;
};
template <typename T>
void launch_axpby(int count, const AxpbyJob<T> *jobs, int max_m, int max_n, hipStream_t st);

// ------------------------------------------------------------ sketches (Alg. A.1)
// Gaussian block Omega(i, j), i < m, j in [c0, c0 + nc) of instance key
// (seed, key1), stored real in out (leading dimension ld) at column j - cbase.
struct GaussJob {
  double *out;
  int ld, m, c0, nc, cbase;
  uint32_t key1;
};
void launch_gaussian(int count, const GaussJob *jobs, uint32_t seed, int max_m, int max_nc,
                     hipStream_t st);

// Y(:, 0:nc) = S(m x m complex T) * Om(m x nc real double)
template <typename T> struct SampleJob {
  const cplx<T> *S;
  const double *Om;
  cplx<T> *Y;
  int ldS, ldO, ldY, m, nc;
};
template <typename T>
void launch_sample(int count, const SampleJob<T> *jobs, int max_m, int max_nc, hipStream_t st);
// the same product for complex64 S on bf16 matrix cores with fp32
// accumulation: split = 1 rounds the operands to bf16, split = 2 keeps a bf16
// head and tail of each operand (three products)
void launch_sample_bf16(int count, const SampleJob<float> *jobs, int max_m, int max_nc, int split,
                        hipStream_t st);

// One cluster of one compression instance at the current tree level.
// Layout of an instance's HSS generators: per cluster offsets (elements of
// cplx<T>) into the instance generator pool, capacities fixed by the host.
struct HssCluster {
  int start, size;      // index range in the instance's ordering
  int left, right;      // children (cluster ids within the instance) or -1
  int level;            // depth in the cluster tree (root 0, level order)
  int rows_cap, k_cap;  // capacity of U (rows_cap x k_cap)
  long U, Om, Sr, D, B12, B21;  // offsets in the instance generator pool
  int sk;               // offset of skeleton ids in the instance int pool
  long W;               // compression scratch offset (relative to the instance)
  long XH;              // matvec scratch offset (relative to the job)
};
constexpr int kMaxLev = 24;   // cluster-tree levels of one instance
constexpr int kXC = 16;       // columns of one HSS matvec job
struct HssInstance {
  int m;                // matrix size
  int ncl;              // clusters (level order, root = 0)
  int nlev;             // tree levels; level l holds clusters [lev_off[l], lev_off[l+1])
  int lev_off[kMaxLev + 1];
  int cl_off;           // first cluster in the global cluster array
  int s;                // sample columns (k + r)
  int k;                // rank cap of this round
  long pool;            // offset of this instance in the generator pool
  long ipool;           // offset in the int pool
  long soff;            // offset of the dense operator S (front pool)
  int ldS;
  long yoff;            // offset of the samples Y = S Omega (sample pool)
  long ooff;            // offset of Omega (real pool)
  int ldY;
  long woff;            // scratch offset (two rows_cap x s blocks per cluster)
  int pre;              // 1: D and B blocks are written into the pool before
                        // each level's launch (operators not formed densely)
  int eop;              // entry operator of such an instance (-1: dense S)
};
struct HssItem {
  int inst, cl;         // instance, cluster id within it
};
// Size classes of one compression launch (every item of the launch fits its
// class): clusters of at most 64 rows in 256-thread workgroups (s <= 64,
// s <= 128, any s); larger clusters that fit the 1024-thread register path
// (at most kRegRows rows, s <= kRegCols; complex64), with tiles for at most
// 128 rows and s <= 64 or s <= 128; any other cluster (global-memory QR).
constexpr int kRegRows = 256, kRegCols = 192;
enum : int {
  kCls256 = 0, kCls1024 = 1, kClsGlobal = 2, kCls256S64 = 3, kCls256S128 = 4,
  kCls1024R128S64 = 5, kCls1024R128S128 = 6
};
template <typename T>
void launch_compress_level(int count, const HssItem *items, const HssInstance *inst,
                           const HssCluster *cl, cplx<T> *pool, int *ipool, int *rank,
                           const cplx<T> *front, const cplx<T> *Y, const double *Om,
                           cplx<T> *scratch, double id_tol, int size_class, hipStream_t st);
// Per job (nc <= kXC columns of one instance): out = H X for the compressed
// H, with X given (ldX) or the identity columns c0.. when X is null; if Yref
// is given, add ||Yref - H X||_F^2 to *err2 and ||Yref||_F^2 to *ref2 (both
// zeroed by the caller) instead of writing out.  Scratch per job: 2 k_cap
// kXC per cluster at XH.  nlev, max_width, max_ncl: the largest level count,
// clusters in one level and clusters of the launch's instances.
template <typename T> struct MatvecJob {
  int inst;
  const double *X;      // real input (m x nc), or null for identity columns c0..
  int ldX, nc, c0;
  cplx<T> *out;         // m x nc output (ldO) or null
  int ldO;
  const cplx<T> *Yref;  // reference samples (ldR) or null
  int ldR;
  double *err2, *ref2;
  long woff;            // scratch offset for the sweep vectors
};
template <typename T>
void launch_hss_matvec(int count, const MatvecJob<T> *jobs, const HssInstance *inst,
                       const HssCluster *cl, const cplx<T> *pool, const int *rank,
                       cplx<T> *scratch, int nlev, int max_width, int max_ncl, hipStream_t st);

// ------------------------------------------------------------ apply (Alg. 3.1)
// y = x(perm) (inverse = 0) or y(perm) = x (inverse = 1), n x nrhs
void launch_permute(int n, int nrhs, const int *perm, const c128 *x, long ldx, c128 *y,
                    long ldy, int inverse, hipStream_t st);
// Tile shapes of the (non-transposed) apply sweeps: rows of the output per
// 256-thread workgroup and right-hand sides per thread.
struct ApplyCfg {
  int rows, rb;
};
constexpr int kNumApplyCfgs = 6;
extern const ApplyCfg kApplyCfgs[kNumApplyCfgs];
// Up-sweep of one tree depth: t = x(I); x(I) = A_ii^-1 t; x(B) += L t
// (trans: A_ii^-T t and R^T t).  x is in elimination order (ld n); tb is an
// n x nrhs staging buffer that receives a copy of the I blocks first.  cfg
// indexes kApplyCfgs (ignored for trans).
template <typename T>
void launch_apply_up(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
                     const int *bpos, c128 *tb, c128 *x, int n, int nrhs, int trans, int max_ni,
                     int max_f, int cfg, hipStream_t st);
// Down-sweep of one tree depth: x(I) += R x(B) (trans: L^T x(B)).
template <typename T>
void launch_apply_down(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
                       const int *bpos, c128 *x, int n, int nrhs, int trans, int max_nb,
                       int max_ni, int cfg, hipStream_t st);

// ------------------------------------------------------------ Krylov
// Systems of a vector block (n rows x nrhs columns): the rows split into np
// parts [off[p], off[p+1]) (device array), rpart[k] is the part of row k
// (device array, or null when np == 1); system s = r * np + p.  Per-system
// arrays (h, norms, scale, cnt) are indexed i * nseg + s, nseg = np * nrhs.
struct Segs {
  int np;
  const int *off;
  const int *rpart;
};
// h[i*nseg + s] = sum over system s of conj(V_i) w, i < cnt; V_i at V + i*stride
void launch_mdot(int n, int nrhs, const Segs &g, int cnt, const c128 *V, long stride,
                 const c128 *w, c128 *h, c128 *partial, int nblk, hipStream_t st);
// w -= sum_{i<cnt} V_i h[i*nseg + s] on each system s
void launch_mupdate(int n, int nrhs, const Segs &g, int cnt, const c128 *V, long stride,
                    const c128 *h, c128 *w, hipStream_t st);
// norms[s] = ||w on system s||_2
void launch_norms(int n, int nrhs, const Segs &g, const c128 *w, double *norms, double *partial,
                  int nblk, hipStream_t st);
// out = in / scale[s] on system s (zero when scale[s] == 0)
void launch_scale(int n, int nrhs, const Segs &g, const c128 *in, const double *scale, c128 *out,
                  hipStream_t st);
// y = a - b
void launch_sub(int n, int nrhs, const c128 *a, long lda, const c128 *b, long ldb, c128 *y,
                long ldy, hipStream_t st);
// x += sum_{i<cnt[s]} Z_i y[i*nseg + s] on each system s
void launch_xupdate(int n, int nrhs, const Segs &g, const int *cnt, const c128 *Z, long stride,
                    const c128 *y, c128 *x, long ldx, hipStream_t st);
// Arnoldi column j bookkeeping for every system: store h, apply the previous
// Givens rotations, build the new one, update g; res[s] = |g_{j+1}|.
void launch_givens(int nseg, int j, int m, c128 *H, const c128 *hcol, const double *hnext,
                   double *cs, c128 *sn, c128 *g, double *res, const int *active,
                   hipStream_t st);
// back substitution H(0:cnt,0:cnt) y = g per system
void launch_hsolve(int nseg, int m, const c128 *H, const c128 *g, const int *cnt, c128 *y,
                   hipStream_t st);
void launch_fill(long n, c128 v, c128 *x, hipStream_t st);
// y = conj(x), n x nrhs (x may equal y)
void launch_conj(long n, int nrhs, const c128 *x, long ldx, c128 *y, long ldy, hipStream_t st);

}  // namespace hssx
