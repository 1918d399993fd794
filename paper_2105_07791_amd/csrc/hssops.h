// Batched building blocks of the HSS arithmetic (Sec. 2.2, Sec. 3.3-3.5):
// small complex products, block copies, row gathers between index spaces,
// products with the sparse couplings between sibling boxes, and entry
// extraction from operators given in generator form.  Every launcher takes
// a device array of jobs (each job with its own sizes, leading dimensions
// and absolute pointers) and enqueues one launch on the given stream.
#pragma once

#include "common.h"
#include "kernels.h"

namespace hssx {

// C = alpha op(A) op(B) + beta C, op = identity or transpose (no conjugate:
// the operators are complex symmetric), column-major; beta is 0 or 1.
template <typename T> struct BgJob {
  const cplx<T> *A, *B;
  cplx<T> *C;
  int lda, ldb, ldc, M, N, K;
  int ta, tb, beta;
  T ar, ai;   // alpha
};
// one 32 x 32 output tile of one job, with a copy of the job so that a
// workgroup reads its whole description in one load
template <typename T> struct BgTask {
  BgJob<T> jb;
  int tm, tn;
};
template <typename T>
void launch_bgemm(int ntiles, const BgTask<T> *tasks, hipStream_t st);

// Block copies: mode 0 dst = s src, 1 dst = s src^T, 2 dst = I, 3 dst = 0,
// 4 dst += s src (m x n block of dst; src m x n, or n x m for mode 1).
template <typename T> struct CopyJob {
  const cplx<T> *src;
  cplx<T> *dst;
  int lds, ldd, m, n, mode;
  T s;
};
template <typename T>
void launch_copy(int count, const CopyJob<T> *jobs, long max_elems, hipStream_t st);

// Row gather / scatter with conversion: for r < nrows, column j < nc,
//   v = src[smap ? smap[r] : r][j] (zero when smap[r] < 0),
//   dst[dmap ? dmap[r] : r][j] = s v (mode 0) or += s v (mode 1) (skipped
//   when dmap[r] < 0).  Ts: double (a real sketch), c64 or c128.
template <typename Ts, typename Td> struct GatherJob {
  const Ts *src;
  Td *dst;
  long lds, ldd;
  const int *smap, *dmap;
  int nrows, nc, mode;
  double s;
};
template <typename Ts, typename Td>
void launch_gather(int count, const GatherJob<Ts, Td> *jobs, long max_elems, hipStream_t st);

// Sparse product with a coupling block stored as a row list: for r < nrows,
//   t = sum_{e in [rp[r], rp[r+1])} val[vi[e]] X[cp[e]][j],
//   Y[r][j] = s t (acc = 0) or += s t (acc = 1).  Values are read from the
//   operator's CSR values (complex128) and rounded to T.
template <typename T> struct SpJob {
  const int *rp, *cp, *vi;
  int nrows, nc, acc;
  const cplx<T> *X;
  long ldx;
  cplx<T> *Y;
  long ldy;
  T s;
};
template <typename T>
void launch_spmm(int count, const SpJob<T> *jobs, const c128 *val, long max_elems, hipStream_t st);

// dst[ri[e] + (coff + ci[e]) ld] = val[vi[e]] (or 1 when vi[e] < 0), e < cnt
template <typename T> struct FillJob {
  const int *ri, *ci, *vi;
  int cnt, ld, coff;
  cplx<T> *dst;
};
template <typename T>
void launch_fill_coo(int count, const FillJob<T> *jobs, const c128 *val, int max_cnt,
                     hipStream_t st);

// P (m x n) and Q (n x m) both become (P + Q^T) / 2 and its transpose; P may
// equal Q (a square block made symmetric in place).
template <typename T> struct SymJob {
  cplx<T> *P, *Q;
  int ldp, ldq, m, n;
};
template <typename T>
void launch_symmetrize(int count, const SymJob<T> *jobs, long max_elems, hipStream_t st);

// ---------------------------------------------------------------- entries
// One cluster of a nested-basis symmetric HSS matrix prepared for entry
// access: Uf is the transpose of the cluster's full basis (k x size, ld k;
// the basis is the product of the transfer matrices down to the leaves,
// eq. 2.3), UB the transpose of that basis times the coupling block towards
// the sibling (k_sibling x size, ld k_sibling), D the diagonal block of a
// leaf.  Then for positions i, j in different leaves, with a, b the children
// of their lowest common ancestor containing i, j:
//   H(i, j) = UB_a(:, i) . Uf_b(:, j)   (contiguous columns).
template <typename T> struct EntCl {
  int start, size, left, right, parent, level, k, ldD;
  const cplx<T> *D, *Uf, *UB;
};
template <typename T> struct EntView {
  const EntCl<T> *cl;
  const int *leaf_of;   // position -> leaf cluster id
};
template <typename T>
__device__ __forceinline__ cplx<T> hss_entry(const EntView<T> &V, int i, int j) {
  int a = V.leaf_of[i], b = V.leaf_of[j];
  const EntCl<T> *C = V.cl;
  if (a == b) {
    const EntCl<T> &c = C[a];
    return c.D[(i - c.start) + (long)(j - c.start) * c.ldD];
  }
  while (C[a].level > C[b].level) a = C[a].parent;
  while (C[b].level > C[a].level) b = C[b].parent;
  while (C[a].parent != C[b].parent) {
    a = C[a].parent;
    b = C[b].parent;
  }
  const EntCl<T> &ca = C[a], &cb = C[b];
  cplx<T> v = czero<T>();
  const cplx<T> *u = ca.UB + (long)(i - ca.start) * cb.k, *w = cb.Uf + (long)(j - cb.start) * cb.k;
  for (int t = 0; t < cb.k; ++t) cfma(v, u[t], w[t]);
  return v;
}

// Entries of an operator compressed without being formed (Sec. 3.5):
//  kind 0: the Schur complement S(sigma) = A_bb - Y_B C Y_B^T on sigma's
//          boundary order, A_bb from the children's compressed Schur
//          complements (same child) or from A (different children);
//  kind 1: the inner Schur complement S~ = S_ii^nu - A~(nu,mu) X A~(mu,nu)
//          on nu's interior order, X = (S_ii^mu)^-1 in HSS form.
template <typename T> struct EntryOp {
  int kind;
  EntView<T> H0, H1;              // kind 0: mu's and nu's S; kind 1: X and nu's S
  const int *bchild, *bcpos, *gid;
  const cplx<T> *YC, *YB;         // kind 0: (Y_B C)^T and Y_B^T (r x nb, ld r)
  int r;
  const int *rp, *cp, *vi;        // kind 1: A~(nu,mu) rows
};

// out[e] = H(ij[2e], ij[2e+1]) for e < n
template <typename T>
void launch_entries_list(EntView<T> view, const int *ij, int n, cplx<T> *out, hipStream_t st);

template <typename T>
void launch_entries(int count, const HssItem *items, const HssInstance *inst,
                    const HssCluster *cl, cplx<T> *pool, const int *ipool, const int *rank,
                    const EntryOp<T> *ops, const int *rowptr, const int *col, const c128 *val,
                    hipStream_t st);

}  // namespace hssx
