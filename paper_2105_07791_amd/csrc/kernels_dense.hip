// Dense fronts of the nested-dissection elimination (eqs. 3.2-3.5).
//
// front_assemble: F(p, q) = S_child(p, q) when both front entries belong to
// the same child's boundary (entry source code 2 pos + child, -1 for none) (the child's Schur complement, held in the
// trailing block of the child's front), else A(p, q) from the CSR (eq. 3.4);
// the appended ni columns start as [I; 0].
//
// eliminate: Gauss-Jordan elimination of the first ne columns with partial
// pivoting among the first ne rows.  On the augmented front this yields in
// one pass A_ii^-1, A_ii^-1 A_ib (negated into R, eq. 3.3b), L = -A_bi A_ii^-1
// (eq. 3.3a) and the Schur complement S (eq. 3.5).  One workgroup per job;
// each thread owns whole rows during an elimination step, so the multiplier
// column can be cleared without an extra barrier.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr int kThreads = 256;

template <typename T, typename Tc>
__global__ __launch_bounds__(kThreads) void front_assemble_kernel(
    const int *__restrict__ nodes, const FrontDesc *__restrict__ desc,
    const int *__restrict__ src_gid, const int *__restrict__ src_code,
    const int *__restrict__ rowptr,
    const int *__restrict__ col, const c128 *__restrict__ val,
    const cplx<Tc> *__restrict__ cpool, cplx<T> *__restrict__ opool) {
  const FrontDesc d = desc[nodes[blockIdx.x]];
  const long f = d.f;
  const long total = f * (f + d.ni);
  const long per = (long)kThreads * 16;
  long e0 = (long)blockIdx.y * per;
  if (e0 >= total) return;
  long e1 = e0 + per < total ? e0 + per : total;
  const int *gid = src_gid + d.src_off;
  const int *code = src_code + d.src_off;
  cplx<T> *F = opool + d.foff;
  for (long e = e0 + threadIdx.x; e < e1; e += kThreads) {
    int p = (int)(e % f), q = (int)(e / f);
    cplx<T> v;
    if (q >= f) {
      v = mk((T)(p == q - f ? 1 : 0), (T)0);
    } else {
      const int ep = code[p], eq = code[q];
      if (ep >= 0 && eq >= 0 && (ep & 1) == (eq & 1)) {
        const FrontDesc c = desc[(ep & 1) == 0 ? d.lo : d.hi];
        v = ccast<T>(cpool[c.foff + (long)(c.ni + (ep >> 1)) + (long)(c.ni + (eq >> 1)) * c.f]);
      } else {
        int gi = gid[p], gj = gid[q];
        c128 a = czero<double>();
        // sorted columns: most pairs of a large front lie outside row gi's
        // column range and are rejected by its two ends; the rest bisect
        int lo = rowptr[gi], hi = rowptr[gi + 1] - 1;
        if (lo <= hi && gj >= col[lo] && gj <= col[hi]) {
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (col[mid] < gj) lo = mid + 1;
            else hi = mid;
          }
          if (col[lo] == gj) a = val[lo];
        }
        v = ccast<T>(a);
      }
    }
    F[e] = v;
  }
}

// Gauss-Jordan of a small front staged in LDS (dynamic shared memory holds
// the m x ncols front with leading dimension m).  Per pivot: wave 0 finds
// the pivot (DPP argmax, ties to the lowest row) and its inverse; one pass
// over the columns exchanges the two rows and scales the pivot row; one pass
// over (row, column) pairs applies the rank-1 update, every thread busy.
// The pivot columns are written as the identity at the end (they are never
// read again), and R = F(0:ne, ne:m) is negated on the way out.
//
// Persistent launch over a work queue: the grid holds as many workgroups as
// fit on the device at once, and each takes the next front from a device
// counter (jobs are listed by decreasing cost, so the uneven fronts of a
// level are balanced longest first).  Every workgroup leaves the loop once
// the counter passes the job count.
template <typename T>
__global__ __launch_bounds__(kThreads) void eliminate_lds_kernel(const ElimJob<T> *__restrict__ jobs,
                                                                int count, int *__restrict__ queue,
                                                                int *__restrict__ err_node) {
  extern __shared__ unsigned char smem_raw[];
  cplx<T> *Fs = reinterpret_cast<cplx<T> *>(smem_raw);
  __shared__ int s_piv, s_job;
  __shared__ cplx<T> s_inv;
  const int tid = threadIdx.x;
  for (;;) {
  if (tid == 0) s_job = atomicAdd(queue, 1);
  __syncthreads();
  const int job = s_job;
  if (job >= count) break;
  const ElimJob<T> jb = jobs[job];
  const int m = jb.m, nc = jb.ncols, ne = jb.ne;
  const long ld = jb.ld;
  for (int e = tid; e < m * nc; e += kThreads) {
    const int i = e % m, j = e / m;
    Fs[e] = jb.ptr[i + (long)j * ld];
  }
  __syncthreads();
  for (int p = 0; p < ne; ++p) {
    if (tid < 64) {
      T best = (T)-1;
      int bi = 0x7fffffff;
      for (int i = p + tid; i < ne; i += 64) {
        const T a = cabs1(Fs[i + p * m]);
        if (a > best || (a == best && i < bi)) { best = a; bi = i; }
      }
      wave_argmax(best, bi);
      if (tid == 0) {
        const bool zero = !(best > (T)0);
        if (zero) atomicCAS(err_node, -1, jb.node);
        s_piv = zero ? p : bi;
        s_inv = zero ? czero<T>() : cinv(Fs[bi + p * m]);
      }
    }
    __syncthreads();
    const int pv = s_piv;
    const cplx<T> inv = s_inv;
    for (int j = p + tid; j < nc; j += kThreads) {
      const cplx<T> a = Fs[p + j * m], b = Fs[pv + j * m];
      Fs[pv + j * m] = a;
      Fs[p + j * m] = j == p ? mk((T)1, (T)0) : b * inv;
    }
    __syncthreads();
    // rank-1 update in register tiles of 4 rows (strided by rs, so that
    // neighbouring threads touch neighbouring rows) by 4 columns: the pivot
    // column's and the pivot row's entries are read once per tile, not once
    // per element
    const int w = nc - p - 1, rs = (m + 3) >> 2, tj = (w + 3) >> 2;
    for (int e = tid; e < rs * tj; e += kThreads) {
      const int i0 = e % rs, j0 = p + 1 + ((e / rs) << 2);
      cplx<T> a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + r * rs;
        a[r] = (i < m && i != p) ? Fs[i + p * m] : czero<T>();
      }
#pragma unroll
      for (int c = 0; c < 4; ++c) b[c] = j0 + c < nc ? Fs[p + (j0 + c) * m] : czero<T>();
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        if (j0 + c >= nc) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int i = i0 + r * rs;
          if (i < m && i != p) cfms(Fs[i + (j0 + c) * m], a[r], b[c]);
        }
      }
    }
    __syncthreads();
  }
  for (int e = tid; e < m * nc; e += kThreads) {
    const int i = e % m, j = e / m;
    cplx<T> v = Fs[e];
    if (j < ne) v = mk((T)(i == j ? 1 : 0), (T)0);
    else if (jb.negate_r && i < ne && j < m) v = -v;
    jb.ptr[i + (long)j * ld] = v;
  }
  __syncthreads();   // Fs and s_job are reused by the next front
  }
}

// Gauss-Jordan on small square blocks held in registers, inverting in place:
// a job's last ne columns hold the identity on input and are not read; the
// kernel works on the first W = ncols - ne columns and writes the inverse of
// the leading block into those last columns.  NT threads, RG row groups x
// NT / RG column groups; thread (i0, cg) keeps rows i0 + RG r (r < RPT) of
// working columns cg CPT .. cg CPT + CPT - 1; the RG threads of a column
// group sit in one wavefront.  Rows are not swapped: step p picks the
// unused row of largest |.|_1 in column p (ties to the smaller row) as the
// pivot row r_p, scales it and removes column p from every other row; slot p
// then holds column r_p of the accumulated row operations (the identity
// column that only row r_p touched until this step), i.e. row r_q of slot p
// is entry (q, r_p) of the inverse.  The write-back puts row r_q in position
// q, the identity in the leading block and the inverse in the last block.
// Per step only column p passes through LDS (double-buffered: one barrier a
// step); the pivot row comes by lane shuffles.  Jobs have m == ne <= RG RPT
// <= 128, W <= (NT / RG) CPT and no negated R block; the workgroups take jobs
// from the counter *queue.
template <typename T, int NT, int RG, int RPT, int CPT>
__global__ __launch_bounds__(NT) void eliminate_reg_kernel(const ElimJob<T> *__restrict__ jobs,
                                                           int count, int *__restrict__ queue,
                                                           int *__restrict__ err_node) {
  constexpr int MR = RG * RPT;
  static_assert(MR <= 128 && (RG == 16 || RG == 32) && NT % 64 == 0, "at most 128 rows");
  __shared__ T s_abs[2][128];
  __shared__ cplx<T> s_col[2][128];
  __shared__ int s_order[128], s_pos[128];
  __shared__ int s_job;
  const int tid = threadIdx.x, i0 = tid % RG, cg = tid / RG, lane = tid & 63;
  for (;;) {
    if (tid == 0) s_job = atomicAdd(queue, 1);
    if (tid < 128) s_pos[tid] = -1;
    __syncthreads();
    const int job = s_job;
    if (job >= count) break;
    const ElimJob<T> jb = jobs[job];
    const int m = jb.m, w = jb.ncols - jb.m;
    const long ld = jb.ld;
    cplx<T> F[RPT][CPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r)
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int i = i0 + r * RG, j = cg * CPT + c;
        F[r][c] = (i < m && j < w) ? jb.ptr[i + (long)j * ld] : czero<T>();
      }
    unsigned long long used0 = 0, used1 = 0;   // rows taken as pivots (0-63, 64-127)
    for (int p = 0; p < m; ++p) {
      const int b = p & 1;
      const bool pcol = cg == p / CPT;   // this thread holds slot p
      const int pc = p % CPT;
      // column p, published by its owners (unused rows with their magnitude)
      if (pcol) {
#pragma unroll
        for (int c = 0; c < CPT; ++c)
          if (c == pc) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
              const int i = i0 + r * RG;
              if (i < m) {
                s_col[b][i] = F[r][c];
                const bool u = i < 64 ? ((used0 >> i) & 1ull) : ((used1 >> (i - 64)) & 1ull);
                s_abs[b][i] = u ? (T)-1 : cabs1(F[r][c]);
              }
            }
          }
      }
      __syncthreads();
      // every wave finds the same pivot
      T best = lane < m ? s_abs[b][lane] : (T)-2;
      int bi = lane;
      if (MR > 64 && lane + 64 < m) {
        const T o = s_abs[b][lane + 64];
        if (o > best) { best = o; bi = lane + 64; }
      }
      wave_argmax(best, bi);
      const bool zero = !(best > (T)0);
      // a zero (or NaN) column takes the first unused row and is reported
      const int first = ~used0 ? __builtin_ctzll(~used0) : 64 + __builtin_ctzll(~used1);
      const int pv = zero ? first : bi;
      const cplx<T> inv = zero ? czero<T>() : cinv(s_col[b][pv]);
      if (tid == 0) {
        if (zero) atomicCAS(err_node, -1, jb.node);
        s_order[p] = pv;
      }
      if (pv < 64) used0 |= 1ull << pv;
      else used1 |= 1ull << (pv - 64);
      // the pivot row, scaled: the lane of this 16-lane group that holds row
      // pv holds it for the same columns (same wavefront), so it comes by a
      // lane shuffle, not through LDS; its slot p becomes inv and is left out
      // of the update (0 in prow)
      const int rr = pv / RG, src = (lane & ~(RG - 1)) | (pv % RG);
      const bool owner = i0 == pv % RG;
      cplx<T> prow[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        cplx<T> v = czero<T>();
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (r == rr) v = F[r][c];
        v = mk(__shfl(v.re, src), __shfl(v.im, src));
        const bool isp = pcol && c == pc;
        const cplx<T> sv = v * inv;
        prow[c] = isp ? czero<T>() : sv;
        if (owner) {
#pragma unroll
          for (int r = 0; r < RPT; ++r)
            if (r == rr) F[r][c] = isp ? inv : sv;
        }
      }
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = i0 + r * RG;
        if (i < m && i != pv) {
          const cplx<T> a = s_col[b][i];
#pragma unroll
          for (int c = 0; c < CPT; ++c) {
            cfms(F[r][c], a, prow[c]);
            // slot p of the other rows: -a inv
            if (pcol && c == pc) F[r][c] = -(a * inv);
          }
        }
      }
    }
    __syncthreads();   // the last step's s_order entry
    for (int t = tid; t < m; t += NT) s_pos[s_order[t]] = t;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = i0 + r * RG;
      const int q = i < m ? s_pos[i] : -1;
      if (q < 0) continue;
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        const int j = cg * CPT + c;
        if (j >= w) continue;
        if (j < m) {
          jb.ptr[q + (long)j * ld] = mk((T)(q == j ? 1 : 0), (T)0);
          jb.ptr[q + (long)(w + s_order[j]) * ld] = F[r][c];
        } else {
          jb.ptr[q + (long)j * ld] = F[r][c];
        }
      }
    }
    __syncthreads();   // s_job, s_order and s_pos are reused by the next job
  }
}

template <typename T>
__device__ void block_argmax(T &v, int &idx, T *sv, int *si) {
  // wave reduction then across waves; ties keep the smaller index
  for (int off = 32; off > 0; off >>= 1) {
    T ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) { sv[w] = v; si[w] = idx; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < kThreads / 64; ++k)
      if (sv[k] > sv[0] || (sv[k] == sv[0] && si[k] < si[0])) { sv[0] = sv[k]; si[0] = si[k]; }
  }
  __syncthreads();
  v = sv[0];
  idx = si[0];
  __syncthreads();
}

template <typename T>
__global__ __launch_bounds__(kThreads) void eliminate_kernel(const ElimJob<T> *__restrict__ jobs,
                                                            int *__restrict__ err_node) {
  __shared__ T sv[kThreads / 64];
  __shared__ int si[kThreads / 64];
  const ElimJob<T> jb = jobs[blockIdx.x];
  cplx<T> *F = jb.ptr;
  const long ld = jb.ld;
  const int m = jb.m, nc = jb.ncols, ne = jb.ne;
  const int tid = threadIdx.x;
  for (int p = 0; p < ne; ++p) {
    T best = (T)-1;
    int bi = 0x7fffffff;
    for (int i = p + tid; i < ne; i += kThreads) {
      T a = cabs1(F[i + p * ld]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    block_argmax(best, bi, sv, si);
    const bool zero = !(best > (T)0);
    if (zero && tid == 0) atomicCAS(err_node, -1, jb.node);
    const int piv = zero ? p : bi;
    if (piv != p) {
      for (int j = p + tid; j < nc; j += kThreads) {
        cplx<T> a = F[p + j * ld];
        F[p + j * ld] = F[piv + j * ld];
        F[piv + j * ld] = a;
      }
    }
    __syncthreads();
    const cplx<T> inv = zero ? czero<T>() : cinv(F[p + p * ld]);
    for (int j = p + 1 + tid; j < nc; j += kThreads) F[p + j * ld] = F[p + j * ld] * inv;
    __syncthreads();
    for (int i = tid; i < m; i += kThreads) {
      if (i == p) continue;
      const cplx<T> l = F[i + p * ld];
      for (int j = p + 1; j < nc; ++j) cfms(F[i + j * ld], l, F[p + j * ld]);
      F[i + p * ld] = czero<T>();
    }
    if (tid == 0) F[p + p * ld] = mk((T)1, (T)0);
    __syncthreads();
  }
  if (!jb.negate_r) return;
  const int nb = m - ne;
  for (long t = tid; t < (long)ne * nb; t += kThreads) {
    int l = (int)(t % ne), c = (int)(t / ne);
    long e = l + (long)(ne + c) * ld;
    F[e] = -F[e];
  }
}


// ---------------------------------------------------------------- blocked GJ
constexpr int kNB = 32;   // largest panel width
constexpr int kTile = 64; // trailing-update tile (rows and columns)

template <typename T>
__global__ __launch_bounds__(kThreads) void panel_kernel(const PanelJob<T> *__restrict__ jobs,
                                                        int *__restrict__ err_node) {
  __shared__ T sv[kThreads / 64];
  __shared__ int si[kThreads / 64];
  const PanelJob<T> jb = jobs[blockIdx.x];
  const int rows = jb.ne - jb.p0, nb = jb.nb, tid = threadIdx.x;
  const long ld = jb.ld;
  cplx<T> *W = jb.W;
  for (int e = tid; e < rows * nb; e += kThreads) {
    int i = e % rows, t = e / rows;
    W[e] = jb.F[(jb.p0 + i) + (long)(jb.p0 + t) * ld];
  }
  __syncthreads();
  for (int t = 0; t < nb; ++t) {
    T best = (T)-1;
    int bi = 0x7fffffff;
    for (int i = t + tid; i < rows; i += kThreads) {
      T a = cabs1(W[i + (long)t * rows]);
      if (a > best || (a == best && i < bi)) { best = a; bi = i; }
    }
    block_argmax(best, bi, sv, si);
    const bool zero = !(best > (T)0);
    if (zero && tid == 0) atomicCAS(err_node, -1, jb.node);
    const int pv = zero ? t : bi;
    if (tid == 0) jb.piv[t] = jb.p0 + pv;
    if (pv != t)
      for (int c = tid; c < nb; c += kThreads) {
        cplx<T> a = W[t + (long)c * rows];
        W[t + (long)c * rows] = W[pv + (long)c * rows];
        W[pv + (long)c * rows] = a;
      }
    __syncthreads();
    const cplx<T> inv = zero ? czero<T>() : cinv(W[t + (long)t * rows]);
    for (int i = t + 1 + tid; i < rows; i += kThreads) {
      cplx<T> l = W[i + (long)t * rows] * inv;
      W[i + (long)t * rows] = l;
      for (int c = t + 1; c < nb; ++c) cfms(W[i + (long)c * rows], l, W[t + (long)c * rows]);
    }
    __syncthreads();
  }
  // G = (L11 U11)^-1, one column per thread, the column in registers
  // (unrolled substitutions; entries beyond nb stay zero)
  for (int c = tid; c < nb; c += kThreads) {
    cplx<T> z[kNB];
#pragma unroll
    for (int i = 0; i < kNB; ++i) {
      cplx<T> v = mk((T)(i == c ? 1 : 0), (T)0);
      if (i < nb) {
#pragma unroll
        for (int j = 0; j < i; ++j) cfms(v, W[i + (long)j * rows], z[j]);
      }
      z[i] = i < nb ? v : czero<T>();
    }
#pragma unroll
    for (int i = kNB - 1; i >= 0; --i) {
      if (i < nb) {
        cplx<T> v = z[i];
#pragma unroll
        for (int j = i + 1; j < kNB; ++j)
          if (j < nb) cfms(v, W[i + (long)j * rows], z[j]);
        z[i] = v * cinv(W[i + (long)i * rows]);
      }
    }
#pragma unroll
    for (int i = 0; i < kNB; ++i)
      if (i < nb) jb.G[i + (long)c * nb] = z[i];
  }
}

// Register-resident panel factorization: NT threads (512, or 256 / 128 when
// no panel of the launch has more rows), thread tid owns panel rows tid + NT q
// (q < RQ) across all NBW columns; pivot search by
// wavefront shuffles, the pivot row broadcast and row exchanges through LDS.
// Same results as panel_kernel (cabs1 pivots, lowest row on ties).
constexpr int kPT = 512;
template <typename T, int NBW, int RQ, int NT = kPT>
__global__ __launch_bounds__(NT) void panel_reg_kernel(const PanelJob<T> *__restrict__ jobs,
                                                        int *__restrict__ err_node) {
  // wavefront maxima and exchanged rows, double-buffered by step parity so
  // that a step needs two barriers
  __shared__ T sv[2][NT / 64];
  __shared__ int si[2][NT / 64];
  __shared__ cplx<T> prowb[2][NBW], trowb[2][NBW];
  __shared__ cplx<T> LU[NBW][NBW + 1];
  const PanelJob<T> jb = jobs[blockIdx.x];
  const int rows = jb.ne - jb.p0, nb = jb.nb, tid = threadIdx.x;
  const long ld = jb.ld;
  cplx<T> w[RQ][NBW];
#pragma unroll
  for (int q = 0; q < RQ; ++q) {
    const int i = tid + NT * q;
#pragma unroll
    for (int c = 0; c < NBW; ++c)
      w[q][c] = (i < rows && c < nb) ? jb.F[(jb.p0 + i) + (long)(jb.p0 + c) * ld] : czero<T>();
  }
  // the pivot steps are unrolled, so t and every column index are
  // compile-time constants: no per-column predicates on the step, and the
  // update touches only the columns right of the pivot
#pragma clang loop unroll(full)
  for (int t = 0; t < NBW; ++t) {
    if (t < nb) {
    const int par = t & 1;
    cplx<T> *prow = prowb[par], *trow = trowb[par];
    T best = (T)-1;
    int bi = 0x7fffffff;
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + NT * q;
      cplx<T> wt = czero<T>();
#pragma unroll
      for (int c = 0; c < NBW; ++c)
        if (c == t) wt = w[q][c];
      const T a = cabs1(wt);
      if (i >= t && i < rows && (a > best || (a == best && i < bi))) { best = a; bi = i; }
    }
    wave_argmax(best, bi);
    if ((tid & 63) == 0) { sv[par][tid / 64] = best; si[par][tid / 64] = bi; }
    lds_barrier();
    best = sv[par][0];
    bi = si[par][0];
#pragma unroll
    for (int k = 1; k < NT / 64; ++k)
      if (sv[par][k] > best || (sv[par][k] == best && si[par][k] < bi)) {
        best = sv[par][k];
        bi = si[par][k];
      }
    const bool zero = !(best > (T)0);
    if (zero && tid == 0) atomicCAS(err_node, -1, jb.node);
    const int pv = zero ? t : bi;
    if (tid == 0) jb.piv[t] = jb.p0 + pv;
    // exchange rows t and pv; the pivot row ends in prow
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + NT * q;
      if (i == pv) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) prow[c] = w[q][c];
      }
      if (i == t) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) trow[c] = w[q][c];
      }
    }
    lds_barrier();
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + NT * q;
      if (i == t) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) w[q][c] = prow[c];
      } else if (i == pv) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) w[q][c] = trow[c];
      }
    }
    const cplx<T> inv = zero ? czero<T>() : cinv(prow[t]);
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + NT * q;
      if (i > t && i < rows) {
        cplx<T> l = czero<T>();
#pragma unroll
        for (int c = 0; c < NBW; ++c)
          if (c == t) l = w[q][c];
        l = l * inv;
#pragma unroll
        for (int c = 0; c < NBW; ++c) {
          if (c == t) w[q][c] = l;
          else if (c > t) cfms(w[q][c], l, prow[c]);
        }
      }
    }
    }
  }
  // L11 U11 to LDS, then G = (L11 U11)^-1, one column per thread with the
  // column in registers (unrolled substitutions; LU read by broadcast).
  // Entries beyond nb are zero (the panel columns past nb were loaded as 0).
  if (tid < nb) {
#pragma unroll
    for (int c = 0; c < NBW; ++c) LU[tid][c] = w[0][c];
  }
  __syncthreads();
  if (tid < nb) {
    const int c = tid;
    cplx<T> z[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      cplx<T> v = mk((T)(i == c ? 1 : 0), (T)0);
#pragma unroll
      for (int j = 0; j < i; ++j) cfms(v, LU[i][j], z[j]);
      z[i] = i < nb ? v : czero<T>();
    }
#pragma unroll
    for (int i = NBW - 1; i >= 0; --i) {
      if (i < nb) {
        cplx<T> v = z[i];
#pragma unroll
        for (int j = i + 1; j < NBW; ++j) cfms(v, LU[i][j], z[j]);
        z[i] = v * cinv(LU[i][i]);
      }
    }
#pragma unroll
    for (int i = 0; i < NBW; ++i)
      if (i < nb) jb.G[i + (long)c * nb] = z[i];
  }
}

// Tall panels (more rows than the register file of one workgroup holds):
// the rows stay in the panel copy W (global memory, L2-resident).  Panel row
// i belongs to thread i mod kTT for the whole panel, so a thread only reads
// rows it wrote itself; the pivot row and the row it displaces reach the
// other threads through LDS (double-buffered by step parity: two barriers
// per step).  The pivot search issues the loads of all of a thread's rows at
// once; the update then takes the rows one at a time (a whole row per load
// batch).  Same results as panel_kernel (cabs1 pivots, lowest row on ties).
constexpr int kTT = 512;
template <typename T, int NBW, int RQ>
__global__ __launch_bounds__(kTT) void panel_tall_kernel(const PanelJob<T> *__restrict__ jobs,
                                                         int *__restrict__ err_node) {
  __shared__ T sv[2][kTT / 64];
  __shared__ int si[2][kTT / 64];
  __shared__ cplx<T> prowb[2][NBW], trowb[2][NBW];
  __shared__ cplx<T> LU[NBW][NBW + 1];
  const PanelJob<T> jb = jobs[blockIdx.x];
  const int rows = jb.ne - jb.p0, nb = jb.nb, tid = threadIdx.x;
  const long ld = jb.ld;
  cplx<T> *W = jb.W;
#pragma unroll 1
  for (int q = 0; q < RQ; ++q) {
    const int i = tid + kTT * q;
    if (i >= rows) break;
    cplx<T> r[NBW];
#pragma unroll
    for (int c = 0; c < NBW; ++c)
      r[c] = c < nb ? jb.F[(jb.p0 + i) + (long)(jb.p0 + c) * ld] : czero<T>();
#pragma unroll
    for (int c = 0; c < NBW; ++c)
      if (c < nb) W[i + (long)c * rows] = r[c];
  }
  for (int t = 0; t < nb; ++t) {
    const int par = t & 1;
    cplx<T> *prow = prowb[par], *trow = trowb[par];
    T best = (T)-1;
    int bi = 0x7fffffff;
    T a[RQ];
#pragma unroll
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + kTT * q;
      a[q] = (i >= t && i < rows) ? cabs1(W[i + (long)t * rows]) : (T)-1;
    }
#pragma unroll
    for (int q = 0; q < RQ; ++q)
      if (a[q] > best) { best = a[q]; bi = tid + kTT * q; }   // rows ascend with q
    wave_argmax(best, bi);
    if ((tid & 63) == 0) { sv[par][tid / 64] = best; si[par][tid / 64] = bi; }
    lds_barrier();
    best = sv[par][0];
    bi = si[par][0];
#pragma unroll
    for (int k = 1; k < kTT / 64; ++k)
      if (sv[par][k] > best || (sv[par][k] == best && si[par][k] < bi)) {
        best = sv[par][k];
        bi = si[par][k];
      }
    const bool zero = !(best > (T)0);
    if (zero && tid == 0) atomicCAS(err_node, -1, jb.node);
    const int pv = zero ? t : bi;
    if (tid == 0) jb.piv[t] = jb.p0 + pv;
    // the owners of rows pv and t publish them
#pragma unroll 1
    for (int q = 0; q < RQ; ++q) {
      const int i = tid + kTT * q;
      if (i != pv && i != t) continue;
      cplx<T> r[NBW];
#pragma unroll
      for (int c = 0; c < NBW; ++c) r[c] = c < nb ? W[i + (long)c * rows] : czero<T>();
      if (i == pv) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) prow[c] = r[c];
      }
      if (i == t) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) trow[c] = r[c];
      }
    }
    lds_barrier();
    const cplx<T> inv = zero ? czero<T>() : cinv(prow[t]);
    // two rows per batch: both rows' loads are in flight before either is
    // updated and stored
    static_assert(RQ % 2 == 0, "rows are updated in pairs");
#pragma unroll 1
    for (int q = 0; q < RQ; q += 2) {
      const int ia = tid + kTT * q, ib = ia + kTT;
      if (ia >= rows) break;
      // row t takes the pivot row (the U row stays unscaled)
      if (ia == t || ib == t) {
        const int it = ia == t ? ia : ib;
#pragma unroll
        for (int c = 0; c < NBW; ++c)
          if (c < nb) W[it + (long)c * rows] = prow[c];
      }
      // row pv takes the displaced row t; every row below t is updated
      const bool ua = ia > t, ub = ib > t && ib < rows;
      const bool swa = ia == pv, swb = ib == pv;
      cplx<T> ra[NBW], rb[NBW];
#pragma unroll
      for (int c = 0; c < NBW; ++c) {
        ra[c] = !ua ? czero<T>()
                : swa ? trow[c]
                : (c >= t && c < nb) ? W[ia + (long)c * rows] : czero<T>();
        rb[c] = !ub ? czero<T>()
                : swb ? trow[c]
                : (c >= t && c < nb) ? W[ib + (long)c * rows] : czero<T>();
      }
      cplx<T> la = czero<T>(), lb = czero<T>();
#pragma unroll
      for (int c = 0; c < NBW; ++c)
        if (c == t) {
          la = ra[c] * inv;
          lb = rb[c] * inv;
        }
#pragma unroll
      for (int c = 0; c < NBW; ++c)
        if (c > t && c < nb) {
          cfms(ra[c], la, prow[c]);
          cfms(rb[c], lb, prow[c]);
        }
      if (ua) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) {
          if (c == t) W[ia + (long)c * rows] = la;
          else if ((c > t || swa) && c < nb) W[ia + (long)c * rows] = ra[c];
        }
      }
      if (ub) {
#pragma unroll
        for (int c = 0; c < NBW; ++c) {
          if (c == t) W[ib + (long)c * rows] = lb;
          else if ((c > t || swb) && c < nb) W[ib + (long)c * rows] = rb[c];
        }
      }
    }
  }
  // L11 U11 (rows 0 .. nb - 1, owned by threads 0 .. nb - 1) to LDS, then
  // G = (L11 U11)^-1 as in panel_reg_kernel
  if (tid < nb) {
#pragma unroll
    for (int c = 0; c < NBW; ++c) LU[tid][c] = c < nb ? W[tid + (long)c * rows] : czero<T>();
  }
  __syncthreads();
  if (tid < nb) {
    const int c = tid;
    cplx<T> z[NBW];
#pragma unroll
    for (int i = 0; i < NBW; ++i) {
      cplx<T> v = mk((T)(i == c ? 1 : 0), (T)0);
#pragma unroll
      for (int j = 0; j < i; ++j) cfms(v, LU[i][j], z[j]);
      z[i] = i < nb ? v : czero<T>();
    }
#pragma unroll
    for (int i = NBW - 1; i >= 0; --i) {
      if (i < nb) {
        cplx<T> v = z[i];
#pragma unroll
        for (int j = i + 1; j < NBW; ++j) cfms(v, LU[i][j], z[j]);
        z[i] = v * cinv(LU[i][i]);
      }
    }
#pragma unroll
    for (int i = 0; i < NBW; ++i)
      if (i < nb) jb.G[i + (long)c * nb] = z[i];
  }
}

template <typename T>
__global__ void swap_kernel(const PanelJob<T> *__restrict__ jobs) {
  const PanelJob<T> jb = jobs[blockIdx.y];
  int j = jb.p0 + blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= jb.ncols) return;
  cplx<T> *col = jb.F + (long)j * jb.ld;
  for (int t = 0; t < jb.nb; ++t) {
    int r = jb.piv[t];
    if (r != jb.p0 + t) {
      cplx<T> a = col[jb.p0 + t];
      col[jb.p0 + t] = col[r];
      col[r] = a;
    }
  }
}

template <typename T>
__global__ void gemm_a_kernel(const PanelJob<T> *__restrict__ jobs) {
  const PanelJob<T> jb = jobs[blockIdx.y];
  const int J = jb.ncols - jb.p0 - jb.nb;
  long e = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (e >= (long)J * jb.nb) return;
  int t = (int)(e % jb.nb), c = (int)(e / jb.nb);
  const cplx<T> *col = jb.F + (long)(jb.p0 + jb.nb + c) * jb.ld + jb.p0;
  cplx<T> acc = czero<T>();
  for (int u = 0; u < jb.nb; ++u) cfma(acc, jb.G[t + (long)u * jb.nb], col[u]);
  jb.Y[t + (long)c * jb.nb] = acc;
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));
typedef double doublex4_t __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<float> {
  using V = floatx4_t;
  static constexpr int KB = 32;   // panel width
  __device__ static V fma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // output row of register r in lane group g (lanes 16 g .. 16 g + 15)
  __device__ static int drow(int g, int r) { return 4 * g + r; }
};
template <> struct MfmaAcc<double> {
  using V = doublex4_t;
  static constexpr int KB = 16;
  __device__ static V fma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int g, int r) { return g + 4 * r; }
};

// Trailing update on the matrix cores (16x16x4 MFMA in the factor's real
// precision).  The tile is computed transposed, D = C^T = Y^T A^T, on the
// real and imaginary parts (Re D = Yr^T Ar^T - Yi^T Ai^T, Im D = Yi^T Ar^T +
// Yr^T Ai^T), so each output register of a lane group holds 16 consecutive
// rows of one column of F and the read-modify-write is coalesced.  Four waves
// cover the 64 x 64 tile as 2 x 2 blocks of 32 x 32; each wave keeps 2 x 2
// blocks of 16 x 16 for both parts.
template <typename T>
__global__ __launch_bounds__(256) void gemm_b_mfma_kernel(const PanelJob<T> *__restrict__ jobs) {
  using M = MfmaAcc<T>;
  constexpr int KB = M::KB;
  __shared__ cplx<T> As[kTile][KB + 1];
  __shared__ cplx<T> Ys[KB][kTile];
  const PanelJob<T> jb = jobs[blockIdx.z];
  const int J = jb.ncols - jb.p0 - jb.nb;
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  if (i0 >= jb.m || j0 >= J) return;
  const int nb = jb.nb, tid = threadIdx.x;
  const long ld = jb.ld;
  // panel columns beyond nb are zero so that the K loop runs in steps of 4.
  // All global loads are issued before the LDS writes: the loads go through
  // generic pointers that may alias LDS, so interleaving them with the
  // writes would wait out each load before the next.
  constexpr int kPE = kTile * KB / 256;
  cplx<T> ra[kPE], ry[kPE];
#pragma unroll
  for (int u = 0; u < kPE; ++u) {
    const int e = tid + 256 * u;
    const int r = e % kTile, t = e / kTile, i = i0 + r;
    ra[u] = (i < jb.m && t < nb) ? jb.F[i + (long)(jb.p0 + t) * ld] : czero<T>();
    const int ty = e % KB, c = e / KB;
    ry[u] = ((j0 + c) < J && ty < nb) ? jb.Y[ty + (long)(j0 + c) * nb] : czero<T>();
  }
#pragma unroll
  for (int u = 0; u < kPE; ++u) {
    const int e = tid + 256 * u;
    As[e % kTile][e / kTile] = ra[u];
    Ys[e % KB][e / KB] = ry[u];
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int wr = 32 * (w & 1), wc = 32 * (w >> 1);
  const int q = lane & 15, kq = lane >> 4;
  typename M::V dr[2][2], di[2][2];
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      dr[bc][bi] = typename M::V{0, 0, 0, 0};
      di[bc][bi] = typename M::V{0, 0, 0, 0};
    }
  const int nbr = (nb + 3) & ~3;
  for (int t0 = 0; t0 < nbr; t0 += 4) {
    const int t = t0 + kq;
    cplx<T> y[2], a[2];
#pragma unroll
    for (int bc = 0; bc < 2; ++bc) y[bc] = Ys[t][wc + 16 * bc + q];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) a[bi] = As[wr + 16 * bi + q][t];
#pragma unroll
    for (int bc = 0; bc < 2; ++bc)
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        dr[bc][bi] = M::fma(y[bc].re, a[bi].re, dr[bc][bi]);
        dr[bc][bi] = M::fma(-y[bc].im, a[bi].im, dr[bc][bi]);
        di[bc][bi] = M::fma(y[bc].im, a[bi].re, di[bc][bi]);
        di[bc][bi] = M::fma(y[bc].re, a[bi].im, di[bc][bi]);
      }
  }
  // lane (q, kq), register r: C row i0 + wr + 16 bi + q, column
  // j0 + wc + 16 bc + drow(kq, r) (the output row of D).  The tile of C is
  // read completely before the first store (see the staging above).
  cplx<T> cv[2][4][2];
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = j0 + wc + 16 * bc + M::drow(kq, r);
      const cplx<T> *col = jb.F + (long)(jb.p0 + nb + c) * ld;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int i = i0 + wr + 16 * bi + q;
        const bool upd = c < J && i < jb.m && !(i >= jb.p0 && i < jb.p0 + nb);
        cv[bc][r][bi] = upd ? col[i] : czero<T>();
      }
    }
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int cl = wc + 16 * bc + M::drow(kq, r), c = j0 + cl;
      if (c >= J) continue;
      cplx<T> *col = jb.F + (long)(jb.p0 + nb + c) * ld;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int i = i0 + wr + 16 * bi + q;
        if (i >= jb.m) continue;
        if (i >= jb.p0 && i < jb.p0 + nb) col[i] = Ys[i - jb.p0][cl];
        else col[i] = cv[bc][r][bi] - mk(dr[bc][bi][r], di[bc][bi][r]);
      }
    }
}

// C -= A B on the matrix cores, one 64 x 64 tile of C per workgroup, K in
// chunks of the panel width staged through LDS; the tile is computed
// transposed (D = C^T = B^T A^T) as in the trailing update.
template <typename T>
__global__ __launch_bounds__(256) void gemm_sub_mfma_kernel(const GemmJob<T> *__restrict__ jobs) {
  using M = MfmaAcc<T>;
  constexpr int KB = M::KB;
  __shared__ cplx<T> As[kTile][KB + 1];
  __shared__ cplx<T> Bs[KB][kTile];
  const GemmJob<T> jb = jobs[blockIdx.z];
  const int i0 = blockIdx.x * kTile, j0 = blockIdx.y * kTile;
  if (i0 >= jb.M || j0 >= jb.N) return;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int wr = 32 * (w & 1), wc = 32 * (w >> 1);
  const int q = lane & 15, kq = lane >> 4;
  typename M::V dr[2][2], di[2][2];
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) {
      dr[bc][bi] = typename M::V{0, 0, 0, 0};
      di[bc][bi] = typename M::V{0, 0, 0, 0};
    }
  constexpr int kPE = kTile * KB / 256;
  for (int k0 = 0; k0 < jb.K; k0 += KB) {
    // all global loads of the chunk before its LDS writes (generic pointers
    // may alias LDS: interleaved, each load would be waited out)
    cplx<T> ra[kPE], rb[kPE];
#pragma unroll
    for (int u = 0; u < kPE; ++u) {
      const int e = tid + 256 * u;
      const int r = e % kTile, t = e / kTile, i = i0 + r, k = k0 + t;
      ra[u] = (i < jb.M && k < jb.K) ? jb.A[i + (long)k * jb.lda] : czero<T>();
      const int tb = e % KB, c = e / KB, kb = k0 + tb, j = j0 + c;
      rb[u] = (j < jb.N && kb < jb.K) ? jb.B[kb + (long)j * jb.ldb] : czero<T>();
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPE; ++u) {
      const int e = tid + 256 * u;
      As[e % kTile][e / kTile] = ra[u];
      Bs[e % KB][e / KB] = rb[u];
    }
    __syncthreads();
#pragma unroll
    for (int t0 = 0; t0 < KB; t0 += 4) {
      const int t = t0 + kq;
      cplx<T> y[2], a[2];
#pragma unroll
      for (int bc = 0; bc < 2; ++bc) y[bc] = Bs[t][wc + 16 * bc + q];
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) a[bi] = As[wr + 16 * bi + q][t];
#pragma unroll
      for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) {
          dr[bc][bi] = M::fma(y[bc].re, a[bi].re, dr[bc][bi]);
          dr[bc][bi] = M::fma(-y[bc].im, a[bi].im, dr[bc][bi]);
          di[bc][bi] = M::fma(y[bc].im, a[bi].re, di[bc][bi]);
          di[bc][bi] = M::fma(y[bc].re, a[bi].im, di[bc][bi]);
        }
    }
  }
  // the tile of C is read completely before the first store
  cplx<T> cv[2][4][2];
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = j0 + wc + 16 * bc + M::drow(kq, r);
      const cplx<T> *col = jb.C + (long)c * jb.ldc;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int i = i0 + wr + 16 * bi + q;
        cv[bc][r][bi] = (c < jb.N && i < jb.M) ? col[i] : czero<T>();
      }
    }
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int c = j0 + wc + 16 * bc + M::drow(kq, r);
      if (c >= jb.N) continue;
      cplx<T> *col = jb.C + (long)c * jb.ldc;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
        const int i = i0 + wr + 16 * bi + q;
        if (i < jb.M) col[i] = cv[bc][r][bi] - mk(dr[bc][bi][r], di[bc][bi][r]);
      }
    }
}

template <typename T>
__global__ void axpby_kernel(const AxpbyJob<T> *__restrict__ jobs) {
  const AxpbyJob<T> jb = jobs[blockIdx.z];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int j = blockIdx.y;
  if (i >= jb.m || j >= jb.n) return;
  cplx<T> v = jb.dst[i + (long)j * jb.ld_dst];
  if (jb.s1) v = v + jb.a * jb.s1[i + (long)j * jb.ld1];
  if (jb.s2) v = v + jb.b * jb.s2[i + (long)j * jb.ld2];
  jb.dst[i + (long)j * jb.ld_dst] = v;
}

}  // namespace

template <typename T, typename Tc>
void launch_front_assemble(int count, const int *nodes, const FrontDesc *desc,
                           const int *src_gid, const int *src_code,
                           const int *rowptr, const int *col, const c128 *val,
                           const cplx<Tc> *cpool, cplx<T> *opool, hipStream_t st, int max_f) {
  if (count <= 0) return;
  long per = (long)kThreads * 16;
  int ny = ceil_div((long)max_f * (2L * max_f), per);
  hipLaunchKernelGGL((front_assemble_kernel<T, Tc>), dim3(count, ny), dim3(kThreads), 0, st,
                     nodes, desc, src_gid, src_code, rowptr, col, val, cpool, opool);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_eliminate(int count, const ElimJob<T> *jobs, int *err_node, hipStream_t st,
                      size_t lds_bytes, int *queue) {
  if (count <= 0) return;
  if (lds_bytes > 0) {
    HSSX_CHECK(queue != nullptr, HSSX_EINVAL, "LDS elimination needs a work-queue counter");
    if (lds_bytes > 65536)
      HSSX_HIP(hipFuncSetAttribute(reinterpret_cast<const void *>(&eliminate_lds_kernel<T>),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes));
    // as many workgroups as are resident at once: LDS (160 KiB per CU) and
    // 8 workgroups of 256 threads per CU, 256 CUs
    int dev = 0, cus = 256;
    HSSX_HIP(hipGetDevice(&dev));
    HSSX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int per_cu = std::max(1, std::min(8, (int)((160 * 1024) / (lds_bytes + 64))));
    const int grid = std::max(1, std::min(count, cus * per_cu));
    hipLaunchKernelGGL(eliminate_lds_kernel<T>, dim3(grid), dim3(kThreads), lds_bytes, st, jobs,
                       count, queue, err_node);
  }
  else
    hipLaunchKernelGGL(eliminate_kernel<T>, dim3(count), dim3(kThreads), 0, st, jobs, err_node);
  HSSX_HIP(hipGetLastError());
}


template <typename T>
int eliminate_reg_max_cols(int max_m) {
  constexpr bool kF32 = sizeof(T) == sizeof(float);
  if (max_m <= 64) return kF32 ? 320 : 192;
  if (max_m <= 128) return kF32 ? 320 : 128;
  return 0;
}

template <typename T>
bool launch_eliminate_reg(int count, const ElimJob<T> *jobs, int *err_node, hipStream_t st,
                          int max_m, int max_nc, int *queue) {
  if (count <= 0) return true;
  constexpr bool kF32 = sizeof(T) == sizeof(float);
  // max_nc: largest working width ncols - m
  if (max_m > 128 || max_nc > eliminate_reg_max_cols<T>(max_m) || !queue) return false;
  int dev = 0, cus = 256;
  HSSX_HIP(hipGetDevice(&dev));
  HSSX_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
#define HSSX_GJR(NT, RG, R, C)                                                                  \
  hipLaunchKernelGGL((eliminate_reg_kernel<T, NT, RG, R, C>),                                   \
                     dim3(std::max(1, std::min(count, cus * (NT == 256 ? 4 : 2)))), dim3(NT), 0, \
                     st, jobs, count, queue, err_node)
  if (max_m <= 64) {
    const int cpt = max_nc <= 64 ? 4 : max_nc <= 128 ? 8 : max_nc <= 192 ? 12 : 20;
    if (max_m <= 16) {
      if (cpt == 4) HSSX_GJR(256, 16, 1, 4);
      else if (cpt == 8) HSSX_GJR(256, 16, 1, 8);
      else if (cpt == 12) HSSX_GJR(256, 16, 1, 12);
      else if constexpr (kF32) HSSX_GJR(256, 16, 1, 20);
    } else {
      if (cpt == 4) HSSX_GJR(256, 16, 4, 4);
      else if (cpt == 8) HSSX_GJR(256, 16, 4, 8);
      else if (cpt == 12) HSSX_GJR(256, 16, 4, 12);
      else if constexpr (kF32) HSSX_GJR(256, 16, 4, 20);
    }
  } else {
    // 512 threads: 32 row groups of 4 rows, 16 column groups
    const int cpt = max_nc <= 128 ? 8 : max_nc <= 192 ? 12 : 20;
    if (cpt == 8) HSSX_GJR(512, 32, 4, 8);
    else if constexpr (kF32) {
      if (cpt == 12) HSSX_GJR(512, 32, 4, 12);
      else HSSX_GJR(512, 32, 4, 20);
    }
  }
#undef HSSX_GJR
  HSSX_HIP(hipGetLastError());
  return true;
}

template <typename T>
void launch_panel_step(int count, const PanelJob<T> *jobs, int max_m, int max_cols,
                       int max_prows, int max_nb, int *err_node, hipStream_t st) {
  if (count <= 0) return;
  constexpr int NBW = sizeof(T) == sizeof(float) ? 32 : 16;
  if (max_nb <= NBW && max_prows <= kPT / 4)
    hipLaunchKernelGGL((panel_reg_kernel<T, NBW, 1, kPT / 4>), dim3(count), dim3(kPT / 4), 0, st,
                       jobs, err_node);
  else if (max_nb <= NBW && max_prows <= kPT / 2)
    hipLaunchKernelGGL((panel_reg_kernel<T, NBW, 1, kPT / 2>), dim3(count), dim3(kPT / 2), 0, st,
                       jobs, err_node);
  else if (max_nb <= NBW && max_prows <= kPT)
    hipLaunchKernelGGL((panel_reg_kernel<T, NBW, 1>), dim3(count), dim3(kPT), 0, st, jobs, err_node);
  else if (max_nb <= NBW && max_prows <= 2 * kPT)
    hipLaunchKernelGGL((panel_reg_kernel<T, NBW, 2>), dim3(count), dim3(kPT), 0, st, jobs, err_node);
  else if (max_nb <= NBW && max_prows <= 3 * kPT)
    hipLaunchKernelGGL((panel_reg_kernel<T, NBW, 3>), dim3(count), dim3(kPT), 0, st, jobs, err_node);
  else if (max_nb <= NBW && max_prows <= 4 * kTT)
    hipLaunchKernelGGL((panel_tall_kernel<T, NBW, 4>), dim3(count), dim3(kTT), 0, st, jobs, err_node);
  else if (max_nb <= NBW && max_prows <= 8 * kTT)
    hipLaunchKernelGGL((panel_tall_kernel<T, NBW, 8>), dim3(count), dim3(kTT), 0, st, jobs, err_node);
  else if (max_nb <= NBW && max_prows <= 12 * kTT)
    hipLaunchKernelGGL((panel_tall_kernel<T, NBW, 12>), dim3(count), dim3(kTT), 0, st, jobs, err_node);
  else
    hipLaunchKernelGGL(panel_kernel<T>, dim3(count), dim3(kThreads), 0, st, jobs, err_node);
  hipLaunchKernelGGL(swap_kernel<T>, dim3(ceil_div(max_cols, 256), count), dim3(256), 0, st, jobs);
  hipLaunchKernelGGL(gemm_a_kernel<T>, dim3(ceil_div((long)max_cols * kNB, 256), count), dim3(256),
                     0, st, jobs);
  hipLaunchKernelGGL(gemm_b_mfma_kernel<T>, dim3(ceil_div(max_m, kTile), ceil_div(max_cols, kTile), count),
                     dim3(256), 0, st, jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_gemm_sub(int count, const GemmJob<T> *jobs, int max_m, int max_n, hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return;
  hipLaunchKernelGGL(gemm_sub_mfma_kernel<T>, dim3(ceil_div(max_m, kTile), ceil_div(max_n, kTile), count),
                     dim3(256), 0, st, jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_axpby(int count, const AxpbyJob<T> *jobs, int max_m, int max_n, hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return;
  hipLaunchKernelGGL(axpby_kernel<T>, dim3(ceil_div(max_m, 256), max_n, count), dim3(256), 0,
                     st, jobs);
  HSSX_HIP(hipGetLastError());
}

#define HSSX_ASM(T, Tc)                                                                      \
  template void launch_front_assemble<T, Tc>(int, const int *, const FrontDesc *, const int *, \
                                             const int *, const int *, const int *,           \
                                             const c128 *, const cplx<Tc> *, cplx<T> *,       \
                                             hipStream_t, int);
HSSX_ASM(double, double)
HSSX_ASM(float, float)
HSSX_ASM(double, float)
#undef HSSX_ASM

#define HSSX_INST(T)                                                                        \
  template void launch_eliminate<T>(int, const ElimJob<T> *, int *, hipStream_t, size_t,    \
                                    int *);                                                 \
  template bool launch_eliminate_reg<T>(int, const ElimJob<T> *, int *, hipStream_t, int, int, \
                                        int *);                                             \
  template int eliminate_reg_max_cols<T>(int);                                              \
  template void launch_panel_step<T>(int, const PanelJob<T> *, int, int, int, int, int *,      \
                                     hipStream_t);                                          \
  template void launch_axpby<T>(int, const AxpbyJob<T> *, int, int, hipStream_t);           \
  template void launch_gemm_sub<T>(int, const GemmJob<T> *, int, int, hipStream_t);
HSSX_INST(double)
HSSX_INST(float)
#undef HSSX_INST

}  // namespace hssx
