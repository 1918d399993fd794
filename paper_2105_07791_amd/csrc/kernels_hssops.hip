// Batched building blocks of the HSS arithmetic: small complex products,
// block copies, row gathers, sparse coupling products, entry extraction.
#include "hssops.h"

namespace hssx {

namespace {

constexpr int kBT = 256;   // threads per workgroup

// 32 x 32 output tile per workgroup, K in steps of 16 staged in LDS; thread
// (tx, ty) = (tid % 16, tid / 16) owns rows tx, tx + 16 and columns ty, ty + 16.
// The next step's global loads are issued before the current step's
// products (two LDS buffers, one barrier per step), so their latency
// overlaps the arithmetic.
template <typename T>
__global__ __launch_bounds__(kBT) void bgemm_kernel(const BgTask<T> *__restrict__ tasks) {
  __shared__ cplx<T> As[2][16][33], Bs[2][16][33];
  const BgTask<T> tl = tasks[blockIdx.x];
  const BgJob<T> &jb = tl.jb;
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = tl.tm * 32, j0 = tl.tn * 32;
  // per-thread staging coordinates (k index within the step, row / column)
  int ak[2], ai[2], bk[2], bj[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + kBT * u;
    if (jb.ta) { ak[u] = e & 15; ai[u] = e >> 4; } else { ai[u] = e & 31; ak[u] = e >> 5; }
    if (jb.tb) { bj[u] = e & 31; bk[u] = e >> 5; } else { bk[u] = e & 15; bj[u] = e >> 4; }
  }
  cplx<T> ra[2], rb[2];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int gi = i0 + ai[u], gk = k0 + ak[u];
      ra[u] = czero<T>();
      if (gi < jb.M && gk < jb.K)
        ra[u] = jb.ta ? jb.A[gk + (long)gi * jb.lda] : jb.A[gi + (long)gk * jb.lda];
      const int gj = j0 + bj[u], gk2 = k0 + bk[u];
      rb[u] = czero<T>();
      if (gj < jb.N && gk2 < jb.K)
        rb[u] = jb.tb ? jb.B[gj + (long)gk2 * jb.ldb] : jb.B[gk2 + (long)gj * jb.ldb];
    }
  };
  cplx<T> acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = czero<T>();
  // the accumulated-into block is read up front, its latency hidden too
  cplx<T> c0[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gi = i0 + tx + 16 * a, gj = j0 + ty + 16 * b;
      c0[a][b] = (jb.beta && gi < jb.M && gj < jb.N) ? jb.C[gi + (long)gj * jb.ldc] : czero<T>();
    }
  fetch(0);
  int buf = 0;
  for (int k0 = 0; k0 < jb.K; k0 += 16) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      As[buf][ak[u]][ai[u]] = ra[u];
      Bs[buf][bk[u]][bj[u]] = rb[u];
    }
    // after this barrier every thread is done with the other buffer's
    // products of the previous step, so the next step may overwrite it
    __syncthreads();
    if (k0 + 16 < jb.K) fetch(k0 + 16);
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const cplx<T> a0 = As[buf][kk][tx], a1 = As[buf][kk][tx + 16];
      const cplx<T> b0 = Bs[buf][kk][ty], b1 = Bs[buf][kk][ty + 16];
      cfma(acc[0][0], a0, b0);
      cfma(acc[0][1], a0, b1);
      cfma(acc[1][0], a1, b0);
      cfma(acc[1][1], a1, b1);
    }
    buf ^= 1;
  }
  const cplx<T> al = mk(jb.ar, jb.ai);
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const int gi = i0 + tx + 16 * a, gj = j0 + ty + 16 * b;
      if (gi < jb.M && gj < jb.N) {
        jb.C[gi + (long)gj * jb.ldc] = c0[a][b] + al * acc[a][b];
      }
    }
}

template <typename T>
__global__ __launch_bounds__(kBT) void copy_kernel(const CopyJob<T> *__restrict__ jobs) {
  const CopyJob<T> jb = jobs[blockIdx.y];
  const long tot = (long)jb.m * jb.n;
  for (long e = blockIdx.x * (long)kBT + threadIdx.x; e < tot; e += (long)gridDim.x * kBT) {
    const int i = (int)(e % jb.m), j = (int)(e / jb.m);
    cplx<T> *d = jb.dst + i + (long)j * jb.ldd;
    switch (jb.mode) {
      case 0: *d = jb.s * jb.src[i + (long)j * jb.lds]; break;
      case 1: *d = jb.s * jb.src[j + (long)i * jb.lds]; break;
      case 2: *d = mk((T)(i == j ? 1 : 0), (T)0); break;
      case 3: *d = czero<T>(); break;
      default: *d = *d + jb.s * jb.src[i + (long)j * jb.lds]; break;
    }
  }
}

template <typename Ts> __device__ __forceinline__ c128 load_any(const Ts *p);
template <> __device__ __forceinline__ c128 load_any<double>(const double *p) {
  return mk(*p, 0.0);
}
template <> __device__ __forceinline__ c128 load_any<c64>(const c64 *p) {
  return ccast<double>(*p);
}
template <> __device__ __forceinline__ c128 load_any<c128>(const c128 *p) { return *p; }

template <typename Ts, typename Td>
__global__ __launch_bounds__(kBT) void gather_kernel(const GatherJob<Ts, Td> *__restrict__ jobs) {
  using TD = decltype(Td::re);
  const GatherJob<Ts, Td> jb = jobs[blockIdx.y];
  const long tot = (long)jb.nrows * jb.nc;
  for (long e = blockIdx.x * (long)kBT + threadIdx.x; e < tot; e += (long)gridDim.x * kBT) {
    const int r = (int)(e % jb.nrows), j = (int)(e / jb.nrows);
    const int dr = jb.dmap ? jb.dmap[r] : r;
    if (dr < 0) continue;
    const int sr = jb.smap ? jb.smap[r] : r;
    c128 v = sr < 0 ? czero<double>() : load_any<Ts>(jb.src + sr + (long)j * jb.lds);
    v = jb.s * v;
    Td *d = jb.dst + dr + (long)j * jb.ldd;
    const Td w = mk((TD)v.re, (TD)v.im);
    *d = jb.mode ? *d + w : w;
  }
}

template <typename T>
__global__ __launch_bounds__(kBT) void spmm_kernel(const SpJob<T> *__restrict__ jobs,
                                                   const c128 *__restrict__ val) {
  const SpJob<T> jb = jobs[blockIdx.y];
  const long tot = (long)jb.nrows * jb.nc;
  for (long e = blockIdx.x * (long)kBT + threadIdx.x; e < tot; e += (long)gridDim.x * kBT) {
    const int r = (int)(e % jb.nrows), j = (int)(e / jb.nrows);
    cplx<T> t = czero<T>();
    for (int q = jb.rp[r]; q < jb.rp[r + 1]; ++q)
      cfma(t, ccast<T>(val[jb.vi[q]]), jb.X[jb.cp[q] + (long)j * jb.ldx]);
    cplx<T> *y = jb.Y + r + (long)j * jb.ldy;
    t = jb.s * t;
    *y = jb.acc ? *y + t : t;
  }
}

template <typename T>
__global__ __launch_bounds__(kBT) void fill_coo_kernel(const FillJob<T> *__restrict__ jobs,
                                                       const c128 *__restrict__ val) {
  const FillJob<T> jb = jobs[blockIdx.y];
  for (int e = blockIdx.x * kBT + threadIdx.x; e < jb.cnt; e += gridDim.x * kBT) {
    const int v = jb.vi[e];
    jb.dst[jb.ri[e] + (long)(jb.coff + jb.ci[e]) * jb.ld] = v < 0 ? mk((T)1, (T)0) : ccast<T>(val[v]);
  }
}

template <typename T>
__global__ __launch_bounds__(kBT) void symmetrize_kernel(const SymJob<T> *__restrict__ jobs) {
  const SymJob<T> jb = jobs[blockIdx.y];
  const long tot = (long)jb.m * jb.n;
  const bool same = jb.P == jb.Q;
  for (long e = blockIdx.x * (long)kBT + threadIdx.x; e < tot; e += (long)gridDim.x * kBT) {
    const int i = (int)(e % jb.m), j = (int)(e / jb.m);
    if (same && i > j) continue;
    cplx<T> *p = jb.P + i + (long)j * jb.ldp, *q = jb.Q + j + (long)i * jb.ldq;
    const cplx<T> v = (T)0.5 * (*p + *q);
    *p = v;
    *q = v;
  }
}

// Entry of the operator of a compression that is not formed densely.
template <typename T>
__device__ cplx<T> op_entry(const EntryOp<T> &op, int i, int j, const int *__restrict__ rowptr,
                            const int *__restrict__ col, const c128 *__restrict__ val) {
  cplx<T> v;
  if (op.kind == 0) {
    const int ci = op.bchild[i], cj = op.bchild[j];
    if (ci == cj) {
      v = hss_entry(ci ? op.H1 : op.H0, op.bcpos[i], op.bcpos[j]);
    } else {
      // coupling of the two children through A (sorted CSR columns)
      const int gi = op.gid[i], gj = op.gid[j];
      int lo = rowptr[gi], hi = rowptr[gi + 1] - 1;
      v = czero<T>();
      if (lo <= hi && gj >= col[lo] && gj <= col[hi]) {
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (col[mid] < gj) lo = mid + 1;
          else hi = mid;
        }
        if (col[lo] == gj) v = ccast<T>(val[lo]);
      }
    }
    const cplx<T> *yc = op.YC + (long)i * op.r, *yb = op.YB + (long)j * op.r;
    for (int t = 0; t < op.r; ++t) cfms(v, yc[t], yb[t]);
  } else {
    v = hss_entry(op.H1, i, j);
    for (int e = op.rp[i]; e < op.rp[i + 1]; ++e) {
      const cplx<T> a = ccast<T>(val[op.vi[e]]);
      for (int f = op.rp[j]; f < op.rp[j + 1]; ++f) {
        const cplx<T> b = ccast<T>(val[op.vi[f]]);
        cfms(v, a * hss_entry(op.H0, op.cp[e], op.cp[f]), b);
      }
    }
  }
  return v;
}

// kEntSplit workgroups per (instance, cluster): a leaf's diagonal block
// D = S(I, I), or an internal cluster's B12 = S(sk_l, sk_r) with
// B21 = B12^T (the operators are symmetric), written where the compression
// kernel reads them.
constexpr int kEntSplit = 8;
template <typename T>
__global__ __launch_bounds__(kBT) void entries_kernel(
    const HssItem *__restrict__ items, const HssInstance *__restrict__ insts,
    const HssCluster *__restrict__ cls, cplx<T> *__restrict__ pool, const int *__restrict__ ipool,
    const int *__restrict__ rank, const EntryOp<T> *__restrict__ ops,
    const int *__restrict__ rowptr, const int *__restrict__ col, const c128 *__restrict__ val) {
  const HssItem it = items[blockIdx.x];
  const HssInstance &I = insts[it.inst];
  const EntryOp<T> &op = ops[I.eop];
  const HssCluster C = cls[I.cl_off + it.cl];
  cplx<T> *P = pool + I.pool;
  const int t0 = blockIdx.y * kBT + threadIdx.x, stride = kEntSplit * kBT;
  if (C.left < 0) {
    const int rows = C.size;
    cplx<T> *D = P + C.D;
    for (int e = t0; e < rows * rows; e += stride)
      D[e] = op_entry(op, C.start + e % rows, C.start + e / rows, rowptr, col, val);
    return;
  }
  const HssCluster L = cls[I.cl_off + C.left], R = cls[I.cl_off + C.right];
  const int kl = rank[I.cl_off + C.left], kr = rank[I.cl_off + C.right];
  const int *skl = ipool + I.ipool + L.sk, *skr = ipool + I.ipool + R.sk;
  cplx<T> *B12 = P + C.B12, *B21 = P + C.B21;
  for (int e = t0; e < kl * kr; e += stride) {
    const int a = e % kl, b = e / kl;
    const cplx<T> v = op_entry(op, skl[a], skr[b], rowptr, col, val);
    B12[e] = v;
    B21[b + (long)a * kr] = v;
  }
}

template <typename T>
__global__ __launch_bounds__(kBT) void entries_list_kernel(EntView<T> V, const int *__restrict__ ij,
                                                           int n, cplx<T> *__restrict__ out) {
  const int e = blockIdx.x * kBT + threadIdx.x;
  if (e < n) out[e] = hss_entry(V, ij[2 * e], ij[2 * e + 1]);
}

inline int grid_for(long elems) {
  return (int)std::max(1L, std::min(1024L, (elems + kBT - 1) / kBT));
}

}  // namespace

template <typename T>
void launch_bgemm(int ntiles, const BgTask<T> *tasks, hipStream_t st) {
  if (ntiles <= 0) return;
  hipLaunchKernelGGL(bgemm_kernel<T>, dim3(ntiles), dim3(kBT), 0, st, tasks);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_copy(int count, const CopyJob<T> *jobs, long max_elems, hipStream_t st) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(copy_kernel<T>, dim3(grid_for(max_elems), count), dim3(kBT), 0, st, jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename Ts, typename Td>
void launch_gather(int count, const GatherJob<Ts, Td> *jobs, long max_elems, hipStream_t st) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL((gather_kernel<Ts, Td>), dim3(grid_for(max_elems), count), dim3(kBT), 0, st,
                     jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_spmm(int count, const SpJob<T> *jobs, const c128 *val, long max_elems,
                 hipStream_t st) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(spmm_kernel<T>, dim3(grid_for(max_elems), count), dim3(kBT), 0, st, jobs,
                     val);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_fill_coo(int count, const FillJob<T> *jobs, const c128 *val, int max_cnt,
                     hipStream_t st) {
  if (count <= 0 || max_cnt <= 0) return;
  hipLaunchKernelGGL(fill_coo_kernel<T>, dim3(grid_for(max_cnt), count), dim3(kBT), 0, st, jobs,
                     val);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_symmetrize(int count, const SymJob<T> *jobs, long max_elems, hipStream_t st) {
  if (count <= 0 || max_elems <= 0) return;
  hipLaunchKernelGGL(symmetrize_kernel<T>, dim3(grid_for(max_elems), count), dim3(kBT), 0, st,
                     jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_entries(int count, const HssItem *items, const HssInstance *inst,
                    const HssCluster *cl, cplx<T> *pool, const int *ipool, const int *rank,
                    const EntryOp<T> *ops, const int *rowptr, const int *col, const c128 *val,
                    hipStream_t st) {
  if (count <= 0) return;
  hipLaunchKernelGGL(entries_kernel<T>, dim3(count, kEntSplit), dim3(kBT), 0, st, items, inst, cl,
                     pool, ipool, rank, ops, rowptr, col, val);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_entries_list(EntView<T> view, const int *ij, int n, cplx<T> *out, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(entries_list_kernel<T>, dim3((n + kBT - 1) / kBT), dim3(kBT), 0, st, view,
                     ij, n, out);
  HSSX_HIP(hipGetLastError());
}

#define HSSX_OPS_INST(T)                                                                       \
  template void launch_entries_list<T>(EntView<T>, const int *, int, cplx<T> *, hipStream_t);  \
  template void launch_bgemm<T>(int, const BgTask<T> *, hipStream_t);                          \
  template void launch_copy<T>(int, const CopyJob<T> *, long, hipStream_t);                    \
  template void launch_spmm<T>(int, const SpJob<T> *, const c128 *, long, hipStream_t);        \
  template void launch_fill_coo<T>(int, const FillJob<T> *, const c128 *, int, hipStream_t);   \
  template void launch_symmetrize<T>(int, const SymJob<T> *, long, hipStream_t);               \
  template void launch_entries<T>(int, const HssItem *, const HssInstance *,                  \
                                  const HssCluster *, cplx<T> *, const int *, const int *,     \
                                  const EntryOp<T> *, const int *, const int *, const c128 *,  \
                                  hipStream_t);
HSSX_OPS_INST(double)
HSSX_OPS_INST(float)
#undef HSSX_OPS_INST

#define HSSX_GATHER_INST(Ts, Td) \
  template void launch_gather<Ts, Td>(int, const GatherJob<Ts, Td> *, long, hipStream_t);
HSSX_GATHER_INST(double, c64)
HSSX_GATHER_INST(double, c128)
HSSX_GATHER_INST(c64, c64)
HSSX_GATHER_INST(c64, c128)
HSSX_GATHER_INST(c128, c64)
HSSX_GATHER_INST(c128, c128)
#undef HSSX_GATHER_INST

}  // namespace hssx
