// Application of P^-1 = R^-1 D^-1 L^-1 (Algorithm 3.1) on vectors held in
// elimination order.
//
// The bottom-up sweep b(B) += L b(I) and the block-diagonal solve
// b(I) <- A_ii^-1 b(I) are fused per node: once a node's L-step has run no
// later L-step reads or writes its I block, so the solve can follow
// immediately.  With the Gauss-Jordan front, rows [0, f) of the appended
// column block F(:, f:f+ni) are exactly [A_ii^-1 ; L], so the fused up-step
// is one small product with t = b(I) staged in LDS.  Nodes of one tree depth
// have disjoint I and B sets (boxes of one depth are disjoint and
// B(sigma) lies inside sigma's box), so a depth is one launch.  The top-down
// sweep b(I) += R b(B) reads ancestors' blocks only.
//
// The transposed apply (P^-T) uses R^T in the up-sweep, A_ii^-T for the
// solve and L^T in the down-sweep.  The plain apply runs tiled products whose
// tile shape (one of kApplyCfgs) is chosen per tree depth by the caller.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr int kT = 256;

__global__ void permute_kernel(int n, int nrhs, const int *__restrict__ perm,
                               const c128 *__restrict__ x, long ldx, c128 *__restrict__ y,
                               long ldy, int inverse) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  if (inverse) y[perm[k] + r * ldy] = x[k + r * ldx];
  else y[k + r * ldy] = x[perm[k] + r * ldx];
}

constexpr int kRows = 64;   // output rows per workgroup

// copy the I blocks of one depth's nodes into the staging buffer (same
// positions), so that the up-sweep can overwrite x(I) while other
// workgroups of the same node still read t
__global__ void stage_kernel(const int *__restrict__ nodes, const FrontDesc *__restrict__ desc,
                             const c128 *__restrict__ x, c128 *__restrict__ tb, int n, int nrhs) {
  const FrontDesc d = desc[nodes[blockIdx.x]];
  long e = blockIdx.y * (long)blockDim.x + threadIdx.x;
  if (e >= (long)d.ni * nrhs) return;
  int i = (int)(e % d.ni), r = (int)(e / d.ni);
  long pos = d.ioff + i + (long)r * n;
  tb[pos] = x[pos];
}

// grid: (node, row tile of [0, f), rhs chunk); LDS holds t = x(I) (ni x rc)
template <typename T>
__global__ __launch_bounds__(kT) void apply_up_kernel(const int *__restrict__ nodes,
                                                      const FrontDesc *__restrict__ desc,
                                                      const cplx<T> *__restrict__ pool,
                                                      const int *__restrict__ bpos,
                                                      const c128 *__restrict__ tb,
                                                      c128 *__restrict__ x, int n, int nrhs,
                                                      int trans, int rc) {
  extern __shared__ c128 tsh[];
  const FrontDesc d = desc[nodes[blockIdx.x]];
  const int ni = d.ni, f = d.f;
  const int i0 = blockIdx.y * kRows;
  if (ni == 0 || i0 >= f) return;
  const int r0 = blockIdx.z * rc;
  const int nr = min(rc, nrhs - r0);
  if (nr <= 0) return;
  const cplx<T> *F = pool + d.foff;
  const int *bp = bpos + d.bpos_off;
  for (int e = threadIdx.x; e < ni * nr; e += kT) {
    int i = e % ni, r = e / ni;
    tsh[e] = tb[d.ioff + i + (long)(r0 + r) * n];
  }
  __syncthreads();
  const int i = i0 + threadIdx.x % kRows;
  if (i >= f) return;
  for (int r = threadIdx.x / kRows; r < nr; r += kT / kRows) {
    c128 acc = czero<double>();
    const c128 *t = tsh + (long)r * ni;
    if (!trans) {
      // [A_ii^-1 ; L](i, :) = F(i, f + l)
      for (int l = 0; l < ni; ++l) cfma(acc, ccast<double>(F[i + (long)(f + l) * f]), t[l]);
    } else if (i < ni) {
      // A_ii^-T(i, l) = F(l, f + i)
      for (int l = 0; l < ni; ++l) cfma(acc, ccast<double>(F[l + (long)(f + i) * f]), t[l]);
    } else {
      // R^T(b, l) = F(l, ni + b)
      const int b = i - ni;
      for (int l = 0; l < ni; ++l) cfma(acc, ccast<double>(F[l + (long)(ni + b) * f]), t[l]);
    }
    if (i < ni) {
      x[d.ioff + i + (long)(r0 + r) * n] = acc;
    } else {
      long pos = bp[i - ni] + (long)(r0 + r) * n;
      x[pos] = x[pos] + acc;
    }
  }
}

// grid: (node, row tile of [0, ni), rhs chunk); LDS holds x(B) (nb x rc)
template <typename T>
__global__ __launch_bounds__(kT) void apply_down_kernel(const int *__restrict__ nodes,
                                                        const FrontDesc *__restrict__ desc,
                                                        const cplx<T> *__restrict__ pool,
                                                        const int *__restrict__ bpos,
                                                        c128 *__restrict__ x, int n, int nrhs,
                                                        int trans, int rc) {
  extern __shared__ c128 tsh[];
  const FrontDesc d = desc[nodes[blockIdx.x]];
  const int ni = d.ni, nb = d.nb, f = d.f;
  const int i0 = blockIdx.y * kRows;
  if (ni == 0 || nb == 0 || i0 >= ni) return;
  const int r0 = blockIdx.z * rc;
  const int nr = min(rc, nrhs - r0);
  if (nr <= 0) return;
  const cplx<T> *F = pool + d.foff;
  const int *bp = bpos + d.bpos_off;
  for (int e = threadIdx.x; e < nb * nr; e += kT) {
    int b = e % nb, r = e / nb;
    tsh[e] = x[bp[b] + (long)(r0 + r) * n];
  }
  __syncthreads();
  const int i = i0 + threadIdx.x % kRows;
  if (i >= ni) return;
  for (int r = threadIdx.x / kRows; r < nr; r += kT / kRows) {
    c128 acc = x[d.ioff + i + (long)(r0 + r) * n];
    const c128 *t = tsh + (long)r * nb;
    if (!trans) {
      for (int b = 0; b < nb; ++b) cfma(acc, ccast<double>(F[i + (long)(ni + b) * f]), t[b]);
    } else {
      // L^T(i, b) = L(b, i) = F(ni + b, f + i)
      for (int b = 0; b < nb; ++b) cfma(acc, ccast<double>(F[ni + b + (long)(f + i) * f]), t[b]);
    }
    x[d.ioff + i + (long)(r0 + r) * n] = acc;
  }
}

// Tiled forms of the two sweeps (no transpose): out(i, r) = sum_l F(i, l)
// t(l, r) as a product over 32-entry chunks of l staged in LDS.  ROWS output
// rows per workgroup, 256 / ROWS right-hand-side groups, RB right-hand sides
// per thread held in registers, so every factor entry is read once per
// workgroup.
template <typename T, int ROWS, int RB>
__global__ __launch_bounds__(kT) void apply_up_tiled(const int *__restrict__ nodes,
                                                     const FrontDesc *__restrict__ desc,
                                                     const cplx<T> *__restrict__ pool,
                                                     const int *__restrict__ bpos,
                                                     const c128 *__restrict__ tb,
                                                     c128 *__restrict__ x, int n, int nrhs) {
  constexpr int G = kT / ROWS, RC = G * RB, KC = 32;
  __shared__ c128 ts[KC][RC];
  const FrontDesc d = desc[nodes[blockIdx.x]];
  const int ni = d.ni, f = d.f;
  const int i0 = blockIdx.y * ROWS, r0 = blockIdx.z * RC;
  if (ni == 0 || i0 >= f || r0 >= nrhs) return;
  const cplx<T> *F = pool + d.foff + (long)f * f;   // [A_ii^-1 ; L] = F(:, f:f+ni)
  const int tid = threadIdx.x, g = tid / ROWS, i = i0 + tid % ROWS;
  c128 acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = czero<double>();
  for (int l0 = 0; l0 < ni; l0 += KC) {
    __syncthreads();
    for (int e = tid; e < KC * RC; e += kT) {
      const int ll = e % KC, rr = e / KC, l = l0 + ll, r = r0 + rr;
      ts[ll][rr] = (l < ni && r < nrhs) ? tb[d.ioff + l + (long)r * n] : czero<double>();
    }
    __syncthreads();
    if (i < f) {
      const int lm = min(KC, ni - l0);
      for (int ll = 0; ll < lm; ++ll) {
        const c128 fv = ccast<double>(F[i + (long)(l0 + ll) * f]);
#pragma unroll
        for (int q = 0; q < RB; ++q) cfma(acc[q], fv, ts[ll][g + G * q]);
      }
    }
  }
  if (i >= f) return;
  const int *bp = bpos + d.bpos_off;
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int r = r0 + g + G * q;
    if (r >= nrhs) continue;
    if (i < ni) {
      x[d.ioff + i + (long)r * n] = acc[q];
    } else {
      const long pos = bp[i - ni] + (long)r * n;
      x[pos] = x[pos] + acc[q];
    }
  }
}

template <typename T, int ROWS, int RB>
__global__ __launch_bounds__(kT) void apply_down_tiled(const int *__restrict__ nodes,
                                                       const FrontDesc *__restrict__ desc,
                                                       const cplx<T> *__restrict__ pool,
                                                       const int *__restrict__ bpos,
                                                       c128 *__restrict__ x, int n, int nrhs) {
  constexpr int G = kT / ROWS, RC = G * RB, KC = 32;
  __shared__ c128 ts[KC][RC];
  const FrontDesc d = desc[nodes[blockIdx.x]];
  const int ni = d.ni, nb = d.nb, f = d.f;
  const int i0 = blockIdx.y * ROWS, r0 = blockIdx.z * RC;
  if (ni == 0 || nb == 0 || i0 >= ni || r0 >= nrhs) return;
  const cplx<T> *F = pool + d.foff + (long)ni * f;   // R = F(0:ni, ni:f)
  const int *bp = bpos + d.bpos_off;
  const int tid = threadIdx.x, g = tid / ROWS, i = i0 + tid % ROWS;
  c128 acc[RB];
#pragma unroll
  for (int q = 0; q < RB; ++q) acc[q] = czero<double>();
  for (int b0 = 0; b0 < nb; b0 += KC) {
    __syncthreads();
    for (int e = tid; e < KC * RC; e += kT) {
      const int bb = e % KC, rr = e / KC, b = b0 + bb, r = r0 + rr;
      ts[bb][rr] = (b < nb && r < nrhs) ? x[bp[b] + (long)r * n] : czero<double>();
    }
    __syncthreads();
    if (i < ni) {
      const int bm = min(KC, nb - b0);
      for (int bb = 0; bb < bm; ++bb) {
        const c128 fv = ccast<double>(F[i + (long)(b0 + bb) * f]);
#pragma unroll
        for (int q = 0; q < RB; ++q) cfma(acc[q], fv, ts[bb][g + G * q]);
      }
    }
  }
  if (i >= ni) return;
#pragma unroll
  for (int q = 0; q < RB; ++q) {
    const int r = r0 + g + G * q;
    if (r >= nrhs) continue;
    const long pos = d.ioff + i + (long)r * n;
    x[pos] = x[pos] + acc[q];
  }
}

int rhs_chunk(int nrhs, int rows) {
  // stage at most 4096 complex doubles (64 KiB) of the input block in LDS
  int rc = rows > 0 ? 4096 / rows : nrhs;
  if (rc < 1) rc = 1;
  return rc < nrhs ? rc : nrhs;
}

}  // namespace

void launch_permute(int n, int nrhs, const int *perm, const c128 *x, long ldx, c128 *y, long ldy,
                    int inverse, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(permute_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, perm,
                     x, ldx, y, ldy, inverse);
  HSSX_HIP(hipGetLastError());
}

// tile configurations of the tiled sweeps: output rows per workgroup and
// right-hand sides per thread
const ApplyCfg kApplyCfgs[kNumApplyCfgs] = {{256, 1}, {128, 2}, {64, 4}, {64, 8}, {64, 16},
                                             {32, 8}};

namespace {

template <typename T, int ROWS, int RB>
void up_tiled(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
              const int *bpos, const c128 *tb, c128 *x, int n, int nrhs, int max_f,
              hipStream_t st) {
  constexpr int RC = (kT / ROWS) * RB;
  hipLaunchKernelGGL((apply_up_tiled<T, ROWS, RB>), dim3(count, ceil_div(max_f, ROWS),
                     ceil_div(nrhs, RC)), dim3(kT), 0, st, nodes, desc, pool, bpos, tb, x, n, nrhs);
}

template <typename T, int ROWS, int RB>
void down_tiled(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
                const int *bpos, c128 *x, int n, int nrhs, int max_ni, hipStream_t st) {
  constexpr int RC = (kT / ROWS) * RB;
  hipLaunchKernelGGL((apply_down_tiled<T, ROWS, RB>), dim3(count, ceil_div(max_ni, ROWS),
                     ceil_div(nrhs, RC)), dim3(kT), 0, st, nodes, desc, pool, bpos, x, n, nrhs);
}

}  // namespace

template <typename T>
void launch_apply_up(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
                     const int *bpos, c128 *tb, c128 *x, int n, int nrhs, int trans, int max_ni,
                     int max_f, int cfg, hipStream_t st) {
  if (count <= 0 || max_ni <= 0) return;
  hipLaunchKernelGGL(stage_kernel, dim3(count, ceil_div((long)max_ni * nrhs, 256)), dim3(256), 0,
                     st, nodes, desc, x, tb, n, nrhs);
  if (!trans) {
    switch (cfg) {
      case 0: up_tiled<T, 256, 1>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
      case 1: up_tiled<T, 128, 2>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
      case 2: up_tiled<T, 64, 4>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
      case 3: up_tiled<T, 64, 8>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
      case 4: up_tiled<T, 64, 16>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
      default: up_tiled<T, 32, 8>(count, nodes, desc, pool, bpos, tb, x, n, nrhs, max_f, st); break;
    }
  } else {
    HSSX_CHECK(max_ni <= 4096, HSSX_EINVAL, "interior block larger than the apply kernel stages");
    int rc = rhs_chunk(nrhs, max_ni);
    size_t lds = (size_t)rc * max_ni * sizeof(c128);
    hipLaunchKernelGGL(apply_up_kernel<T>, dim3(count, ceil_div(max_f, kRows), ceil_div(nrhs, rc)),
                       dim3(kT), lds, st, nodes, desc, pool, bpos, tb, x, n, nrhs, trans, rc);
  }
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_apply_down(int count, const int *nodes, const FrontDesc *desc, const cplx<T> *pool,
                       const int *bpos, c128 *x, int n, int nrhs, int trans, int max_nb,
                       int max_ni, int cfg, hipStream_t st) {
  if (count <= 0 || max_nb <= 0 || max_ni <= 0) return;
  if (!trans) {
    switch (cfg) {
      case 0: down_tiled<T, 256, 1>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
      case 1: down_tiled<T, 128, 2>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
      case 2: down_tiled<T, 64, 4>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
      case 3: down_tiled<T, 64, 8>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
      case 4: down_tiled<T, 64, 16>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
      default: down_tiled<T, 32, 8>(count, nodes, desc, pool, bpos, x, n, nrhs, max_ni, st); break;
    }
  } else {
    HSSX_CHECK(max_nb <= 4096, HSSX_EINVAL, "boundary block larger than the apply kernel stages");
    int rc = rhs_chunk(nrhs, max_nb);
    size_t lds = (size_t)rc * max_nb * sizeof(c128);
    hipLaunchKernelGGL(apply_down_kernel<T>, dim3(count, ceil_div(max_ni, kRows), ceil_div(nrhs, rc)),
                       dim3(kT), lds, st, nodes, desc, pool, bpos, x, n, nrhs, trans, rc);
  }
  HSSX_HIP(hipGetLastError());
}

#define HSSX_INST(T)                                                                          \
  template void launch_apply_up<T>(int, const int *, const FrontDesc *, const cplx<T> *,      \
                                   const int *, c128 *, c128 *, int, int, int, int, int, int, \
                                   hipStream_t);                                              \
  template void launch_apply_down<T>(int, const int *, const FrontDesc *, const cplx<T> *,    \
                                     const int *, c128 *, int, int, int, int, int, int,       \
                                     hipStream_t);
HSSX_INST(double)
HSSX_INST(float)
#undef HSSX_INST

}  // namespace hssx
