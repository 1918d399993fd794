// Restarted GMRES building blocks (eq. 1.2, Sec. 4), FP64, batched over
// independent systems that each own their Krylov basis.  A vector block has
// n rows and nrhs columns (column-major); the rows split into np parts (the
// problems of a batch, np = 1 for a single problem), and system
// s = r * np + p is rows [off[p], off[p+1]) of column r.  Basis vector i of
// all systems is the block V + i * stride.  Reductions are two-stage with a
// fixed order, so results do not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr int kT = 256;

__device__ inline int seg_of(const Segs &g, int k, int r) {
  return r * g.np + (g.rpart ? g.rpart[k] : 0);
}

// partial[(blk * cnt + i) * nseg + s] = sum over the block's rows of system s
__global__ __launch_bounds__(kT) void mdot_partial(int n, Segs g, int cnt,
                                                   const c128 *__restrict__ V, long stride,
                                                   const c128 *__restrict__ w,
                                                   c128 *__restrict__ partial, int nblk) {
  __shared__ c128 red[kT];
  const int i = blockIdx.y, s = blockIdx.z, blk = blockIdx.x;
  const int r = s / g.np, p = s % g.np;
  const int o = g.off[p], len = g.off[p + 1] - o;
  const int nseg = gridDim.z;
  const c128 *v = V + i * stride + (long)r * n + o;
  const c128 *x = w + (long)r * n + o;
  c128 acc = czero<double>();
  for (long k = (long)blk * kT + threadIdx.x; k < len; k += (long)nblk * kT)
    cfma(acc, conj(v[k]), x[k]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int q = kT / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[((long)blk * cnt + i) * nseg + s] = red[0];
}

__global__ void mdot_final(int cnt, int nseg, const c128 *__restrict__ partial, int nblk,
                           c128 *__restrict__ h) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * nseg) return;
  c128 acc = czero<double>();
  for (int b = 0; b < nblk; ++b) acc = acc + partial[(long)b * cnt * nseg + t];
  h[t] = acc;
}

__global__ void mupdate_kernel(int n, int nrhs, Segs g, int cnt, const c128 *__restrict__ V,
                               long stride, const c128 *__restrict__ h, c128 *__restrict__ w) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  const int s = seg_of(g, k, r), nseg = g.np * nrhs;
  c128 acc = w[t];
  for (int i = 0; i < cnt; ++i) cfms(acc, V[i * stride + t], h[i * nseg + s]);
  w[t] = acc;
}

__global__ __launch_bounds__(kT) void norm_partial(int n, Segs g, const c128 *__restrict__ w,
                                                   double *__restrict__ partial, int nblk) {
  __shared__ double red[kT];
  const int s = blockIdx.y, blk = blockIdx.x, nseg = gridDim.y;
  const int r = s / g.np, p = s % g.np;
  const int o = g.off[p], len = g.off[p + 1] - o;
  const c128 *x = w + (long)r * n + o;
  double acc = 0.0;
  for (long k = (long)blk * kT + threadIdx.x; k < len; k += (long)nblk * kT) acc += abs2(x[k]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int q = kT / 2; q > 0; q >>= 1) {
    if (threadIdx.x < q) red[threadIdx.x] += red[threadIdx.x + q];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)blk * nseg + s] = red[0];
}

__global__ void norm_final(int nseg, const double *__restrict__ partial, int nblk,
                           double *__restrict__ norms) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nseg) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[(long)b * nseg + s];
  norms[s] = sqrt(acc);
}

__global__ void scale_kernel(int n, int nrhs, Segs g, const c128 *__restrict__ in,
                             const double *__restrict__ scale, c128 *__restrict__ out) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  double sc = scale[seg_of(g, k, r)];
  out[t] = sc > 0.0 ? (1.0 / sc) * in[t] : czero<double>();
}

__global__ void sub_kernel(int n, int nrhs, const c128 *__restrict__ a, long lda,
                           const c128 *__restrict__ b, long ldb, c128 *__restrict__ y, long ldy) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  y[k + r * ldy] = a[k + r * lda] - b[k + r * ldb];
}

__global__ void xupdate_kernel(int n, int nrhs, Segs g, const int *__restrict__ cnt,
                               const c128 *__restrict__ Z, long stride, const c128 *__restrict__ y,
                               c128 *__restrict__ x, long ldx) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  const int s = seg_of(g, k, r), nseg = g.np * nrhs;
  c128 acc = x[k + r * ldx];
  for (int i = 0; i < cnt[s]; ++i) cfma(acc, Z[i * stride + t], y[i * nseg + s]);
  x[k + r * ldx] = acc;
}

// H layout: H[(col * (m + 1) + row) * nseg + s]
__global__ void givens_kernel(int nseg, int j, int m, c128 *__restrict__ H,
                              const c128 *__restrict__ hcol, const double *__restrict__ hnext,
                              double *__restrict__ cs, c128 *__restrict__ sn, c128 *__restrict__ g,
                              double *__restrict__ res, const int *__restrict__ active) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nseg) return;
  if (!active[r]) return;
  auto Hat = [&](int row) -> c128 & { return H[((long)j * (m + 1) + row) * nseg + r]; };
  for (int i = 0; i <= j; ++i) Hat(i) = hcol[i * nseg + r];
  Hat(j + 1) = mk(hnext[r], 0.0);
  for (int i = 0; i < j; ++i) {
    c128 a = Hat(i), b = Hat(i + 1);
    double c = cs[i * nseg + r];
    c128 s = sn[i * nseg + r];
    Hat(i) = mk(c * a.re, c * a.im) + s * b;
    Hat(i + 1) = mk(c * b.re, c * b.im) - conj(s) * a;
  }
  c128 a = Hat(j), b = Hat(j + 1);
  double na = sqrt(abs2(a)), nb = sqrt(abs2(b));
  double c;
  c128 s;
  if (nb == 0.0) { c = 1.0; s = czero<double>(); }
  else if (na == 0.0) { c = 0.0; s = mk(1.0, 0.0); }
  else {
    double nu = hypot(na, nb);
    c = na / nu;
    s = (1.0 / (na * nu)) * (a * conj(b));
  }
  cs[j * nseg + r] = c;
  sn[j * nseg + r] = s;
  Hat(j) = mk(c * a.re, c * a.im) + s * b;
  Hat(j + 1) = czero<double>();
  c128 gj = g[j * nseg + r];
  g[(j + 1) * nseg + r] = -(conj(s) * gj);
  g[j * nseg + r] = mk(c * gj.re, c * gj.im);
  res[r] = sqrt(abs2(g[(j + 1) * nseg + r]));
}

__global__ void hsolve_kernel(int nseg, int m, const c128 *__restrict__ H,
                              const c128 *__restrict__ g, const int *__restrict__ cnt,
                              c128 *__restrict__ y) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nseg) return;
  int k = cnt[r];
  for (int i = k - 1; i >= 0; --i) {
    c128 v = g[i * nseg + r];
    for (int l = i + 1; l < k; ++l) cfms(v, H[((long)l * (m + 1) + i) * nseg + r], y[l * nseg + r]);
    c128 d = H[((long)i * (m + 1) + i) * nseg + r];
    y[i * nseg + r] = v * cinv(d);
  }
}

__global__ void fill_kernel(long n, c128 v, c128 *__restrict__ x) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

__global__ void conj_kernel(long n, int nrhs, const c128 *x, long ldx, c128 *y, long ldy) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= n * nrhs) return;
  const long i = t % n, r = t / n;
  y[i + r * ldy] = conj(x[i + r * ldx]);
}

}  // namespace

void launch_mdot(int n, int nrhs, const Segs &g, int cnt, const c128 *V, long stride,
                 const c128 *w, c128 *h, c128 *partial, int nblk, hipStream_t st) {
  if (cnt <= 0) return;
  const int nseg = g.np * nrhs;
  hipLaunchKernelGGL(mdot_partial, dim3(nblk, cnt, nseg), dim3(kT), 0, st, n, g, cnt, V, stride,
                     w, partial, nblk);
  hipLaunchKernelGGL(mdot_final, dim3(ceil_div((long)cnt * nseg, 256)), dim3(256), 0, st, cnt,
                     nseg, partial, nblk, h);
  HSSX_HIP(hipGetLastError());
}

void launch_mupdate(int n, int nrhs, const Segs &g, int cnt, const c128 *V, long stride,
                    const c128 *h, c128 *w, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(mupdate_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, g, cnt,
                     V, stride, h, w);
  HSSX_HIP(hipGetLastError());
}

void launch_norms(int n, int nrhs, const Segs &g, const c128 *w, double *norms, double *partial,
                  int nblk, hipStream_t st) {
  const int nseg = g.np * nrhs;
  hipLaunchKernelGGL(norm_partial, dim3(nblk, nseg), dim3(kT), 0, st, n, g, w, partial, nblk);
  hipLaunchKernelGGL(norm_final, dim3(ceil_div(nseg, 256)), dim3(256), 0, st, nseg, partial, nblk,
                     norms);
  HSSX_HIP(hipGetLastError());
}

void launch_scale(int n, int nrhs, const Segs &g, const c128 *in, const double *scale, c128 *out,
                  hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(scale_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, g, in,
                     scale, out);
  HSSX_HIP(hipGetLastError());
}

void launch_sub(int n, int nrhs, const c128 *a, long lda, const c128 *b, long ldb, c128 *y,
                long ldy, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(sub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, a, lda, b,
                     ldb, y, ldy);
  HSSX_HIP(hipGetLastError());
}

void launch_xupdate(int n, int nrhs, const Segs &g, const int *cnt, const c128 *Z, long stride,
                    const c128 *y, c128 *x, long ldx, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(xupdate_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, g, cnt,
                     Z, stride, y, x, ldx);
  HSSX_HIP(hipGetLastError());
}

void launch_givens(int nseg, int j, int m, c128 *H, const c128 *hcol, const double *hnext,
                   double *cs, c128 *sn, c128 *g, double *res, const int *active,
                   hipStream_t st) {
  hipLaunchKernelGGL(givens_kernel, dim3(ceil_div(nseg, 64)), dim3(64), 0, st, nseg, j, m, H,
                     hcol, hnext, cs, sn, g, res, active);
  HSSX_HIP(hipGetLastError());
}

void launch_hsolve(int nseg, int m, const c128 *H, const c128 *g, const int *cnt, c128 *y,
                   hipStream_t st) {
  hipLaunchKernelGGL(hsolve_kernel, dim3(ceil_div(nseg, 64)), dim3(64), 0, st, nseg, m, H, g, cnt,
                     y);
  HSSX_HIP(hipGetLastError());
}

void launch_fill(long n, c128 v, c128 *x, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, v, x);
  HSSX_HIP(hipGetLastError());
}

void launch_conj(long n, int nrhs, const c128 *x, long ldx, c128 *y, long ldy, hipStream_t st) {
  if (n <= 0 || nrhs <= 0) return;
  hipLaunchKernelGGL(conj_kernel, dim3(ceil_div(n * nrhs, 256)), dim3(256), 0, st, n, nrhs, x, ldx,
                     y, ldy);
  HSSX_HIP(hipGetLastError());
}

}  // namespace hssx
