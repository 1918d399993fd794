// Restarted GMRES building blocks (eq. 1.2, Sec. 4), FP64, batched over
// right-hand sides that each own their Krylov basis.  Basis vector i of all
// right-hand sides is the n x nrhs block V + i * stride.  Reductions are
// two-stage with a fixed order, so results do not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr int kT = 256;

// partial[(blk * cnt + i) * nrhs + r] = sum over the block's rows
__global__ __launch_bounds__(kT) void mdot_partial(int n, int nrhs, int cnt,
                                                   const c128 *__restrict__ V, long stride,
                                                   const c128 *__restrict__ w,
                                                   c128 *__restrict__ partial, int nblk) {
  __shared__ c128 red[kT];
  const int i = blockIdx.y, r = blockIdx.z, blk = blockIdx.x;
  const c128 *v = V + i * stride + (long)r * n;
  const c128 *x = w + (long)r * n;
  c128 acc = czero<double>();
  for (long k = (long)blk * kT + threadIdx.x; k < n; k += (long)nblk * kT)
    cfma(acc, conj(v[k]), x[k]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = red[threadIdx.x] + red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[((long)blk * cnt + i) * nrhs + r] = red[0];
}

__global__ void mdot_final(int cnt, int nrhs, const c128 *__restrict__ partial, int nblk,
                           c128 *__restrict__ h) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= cnt * nrhs) return;
  c128 acc = czero<double>();
  for (int b = 0; b < nblk; ++b) acc = acc + partial[(long)b * cnt * nrhs + t];
  h[t] = acc;
}

__global__ void mupdate_kernel(int n, int nrhs, int cnt, const c128 *__restrict__ V, long stride,
                               const c128 *__restrict__ h, c128 *__restrict__ w) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  c128 acc = w[t];
  for (int i = 0; i < cnt; ++i) cfms(acc, V[i * stride + (long)r * n + k], h[i * nrhs + r]);
  w[t] = acc;
}

__global__ __launch_bounds__(kT) void norm_partial(int n, int nrhs, const c128 *__restrict__ w,
                                                   double *__restrict__ partial, int nblk) {
  __shared__ double red[kT];
  const int r = blockIdx.y, blk = blockIdx.x;
  const c128 *x = w + (long)r * n;
  double acc = 0.0;
  for (long k = (long)blk * kT + threadIdx.x; k < n; k += (long)nblk * kT) acc += abs2(x[k]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[(long)blk * nrhs + r] = red[0];
}

__global__ void norm_final(int nrhs, const double *__restrict__ partial, int nblk,
                           double *__restrict__ norms) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  double acc = 0.0;
  for (int b = 0; b < nblk; ++b) acc += partial[(long)b * nrhs + r];
  norms[r] = sqrt(acc);
}

__global__ void scale_kernel(int n, int nrhs, const c128 *__restrict__ in,
                             const double *__restrict__ scale, c128 *__restrict__ out) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int r = (int)(t / n);
  double s = scale[r];
  out[t] = s > 0.0 ? (1.0 / s) * in[t] : czero<double>();
}

__global__ void sub_kernel(int n, int nrhs, const c128 *__restrict__ a, long lda,
                           const c128 *__restrict__ b, long ldb, c128 *__restrict__ y, long ldy) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  y[k + r * ldy] = a[k + r * lda] - b[k + r * ldb];
}

__global__ void xupdate_kernel(int n, int nrhs, const int *__restrict__ cnt,
                               const c128 *__restrict__ Z, long stride, const c128 *__restrict__ y,
                               c128 *__restrict__ x, long ldx) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int k = (int)(t % n), r = (int)(t / n);
  c128 acc = x[k + r * ldx];
  for (int i = 0; i < cnt[r]; ++i) cfma(acc, Z[i * stride + (long)r * n + k], y[i * nrhs + r]);
  x[k + r * ldx] = acc;
}

// H layout: H[(col * (m + 1) + row) * nrhs + r]
__global__ void givens_kernel(int nrhs, int j, int m, c128 *__restrict__ H,
                              const c128 *__restrict__ hcol, const double *__restrict__ hnext,
                              double *__restrict__ cs, c128 *__restrict__ sn, c128 *__restrict__ g,
                              double *__restrict__ res, const int *__restrict__ active) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  if (!active[r]) return;
  auto Hat = [&](int row) -> c128 & { return H[((long)j * (m + 1) + row) * nrhs + r]; };
  for (int i = 0; i <= j; ++i) Hat(i) = hcol[i * nrhs + r];
  Hat(j + 1) = mk(hnext[r], 0.0);
  for (int i = 0; i < j; ++i) {
    c128 a = Hat(i), b = Hat(i + 1);
    double c = cs[i * nrhs + r];
    c128 s = sn[i * nrhs + r];
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
  cs[j * nrhs + r] = c;
  sn[j * nrhs + r] = s;
  Hat(j) = mk(c * a.re, c * a.im) + s * b;
  Hat(j + 1) = czero<double>();
  c128 gj = g[j * nrhs + r];
  g[(j + 1) * nrhs + r] = -(conj(s) * gj);
  g[j * nrhs + r] = mk(c * gj.re, c * gj.im);
  res[r] = sqrt(abs2(g[(j + 1) * nrhs + r]));
}

__global__ void hsolve_kernel(int nrhs, int m, const c128 *__restrict__ H,
                              const c128 *__restrict__ g, const int *__restrict__ cnt,
                              c128 *__restrict__ y) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrhs) return;
  int k = cnt[r];
  for (int i = k - 1; i >= 0; --i) {
    c128 v = g[i * nrhs + r];
    for (int l = i + 1; l < k; ++l) cfms(v, H[((long)l * (m + 1) + i) * nrhs + r], y[l * nrhs + r]);
    c128 d = H[((long)i * (m + 1) + i) * nrhs + r];
    y[i * nrhs + r] = v * cinv(d);
  }
}

__global__ void fill_kernel(long n, c128 v, c128 *__restrict__ x) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t < n) x[t] = v;
}

}  // namespace

void launch_mdot(int n, int nrhs, int cnt, const c128 *V, long stride, const c128 *w, c128 *h,
                 c128 *partial, int nblk, hipStream_t st) {
  if (cnt <= 0) return;
  hipLaunchKernelGGL(mdot_partial, dim3(nblk, cnt, nrhs), dim3(kT), 0, st, n, nrhs, cnt, V, stride,
                     w, partial, nblk);
  hipLaunchKernelGGL(mdot_final, dim3(ceil_div((long)cnt * nrhs, 256)), dim3(256), 0, st, cnt,
                     nrhs, partial, nblk, h);
  HSSX_HIP(hipGetLastError());
}

void launch_mupdate(int n, int nrhs, int cnt, const c128 *V, long stride, const c128 *h, c128 *w,
                    hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(mupdate_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, cnt, V,
                     stride, h, w);
  HSSX_HIP(hipGetLastError());
}

void launch_norms(int n, int nrhs, const c128 *w, double *norms, double *partial, int nblk,
                  hipStream_t st) {
  hipLaunchKernelGGL(norm_partial, dim3(nblk, nrhs), dim3(kT), 0, st, n, nrhs, w, partial, nblk);
  hipLaunchKernelGGL(norm_final, dim3(ceil_div(nrhs, 256)), dim3(256), 0, st, nrhs, partial, nblk,
                     norms);
  HSSX_HIP(hipGetLastError());
}

void launch_scale(int n, int nrhs, const c128 *in, const double *scale, c128 *out,
                  hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(scale_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, in, scale,
                     out);
  HSSX_HIP(hipGetLastError());
}

void launch_sub(int n, int nrhs, const c128 *a, long lda, const c128 *b, long ldb, c128 *y,
                long ldy, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(sub_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, a, lda, b,
                     ldb, y, ldy);
  HSSX_HIP(hipGetLastError());
}

void launch_xupdate(int n, int nrhs, const int *cnt, int maxcnt, const c128 *Z, long stride,
                    const c128 *y, c128 *x, long ldx, hipStream_t st) {
  (void)maxcnt;
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(xupdate_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, cnt, Z,
                     stride, y, x, ldx);
  HSSX_HIP(hipGetLastError());
}

void launch_givens(int nrhs, int j, int m, c128 *H, const c128 *hcol, const double *hnext,
                   double *cs, c128 *sn, c128 *g, double *res, const int *active,
                   hipStream_t st) {
  hipLaunchKernelGGL(givens_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, st, nrhs, j, m, H,
                     hcol, hnext, cs, sn, g, res, active);
  HSSX_HIP(hipGetLastError());
}

void launch_hsolve(int nrhs, int m, const c128 *H, const c128 *g, const int *cnt, c128 *y,
                   hipStream_t st) {
  hipLaunchKernelGGL(hsolve_kernel, dim3(ceil_div(nrhs, 64)), dim3(64), 0, st, nrhs, m, H, g, cnt,
                     y);
  HSSX_HIP(hipGetLastError());
}

void launch_fill(long n, c128 v, c128 *x, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, n, v, x);
  HSSX_HIP(hipGetLastError());
}

}  // namespace hssx
