// P1 Galerkin assembly, mass load, SpMV and the adjoint dA/ds contraction
// on the structured N x N grid (Sec. 4.2, eq. 4.2 with absorbing boundary).
//
// A = K - omega^2 M[s^2] - i omega G[s] in CSR with the fixed 7-point
// pattern (columns sorted: -N-1, -N, -1, 0, +1, +N, +N+1).  Each thread
// builds one row; entry (i,j) is evaluated for the ordered pair
// (lo, hi) = (min, max) by visiting the four cells around lo in global cell
// order (triangle SW-SE-NE before SW-NE-NW) and then the boundary edge they
// share, so (i,j) and (j,i) run the identical computation: A is bitwise
// symmetric and the assembly uses no atomics.
//
// Closed forms (barycentric monomials): int_T l_l l_a l_b = 2|T| * {1/20 if
// l=a=b, 1/60 if two equal, 1/120 if distinct}; int_e l_l l_a l_b = |e| *
// {1/4, 1/12}.  The load matrix M[1]_ab = 2|T| * {1/12, 1/24}.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

__device__ __forceinline__ double tri3(int l, int a, int b) {
  if (l == a && a == b) return 1.0 / 20.0;
  if (l == a || l == b || a == b) return 1.0 / 60.0;
  return 1.0 / 120.0;
}

struct Tri {
  int v[3];
};

// triangle t (0/1) of cell (cx, cy)
__device__ __forceinline__ Tri cell_tri(int N, int cx, int cy, int t) {
  Tri T;
  int sw = cy * N + cx, se = sw + 1, ne = sw + N + 1, nw = sw + N;
  T.v[0] = sw;
  T.v[1] = t == 0 ? se : ne;
  T.v[2] = t == 0 ? ne : nw;
  return T;
}

__device__ __forceinline__ int local_index(const Tri &T, int g) {
  return T.v[0] == g ? 0 : (T.v[1] == g ? 1 : (T.v[2] == g ? 2 : -1));
}

// K_ab, M[w]_ab (w = s^2), M[1]_ab of one triangle for local vertices a, b.
__device__ void tri_terms(int N, double h, const Tri &T, int a, int b,
                          const double *s, double &k, double &m, double &m1) {
  double px[3], py[3];
  for (int q = 0; q < 3; ++q) {
    px[q] = (double)(T.v[q] % N) * h;
    py[q] = (double)(T.v[q] / N) * h;
  }
  double det = (px[1] - px[0]) * (py[2] - py[0]) - (py[1] - py[0]) * (px[2] - px[0]);
  double area = 0.5 * fabs(det);
  // grad l_q = rot(p_{q+2} - p_{q+1}) / det
  double gax = (py[(a + 2) % 3] - py[(a + 1) % 3]) / det;
  double gay = -(px[(a + 2) % 3] - px[(a + 1) % 3]) / det;
  double gbx = (py[(b + 2) % 3] - py[(b + 1) % 3]) / det;
  double gby = -(px[(b + 2) % 3] - px[(b + 1) % 3]) / det;
  k = area * (gax * gbx + gay * gby);
  double acc = 0.0;
  for (int l = 0; l < 3; ++l) {
    double w = s[T.v[l]] * s[T.v[l]];
    acc += w * tri3(l, a, b);
  }
  m = 2.0 * area * acc;
  m1 = 2.0 * area * (a == b ? 1.0 / 12.0 : 1.0 / 24.0);
}

// Boundary edges in global order: south (k), east, north, west.
// Edge e of side q joins (e-th, e+1-th) node along that side.
__device__ __forceinline__ void side_edge(int N, int q, int e, int &u, int &v) {
  if (q == 0) { u = e; v = e + 1; }
  else if (q == 1) { u = e * N + N - 1; v = (e + 1) * N + N - 1; }
  else if (q == 2) { u = (N - 1) * N + e; v = u + 1; }
  else { u = e * N; v = (e + 1) * N; }
}

// sum over boundary edges containing both gi and gj of sum_l s_l int l_l l_a l_b
__device__ double edge_terms(int N, double h, int gi, int gj, const double *s) {
  int xi = gi % N, yi = gi / N;
  double acc = 0.0;
  for (int q = 0; q < 4; ++q) {
    // candidate edge indices along side q touching node gi
    int along;
    bool on;
    if (q == 0) { on = yi == 0; along = xi; }
    else if (q == 1) { on = xi == N - 1; along = yi; }
    else if (q == 2) { on = yi == N - 1; along = xi; }
    else { on = xi == 0; along = yi; }
    if (!on) continue;
    for (int e = along - 1; e <= along; ++e) {
      if (e < 0 || e >= N - 1) continue;
      int u, v;
      side_edge(N, q, e, u, v);
      bool hi_ = (u == gi || v == gi), hj = (u == gj || v == gj);
      if (!(hi_ && hj)) continue;
      int a = (u == gi) ? 0 : 1, b = (u == gj) ? 0 : 1;
      double su = s[u], sv = s[v];
      // int_e l_l l_a l_b / |e|: 1/4 if all equal, 1/12 otherwise
      double t0 = (0 == a && a == b) ? 0.25 : 1.0 / 12.0;
      double t1 = (1 == a && a == b) ? 0.25 : 1.0 / 12.0;
      acc += h * (su * t0 + sv * t1);
    }
  }
  return acc;
}

__global__ void assemble_kernel(int N, double omega, const double *__restrict__ s,
                                const int *__restrict__ rowptr, const int *__restrict__ col,
                                c128 *__restrict__ val, double *__restrict__ mval) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * N) return;
  double h = 1.0 / (N - 1);
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) {
    // entry (i, j) and (j, i) run the identical computation on the ordered
    // pair (lo, hi), so the matrix is symmetric bit for bit
    const int lo = min(i, col[p]), hi = max(i, col[p]);
    const int xl = lo % N, yl = lo / N;
    double k = 0.0, m = 0.0, m1 = 0.0;
    // cells around node lo in global cell order
    for (int cy = yl - 1; cy <= yl; ++cy)
      for (int cx = xl - 1; cx <= xl; ++cx) {
        if (cx < 0 || cy < 0 || cx >= N - 1 || cy >= N - 1) continue;
        for (int t = 0; t < 2; ++t) {
          Tri T = cell_tri(N, cx, cy, t);
          int a = local_index(T, lo), b = local_index(T, hi);
          if (a < 0 || b < 0) continue;
          double kk, mm, mm1;
          tri_terms(N, h, T, a, b, s, kk, mm, mm1);
          k += kk;
          m += mm;
          m1 += mm1;
        }
      }
    double g = edge_terms(N, h, lo, hi, s);
    val[p] = mk(k - omega * omega * m, -omega * g);
    mval[p] = m1;
  }
}

// ---------------------------------------------------------------- elastic
// Time-harmonic P1 elasticity (DOF 2 v + c): A = K[lam, mu] - omega^2 M[rho]
// - i omega C with the Lysmer-Kuhlemeyer boundary term.  Per triangle and
// local vertices a, b, components i, j:
//   K = lam_T g_a[i] g_b[j] + mu_T (delta_ij g_a.g_b + g_a[j] g_b[i]),
//   lam_T, mu_T = area times the vertex mean; M = delta_ij 2|T| sum_l rho_l
//   int l_l l_a l_b; on boundary edges C = delta_ij h sum_l z_l int l_l l_a l_b
//   with z = rho c_p for the normal component and rho c_s for the tangential.
__device__ void tri_terms_el(int N, double h, const Tri &T, int a, int i, int b, int j,
                             const double *lam, const double *mu, const double *rho,
                             double &k, double &m, double &m1) {
  double px[3], py[3];
  for (int q = 0; q < 3; ++q) {
    px[q] = (double)(T.v[q] % N) * h;
    py[q] = (double)(T.v[q] / N) * h;
  }
  double det = (px[1] - px[0]) * (py[2] - py[0]) - (py[1] - py[0]) * (px[2] - px[0]);
  double area = 0.5 * fabs(det);
  double ga[2], gb[2];
  ga[0] = (py[(a + 2) % 3] - py[(a + 1) % 3]) / det;
  ga[1] = -(px[(a + 2) % 3] - px[(a + 1) % 3]) / det;
  gb[0] = (py[(b + 2) % 3] - py[(b + 1) % 3]) / det;
  gb[1] = -(px[(b + 2) % 3] - px[(b + 1) % 3]) / det;
  const double lt = (lam[T.v[0]] + lam[T.v[1]] + lam[T.v[2]]) / 3.0 * area;
  const double mt = (mu[T.v[0]] + mu[T.v[1]] + mu[T.v[2]]) / 3.0 * area;
  const double gg = ga[0] * gb[0] + ga[1] * gb[1];
  k = lt * ga[i] * gb[j] + mt * ((i == j ? gg : 0.0) + ga[j] * gb[i]);
  m = 0.0;
  m1 = 0.0;
  if (i == j) {
    double acc = 0.0;
    for (int l = 0; l < 3; ++l) acc += rho[T.v[l]] * tri3(l, a, b);
    m = 2.0 * area * acc;
    m1 = 2.0 * area * (a == b ? 1.0 / 12.0 : 1.0 / 24.0);
  }
}

// boundary term of the DOF pair (gi, ci), (gj, cj): nonzero for ci == cj only
__device__ double edge_terms_el(int N, double h, int gi, int gj, int c, const double *lam,
                                const double *mu, const double *rho) {
  int xi = gi % N, yi = gi / N;
  double acc = 0.0;
  for (int q = 0; q < 4; ++q) {
    int along;
    bool on;
    if (q == 0) { on = yi == 0; along = xi; }
    else if (q == 1) { on = xi == N - 1; along = yi; }
    else if (q == 2) { on = yi == N - 1; along = xi; }
    else { on = xi == 0; along = yi; }
    if (!on) continue;
    // normal component: y on the south/north sides, x on east/west
    const bool normal = (q == 0 || q == 2) ? c == 1 : c == 0;
    for (int e = along - 1; e <= along; ++e) {
      if (e < 0 || e >= N - 1) continue;
      int u, v;
      side_edge(N, q, e, u, v);
      bool hi_ = (u == gi || v == gi), hj = (u == gj || v == gj);
      if (!(hi_ && hj)) continue;
      int a = (u == gi) ? 0 : 1, b = (u == gj) ? 0 : 1;
      const double zu = normal ? sqrt(rho[u] * (lam[u] + 2.0 * mu[u])) : sqrt(rho[u] * mu[u]);
      const double zv = normal ? sqrt(rho[v] * (lam[v] + 2.0 * mu[v])) : sqrt(rho[v] * mu[v]);
      double t0 = (0 == a && a == b) ? 0.25 : 1.0 / 12.0;
      double t1 = (1 == a && a == b) ? 0.25 : 1.0 / 12.0;
      acc += h * (zu * t0 + zv * t1);
    }
  }
  return acc;
}

__global__ void assemble_elastic_kernel(int N, double omega, const double *__restrict__ lam,
                                        const double *__restrict__ mu,
                                        const double *__restrict__ rho,
                                        const int *__restrict__ rowptr,
                                        const int *__restrict__ col, c128 *__restrict__ val,
                                        double *__restrict__ mval) {
  int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * N * N) return;
  double h = 1.0 / (N - 1);
  for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
    // the ordered DOF pair (lo, hi): bitwise symmetric, no atomics
    const int lo = min(r, col[p]), hi = max(r, col[p]);
    const int vl = lo / 2, il = lo % 2, vh = hi / 2, ih = hi % 2;
    const int xl = vl % N, yl = vl / N;
    double k = 0.0, m = 0.0, m1 = 0.0;
    for (int cy = yl - 1; cy <= yl; ++cy)
      for (int cx = xl - 1; cx <= xl; ++cx) {
        if (cx < 0 || cy < 0 || cx >= N - 1 || cy >= N - 1) continue;
        for (int t = 0; t < 2; ++t) {
          Tri T = cell_tri(N, cx, cy, t);
          int a = local_index(T, vl), b = local_index(T, vh);
          if (a < 0 || b < 0) continue;
          double kk, mm, mm1;
          tri_terms_el(N, h, T, a, il, b, ih, lam, mu, rho, kk, mm, mm1);
          k += kk;
          m += mm;
          m1 += mm1;
        }
      }
    double g = il == ih ? edge_terms_el(N, h, vl, vh, il, lam, mu, rho) : 0.0;
    val[p] = mk(k - omega * omega * m, -omega * g);
    mval[p] = m1;
  }
}

// b = M[1] f  (f real n x nrhs, b complex)
__global__ void load_kernel(int n, int nrhs, const int *__restrict__ rowptr,
                            const int *__restrict__ col, const double *__restrict__ mval,
                            const double *__restrict__ f, long ldf, c128 *__restrict__ b, long ldb) {
  long t = blockIdx.x * (long)blockDim.x + threadIdx.x;
  if (t >= (long)n * nrhs) return;
  int i = (int)(t % n), r = (int)(t / n);
  double acc = 0.0;
  for (int p = rowptr[i]; p < rowptr[i + 1]; ++p) acc += mval[p] * f[col[p] + r * ldf];
  b[i + r * ldb] = mk(acc, 0.0);
}

// One thread per row: the row's <= 7 entries are read once and reused for
// every right-hand side; for a fixed rhs a wavefront touches consecutive rows,
// so x and y accesses stay coalesced.
// One row per thread, the row's W (7: scalar stencil, 14: 2 x 2 blocks,
// 24: P2 triangle blocks)
// entries held in registers across the right-hand sides.
template <int W>
__global__ __launch_bounds__(256) void spmv_kernel(int n, int nrhs, const int *__restrict__ rowptr,
                                                   const int *__restrict__ col,
                                                   const c128 *__restrict__ val,
                                                   const c128 *__restrict__ x, long ldx,
                                                   c128 *__restrict__ y, long ldy) {
  // workgroups go round-robin to the 8 XCDs: give each XCD one contiguous
  // eighth of the rows, so the neighbouring rows a row's columns reach are
  // mostly read through the same XCD's L2 (the grid is a multiple of 8)
  const int per = gridDim.x / 8;
  const int blk = (blockIdx.x % 8) * per + blockIdx.x / 8;
  int i = blk * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = rowptr[i], cnt = rowptr[i + 1] - p0;
  int cj[W];
  c128 a[W];
#pragma unroll
  for (int q = 0; q < W; ++q) {
    cj[q] = q < cnt ? col[p0 + q] : i;
    a[q] = q < cnt ? val[p0 + q] : czero<double>();
  }
  for (int r = 0; r < nrhs; ++r) {
    const c128 *xr = x + r * ldx;
    c128 acc = czero<double>();
#pragma unroll
    for (int q = 0; q < W; ++q) cfma(acc, a[q], xr[cj[q]]);
    y[i + r * ldy] = acc;
  }
}

// grad[l] += -Re sum_r sum_{a,b} lam_a (dA/ds_l)_ab x_b, one thread per node l.
// dA/ds_l = -omega^2 * 2 s_l * Mtri_l - i omega * Gedge_l where Mtri_l(a,b) =
// sum_{T ni l,a,b} int l_l l_a l_b and Gedge_l likewise on boundary edges.
__global__ void dads_kernel(int N, double omega, const double *__restrict__ s, int nrhs,
                            const c128 *__restrict__ lam, const c128 *__restrict__ x, long ld,
                            double *__restrict__ grad, int conj_lam) {
  int l = blockIdx.x * blockDim.x + threadIdx.x;
  int n = N * N;
  if (l >= n) return;
  double h = 1.0 / (N - 1);
  int xl = l % N, yl = l / N;
  double total = 0.0;
  for (int r = 0; r < nrhs; ++r) {
    const c128 *lr = lam + (long)r * ld;
    const c128 *xr = x + (long)r * ld;
    c128 accT = czero<double>();   // sum_T 2|T| sum_ab c(l,a,b) lam_a x_b
    for (int cy = yl - 1; cy <= yl; ++cy)
      for (int cx = xl - 1; cx <= xl; ++cx) {
        if (cx < 0 || cy < 0 || cx >= N - 1 || cy >= N - 1) continue;
        for (int t = 0; t < 2; ++t) {
          Tri T = cell_tri(N, cx, cy, t);
          int ll = local_index(T, l);
          if (ll < 0) continue;
          double area = 0.5 * h * h;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
              double c = 2.0 * area * tri3(ll, a, b);
              const c128 la = conj_lam ? conj(lr[T.v[a]]) : lr[T.v[a]];
              cfma(accT, mk(c, 0.0), la * xr[T.v[b]]);
            }
        }
      }
    c128 accE = czero<double>();   // sum_e |e| sum_ab c_e(l,a,b) lam_a x_b
    for (int q = 0; q < 4; ++q) {
      int along;
      bool on;
      if (q == 0) { on = yl == 0; along = xl; }
      else if (q == 1) { on = xl == N - 1; along = yl; }
      else if (q == 2) { on = yl == N - 1; along = xl; }
      else { on = xl == 0; along = yl; }
      if (!on) continue;
      for (int e = along - 1; e <= along; ++e) {
        if (e < 0 || e >= N - 1) continue;
        int u, v;
        side_edge(N, q, e, u, v);
        int ll = (u == l) ? 0 : 1;
        int vv[2] = {u, v};
        for (int a = 0; a < 2; ++a)
          for (int b = 0; b < 2; ++b) {
            double c = (ll == a && a == b) ? 0.25 : 1.0 / 12.0;
            const c128 la = conj_lam ? conj(lr[vv[a]]) : lr[vv[a]];
            cfma(accE, mk(h * c, 0.0), la * xr[vv[b]]);
          }
      }
    }
    // lam^T dA x = -2 omega^2 s_l accT - i omega accE
    c128 val = mk(-2.0 * omega * omega * s[l] * accT.re + omega * accE.im,
                  -2.0 * omega * omega * s[l] * accT.im - omega * accE.re);
    total += -val.re;
  }
  grad[l] += total;
}

}  // namespace

void launch_assemble(int N, double omega, const double *s, const int *rowptr, const int *col,
                     c128 *val, double *mval, hipStream_t st) {
  int n = N * N;
  hipLaunchKernelGGL(assemble_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, N, omega, s,
                     rowptr, col, val, mval);
  HSSX_HIP(hipGetLastError());
}

void launch_assemble_elastic(int N, double omega, const double *lam, const double *mu,
                             const double *rho, const int *rowptr, const int *col, c128 *val,
                             double *mval, hipStream_t st) {
  int n = 2 * N * N;
  hipLaunchKernelGGL(assemble_elastic_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, N, omega,
                     lam, mu, rho, rowptr, col, val, mval);
  HSSX_HIP(hipGetLastError());
}

void launch_load(int n, int nrhs, const int *rowptr, const int *col, const double *mval,
                 const double *f, long ldf, c128 *b, long ldb, hipStream_t st) {
  long tot = (long)n * nrhs;
  hipLaunchKernelGGL(load_kernel, dim3(ceil_div(tot, 256)), dim3(256), 0, st, n, nrhs, rowptr,
                     col, mval, f, ldf, b, ldb);
  HSSX_HIP(hipGetLastError());
}

void launch_spmv(int n, int nrhs, const int *rowptr, const int *col, const c128 *val,
                 const c128 *x, long ldx, c128 *y, long ldy, int row_max, hipStream_t st) {
  const dim3 grid(8 * ceil_div(ceil_div(n, 256), 8));
  if (row_max <= 7)
    hipLaunchKernelGGL(spmv_kernel<7>, grid, dim3(256), 0, st, n, nrhs, rowptr, col, val, x, ldx,
                       y, ldy);
  else if (row_max <= 14)
    hipLaunchKernelGGL(spmv_kernel<14>, grid, dim3(256), 0, st, n, nrhs, rowptr, col, val, x, ldx,
                       y, ldy);
  else if (row_max <= 24)
    hipLaunchKernelGGL(spmv_kernel<24>, grid, dim3(256), 0, st, n, nrhs, rowptr, col, val, x, ldx,
                       y, ldy);
  else
    throw Error(HSSX_EINVAL, "rows longer than 24 entries");
  HSSX_HIP(hipGetLastError());
}

void launch_dads(int N, double omega, const double *s, int nrhs, const c128 *lam,
                 const c128 *x, long ld, double *grad, int conj_lam, hipStream_t st) {
  int n = N * N;
  hipLaunchKernelGGL(dads_kernel, dim3(ceil_div(n, 256)), dim3(256), 0, st, N, omega, s, nrhs,
                     lam, x, ld, grad, conj_lam);
  HSSX_HIP(hipGetLastError());
}

}  // namespace hssx
