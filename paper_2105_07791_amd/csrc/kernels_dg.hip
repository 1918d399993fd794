// Symmetric interior-penalty DG assembly with P1 or P2 elements for the
// Helmholtz operator (the IPDG discretization of Sec. 4.1-4.2 and 4.6) on the
// structured mesh:
//
//   a(u,v) = sum_T int_T grad u . grad v - k^2 u v
//          + sum_{interior F} -int {grad u . n}[v] - int {grad v . n}[u]
//                              + tau_F int [u][v]
//          + boundary terms,                          tau_F = 10 p^2 / |F|,
//
// the boundary terms being either the absorbing -i int_F k u v or the
// homogeneous Dirichlet condition, imposed like an interior face with zero
// outside: -int_F (grad u . n) v - int_F (grad v . n) u + tau_F int_F u v.
// k^2 = omega^2 (P1 interpolant of the vertex values s^2), k on boundary faces
// = omega (P1 interpolant of s).  Cells (i, j) of side h = 1/Nc hold the lower
// triangle (i,j),(i+1,j),(i+1,j+1) (element 2 c) and the upper triangle
// (i,j),(i+1,j+1),(i,j+1) (element 2 c + 1), c = j Nc + i; DOF NB e + a with
// the nodal basis of degree p (NB = 3: the vertices; NB = 6: the vertices,
// then the midpoints of (v0,v1), (v1,v2), (v2,v0)).
//
// Each thread builds one CSR row.  Entry (r, c) is evaluated for the ordered
// pair (min, max) with the same quadrature and summation order from either
// side, so A is bitwise symmetric without atomics.  Volume integrals use a
// collapsed 4 x 4 Gauss-Legendre rule, face integrals 4-point Gauss-Legendre.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr double kPenaltyBase = 10.0;   // tau_F |F| = 10 p^2

// Gauss-Legendre on [0, 1]: nodes and weights of the 4-point rule
__device__ __forceinline__ void gl4(int q, double &t, double &w) {
  const double a = 0.3399810435848562648, b = 0.8611363115940525752;
  const double wa = 0.6521451548625461426, wb = 0.3478548451374538574;
  const double tt[4] = {-b, -a, a, b};
  const double ww[4] = {wb, wa, wa, wb};
  t = 0.5 * (tt[q] + 1.0);
  w = 0.5 * ww[q];
}

struct Elem {
  double x[3], y[3];
  int vid[3];       // vertex ids on the (Nc+1)^2 grid
  double det;       // twice the signed area (> 0: counter-clockwise)
};

__device__ Elem make_elem(int Nc, int e) {
  const int c = e >> 1, t = e & 1, i = c % Nc, j = c / Nc, Nv = Nc + 1;
  const double h = 1.0 / Nc;
  Elem E;
  const int di[2][3] = {{0, 1, 1}, {0, 1, 0}}, dj[2][3] = {{0, 0, 1}, {0, 1, 1}};
  for (int a = 0; a < 3; ++a) {
    const int vi = i + di[t][a], vj = j + dj[t][a];
    E.vid[a] = vj * Nv + vi;
    E.x[a] = vi * h;
    E.y[a] = vj * h;
  }
  E.det = (E.x[1] - E.x[0]) * (E.y[2] - E.y[0]) - (E.y[1] - E.y[0]) * (E.x[2] - E.x[0]);
  return E;
}

// barycentric coordinates of (px, py) and their gradients
__device__ void bary(const Elem &E, double px, double py, double lam[3], double g[3][2]) {
  for (int a = 0; a < 3; ++a) {
    const int b = (a + 1) % 3, c = (a + 2) % 3;
    const double ax = E.x[b] - px, ay = E.y[b] - py, bx = E.x[c] - px, by = E.y[c] - py;
    lam[a] = (ax * by - ay * bx) / E.det;
    g[a][0] = (E.y[b] - E.y[c]) / E.det;
    g[a][1] = (E.x[c] - E.x[b]) / E.det;
  }
}

// nodal function a (of NB per element) of E at (px, py): value and gradient
template <int NB>
__device__ void shape(const Elem &E, int a, double px, double py, double &phi, double &gx,
                      double &gy) {
  double lam[3], g[3][2];
  bary(E, px, py, lam, g);
  if (NB == 3) {
    phi = lam[a];
    gx = g[a][0];
    gy = g[a][1];
  } else if (a < 3) {
    phi = lam[a] * (2.0 * lam[a] - 1.0);
    gx = (4.0 * lam[a] - 1.0) * g[a][0];
    gy = (4.0 * lam[a] - 1.0) * g[a][1];
  } else {
    const int p = a - 3, q = (a - 2) % 3;   // edges (0,1), (1,2), (2,0)
    phi = 4.0 * lam[p] * lam[q];
    gx = 4.0 * (lam[q] * g[p][0] + lam[p] * g[q][0]);
    gy = 4.0 * (lam[q] * g[p][1] + lam[p] * g[q][1]);
  }
}

// neighbour across local face f of element e (-1: domain boundary)
__device__ int face_nbr(int Nc, int e, int f) {
  const int c = e >> 1, t = e & 1, i = c % Nc, j = c / Nc;
  if (t == 0) {
    if (f == 0) return j > 0 ? 2 * ((j - 1) * Nc + i) + 1 : -1;       // south
    if (f == 1) return i < Nc - 1 ? 2 * (j * Nc + i + 1) + 1 : -1;    // east
    return e + 1;                                                     // diagonal
  }
  if (f == 0) return e - 1;                                           // diagonal
  if (f == 1) return j < Nc - 1 ? 2 * ((j + 1) * Nc + i) : -1;        // north
  return i > 0 ? 2 * (j * Nc + i - 1) : -1;                           // west
}

// face f of E: start point, direction, length and unit outward normal
__device__ void face_geom(const Elem &E, int f, double &sx, double &sy, double &dx, double &dy,
                          double &L, double &nx, double &ny) {
  const int a = f, b = (f + 1) % 3;
  sx = E.x[a];
  sy = E.y[a];
  dx = E.x[b] - E.x[a];
  dy = E.y[b] - E.y[a];
  L = sqrt(dx * dx + dy * dy);
  nx = dy / L;
  ny = -dx / L;
}

// same-element entry (a, b) of element e: volume terms, the same-side terms
// of its interior faces and its boundary faces (absorbing, or Dirichlet when
// dir is set)
template <int NB>
__device__ void dg_self(int Nc, double omega, const double *s, int dir, int e, int a, int b,
                        double &re, double &im, double &m1) {
  constexpr double kPenalty = kPenaltyBase * (NB == 3 ? 1 : 4);
  const Elem E = make_elem(Nc, e);
  const double area2 = fabs(E.det);
  double k = 0, m = 0, mm = 0;
  for (int qu = 0; qu < 4; ++qu)
    for (int qv = 0; qv < 4; ++qv) {
      double u, wu, v, wv;
      gl4(qu, u, wu);
      gl4(qv, v, wv);
      const double xi = u, eta = v * (1.0 - u), w = wu * wv * (1.0 - u) * area2;
      const double px = E.x[0] + xi * (E.x[1] - E.x[0]) + eta * (E.x[2] - E.x[0]);
      const double py = E.y[0] + xi * (E.y[1] - E.y[0]) + eta * (E.y[2] - E.y[0]);
      const double l0 = 1.0 - xi - eta;
      const double s2 = l0 * s[E.vid[0]] * s[E.vid[0]] + xi * s[E.vid[1]] * s[E.vid[1]] +
                        eta * s[E.vid[2]] * s[E.vid[2]];
      double pa, gax, gay, pb, gbx, gby;
      shape<NB>(E, a, px, py, pa, gax, gay);
      shape<NB>(E, b, px, py, pb, gbx, gby);
      k += w * (gax * gbx + gay * gby);
      m += w * omega * omega * s2 * pa * pb;
      mm += w * pa * pb;
    }
  double fre = 0, fim = 0;
  for (int f = 0; f < 3; ++f) {
    const int en = face_nbr(Nc, e, f);
    double sx, sy, dx, dy, L, nx, ny;
    face_geom(E, f, sx, sy, dx, dy, L, nx, ny);
    const double tau = kPenalty / L;
    for (int q = 0; q < 4; ++q) {
      double t, w;
      gl4(q, t, w);
      w *= L;
      const double px = sx + t * dx, py = sy + t * dy;
      double pa, gax, gay, pb, gbx, gby;
      shape<NB>(E, a, px, py, pa, gax, gay);
      shape<NB>(E, b, px, py, pb, gbx, gby);
      if (en >= 0) {
        fre += w * (-0.5 * (gbx * nx + gby * ny) * pa - 0.5 * (gax * nx + gay * ny) * pb +
                    tau * pa * pb);
      } else if (dir) {
        fre += w * (-(gbx * nx + gby * ny) * pa - (gax * nx + gay * ny) * pb + tau * pa * pb);
      } else {
        const int v0 = E.vid[f], v1 = E.vid[(f + 1) % 3];
        const double kb = omega * ((1.0 - t) * s[v0] + t * s[v1]);
        fim -= w * kb * pa * pb;
      }
    }
  }
  re = k - m + fre;
  im = fim;
  m1 = mm;
}

// cross entry between DOF a of element e1 and DOF b of face neighbour e2 > e1
template <int NB>
__device__ double dg_cross(int Nc, int e1, int a, int e2, int b) {
  constexpr double kPenalty = kPenaltyBase * (NB == 3 ? 1 : 4);
  const Elem E1 = make_elem(Nc, e1), E2 = make_elem(Nc, e2);
  int f = 0;
  while (f < 3 && face_nbr(Nc, e1, f) != e2) ++f;
  double sx, sy, dx, dy, L, nx, ny;
  face_geom(E1, f, sx, sy, dx, dy, L, nx, ny);   // normal from e1 (+) to e2 (-)
  const double tau = kPenalty / L;
  double acc = 0;
  for (int q = 0; q < 4; ++q) {
    double t, w;
    gl4(q, t, w);
    w *= L;
    const double px = sx + t * dx, py = sy + t * dy;
    double pa, gax, gay, pb, gbx, gby;
    shape<NB>(E1, a, px, py, pa, gax, gay);
    shape<NB>(E2, b, px, py, pb, gbx, gby);
    // row side +, column side -: signs s_r = 1, s_c = -1
    acc += w * (-0.5 * (gbx * nx + gby * ny) * pa + 0.5 * (gax * nx + gay * ny) * pb -
                tau * pa * pb);
  }
  return acc;
}

template <int NB>
__global__ void assemble_dg_kernel(int Nc, double omega, const double *__restrict__ s, int dir,
                                   const int *__restrict__ rowptr, const int *__restrict__ col,
                                   c128 *__restrict__ val, double *__restrict__ mval) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= 2 * NB * Nc * Nc) return;
  for (int p = rowptr[r]; p < rowptr[r + 1]; ++p) {
    const int lo = min(r, col[p]), hi = max(r, col[p]);
    const int e1 = lo / NB, a = lo % NB, e2 = hi / NB, b = hi % NB;
    if (e1 == e2) {
      double re, im, m1;
      dg_self<NB>(Nc, omega, s, dir, e1, a, b, re, im, m1);
      val[p] = mk(re, im);
      mval[p] = m1;
    } else {
      val[p] = mk(dg_cross<NB>(Nc, e1, a, e2, b), 0.0);
      mval[p] = 0.0;
    }
  }
}

}  // namespace

void launch_assemble_dg(int Nc, int deg, int dirichlet, double omega, const double *s,
                        const int *rowptr, const int *col, c128 *val, double *mval,
                        hipStream_t st) {
  const int nb = deg == 1 ? 3 : 6, n = 2 * nb * Nc * Nc;
  if (deg == 1)
    hipLaunchKernelGGL(assemble_dg_kernel<3>, dim3(ceil_div(n, 128)), dim3(128), 0, st, Nc, omega,
                       s, dirichlet, rowptr, col, val, mval);
  else
    hipLaunchKernelGGL(assemble_dg_kernel<6>, dim3(ceil_div(n, 128)), dim3(128), 0, st, Nc, omega,
                       s, dirichlet, rowptr, col, val, mval);
  HSSX_HIP(hipGetLastError());
}

}  // namespace hssx
