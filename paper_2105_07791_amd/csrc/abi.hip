// extern "C" entry points declared in include/hssx.h.  Every call validates
// its arguments, runs under the handle's device, converts exceptions into a
// status code and records the message for hssx_last_error().
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <exception>
#include <mutex>
#include <thread>

#include "engine.h"
#include "prof.h"

using namespace hssx;

namespace {

thread_local std::string g_err;

template <typename F> hssx_status guarded(F &&f) {
  try {
    f();
    return HSSX_OK;
  } catch (const Error &e) {
    g_err = e.what();
    return e.code;
  } catch (const std::bad_alloc &) {
    g_err = "host allocation failed";
    return HSSX_ENOMEM;
  } catch (const std::exception &e) {
    g_err = e.what();
    return HSSX_EINVAL;
  }
}

struct DeviceScope {
  int prev = 0;
  explicit DeviceScope(int d) {
    HSSX_HIP(hipGetDevice(&prev));
    if (prev != d) HSSX_HIP(hipSetDevice(d));
  }
  ~DeviceScope() { (void)hipSetDevice(prev); }
};

hipStream_t S(void *s) { return reinterpret_cast<hipStream_t>(s); }

// the context bound to the calling thread (hssx_bind): handles created
// while it is bound allocate through its allocator
thread_local hssx_ctx_ *g_bound = nullptr;

// Subtree roots of a child's cluster tree: [P0 | P1] split at the root when
// both parts exist (Fig. 4), else the whole tree is the one present part.
void child_roots(const NDNode &c, int &ii, int &bb, int &split) {
  const int nb = (int)c.B.size();
  split = 0;
  ii = bb = -1;
  if (c.ct.count() == 0) return;
  if (c.p0 > 0 && c.p0 < nb) {
    split = 1;
    ii = c.ct.left[0];
    bb = c.ct.right[0];
  } else if (c.p0 == nb) {
    ii = 0;
  } else {
    bb = 0;
  }
}

// Index maps and coupling lists of the HSS-class nodes (eq. 3.4 layout):
// where each position of sigma's front sits in its children's boundaries,
// and the entries of A that couple the two children, split by the blocks
// they fall in (A~_ii both ways, A~_ib as sparse columns, A~_bb).
void build_hss_sym(hssx_fact_ &P, const hssx_op_ &A) {
  const Symbolic &sym = P.sym;
  const int nn = (int)sym.nodes.size();
  P.hsym.clear();
  std::vector<int> pool;
  auto put = [&](const std::vector<int> &v) {
    const long o = (long)pool.size();
    pool.insert(pool.end(), v.begin(), v.end());
    pool.push_back(0);   // no empty arrays
    return o;
  };
  std::vector<int> own(A.n, -1), cpos(A.n, -1), spos(A.n, -1);
  auto csr_index = [&](int r, int c) {
    const int *b = A.h_col.data() + A.h_rowptr[r], *e = A.h_col.data() + A.h_rowptr[r + 1];
    const int *q = std::lower_bound(b, e, c);
    HSSX_CHECK(q != e && *q == c, HSSX_EINVAL, "unsymmetric sparsity pattern");
    return (int)(q - A.h_col.data());
  };
  for (int k = 0; k < nn; ++k) {
    if (P.hss_idx[k] < 0) continue;
    const NDNode &nd = sym.nodes[k], &mu = sym.nodes[nd.lo], &nu = sym.nodes[nd.hi];
    HssSym h;
    h.node = k;
    h.mu = nd.lo;
    h.nu = nd.hi;
    h.pmu = mu.p0;
    h.pnu = nu.p0;
    h.ni = (int)nd.I.size();
    h.nb = (int)nd.B.size();
    h.mmu = (int)mu.B.size();
    h.mnu = (int)nu.B.size();
    child_roots(mu, h.ii_mu, h.bb_mu, h.split_mu);
    child_roots(nu, h.ii_nu, h.bb_nu, h.split_nu);
    HSSX_CHECK(h.ni == h.pmu + h.pnu, HSSX_EINVAL, "interior is not [P0(mu); P0(nu)]");
    for (int i = 0; i < h.pmu; ++i)
      HSSX_CHECK(nd.I[i] == mu.B[i], HSSX_EINVAL, "interior order differs from P0(mu)");
    for (int i = 0; i < h.pnu; ++i)
      HSSX_CHECK(nd.I[h.pmu + i] == nu.B[i], HSSX_EINVAL, "interior order differs from P0(nu)");
    for (int i = 0; i < h.mmu; ++i) { own[mu.B[i]] = 0; cpos[mu.B[i]] = i; }
    for (int i = 0; i < h.mnu; ++i) { own[nu.B[i]] = 1; cpos[nu.B[i]] = i; }
    for (int b = 0; b < h.nb; ++b) spos[nd.B[b]] = b;
    std::vector<int> bchild(h.nb), bcp(h.nb), gid(h.nb), smu(h.nb, -1), snu(h.nb, -1);
    std::vector<int> p1mu(std::max(0, h.mmu - h.pmu)), p1nu(std::max(0, h.mnu - h.pnu));
    for (int b = 0; b < h.nb; ++b) {
      const int v = nd.B[b];
      HSSX_CHECK(own[v] >= 0 && cpos[v] >= (own[v] ? h.pnu : h.pmu), HSSX_EINVAL,
                 "boundary position outside the children's P1 parts");
      bchild[b] = own[v];
      bcp[b] = cpos[v];
      gid[b] = v;
      if (own[v] == 0) {
        smu[b] = cpos[v] - h.pmu;
        p1mu[cpos[v] - h.pmu] = b;
      } else {
        snu[b] = cpos[v] - h.pnu;
        p1nu[cpos[v] - h.pnu] = b;
      }
    }
    // couplings of the two children through A
    std::vector<std::vector<std::pair<int, int>>> imu(h.pmu), inu(h.pnu), bb(h.nb);
    std::vector<std::array<int, 3>> ib;   // I row, B position, value index
    for (int i = 0; i < h.mmu; ++i) {
      const int v = mu.B[i];
      for (int e = A.h_rowptr[v]; e < A.h_rowptr[v + 1]; ++e) {
        const int u = A.h_col[e];
        if (u < 0 || u >= A.n || own[u] != 1) continue;
        const int j = cpos[u], euv = csr_index(u, v);
        const bool vi = i < h.pmu, ui = j < h.pnu;
        if (vi && ui) {
          imu[i].push_back({j, e});
          inu[j].push_back({i, euv});
        } else if (vi) {
          ib.push_back({i, spos[u], e});
        } else if (ui) {
          ib.push_back({h.pmu + j, spos[v], euv});
        } else {
          bb[spos[v]].push_back({spos[u], e});
          bb[spos[u]].push_back({spos[v], euv});
        }
      }
    }
    auto csr = [&](std::vector<std::vector<std::pair<int, int>>> &rows, long &rp, long &cp,
                   long &vi) {
      std::vector<int> r{0}, c, w;
      for (auto &row : rows) {
        std::sort(row.begin(), row.end());
        for (auto &x : row) { c.push_back(x.first); w.push_back(x.second); }
        r.push_back((int)c.size());
      }
      rp = put(r);
      cp = put(c);
      vi = put(w);
    };
    csr(imu, h.imu_rp, h.imu_cp, h.imu_vi);
    csr(inu, h.inu_rp, h.inu_cp, h.inu_vi);
    csr(bb, h.bb_rp, h.bb_cp, h.bb_vi);
    std::sort(ib.begin(), ib.end(), [](const std::array<int, 3> &a, const std::array<int, 3> &b) {
      return a[1] != b[1] ? a[1] < b[1] : a[0] < b[0];
    });
    std::vector<int> ri, ci, vv, yr, yc, yv;
    for (const auto &x : ib) {
      if (yr.empty() || yr.back() != x[1]) {
        yr.push_back(x[1]);
        yc.push_back((int)yc.size());
        yv.push_back(-1);
      }
      ri.push_back(x[0]);
      ci.push_back((int)yc.size() - 1);
      vv.push_back(x[2]);
    }
    h.nib = (int)ri.size();
    h.ncr = (int)yr.size();
    h.ib_ri = put(ri); h.ib_ci = put(ci); h.ib_vi = put(vv);
    h.yb_ri = put(yr); h.yb_ci = put(yc); h.yb_vi = put(yv);
    h.bchild = put(bchild); h.bcpos = put(bcp); h.gid = put(gid);
    h.smu = put(smu); h.snu = put(snu); h.p1mu = put(p1mu); h.p1nu = put(p1nu);
    for (int v : mu.B) own[v] = -1;
    for (int v : nu.B) own[v] = -1;
    P.hsym.push_back(h);
  }
  if (pool.empty()) pool.push_back(0);
  upload(P.hsym_pool, pool);
}

}  // namespace

hssx_fact_::~hssx_fact_() {
  hssx::destroy_graphs(*this);
  if (cap_stream) (void)hipStreamDestroy(cap_stream);
}

namespace {
hssx_status dads(hssx_op A, int nrhs, const void *lambda_dev, const void *x_dev, double *grad_dev,
                 int conj_lam, void *stream) {
  return guarded([&] {
    HSSX_CHECK(A && lambda_dev && x_dev && grad_dev && nrhs >= 1, HSSX_EINVAL, "invalid argument");
    HSSX_CHECK(A->dofs == 1 && A->mesh == kMeshCG, HSSX_EINVAL,
               "the slowness gradient is defined for P1 Helmholtz operators");
    DeviceScope ds(A->device);
    AllocScope as_(A->ctx, stream);
    for (size_t q = 0; q < A->part_N.size(); ++q) {
      const int o = A->part_off[q];
      launch_dads(A->part_N[q], A->part_omega[q], A->s.as<double>() + o, nrhs,
                  (const c128 *)lambda_dev + o, (const c128 *)x_dev + o, A->n, grad_dev + o,
                  conj_lam, S(stream));
    }
  });
}
}  // namespace

extern "C" {

const char *hssx_last_error(void) { return g_err.c_str(); }

hssx_status hssx_assemble(int device, const hssx_problem_desc *desc, const double *s_dev,
                          void *stream, hssx_op *A_out) {
  return guarded([&] {
    HSSX_CHECK(desc && A_out && s_dev, HSSX_EINVAL, "null argument");
    // 32-bit CSR offsets: nnz < 7 N^2 must stay below 2^31
    HSSX_CHECK(desc->N >= 2 && desc->N <= 17000, HSSX_EINVAL, "N out of range");
    HSSX_CHECK(std::isfinite(desc->omega) && desc->omega >= 0, HSSX_EINVAL, "omega");
    *A_out = nullptr;
    DeviceScope ds(device);
    AllocScope as_(g_bound, stream);
    auto A = std::make_unique<hssx_op_>();
    A->device = device;
    A->ctx = g_bound;
    A->N = desc->N;
    A->omega = desc->omega;
    const int N = desc->N, n = N * N;
    A->n = n;
    // fixed 7-point pattern, sorted columns
    A->h_rowptr.resize(n + 1);
    A->h_col.reserve((size_t)7 * n);
    A->h_rowptr[0] = 0;
    static const int ox[7] = {-1, 0, -1, 0, 1, 0, 1}, oy[7] = {-1, -1, 0, 0, 0, 1, 1};
    for (int i = 0; i < n; ++i) {
      int x = i % N, y = i / N;
      for (int t = 0; t < 7; ++t) {
        int u = x + ox[t], v = y + oy[t];
        if (u >= 0 && v >= 0 && u < N && v < N) A->h_col.push_back(v * N + u);
      }
      A->h_rowptr[i + 1] = (int)A->h_col.size();
    }
    A->nnz = (long)A->h_col.size();
    upload(A->rowptr, A->h_rowptr);
    upload(A->col, A->h_col);
    A->val.alloc(A->nnz * sizeof(c128));
    A->mval.alloc(A->nnz * sizeof(double));
    A->s.alloc((size_t)n * sizeof(double));
    HSSX_HIP(hipMemcpyAsync(A->s.p, s_dev, (size_t)n * sizeof(double), hipMemcpyDeviceToDevice, S(stream)));
    launch_assemble(N, desc->omega, A->s.as<double>(), A->rowptr.as<int>(), A->col.as<int>(),
                    A->val.as<c128>(), A->mval.as<double>(), S(stream));
    A->part_N = {N};
    A->part_omega = {desc->omega};
    A->part_off = {0, n};
    upload(A->part_off_dev, A->part_off);
    HSSX_HIP(hipStreamSynchronize(S(stream)));
    *A_out = A.release();
  });
}

hssx_status hssx_assemble_elastic(int device, const hssx_problem_desc *desc, const double *lam_dev,
                                  const double *mu_dev, const double *rho_dev, void *stream,
                                  hssx_op *A_out) {
  return guarded([&] {
    HSSX_CHECK(desc && A_out && lam_dev && mu_dev && rho_dev, HSSX_EINVAL, "null argument");
    // 32-bit CSR offsets: nnz < 28 N^2 must stay below 2^31
    HSSX_CHECK(desc->N >= 2 && desc->N <= 8500, HSSX_EINVAL, "N out of range");
    HSSX_CHECK(std::isfinite(desc->omega) && desc->omega >= 0, HSSX_EINVAL, "omega");
    *A_out = nullptr;
    DeviceScope ds(device);
    AllocScope as_(g_bound, stream);
    hipStream_t st = S(stream);
    auto A = std::make_unique<hssx_op_>();
    A->device = device;
    A->ctx = g_bound;
    A->N = desc->N;
    A->omega = desc->omega;
    A->dofs = 2;
    A->row_max = 14;
    const int N = desc->N, nn = N * N, n = 2 * nn;
    A->n = n;
    // 2 x 2 blocks of the 7-point node stencil, columns sorted
    A->h_rowptr.resize(n + 1);
    A->h_col.reserve((size_t)14 * n);
    A->h_rowptr[0] = 0;
    static const int ox[7] = {-1, 0, -1, 0, 1, 0, 1}, oy[7] = {-1, -1, 0, 0, 0, 1, 1};
    for (int r = 0; r < n; ++r) {
      const int v = r / 2, x = v % N, y = v / N;
      for (int t = 0; t < 7; ++t) {
        int u = x + ox[t], w = y + oy[t];
        if (u >= 0 && w >= 0 && u < N && w < N) {
          A->h_col.push_back(2 * (w * N + u));
          A->h_col.push_back(2 * (w * N + u) + 1);
        }
      }
      A->h_rowptr[r + 1] = (int)A->h_col.size();
    }
    A->nnz = (long)A->h_col.size();
    upload(A->rowptr, A->h_rowptr);
    upload(A->col, A->h_col);
    A->val.alloc(A->nnz * sizeof(c128));
    A->mval.alloc(A->nnz * sizeof(double));
    // material fields kept as [lam; mu; rho]
    A->s.alloc((size_t)3 * nn * sizeof(double));
    double *f = A->s.as<double>();
    HSSX_HIP(hipMemcpyAsync(f, lam_dev, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
    HSSX_HIP(hipMemcpyAsync(f + nn, mu_dev, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
    HSSX_HIP(hipMemcpyAsync(f + 2 * nn, rho_dev, nn * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_assemble_elastic(N, desc->omega, f, f + nn, f + 2 * nn, A->rowptr.as<int>(),
                            A->col.as<int>(), A->val.as<c128>(), A->mval.as<double>(), st);
    A->part_N = {N};
    A->part_omega = {desc->omega};
    A->part_off = {0, n};
    upload(A->part_off_dev, A->part_off);
    HSSX_HIP(hipStreamSynchronize(st));
    *A_out = A.release();
  });
}

namespace {

// the SIPG operators of hssx_assemble_dg and hssx_assemble_ipdg
hssx_status assemble_sipg(int device, int Nc, int deg, int bc, double omega, const double *s_dev,
                          void *stream, hssx_op *A_out) {
  return guarded([&] {
    HSSX_CHECK(A_out && s_dev, HSSX_EINVAL, "null argument");
    HSSX_CHECK(deg == 1 || deg == 2, HSSX_EINVAL, "polynomial degree must be 1 or 2");
    HSSX_CHECK(bc == HSSX_BC_ABSORBING || bc == HSSX_BC_DIRICHLET, HSSX_EINVAL,
               "boundary condition");
    const int nb = deg == 1 ? 3 : 6;
    // 32-bit CSR offsets: nnz < 8 nb^2 Nc^2 must stay below 2^31
    HSSX_CHECK(Nc >= 1 && Nc <= (deg == 1 ? 5400 : 2700), HSSX_EINVAL, "cell count out of range");
    HSSX_CHECK(std::isfinite(omega) && omega >= 0, HSSX_EINVAL, "omega");
    *A_out = nullptr;
    DeviceScope ds(device);
    AllocScope as_(g_bound, stream);
    hipStream_t st = S(stream);
    auto A = std::make_unique<hssx_op_>();
    A->device = device;
    A->ctx = g_bound;
    A->N = Nc;
    A->omega = omega;
    A->dofs = nb;
    A->mesh = kMeshDG;
    A->row_max = 4 * nb;
    const int ne = 2 * Nc * Nc, n = nb * ne, nv = (Nc + 1) * (Nc + 1);
    A->n = n;
    // nb x nb blocks of each triangle with itself and its face neighbours,
    // neighbour elements in increasing id (columns sorted)
    A->h_rowptr.resize(n + 1);
    A->h_col.reserve((size_t)4 * nb * n);
    A->h_rowptr[0] = 0;
    for (int e = 0; e < ne; ++e) {
      const int c = e >> 1, t = e & 1, i = c % Nc, j = c / Nc;
      int el[4], k = 0;
      el[k++] = e;
      el[k++] = t == 0 ? e + 1 : e - 1;
      if (t == 0) {
        if (j > 0) el[k++] = 2 * ((j - 1) * Nc + i) + 1;
        if (i < Nc - 1) el[k++] = 2 * (j * Nc + i + 1) + 1;
      } else {
        if (j < Nc - 1) el[k++] = 2 * ((j + 1) * Nc + i);
        if (i > 0) el[k++] = 2 * (j * Nc + i - 1);
      }
      std::sort(el, el + k);
      for (int a = 0; a < nb; ++a) {
        for (int q = 0; q < k; ++q)
          for (int b = 0; b < nb; ++b) A->h_col.push_back(nb * el[q] + b);
        A->h_rowptr[nb * e + a + 1] = (int)A->h_col.size();
      }
    }
    A->nnz = (long)A->h_col.size();
    upload(A->rowptr, A->h_rowptr);
    upload(A->col, A->h_col);
    A->val.alloc(A->nnz * sizeof(c128));
    A->mval.alloc(A->nnz * sizeof(double));
    A->s.alloc((size_t)nv * sizeof(double));
    HSSX_HIP(hipMemcpyAsync(A->s.p, s_dev, nv * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_assemble_dg(Nc, deg, bc == HSSX_BC_DIRICHLET, omega, A->s.as<double>(),
                       A->rowptr.as<int>(), A->col.as<int>(), A->val.as<c128>(),
                       A->mval.as<double>(), st);
    A->part_N = {Nc};
    A->part_omega = {omega};
    A->part_off = {0, n};
    upload(A->part_off_dev, A->part_off);
    HSSX_HIP(hipStreamSynchronize(st));
    *A_out = A.release();
  });
}

}  // namespace

hssx_status hssx_assemble_dg(int device, const hssx_problem_desc *desc, const double *s_dev,
                             void *stream, hssx_op *A_out) {
  if (!desc) return guarded([] { throw Error(HSSX_EINVAL, "null argument"); });
  return assemble_sipg(device, desc->N, 2, HSSX_BC_ABSORBING, desc->omega, s_dev, stream, A_out);
}

hssx_status hssx_assemble_ipdg(int device, const hssx_ipdg_desc *desc, const double *s_dev,
                               void *stream, hssx_op *A_out) {
  if (!desc) return guarded([] { throw Error(HSSX_EINVAL, "null argument"); });
  return assemble_sipg(device, desc->N, desc->p, desc->bc, desc->omega, s_dev, stream, A_out);
}

hssx_status hssx_op_batch(int count, const hssx_op *parts, void *stream, hssx_op *A_out) {
  return guarded([&] {
    HSSX_CHECK(parts && A_out && count >= 1, HSSX_EINVAL, "invalid argument");
    *A_out = nullptr;
    long n = 0, nnz = 0;
    for (int q = 0; q < count; ++q) {
      HSSX_CHECK(parts[q] && parts[q]->part_N.size() == 1, HSSX_EINVAL,
                 "batch parts must be single-problem operators");
      HSSX_CHECK(parts[q]->device == parts[0]->device, HSSX_EINVAL, "parts on different devices");
      HSSX_CHECK(parts[q]->dofs == 1 && parts[q]->mesh == kMeshCG, HSSX_EINVAL,
                 "batches hold P1 Helmholtz problems");
      n += parts[q]->n;
      nnz += parts[q]->nnz;
    }
    HSSX_CHECK(n < (1L << 31) && nnz < (1L << 31), HSSX_EINVAL, "batch too large for 32-bit indices");
    DeviceScope ds(parts[0]->device);
    AllocScope as_(g_bound, stream);
    hipStream_t st = S(stream);
    auto A = std::make_unique<hssx_op_>();
    A->device = parts[0]->device;
    A->ctx = g_bound;
    A->n = (int)n;
    A->nnz = nnz;
    A->h_rowptr.reserve(n + 1);
    A->h_col.reserve(nnz);
    A->h_rowptr.push_back(0);
    A->part_off.push_back(0);
    std::vector<int> row_part;
    row_part.reserve(n);
    for (int q = 0; q < count; ++q) {
      const hssx_op_ &B = *parts[q];
      const int r0 = A->part_off.back(), e0 = (int)A->h_col.size();
      for (int i = 0; i < B.n; ++i) A->h_rowptr.push_back(e0 + B.h_rowptr[i + 1]);
      for (int c : B.h_col) A->h_col.push_back(r0 + c);
      A->part_N.push_back(B.N);
      A->part_omega.push_back(B.omega);
      A->part_off.push_back(r0 + B.n);
      row_part.insert(row_part.end(), B.n, q);
    }
    upload(A->rowptr, A->h_rowptr);
    upload(A->col, A->h_col);
    upload(A->part_off_dev, A->part_off);
    upload(A->row_part_dev, row_part);
    A->val.alloc(nnz * sizeof(c128));
    A->mval.alloc(nnz * sizeof(double));
    A->s.alloc(n * sizeof(double));
    for (int q = 0; q < count; ++q) {
      const hssx_op_ &B = *parts[q];
      const long e0 = A->h_rowptr[A->part_off[q]], r0 = A->part_off[q];
      HSSX_HIP(hipMemcpyAsync(A->val.as<c128>() + e0, B.val.p, B.nnz * sizeof(c128),
                              hipMemcpyDeviceToDevice, st));
      HSSX_HIP(hipMemcpyAsync(A->mval.as<double>() + e0, B.mval.p, B.nnz * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
      HSSX_HIP(hipMemcpyAsync(A->s.as<double>() + r0, B.s.p, B.n * sizeof(double),
                              hipMemcpyDeviceToDevice, st));
    }
    HSSX_HIP(hipStreamSynchronize(st));
    *A_out = A.release();
  });
}

hssx_status hssx_op_info(hssx_op A, int *n, int *parts, int32_t *part_off) {
  return guarded([&] {
    HSSX_CHECK(A, HSSX_EINVAL, "null operator");
    if (n) *n = A->n;
    if (parts) *parts = (int)A->part_N.size();
    if (part_off) std::memcpy(part_off, A->part_off.data(), A->part_off.size() * sizeof(int));
  });
}

hssx_status hssx_load(hssx_op A, int nrhs, const double *f_dev, long ldf, void *b_dev, long ldb,
                      void *stream) {
  return guarded([&] {
    HSSX_CHECK(A && f_dev && b_dev && nrhs >= 1 && ldf >= A->n && ldb >= A->n, HSSX_EINVAL,
               "invalid argument");
    DeviceScope ds(A->device);
    AllocScope as_(A->ctx, stream);
    launch_load(A->n, nrhs, A->rowptr.as<int>(), A->col.as<int>(), A->mval.as<double>(), f_dev, ldf,
                (c128 *)b_dev, ldb, S(stream));
  });
}

hssx_status hssx_matvec(hssx_op A, int trans, int nrhs, const void *x_dev, long ldx, void *y_dev,
                        long ldy, void *stream) {
  return guarded([&] {
    HSSX_CHECK(A && x_dev && y_dev && nrhs >= 1 && ldx >= A->n && ldy >= A->n, HSSX_EINVAL,
               "invalid argument");
    HSSX_CHECK(x_dev != y_dev, HSSX_EINVAL, "matvec output may not alias its input");
    (void)trans;   // A^T = A
    DeviceScope ds(A->device);
    AllocScope as_(A->ctx, stream);
    launch_spmv(A->n, nrhs, A->rowptr.as<int>(), A->col.as<int>(), A->val.as<c128>(),
                (const c128 *)x_dev, ldx, (c128 *)y_dev, ldy, A->row_max, S(stream));
  });
}

hssx_status hssx_get_csr(hssx_op A, int32_t *rowptr, int32_t *col, double *val, long *nnz_out,
                         void *stream) {
  return guarded([&] {
    HSSX_CHECK(A, HSSX_EINVAL, "null operator");
    DeviceScope ds(A->device);
    AllocScope as_(A->ctx, stream);
    HSSX_HIP(hipStreamSynchronize(S(stream)));
    if (nnz_out) *nnz_out = A->nnz;
    if (rowptr) std::memcpy(rowptr, A->h_rowptr.data(), (A->n + 1) * sizeof(int));
    if (col) std::memcpy(col, A->h_col.data(), A->nnz * sizeof(int));
    if (val) HSSX_HIP(hipMemcpy(val, A->val.p, A->nnz * sizeof(c128), hipMemcpyDeviceToHost));
  });
}

hssx_status hssx_factor(hssx_op A, double tol, int leaf_size, const hssx_factor_opts *opts,
                        void *stream, hssx_fact *P_out) {
  return guarded([&] {
    HSSX_CHECK(A && P_out, HSSX_EINVAL, "null argument");
    HSSX_CHECK(tol > 0 && tol < 1, HSSX_EINVAL, "tol must lie in (0, 1)");
    HSSX_CHECK(leaf_size >= 1, HSSX_EINVAL, "leaf_size must be >= 1");
    *P_out = nullptr;
    hssx_factor_opts o{16, 4, 32, 16, 32, HSSX_C128, 0u, 0.0, 1, 1, 0, 0, 0, 0};
    if (opts) o = *opts;
    HSSX_CHECK(o.beta >= 1 && o.k0 >= 1 && o.r >= 1 && o.r <= 64 && o.max_rounds >= 1,
               HSSX_EINVAL, "invalid factor options");
    HSSX_CHECK(o.dtype == HSSX_C128 || o.dtype == HSSX_C64, HSSX_EINVAL, "dtype");
    HSSX_CHECK(o.sample_bf16 >= 0 && o.sample_bf16 <= 2, HSSX_EINVAL, "sample_bf16 must be 0, 1 or 2");
    HSSX_CHECK(leaf_size >= A->dofs && o.beta >= A->dofs, HSSX_EINVAL,
               "leaf and HSS leaf sizes must hold one grid node's unknowns");
    HSSX_CHECK(!o.sample_bf16 || o.dtype == HSSX_C64, HSSX_EINVAL,
               "bf16 sampling needs a complex64 factor");
    HSSX_CHECK(!o.wide_inverse || o.dtype == HSSX_C64, HSSX_EINVAL,
               "wide_inverse applies to complex64 factors");
    DeviceScope ds(A->device);
    AllocScope as_(g_bound, stream);
    hipStream_t st = S(stream);
    auto P = std::make_unique<hssx_fact_>();
    P->A = A;
    P->ctx = g_bound;
    P->device = A->device;
    P->pattern = A->pattern_key();
    P->dtype = o.dtype;
    P->tol = tol;
    P->leaf = leaf_size;
    P->opts = o;
    auto t0 = std::chrono::steady_clock::now();
    if (A->part_N.size() == 1) {
      P->sym = build_symbolic(A->part_N[0], leaf_size, o.beta,
                              std::min(16, (int)std::thread::hardware_concurrency()), A->dofs,
                              A->mesh);
    } else {
      // the problems' analyses are independent: run them on host threads
      const int np = (int)A->part_N.size();
      std::vector<Symbolic> parts(np);
      std::atomic<int> next{0};
      std::exception_ptr fail;
      std::mutex mu;
      auto work = [&] {
        try {
          for (int q; (q = next++) < np;) parts[q] = build_symbolic(A->part_N[q], leaf_size, o.beta);
        } catch (...) {
          std::lock_guard<std::mutex> g(mu);
          fail = std::current_exception();
        }
      };
      const int nt = std::max(1, std::min(np, std::min(16, (int)std::thread::hardware_concurrency())));
      std::vector<std::thread> pool;
      for (int t = 1; t < nt; ++t) pool.emplace_back(work);
      work();
      for (auto &t : pool) t.join();
      if (fail) std::rethrow_exception(fail);
      P->sym = merge_forest(std::move(parts), A->part_off);
    }
    const Symbolic &sym = P->sym;
    const int nn = (int)sym.nodes.size();
    auto ts = std::chrono::steady_clock::now();
    P->arith.assign(nn, 0);
    P->comp.assign(nn, 0);
    HSSX_CHECK(o.switch_size >= 0, HSSX_EINVAL, "switch_size must be >= 0");
    if (o.switch_size > 0) {
      // size rule: a separator of at least switch_size DOFs, or a child with
      // HSS arithmetic (post-order: children first), keeps the classes
      // monotone up the tree
      for (int k = 0; k < nn; ++k) {
        const NDNode &nd = sym.nodes[k];
        if (nd.leafnode() || o.h_sw < 0) continue;
        P->arith[k] = (int)nd.I.size() >= o.switch_size || P->arith[nd.lo] || P->arith[nd.hi];
      }
    } else {
      for (int k = 0; k < nn; ++k) P->arith[k] = o.h_sw >= 0 && sym.nodes[k].height > o.h_sw;
    }
    for (int k = 0; k < nn; ++k) P->comp[k] = sym.nodes[k].parent >= 0 && P->arith[sym.nodes[k].parent];
    P->node_rank.assign(nn, 0);
    // HSS-class nodes: HSS arithmetic and not a root (a root factors its
    // dense A_ii); they keep no dense front
    P->hss_idx.assign(nn, -1);
    int n_hss = 0;
    for (int k = 0; k < nn; ++k)
      if (P->arith[k] && sym.nodes[k].parent >= 0 && !sym.nodes[k].leafnode()) P->hss_idx[k] = n_hss++;

    // descriptors (sizes and offsets, one pass over the nodes)
    std::vector<FrontDesc> dsc(nn);
    // complex64 factors keep the roots' fronts in complex128, in a buffer of
    // their own (offsets roff)
    const bool split_roots = o.dtype == HSSX_C64;
    long foff = 0, roff = 0, boff = 0, soff = 0;
    double fbytes = 0, flops = 0;   // of the exact multifrontal factorization
    const size_t esz_pool = o.dtype == HSSX_C128 ? sizeof(c128) : sizeof(c64);
    for (int k = 0; k < nn; ++k) {
      const NDNode &nd = sym.nodes[k];
      FrontDesc &d = dsc[k];
      d.ni = (int)nd.I.size();
      d.nb = (int)nd.B.size();
      d.f = d.ni + d.nb;
      const bool in64 = split_roots && nd.parent < 0;
      long &off = in64 ? roff : foff;
      if (P->hss_idx[k] < 0) {
        d.foff = off;
        off += (long)d.f * (d.f + d.ni);
      } else if (P->hss_idx[nd.parent] < 0) {
        // HSS-class child of a dense parent: only its Schur block S (ld f),
        // the expansion the parent's front assembly reads
        d.foff = off - d.ni - (long)d.ni * d.f;
        off += (long)d.f * d.nb;
      } else {
        d.foff = 0;
      }
      d.ioff = nd.offset;
      d.bpos_off = (int)boff;
      boff += d.nb;
      HSSX_CHECK(soff + d.f < (1L << 31), HSSX_EINVAL, "front index space exceeds 32 bits");
      d.src_off = (int)soff;
      soff += d.f;
      d.lo = nd.lo;
      d.hi = nd.hi;
      fbytes += ((double)d.ni * d.ni + 2.0 * d.ni * d.nb) * (in64 ? sizeof(c128) : esz_pool);
      // Gauss-Jordan on f rows x (f + ni) columns, complex multiply-add = 8 flops:
      // sum over pivots p < ni of (f - 1)(f + ni - p - 1)
      flops += 8.0 * (d.f - 1) * ((double)d.ni * (d.f + d.ni - 1) - 0.5 * d.ni * (d.ni - 1.0));
    }
    // front-entry sources: node id, and (child, position in the child's B)
    // packed as 2 pos + child (-1: entry of A); parts filled on host threads
    std::vector<int> bpos(boff), sg(soff), scode(soff);
    const int nparts = (int)sym.part_nodes.size() - 1;
    {
      std::atomic<int> next{0};
      std::exception_ptr fail;
      std::mutex mu;
      auto work = [&] {
        try {
          std::vector<int> owner, opos;
          for (int q; (q = next++) < nparts;) {
            const int k0 = sym.part_nodes[q], k1 = sym.part_nodes[q + 1];
            const int v0 = A->part_off[q], nv = A->part_off[q + 1] - v0;
            owner.assign(nv, -1);
            opos.assign(nv, -1);
            for (int k = k0; k < k1; ++k) {
              const NDNode &nd = sym.nodes[k];
              const FrontDesc &d = dsc[k];
              for (int b = 0; b < d.nb; ++b) bpos[d.bpos_off + b] = sym.iperm[nd.B[b]];
              const bool leaf = nd.leafnode();
              if (!leaf) {
                const NDNode &lo = sym.nodes[nd.lo], &hi = sym.nodes[nd.hi];
                for (size_t b = 0; b < lo.B.size(); ++b) { owner[lo.B[b] - v0] = 0; opos[lo.B[b] - v0] = (int)b; }
                for (size_t b = 0; b < hi.B.size(); ++b) { owner[hi.B[b] - v0] = 1; opos[hi.B[b] - v0] = (int)b; }
              }
              long e = d.src_off;
              auto put = [&](int v) {
                sg[e] = v;
                if (leaf) {
                  scode[e] = -1;
                } else {
                  HSSX_CHECK(owner[v - v0] >= 0, HSSX_EINVAL,
                             "front entry outside the children's boundaries");
                  scode[e] = 2 * opos[v - v0] + owner[v - v0];
                }
                ++e;
              };
              for (int v : nd.I) put(v);
              for (int v : nd.B) put(v);
              if (!leaf) {
                for (int v : sym.nodes[nd.lo].B) owner[v - v0] = -1;
                for (int v : sym.nodes[nd.hi].B) owner[v - v0] = -1;
              }
            }
          }
        } catch (...) {
          std::lock_guard<std::mutex> g(mu);
          fail = std::current_exception();
        }
      };
      const int nt = std::max(1, std::min(nparts, std::min(16, (int)std::thread::hardware_concurrency())));
      std::vector<std::thread> pool;
      for (int t = 1; t < nt; ++t) pool.emplace_back(work);
      work();
      for (auto &t : pool) t.join();
      if (fail) std::rethrow_exception(fail);
    }
    P->h_desc = dsc;
    upload(P->desc, dsc);
    upload(P->bpos, bpos);
    upload(P->src_gid, sg);
    upload(P->src_code, scode);
    upload(P->perm, sym.perm);
    build_hss_sym(*P, *A);
    P->depth_nodes.assign(sym.max_depth + 1, {});
    P->dense_nodes.assign(sym.max_depth + 1, {});
    P->hss_nodes.assign(sym.max_depth + 1, {});
    for (int k = 0; k < nn; ++k) {
      P->depth_nodes[sym.nodes[k].depth].push_back(k);
      (P->hss_idx[k] < 0 ? P->dense_nodes : P->hss_nodes)[sym.nodes[k].depth].push_back(k);
    }
    P->depth_dev.resize(sym.max_depth + 1);
    P->depth_max_ni.assign(sym.max_depth + 1, 0);
    P->depth_max_nb.assign(sym.max_depth + 1, 0);
    P->depth_max_f.assign(sym.max_depth + 1, 0);
    const int D1 = sym.max_depth + 1;
    P->up_fbytes.assign(D1, 0); P->up_velems.assign(D1, 0);
    P->down_fbytes.assign(D1, 0); P->down_velems.assign(D1, 0); P->asm_bytes.assign(D1, 0);
    for (int d = 0; d <= sym.max_depth; ++d) {
      upload(P->depth_dev[d], P->dense_nodes[d]);
      for (int k : P->dense_nodes[d]) {
        const FrontDesc &q = dsc[k];
        const size_t esz = split_roots && sym.nodes[k].parent < 0 ? sizeof(c128) : esz_pool;
        P->depth_max_ni[d] = std::max(P->depth_max_ni[d], q.ni);
        P->depth_max_nb[d] = std::max(P->depth_max_nb[d], q.nb);
        P->depth_max_f[d] = std::max(P->depth_max_f[d], q.f);
        if (q.ni) {
          P->up_fbytes[d] += (double)q.f * q.ni * esz;          // [A_ii^-1; L]
          P->up_velems[d] += 2.0 * q.ni + 2.0 * q.nb;           // t in, x(I) out, x(B) rw
          if (q.nb) {
            P->down_fbytes[d] += (double)q.ni * q.nb * esz;     // R
            P->down_velems[d] += q.nb + 2.0 * q.ni;             // x(B) in, x(I) rw
          }
        }
        P->asm_bytes[d] += (double)q.f * (q.f + q.ni) * esz;
      }
    }
    P->front.alloc(std::max(1L, foff) * esz_pool);
    if (split_roots) P->front64.alloc(std::max(1L, roff) * sizeof(c128));
    auto t1 = std::chrono::steady_clock::now();
    P->stats.ms_symbolic = std::chrono::duration<double, std::milli>(ts - t0).count();
    P->stats.ms_setup = std::chrono::duration<double, std::milli>(t1 - ts).count();
    P->stats.n = A->n;
    P->stats.nodes = nn;
    P->stats.depth = sym.max_depth;
    int nh = 0;
    for (int k = 0; k < nn; ++k) nh += P->arith[k];
    P->stats.n_hss_nodes = nh;
    P->stats.factor_bytes = fbytes;
    P->stats.factor_flops = flops;
    P->stats.exact_factor_bytes = fbytes;
    P->stats.exact_factor_flops = flops;
    factor_numeric(*P, st);
    *P_out = P.release();
  });
}

hssx_status hssx_refactor(hssx_fact P, hssx_op A, void *stream) {
  return guarded([&] {
    HSSX_CHECK(P && A, HSSX_EINVAL, "null argument");
    HSSX_CHECK(P->desc.p != nullptr, HSSX_EINVAL, "handle holds no factorization");
    HSSX_CHECK(A->pattern_key() == P->pattern, HSSX_EINVAL,
               "refactor needs an operator with the factor's pattern (same grids and kind)");
    DeviceScope ds(A->device);
    AllocScope as_(P->ctx, stream);
    P->A = A;
    P->stats.ms_symbolic = 0;
    P->stats.ms_setup = 0;
    std::fill(P->node_rank.begin(), P->node_rank.end(), 0);
    factor_numeric(*P, S(stream));
  });
}

hssx_status hssx_apply(hssx_fact P, int trans, int nrhs, const void *x_dev, long ldx, void *y_dev,
                       long ldy, void *stream) {
  return guarded([&] {
    HSSX_CHECK(P && x_dev && y_dev && nrhs >= 1 && ldx >= P->A->n && ldy >= P->A->n, HSSX_EINVAL,
               "invalid argument");
    DeviceScope ds(P->A->device);
    AllocScope as_(P->ctx, stream);
    hssx::apply(*P, trans ? 1 : 0, nrhs, (const c128 *)x_dev, ldx, (c128 *)y_dev, ldy, S(stream));
  });
}

hssx_status hssx_apply_noalloc(hssx_fact P, int trans, int nrhs, const void *x_dev, long ldx,
                               void *y_dev, long ldy, void *stream) {
  return guarded([&] {
    HSSX_CHECK(P && P->A && x_dev && y_dev && nrhs >= 1 && ldx >= P->A->n && ldy >= P->A->n,
               HSSX_EINVAL, "invalid argument");
    HSSX_CHECK(P->desc.p != nullptr, HSSX_EINVAL, "handle holds no factorization");
    DeviceScope ds(P->device);
    AllocScope as_(P->ctx, stream);
    size_t bytes = 0;
    char *ws = noalloc_workspace(&bytes);
    apply_workspace(*P, trans ? 1 : 0, nrhs, (const c128 *)x_dev, ldx, (c128 *)y_dev, ldy,
                    S(stream), ws, bytes);
  });
}

hssx_status hssx_gmres_solve(hssx_op A, hssx_fact P, int trans, int nrhs, const void *b_dev,
                             long ldb, void *x_dev, long ldx, const hssx_gmres_opts *opts,
                             hssx_gmres_stats *stats, void *stream) {
  hssx_status st = guarded([&] {
    HSSX_CHECK(A && b_dev && x_dev && nrhs >= 1 && ldb >= A->n && ldx >= A->n, HSSX_EINVAL,
               "invalid argument");
    HSSX_CHECK(!P || P->A == A, HSSX_EINVAL, "preconditioner built for another operator");
    hssx_gmres_opts o{50, 1e-8, 1000, 0};
    if (opts) o = *opts;
    HSSX_CHECK(o.m >= 1 && o.m <= 500 && o.tol > 0 && o.maxit >= 1, HSSX_EINVAL, "gmres options");
    HSSX_CHECK(trans >= 0 && trans <= 2, HSSX_EINVAL, "trans must be 0, 1 or 2");
    DeviceScope ds(A->device);
    AllocScope as_(P ? P->ctx : A->ctx, stream);
    gmres(*A, P, trans, nrhs, (const c128 *)b_dev, ldb, (c128 *)x_dev, ldx, o, stats,
          S(stream));
  });
  if (st == HSSX_OK && stats) {
    const int nseg = nrhs * (int)A->part_N.size();
    for (int r = 0; r < nseg; ++r)
      if (!stats[r].converged) { g_err = "GMRES did not reach the tolerance"; return HSSX_ENOCONV; }
  }
  return st;
}

hssx_status hssx_dAds_contract(hssx_op A, int nrhs, const void *lambda_dev, const void *x_dev,
                               double *grad_dev, void *stream) {
  return dads(A, nrhs, lambda_dev, x_dev, grad_dev, 0, stream);
}

hssx_status hssx_dAds_contract_adjoint(hssx_op A, int nrhs, const void *mu_dev, const void *x_dev,
                                       double *grad_dev, void *stream) {
  return dads(A, nrhs, mu_dev, x_dev, grad_dev, 1, stream);
}



hssx_status hssx_analyze(int N, int dofs, int leaf_size, int beta, hssx_fact *P_out) {
  return guarded([&] {
    HSSX_CHECK(P_out && N >= 2 && (dofs == 1 || dofs == 2) && (long)N * N * dofs < (1L << 31) &&
                   leaf_size >= dofs && beta >= dofs,
               HSSX_EINVAL, "invalid argument");
    *P_out = nullptr;
    auto P = std::make_unique<hssx_fact_>();
    P->leaf = leaf_size;
    P->opts.beta = beta;
    P->sym = build_symbolic(N, leaf_size, beta, std::min(16, (int)std::thread::hardware_concurrency()),
                            dofs);
    *P_out = P.release();
  });
}

hssx_status hssx_analyze_ipdg(int Nc, int p, int leaf_size, int beta, hssx_fact *P_out) {
  return guarded([&] {
    const int nb = p == 1 ? 3 : 6;
    HSSX_CHECK(P_out && (p == 1 || p == 2) && Nc >= 1 && Nc <= (p == 1 ? 5400 : 2700) &&
                   leaf_size >= nb && beta >= nb,
               HSSX_EINVAL, "invalid argument");
    *P_out = nullptr;
    auto P = std::make_unique<hssx_fact_>();
    P->leaf = leaf_size;
    P->opts.beta = beta;
    P->sym = build_symbolic(Nc, leaf_size, beta, std::min(16, (int)std::thread::hardware_concurrency()),
                            nb, kMeshDG);
    *P_out = P.release();
  });
}

hssx_status hssx_analyze_dg(int Nc, int leaf_size, int beta, hssx_fact *P_out) {
  return hssx_analyze_ipdg(Nc, 2, leaf_size, beta, P_out);
}

hssx_status hssx_get_perm(hssx_fact P, int32_t *perm_host, long n) {
  return guarded([&] {
    HSSX_CHECK(P && perm_host && n == (long)P->sym.perm.size(), HSSX_EINVAL, "invalid argument");
    std::memcpy(perm_host, P->sym.perm.data(), n * sizeof(int));
  });
}

hssx_status hssx_get_tree(hssx_fact P, int64_t *sizes, int32_t *node_info, int32_t *i_ids,
                          int32_t *i_ptr, int32_t *b_ids, int32_t *b_ptr, int32_t *clusters,
                          int32_t *c_ptr) {
  return guarded([&] {
    HSSX_CHECK(P && sizes, HSSX_EINVAL, "invalid argument");
    const auto &nodes = P->sym.nodes;
    long ti = 0, tb = 0, tc = 0;
    for (const auto &nd : nodes) { ti += nd.I.size(); tb += nd.B.size(); tc += nd.ct.count(); }
    sizes[0] = (int64_t)nodes.size();
    sizes[1] = ti;
    sizes[2] = tb;
    sizes[3] = tc;
    if (!node_info) return;
    HSSX_CHECK(i_ids && i_ptr && b_ids && b_ptr && clusters && c_ptr, HSSX_EINVAL, "null array");
    long pi = 0, pb = 0, pc = 0;
    for (size_t k = 0; k < nodes.size(); ++k) {
      const auto &nd = nodes[k];
      int32_t *ni = node_info + 10 * k;
      ni[0] = nd.x0; ni[1] = nd.x1; ni[2] = nd.y0; ni[3] = nd.y1; ni[4] = nd.lo; ni[5] = nd.hi;
      ni[6] = nd.parent; ni[7] = nd.depth; ni[8] = nd.height; ni[9] = nd.p0;
      i_ptr[k] = (int32_t)pi;
      for (int v : nd.I) i_ids[pi++] = v;
      b_ptr[k] = (int32_t)pb;
      for (int v : nd.B) b_ids[pb++] = v;
      c_ptr[k] = (int32_t)pc;
      for (int c = 0; c < nd.ct.count(); ++c, ++pc) {
        int32_t *cc = clusters + 5 * pc;
        cc[0] = nd.ct.start[c]; cc[1] = nd.ct.size[c]; cc[2] = nd.ct.left[c];
        cc[3] = nd.ct.right[c]; cc[4] = nd.ct.level[c];
      }
    }
    i_ptr[nodes.size()] = (int32_t)pi;
    b_ptr[nodes.size()] = (int32_t)pb;
    c_ptr[nodes.size()] = (int32_t)pc;
  });
}

hssx_status hssx_get_factor_stats(hssx_fact P, hssx_factor_stats *s) {
  return guarded([&] {
    HSSX_CHECK(P && s, HSSX_EINVAL, "invalid argument");
    *s = P->stats;
  });
}

hssx_status hssx_get_schur(hssx_fact P, int node, double *S_host, long ld) {
  return guarded([&] {
    HSSX_CHECK(P && S_host && node >= 0 && node < (int)P->h_desc.size(), HSSX_EINVAL,
               "invalid argument");
    const FrontDesc &d = P->h_desc[node];
    HSSX_CHECK(ld >= d.nb, HSSX_EINVAL, "ld < |B|");
    if (d.nb == 0) return;   // the root: no Schur complement
    DeviceScope ds(P->A->device);
    AllocScope as_(P->ctx, nullptr);
    HSSX_HIP(hipDeviceSynchronize());
    std::vector<c128> e;
    if (expand_schur(*P, node, e)) {   // compressed: expansion of its generators
      for (int j = 0; j < d.nb; ++j)
        for (int i = 0; i < d.nb; ++i) {
          S_host[2 * (i + (long)j * ld)] = e[i + (size_t)j * d.nb].re;
          S_host[2 * (i + (long)j * ld) + 1] = e[i + (size_t)j * d.nb].im;
        }
      return;
    }
    HSSX_CHECK(P->hss_idx.empty() || P->hss_idx[node] < 0, HSSX_EINVAL, "node keeps no Schur complement");
    const size_t esz = P->dtype == HSSX_C128 ? sizeof(c128) : sizeof(c64);
    std::vector<char> buf((size_t)d.f * (d.f + d.ni) * esz);
    HSSX_HIP(hipMemcpy(buf.data(), (char *)P->front.p + d.foff * esz, buf.size(),
                       hipMemcpyDeviceToHost));
    for (int j = 0; j < d.nb; ++j)
      for (int i = 0; i < d.nb; ++i) {
        long e = (d.ni + i) + (long)(d.ni + j) * d.f;
        double re, im;
        if (P->dtype == HSSX_C128) {
          c128 v;
          std::memcpy(&v, buf.data() + e * esz, esz);
          re = v.re; im = v.im;
        } else {
          c64 v;
          std::memcpy(&v, buf.data() + e * esz, esz);
          re = v.re; im = v.im;
        }
        S_host[2 * (i + (long)j * ld)] = re;
        S_host[2 * (i + (long)j * ld) + 1] = im;
      }
  });
}

hssx_status hssx_hss_eval(int device, hssx_dtype dtype, int m, int ncl, const int32_t *tree,
                          const int32_t *rank, const double *gens, int op, int nrhs,
                          const void *x_dev, void *y_dev, long nij, const int32_t *ij,
                          double *vals, void *stream) {
  return guarded([&] {
    HSSX_CHECK(m >= 1 && ncl >= 1 && tree && rank && gens && op >= 0 && op <= 5, HSSX_EINVAL,
               "invalid argument");
    const int base = op == 4 ? 1 : op == 5 ? 3 : op;
    HSSX_CHECK(base >= 2 || (nrhs >= 1 && x_dev && y_dev), HSSX_EINVAL, "vectors");
    HSSX_CHECK(base < 2 || (nij >= 0 && (nij == 0 || (ij && vals))), HSSX_EINVAL, "entry lists");
    HSSX_CHECK(dtype == HSSX_C128 || dtype == HSSX_C64, HSSX_EINVAL, "dtype");
    DeviceScope ds(device);
    AllocScope as_(g_bound, stream);
    hss_eval(dtype, m, ncl, tree, rank, gens, op, nrhs, x_dev, y_dev, nij, ij, vals, S(stream));
  });
}

hssx_status hssx_create(int device, const hssx_allocator *alloc, hssx_ctx *ctx_out) {
  return guarded([&] {
    HSSX_CHECK(ctx_out && alloc && alloc->alloc && alloc->free, HSSX_EINVAL, "invalid argument");
    int count = 0;
    HSSX_HIP(hipGetDeviceCount(&count));
    HSSX_CHECK(device >= 0 && device < count, HSSX_EINVAL, "no such device");
    auto c = std::make_unique<hssx_ctx_>();
    c->device = device;
    c->a = *alloc;
    *ctx_out = c.release();
  });
}

hssx_status hssx_bind(hssx_ctx ctx) {
  g_bound = ctx;
  return HSSX_OK;
}

hssx_status hssx_ctx_stats(hssx_ctx ctx, long *live_bytes, long *allocs, long *frees) {
  return guarded([&] {
    HSSX_CHECK(ctx, HSSX_EINVAL, "null context");
    if (live_bytes) *live_bytes = ctx->live_bytes;
    if (allocs) *allocs = ctx->allocs;
    if (frees) *frees = ctx->frees;
  });
}

void hssx_destroy(hssx_ctx ctx) {
  if (!ctx) return;
  if (g_bound == ctx) g_bound = nullptr;
  int prev = 0;
  const int d = ctx->device;
  const bool dev = hipGetDevice(&prev) == hipSuccess;
  if (dev && prev != d) (void)hipSetDevice(d);
  (void)hipDeviceSynchronize();
  {
    AllocScope as_(ctx, nullptr);
    ctx->arenas.clear();
    ctx->stagings.clear();
  }
  delete ctx;
  if (dev && prev != d) (void)hipSetDevice(prev);
}

hssx_status hssx_prof_enable(int on) {
  return guarded([&] { prof_enable(on != 0); });
}

hssx_status hssx_prof_query(const char *kernel, double *ms, long *launches, double *work) {
  return guarded([&] {
    HSSX_CHECK(kernel, HSSX_EINVAL, "null kernel name");
    prof_query(kernel, ms, launches, work);
  });
}

void hssx_fact_destroy(hssx_fact P) {
  if (P) {
    // the factor's own device id: the operator it refers to may already be
    // destroyed
    int prev = 0;
    const int d = P->device;
    const bool dev = hipGetDevice(&prev) == hipSuccess;
    if (dev && prev != d) (void)hipSetDevice(d);
    delete P;
    if (dev && prev != d) (void)hipSetDevice(prev);
  }
}
void hssx_op_destroy(hssx_op A) { delete A; }

}  // extern "C"
