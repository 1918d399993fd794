// Restarted GMRES for A x = b with the approximate factorization as
// preconditioner (eq. 1.2; Sec. 4: restarted GMRES stopped on the relative
// residual).  All systems advance together, each with its own Krylov basis;
// converged ones are frozen (their step count stops).  A system is one
// right-hand side of one problem: a batch of np problems with nrhs columns
// has np * nrhs systems, system r * np + p being part p of column r.
//
// Left preconditioning (paper): Arnoldi on P^-1 A, stop when
// ||P^-1 (b - A x)|| / ||P^-1 b|| <= target; then the true residual
// ||b - A x|| / ||b|| is checked and, while it is above tol, up to three
// more cycles run with the target scaled by the observed ratio.
// Flexible right preconditioning: z_j = P^-1 v_j, Arnoldi on A z_j, and the
// GMRES residual is the true residual.
// Orthogonalisation: classical Gram-Schmidt applied twice (CGS2).
#include <algorithm>
#include <cmath>

#include "engine.h"

namespace hssx {

namespace {

// scratch taken from the arena for the duration of one solve
struct Scr {
  void *p = nullptr;
  template <typename T> T *as() const { return reinterpret_cast<T *>(p); }
};

void gmres_impl(hssx_op_ &A, hssx_fact_ *P, int trans, int nrhs, const c128 *b, long ldb,
                c128 *x, long ldx, const hssx_gmres_opts &o, hssx_gmres_stats *stats,
                hipStream_t st, Arena &ar, Staging &stg) {
  const int n = A.n, m = o.m;
  const bool left = !o.flexible;
  const long blk = (long)n * nrhs;
  const Segs sg = A.segs();
  const int np = sg.np, nseg = np * nrhs;
  int maxlen = 0;
  for (int q = 0; q < np; ++q) maxlen = std::max(maxlen, A.part_off[q + 1] - A.part_off[q]);
  auto precond = [&](const c128 *in, c128 *out) {
    if (P) apply(*P, trans, nrhs, in, n, out, n, st);
    else HSSX_HIP(hipMemcpyAsync(out, in, blk * sizeof(c128), hipMemcpyDeviceToDevice, st));
  };
  auto matvec = [&](const c128 *in, c128 *out) {
    hipEvent_t pe = prof_begin(st);
    launch_spmv(n, nrhs, A.rowptr.as<int>(), A.col.as<int>(), A.val.as<c128>(), in, n, out, n,
                A.row_max, st);
    // CSR values + column indices once, row pointers, x read and y written per rhs
    prof_end("spmv", st, pe, A.nnz * 20.0 + (n + 1) * 4.0 + 2.0 * blk * sizeof(c128));
  };
  auto take = [&](size_t bytes) {
    Scr q;
    q.p = ar.get<char>(bytes);
    return q;
  };
  Scr V = take((size_t)(m + 1) * blk * sizeof(c128));
  Scr Z = left ? Scr{} : take((size_t)m * blk * sizeof(c128));
  Scr w = take(blk * sizeof(c128)), t1 = take(blk * sizeof(c128));
  Scr xc = take(blk * sizeof(c128)), bc = take(blk * sizeof(c128));
  Scr H = take((size_t)(m + 1) * m * nseg * sizeof(c128));
  Scr cs = take((size_t)m * nseg * sizeof(double));
  Scr sn = take((size_t)m * nseg * sizeof(c128));
  Scr g = take((size_t)(m + 1) * nseg * sizeof(c128));
  Scr y = take((size_t)m * nseg * sizeof(c128));
  Scr hcol = take((size_t)(m + 1) * nseg * sizeof(c128));
  Scr h2 = take((size_t)(m + 1) * nseg * sizeof(c128));
  Scr hn = take(nseg * sizeof(double)), res = take(nseg * sizeof(double));
  Scr nrm = take(nseg * sizeof(double));
  Scr cnt = take(nseg * sizeof(int)), act = take(nseg * sizeof(int));
  const int nblk = std::max(1, std::min(64, ceil_div(maxlen, 256 * 8)));
  Scr part = take((size_t)nblk * (m + 1) * nseg * sizeof(c128));
  Scr partd = take((size_t)nblk * nseg * sizeof(double));

  // hcol += h2 for Arnoldi step j, one descriptor per step, uploaded once
  const AxpbyJob<double> *cgs_job;
  {
    std::vector<AxpbyJob<double>> aj;
    for (int j = 0; j < m; ++j)
      aj.push_back(AxpbyJob<double>{hcol.as<c128>(), h2.as<c128>(), nullptr, (j + 1) * nseg,
                                    (j + 1) * nseg, 0, (j + 1) * nseg, 1, 1.0, 0.0});
    cgs_job = stg.put(aj);
  }

  // contiguous copies of b and x
  HSSX_HIP(hipMemcpy2DAsync(bc.p, n * sizeof(c128), b, ldb * sizeof(c128), n * sizeof(c128), nrhs,
                            hipMemcpyDeviceToDevice, st));
  launch_fill(blk, czero<double>(), xc.as<c128>(), st);

  auto norms_host = [&](const c128 *v, std::vector<double> &out) {
    launch_norms(n, nrhs, sg, v, nrm.as<double>(), partd.as<double>(), nblk, st);
    out.resize(nseg);
    HSSX_HIP(hipMemcpyAsync(out.data(), nrm.p, nseg * sizeof(double), hipMemcpyDeviceToHost, st));
    HSSX_HIP(hipStreamSynchronize(st));
  };

  std::vector<double> bnorm, pbnorm;
  norms_host(bc.as<c128>(), bnorm);
  if (left) {
    precond(bc.as<c128>(), t1.as<c128>());
    norms_host(t1.as<c128>(), pbnorm);
  } else {
    pbnorm = bnorm;
  }
  std::vector<double> target(nseg, o.tol), prec_rel(nseg, 0.0), true_rel(nseg, 0.0);
  std::vector<int> extra(nseg, 0), done(nseg, 0), iters(nseg, 0), conv(nseg, 0);
  for (int r = 0; r < nseg; ++r)
    if (bnorm[r] == 0.0) { done[r] = 1; conv[r] = 1; }
  int total = 0;
  const long stride = blk;
  c128 *Vp = V.as<c128>();
  c128 *Zp = left ? nullptr : Z.as<c128>();

  while (true) {
    // residuals of the current iterate
    matvec(xc.as<c128>(), t1.as<c128>());
    launch_sub(n, nrhs, bc.as<c128>(), n, t1.as<c128>(), n, w.as<c128>(), n, st);
    std::vector<double> tr, pr;
    norms_host(w.as<c128>(), tr);
    if (left) {
      precond(w.as<c128>(), Vp);
      norms_host(Vp, pr);
    } else {
      HSSX_HIP(hipMemcpyAsync(Vp, w.p, blk * sizeof(c128), hipMemcpyDeviceToDevice, st));
      pr = tr;
    }
    std::vector<int> active(nseg, 0);
    bool any = false;
    for (int r = 0; r < nseg; ++r) {
      if (done[r]) continue;
      true_rel[r] = tr[r] / bnorm[r];
      prec_rel[r] = pr[r] / pbnorm[r];
      if (prec_rel[r] <= target[r]) {
        if (true_rel[r] <= o.tol || extra[r] >= 3) {
          done[r] = 1;
          conv[r] = true_rel[r] <= o.tol;
          continue;
        }
        target[r] *= o.tol / true_rel[r];
        ++extra[r];
      }
      if (iters[r] >= o.maxit) { done[r] = 1; continue; }
      active[r] = 1;
      any = true;
    }
    if (!any) break;
    // v0 = r0 / beta (zero for inactive right-hand sides)
    std::vector<double> beta(nseg);
    for (int r = 0; r < nseg; ++r) beta[r] = active[r] ? pr[r] : 0.0;
    HSSX_HIP(hipMemcpyAsync(hn.p, beta.data(), nseg * sizeof(double), hipMemcpyHostToDevice, st));
    launch_scale(n, nrhs, sg, Vp, hn.as<double>(), Vp, st);
    std::vector<c128> g0((size_t)(m + 1) * nseg, czero<double>());
    for (int r = 0; r < nseg; ++r) g0[r] = mk(beta[r], 0.0);
    HSSX_HIP(hipMemcpyAsync(g.p, g0.data(), g0.size() * sizeof(c128), hipMemcpyHostToDevice, st));
    HSSX_HIP(hipMemcpyAsync(act.p, active.data(), nseg * sizeof(int), hipMemcpyHostToDevice, st));
    std::vector<int> count(nseg, 0);
    for (int j = 0; j < m; ++j) {
      c128 *vj = Vp + j * stride;
      if (left) {
        matvec(vj, t1.as<c128>());
        precond(t1.as<c128>(), w.as<c128>());
      } else {
        precond(vj, Zp + j * stride);
        matvec(Zp + j * stride, w.as<c128>());
      }
      launch_mdot(n, nrhs, sg, j + 1, Vp, stride, w.as<c128>(), hcol.as<c128>(), part.as<c128>(),
                  nblk, st);
      launch_mupdate(n, nrhs, sg, j + 1, Vp, stride, hcol.as<c128>(), w.as<c128>(), st);
      launch_mdot(n, nrhs, sg, j + 1, Vp, stride, w.as<c128>(), h2.as<c128>(), part.as<c128>(),
                  nblk, st);
      launch_mupdate(n, nrhs, sg, j + 1, Vp, stride, h2.as<c128>(), w.as<c128>(), st);
      // hcol += h2 (the second Gram-Schmidt pass's coefficients)
      launch_axpby<double>(1, cgs_job + j, (j + 1) * nseg, 1, st);
      launch_norms(n, nrhs, sg, w.as<c128>(), hn.as<double>(), partd.as<double>(), nblk, st);
      launch_scale(n, nrhs, sg, w.as<c128>(), hn.as<double>(), Vp + (j + 1) * stride, st);
      launch_givens(nseg, j, m, H.as<c128>(), hcol.as<c128>(), hn.as<double>(), cs.as<double>(),
                    sn.as<c128>(), g.as<c128>(), res.as<double>(), act.as<int>(), st);
      std::vector<double> rs(nseg);
      HSSX_HIP(hipMemcpyAsync(rs.data(), res.p, nseg * sizeof(double), hipMemcpyDeviceToHost, st));
      HSSX_HIP(hipStreamSynchronize(st));
      ++total;
      bool still = false;
      for (int r = 0; r < nseg; ++r) {
        if (!active[r]) continue;
        ++iters[r];
        count[r] = j + 1;
        if (rs[r] / pbnorm[r] <= target[r] || iters[r] >= o.maxit) active[r] = 0;
        else still = true;
      }
      HSSX_HIP(hipMemcpyAsync(act.p, active.data(), nseg * sizeof(int), hipMemcpyHostToDevice, st));
      if (!still) break;
    }
    HSSX_HIP(hipMemcpyAsync(cnt.p, count.data(), nseg * sizeof(int), hipMemcpyHostToDevice, st));
    launch_hsolve(nseg, m, H.as<c128>(), g.as<c128>(), cnt.as<int>(), y.as<c128>(), st);
    launch_xupdate(n, nrhs, sg, cnt.as<int>(), left ? Vp : Zp, stride, y.as<c128>(), xc.as<c128>(),
                   n, st);
    HSSX_HIP(hipStreamSynchronize(st));
  }
  HSSX_HIP(hipMemcpy2DAsync(x, ldx * sizeof(c128), xc.p, n * sizeof(c128), n * sizeof(c128), nrhs,
                            hipMemcpyDeviceToDevice, st));
  HSSX_HIP(hipStreamSynchronize(st));
  if (stats)
    for (int r = 0; r < nseg; ++r) {
      stats[r].iters = iters[r];
      stats[r].converged = conv[r];
      stats[r].prec_res = prec_rel[r];
      stats[r].true_res = true_rel[r];
    }
  (void)total;
}

}  // namespace

void gmres(hssx_op_ &A, hssx_fact_ *P, int trans, int nrhs, const c128 *b, long ldb, c128 *x,
           long ldx, const hssx_gmres_opts &o, hssx_gmres_stats *stats, hipStream_t st) {
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  std::unique_ptr<Arena> ar = acquire_arena(dev);
  std::unique_ptr<Staging> stg = acquire_staging(dev, st);
  try {
    if (trans == 2) {
      // adjoint system A^H x = b as conj(A^-T conj(b)): the transposed
      // solve with the transposed preconditioner on conjugated data
      c128 *bc = ar->get<c128>((size_t)A.n * nrhs);
      launch_conj(A.n, nrhs, b, ldb, bc, A.n, st);
      gmres_impl(A, P, 1, nrhs, bc, A.n, x, ldx, o, stats, st, *ar, *stg);
      launch_conj(A.n, nrhs, x, ldx, x, ldx, st);
    } else {
      gmres_impl(A, P, trans, nrhs, b, ldb, x, ldx, o, stats, st, *ar, *stg);
    }
  } catch (...) {
    (void)hipStreamSynchronize(st);
    return_arena(dev, std::move(ar));
    return_staging(dev, std::move(stg));
    throw;
  }
  return_arena(dev, std::move(ar));
  return_staging(dev, std::move(stg));
}

}  // namespace hssx
