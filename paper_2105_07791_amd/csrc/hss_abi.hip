// The HSS building blocks of the factorization (telescoping
// product, telescoping inverse and solve, entry access to a matrix and to
// its inverse) on one symmetric HSS matrix given by the caller in generator
// form (Sec. 2.2).
#include <cstring>

#include "engine.h"

using namespace hssx;

namespace {

template <typename T>
void hss_eval_t(int m, int ncl, const int32_t *tree, const int32_t *rank, const double *gens, int op,
              int nrhs, const c128 *X, c128 *Y, long nij, const int32_t *ij, double *vals,
              hipStream_t st) {
  // ops 4 and 5: ops 1 and 3 with the inverse computed in complex128
  const bool wide = op == 4 || op == 5;
  if (wide) op = op == 4 ? 1 : 3;
  HssMat<T> H;
  H.m = m;
  ClusterTree &ct = H.ct;
  ct.start.resize(ncl); ct.size.resize(ncl); ct.left.resize(ncl); ct.right.resize(ncl);
  ct.level.resize(ncl);
  for (int c = 0; c < ncl; ++c) {
    ct.start[c] = tree[5 * c];
    ct.size[c] = tree[5 * c + 1];
    ct.left[c] = tree[5 * c + 2];
    ct.right[c] = tree[5 * c + 3];
    ct.level[c] = tree[5 * c + 4];
  }
  HSSX_CHECK(ct.start[0] == 0 && ct.size[0] == m, HSSX_EINVAL, "root cluster must cover [0, m)");
  for (int c = 0; c < ncl; ++c) {
    const bool lf = ct.left[c] < 0;
    HSSX_CHECK(lf == (ct.right[c] < 0), HSSX_EINVAL, "cluster with one child");
    HSSX_CHECK(ct.size[c] >= 1 && ct.start[c] >= 0 && ct.start[c] + ct.size[c] <= m, HSSX_EINVAL,
               "cluster range outside [0, m)");
    HSSX_CHECK(rank[c] >= 0 && (c > 0 || rank[0] == 0), HSSX_EINVAL, "rank");
    if (!lf) {
      const int l = ct.left[c], r = ct.right[c];
      HSSX_CHECK(l > c && r > c && l < ncl && r < ncl && ct.level[l] == ct.level[c] + 1 &&
                     ct.level[r] == ct.level[c] + 1 && ct.start[l] == ct.start[c] &&
                     ct.start[r] == ct.start[l] + ct.size[l] &&
                     ct.size[l] + ct.size[r] == ct.size[c],
                 HSSX_EINVAL, "clusters must be in level order and split their parent");
    }
  }
  H.k.assign(rank, rank + ncl);
  // generators: sizes, then one device copy in T
  std::vector<long> offU(ncl, -1), offD(ncl, -1), off12(ncl, -1), off21(ncl, -1);
  long tot = 0;
  for (int c = 0; c < ncl; ++c) {
    const bool lf = ct.left[c] < 0;
    const int rows = lf ? ct.size[c] : H.k[ct.left[c]] + H.k[ct.right[c]];
    if (c > 0) { offU[c] = tot; tot += (long)rows * H.k[c]; }
    if (lf) { offD[c] = tot; tot += (long)ct.size[c] * ct.size[c]; }
    else {
      off12[c] = tot; tot += (long)H.k[ct.left[c]] * H.k[ct.right[c]];
      off21[c] = tot; tot += (long)H.k[ct.left[c]] * H.k[ct.right[c]];
    }
    HSSX_CHECK(c == 0 || H.k[c] <= rows, HSSX_EINVAL, "rank above the rows of a basis");
  }
  std::vector<cplx<T>> hg(std::max(1L, tot));
  for (long e = 0; e < tot; ++e) hg[e] = mk((T)gens[2 * e], (T)gens[2 * e + 1]);
  DevBuf g;
  upload(g, hg);
  cplx<T> *gp = g.as<cplx<T>>();
  H.U.assign(ncl, nullptr); H.D.assign(ncl, nullptr); H.B12.assign(ncl, nullptr);
  H.B21.assign(ncl, nullptr);
  for (int c = 0; c < ncl; ++c) {
    if (offU[c] >= 0) H.U[c] = gp + offU[c];
    if (offD[c] >= 0) H.D[c] = gp + offD[c];
    if (off12[c] >= 0) { H.B12[c] = gp + off12[c]; H.B21[c] = gp + off21[c]; }
  }
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  std::unique_ptr<Arena> ar = acquire_arena(dev);
  std::unique_ptr<Staging> sg = acquire_staging(dev, st);
  auto done = [&] {
    (void)hipStreamSynchronize(st);
    return_arena(dev, std::move(ar));
    return_staging(dev, std::move(sg));
  };
  try {
    Alloc<T> al = [&](size_t n) { return ar->get<cplx<T>>(n); };
    const Gen<T> gen = H.gen(0);
    std::vector<HssInv<T>> inv;
    if (op == 1 || op == 3) {
      int *err = ar->get<int>(1);
      int *d0 = sg->put(std::vector<int>{-1});
      HSSX_HIP(hipMemcpyAsync(err, d0, sizeof(int), hipMemcpyDeviceToDevice, st));
      double fl = 0;
      bool done_wide = false;
      if constexpr (sizeof(T) == sizeof(float)) {
        if (wide) {
          Alloc<double> wal = [&](size_t n) { return ar->get<c128>(n); };
          gym_factor_wide(inv, std::vector<const Gen<T> *>{&gen}, std::vector<int>{0}, al, wal,
                          err, *sg, *ar, nullptr, st, &fl);
          done_wide = true;
        }
      }
      if (!done_wide)
        gym_factor(inv, std::vector<const Gen<T> *>{&gen}, std::vector<int>{0}, al, al, err, *sg,
                   *ar, nullptr, st, &fl);
      int bad = -1;
      HSSX_HIP(hipMemcpyAsync(&bad, err, sizeof(int), hipMemcpyDeviceToHost, st));
      HSSX_HIP(hipStreamSynchronize(st));
      HSSX_CHECK(bad < 0, HSSX_ESINGULAR, "zero pivot in a block of the telescoping inverse");
    }
    if (op == 0 || op == 1) {
      cplx<T> *Xt = al((size_t)m * nrhs), *Yt = al((size_t)m * nrhs);
      Prog<T> p;
      p.add(kGwt).gwt.push_back(
          GatherJob<c128, cplx<T>>{X, Xt, m, m, nullptr, nullptr, m, nrhs, 0, 1.0});
      if (op == 0) hss_matvec(p, std::vector<MvItem<T>>{MvItem<T>{&gen, Xt, m, Yt, m, nrhs}}, al);
      else gym_solve(p, std::vector<SolveItem<T>>{SolveItem<T>{&inv[0], Xt, m, Yt, m, nrhs}}, al);
      p.add(kGtw).gtw.push_back(
          GatherJob<cplx<T>, c128>{Yt, Y, m, m, nullptr, nullptr, m, nrhs, 0, 1.0});
      run_prog(p, *sg, nullptr, st);
    } else {
      Prog<T> p;
      Gen<T> xg;
      std::vector<EntPrep<T>> ep(1);
      if (op == 3) {
        std::vector<HssInv<T> *> hs{&inv[0]};
        gym_inverse_blocks(p, hs, al, al);
        xg = inv[0].inv_gen();
        ep[0].g = &xg;
      } else {
        ep[0].g = &gen;
      }
      entry_prep(p, ep, al);
      run_prog(p, *sg, nullptr, st);
      for (long e = 0; e < 2 * nij; ++e)
        HSSX_CHECK(ij[e] >= 0 && ij[e] < m, HSSX_EINVAL, "entry index outside [0, m)");
      EntView<T> v{sg->put(ep[0].cl), sg->put(ep[0].leaf_of)};
      const int *dij = sg->put(std::vector<int>(ij, ij + 2 * nij));
      cplx<T> *out = al((size_t)std::max(1L, nij));
      launch_entries_list<T>(v, dij, (int)nij, out, st);
      std::vector<cplx<T>> h(std::max(1L, nij));
      HSSX_HIP(hipMemcpyAsync(h.data(), out, nij * sizeof(cplx<T>), hipMemcpyDeviceToHost, st));
      HSSX_HIP(hipStreamSynchronize(st));
      for (long e = 0; e < nij; ++e) {
        vals[2 * e] = h[e].re;
        vals[2 * e + 1] = h[e].im;
      }
    }
  } catch (...) {
    done();
    throw;
  }
  done();
}

}  // namespace

namespace hssx {

void hss_eval(hssx_dtype dtype, int m, int ncl, const int32_t *tree, const int32_t *rank,
              const double *gens, int op, int nrhs, const void *x_dev, void *y_dev, long nij,
              const int32_t *ij, double *vals, hipStream_t st) {
  if (dtype == HSSX_C128)
    hss_eval_t<double>(m, ncl, tree, rank, gens, op, nrhs, (const c128 *)x_dev, (c128 *)y_dev, nij,
                       ij, vals, st);
  else
    hss_eval_t<float>(m, ncl, tree, rank, gens, op, nrhs, (const c128 *)x_dev, (c128 *)y_dev, nij,
                      ij, vals, st);
}

}  // namespace hssx
