// Numeric factorization P = LDR (Algorithm 3.4) and its application
// (Algorithm 3.1).
//
// Nodes are processed one tree depth at a time, deepest first; all nodes of
// a depth are independent (their boxes are disjoint).  Per depth:
//   1. assemble the augmented fronts (eq. 3.2 at leaves, eq. 3.4 above);
//   2. nodes with HSS arithmetic (height > h_sw): form the inner Schur
//      complement S~ = S_ii^nu - A~^(nu,mu) (S_ii^mu)^-1 A~^(mu,nu) of the
//      interior block, compress it with Algorithm A.1 on nu's interior
//      cluster tree, and replace S~ by its HSS approximation inside A_ii:
//      the factor then applies exactly the 2x2 block inverse of
//      Algorithm 3.2 whose Schur block is the HSS matrix (Algorithm 3.3);
//   3. Gauss-Jordan elimination of every front (A_ii^-1, R, L, S);
//   4. nodes whose parent uses HSS arithmetic compress S with Algorithm A.1
//      (dense S below the switch, "form S directly in HSS form" above it)
//      and pass the HSS approximation on to the parent's front.
// The compressions of a depth are batched: all instances sample, compress
// level by level, and estimate together; only those whose estimate
// (eq. 2.7) misses the tolerance grow k <- k + r and go round again.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <type_traits>

#include "engine.h"

namespace hssx {

namespace {

// A second stream per device and host thread (default priority) for launches
// that may overlap the factor's own stream, with the events that fork work
// onto it and join it back.  Thread-local, so concurrent factorizations on
// different host threads never share one.
struct SideStream {
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
SideStream &side_stream() {
  thread_local std::map<int, SideStream> per_device;
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  SideStream &x = per_device[dev];
  if (!x.s) {
    HSSX_HIP(hipStreamCreateWithFlags(&x.s, hipStreamNonBlocking));
    HSSX_HIP(hipEventCreateWithFlags(&x.fork, hipEventDisableTiming));
    HSSX_HIP(hipEventCreateWithFlags(&x.join, hipEventDisableTiming));
  }
  return x;
}

}  // namespace

namespace {

template <typename T> struct CompressTask {
  int node = 0, kind = 0;
  int m = 0;
  int k_init = 0;   // initial rank guess (0: the option k0)
  ClusterTree ct;
  cplx<T> *S = nullptr;
  int ldS = 0;
  cplx<T> *target = nullptr;
  int ldT = 0;
  // state / results
  int k = 0, s = 0, rounds = 0, cap = 0;
  double est = 0, est_prev = 0;
  int maxrank = 0;
  bool done = false;
  long ooff = 0, yoff = 0;
};

struct Layout {
  std::vector<HssCluster> cl;
  long pool = 0, ipool = 0, xh = 0;
  // compression scratch per tree level: a cluster's local samples are only
  // used while its own level runs, so the levels share one region
  std::vector<long> level_scratch;
};

// cluster capacities and pool offsets of one instance for rank cap k and s columns
Layout layout_instance(const ClusterTree &ct, int k, int s) {
  Layout L;
  int nc = ct.count();
  L.cl.resize(nc);
  std::vector<int> kcap(nc, 0), rcap(nc, 0);
  for (int c = nc - 1; c >= 0; --c) {
    if (ct.leaf(c)) rcap[c] = ct.size[c];
    else rcap[c] = kcap[ct.left[c]] + kcap[ct.right[c]];
    int kc = std::min(k, std::min(rcap[c], s));
    kcap[c] = c == 0 ? 0 : kc;
  }
  for (int c = 0; c < nc; ++c) {
    HssCluster &h = L.cl[c];
    h.start = ct.start[c];
    h.size = ct.size[c];
    h.left = ct.left[c];
    h.right = ct.right[c];
    h.level = ct.level[c];
    h.rows_cap = rcap[c];
    h.k_cap = kcap[c];
    long r = rcap[c], kk = kcap[c];
    h.U = L.pool; L.pool += std::max(1L, r * kk);
    h.Om = L.pool; L.pool += std::max(1L, kk * s);
    h.Sr = L.pool; L.pool += std::max(1L, kk * s);
    if (ct.leaf(c)) { h.D = L.pool; L.pool += (long)h.size * h.size; } else h.D = 0;
    if (!ct.leaf(c)) {
      long kl = kcap[ct.left[c]], kr = kcap[ct.right[c]];
      h.B12 = L.pool; L.pool += std::max(1L, kl * kr);
      h.B21 = L.pool; L.pool += std::max(1L, kl * kr);
    } else {
      h.B12 = h.B21 = 0;
    }
    h.sk = (int)L.ipool; L.ipool += std::max(1L, kk);
    if ((int)L.level_scratch.size() <= h.level) L.level_scratch.resize(h.level + 1, 0);
    h.W = L.level_scratch[h.level];
    L.level_scratch[h.level] += 3 * r * s + std::max(1L, kk) * std::max(1L, r);
    h.XH = L.xh; L.xh += 2 * std::max(1L, kk) * kXC;
  }
  return L;
}

// nominal flops of one cluster's step of Algorithm A.1 with the rank cap:
// local samples, pivoted QR of S_loc^T (two projections per pivot), the
// interpolation matrix and the reduced sketch
inline double compress_flops(const HssCluster &c, const HssInstance &I) {
  const double s = I.s, rows = c.rows_cap, k = c.k_cap;
  double f = 0;
  if (c.left < 0) f += 4.0 * rows * rows * s;                 // D Omega
  else f += 8.0 * rows * rows * s / 2;                        // B12 Om_r, B21 Om_l
  f += k * rows * s * (3.0 + 16.0);                           // norms + dot + axpy per pivot
  f += 4.0 * (rows - k) * k * k + 8.0 * k * rows * s;         // T and U^T Omega
  return f;
}

// rows of one local sample block the compression kernel holds
constexpr int kMaxLocalRows = 1024;
// acceptance slack of a stalled complex64 estimate, relative to tol
constexpr double kStallSlack = 10.0;

template <typename T>
void compress_batch(std::vector<CompressTask<T>> &tasks, const hssx_factor_opts &o, double tol,
                    double id_tol, Staging &sg, Arena &ar) {
  if (tasks.empty()) return;
  const hipStream_t st = sg.stream();
  const int k0 = o.k0, r = o.r;
  long osz = 0, ysz = 0;
  for (auto &t : tasks) {
    t.k = std::max(1, std::min(std::max(k0, t.k_init), t.m));
    t.s = t.k + r;
    // room for every round up to k >= m (s = k + r samples + r probes)
    t.cap = std::min(t.k + r * (o.max_rounds + 1), t.m + 3 * r);
    t.cap = std::max(t.cap, t.s + r);
    t.ooff = osz;
    t.yoff = ysz;
    osz += (long)t.m * t.cap;
    ysz += (long)t.m * t.cap;
    t.rounds = 0;
    t.done = false;
    HSSX_CHECK(t.cap <= 1024, HSSX_EINVAL, "sample block wider than the compression kernel holds");
    HSSX_CHECK(t.m <= 1 << 24, HSSX_EINVAL, "compression size");
  }
  // sketches and samples live until the last round; each round's generator
  // pools are released once the round has been synchronised
  double *Om = ar.get<double>(osz);
  cplx<T> *Y = ar.get<cplx<T>>(ysz);
  double *d_err = ar.get<double>(2 * tasks.size());

  auto gen_and_sample = [&](const std::vector<int> &ids, bool probe) {
    std::vector<GaussJob> gj;
    std::vector<SampleJob<T>> sj;
    int mm = 0, mc = 0;
    for (int i : ids) {
      auto &t = tasks[i];
      int c0 = probe ? t.s : 0, nc = probe ? r : t.s;
      GaussJob g{Om + t.ooff, t.m, t.m, c0, nc, 0, (uint32_t)(4 * t.node + t.kind)};
      gj.push_back(g);
      SampleJob<T> s{t.S, Om + t.ooff + (long)c0 * t.m, Y + t.yoff + (long)c0 * t.m,
                     t.ldS, t.m, t.m, t.m, nc};
      sj.push_back(s);
      mm = std::max(mm, t.m);
      mc = std::max(mc, nc);
    }
    GaussJob *dg = sg.put(gj);
    SampleJob<T> *ds = sg.put(sj);
    launch_gaussian((int)gj.size(), dg, o.seed, mm, mc, st);
    double sflops = 0;
    for (const auto &q : sj) sflops += 4.0 * q.m * (double)q.m * q.nc;
    hipEvent_t ps = prof_begin(st);
    if constexpr (std::is_same<T, float>::value) {
      if (o.sample_bf16) launch_sample_bf16((int)sj.size(), ds, mm, mc, o.sample_bf16, st);
      else launch_sample<T>((int)sj.size(), ds, mm, mc, st);
    } else {
      launch_sample<T>((int)sj.size(), ds, mm, mc, st);
    }
    prof_end("sample", st, ps, sflops);
  };

  std::vector<int> all(tasks.size());
  for (size_t i = 0; i < tasks.size(); ++i) all[i] = (int)i;
  gen_and_sample(all, false);

  std::vector<int> active = all;
  while (!active.empty()) {
    const Arena::Mark round_mark = ar.mark();
    // ---- layout of the active instances
    std::vector<HssInstance> inst;
    std::vector<HssCluster> cls;
    std::vector<Layout> lay;
    long pool = 0, ipool = 0;
    int max_width = 0, max_ncl = 0;
    std::vector<long> xh_of;     // matvec scratch per job of each instance
    std::vector<long> lev_scr;   // running scratch offset per tree level
    int maxlev = 0;
    for (int i : active) {
      auto &t = tasks[i];
      Layout L = layout_instance(t.ct, t.k, t.s);
      if (lev_scr.size() < L.level_scratch.size()) lev_scr.resize(L.level_scratch.size(), 0);
      for (auto &c : L.cl) c.W += lev_scr[c.level];
      for (size_t l = 0; l < L.level_scratch.size(); ++l) lev_scr[l] += L.level_scratch[l];
      for (const auto &c : L.cl)
        HSSX_CHECK(c.rows_cap <= kMaxLocalRows, HSSX_EINVAL,
                   "local sample block taller than the compression kernel holds");
      HssInstance h{};
      h.m = t.m;
      h.ncl = t.ct.count();
      h.cl_off = (int)cls.size();
      h.s = t.s;
      h.k = t.k;
      h.pool = pool;
      h.ipool = ipool;
      h.soff = 0;
      h.ldS = t.ldS;
      h.yoff = t.yoff;
      h.ooff = t.ooff;
      h.ldY = t.m;
      h.woff = 0;
      // clusters are numbered level by level
      h.nlev = t.ct.depth() + 1;
      HSSX_CHECK(h.nlev <= kMaxLev, HSSX_EINVAL, "cluster tree deeper than the matvec supports");
      for (int l = 0, c = 0; l <= h.nlev; ++l) {
        while (c < h.ncl && t.ct.level[c] < l) ++c;
        h.lev_off[l] = c;
      }
      for (int l = 0; l < h.nlev; ++l) max_width = std::max(max_width, h.lev_off[l + 1] - h.lev_off[l]);
      max_ncl = std::max(max_ncl, h.ncl);
      pool += L.pool;
      ipool += L.ipool;
      xh_of.push_back(L.xh);
      cls.insert(cls.end(), L.cl.begin(), L.cl.end());
      inst.push_back(h);
      maxlev = std::max(maxlev, t.ct.depth());
      lay.push_back(std::move(L));
    }
    // each instance's operator S lives in device memory of its own; the
    // kernel adds soff to a common base, so pass base = nullptr-offset form
    // through per-instance soff relative to the first task's S.
    const cplx<T> *base = tasks[active[0]].S;
    for (size_t a = 0; a < active.size(); ++a) inst[a].soff = tasks[active[a]].S - base;

    HssInstance *d_inst = sg.put(inst);
    HssCluster *d_cls = sg.put(cls);
    cplx<T> *d_pool = ar.get<cplx<T>>(pool);
    int *d_ipool = ar.get<int>(ipool);
    int *d_rank = ar.get<int>(cls.size());
    long scratch = 0;
    for (long v : lev_scr) scratch = std::max(scratch, v);
    cplx<T> *d_scr = ar.get<cplx<T>>(scratch);
    HSSX_HIP(hipMemsetAsync(d_rank, 0, cls.size() * sizeof(int), st));

    // ---- bottom-up compression, one launch per cluster-tree level and size
    // class (clusters of at most 64 rows in small workgroups; the larger
    // ones in large workgroups, split by whether they fit the register path)
    // all levels' work lists go up in one upload
    std::vector<HssItem> all_items;
    std::vector<std::array<long, 4>> launches;   // level, size class, offset, count
    for (int lev = maxlev; lev >= 0; --lev) {
      std::vector<HssItem> items[3];
      for (size_t a = 0; a < active.size(); ++a) {
        for (int c = inst[a].lev_off[std::min(lev, inst[a].nlev)];
             c < inst[a].lev_off[std::min(lev + 1, inst[a].nlev)]; ++c) {
          const int rc = cls[inst[a].cl_off + c].rows_cap;
          const bool reg = rc <= kRegRows && inst[a].s <= kRegCols;
          items[rc <= 64 ? 0 : reg ? 1 : 2].push_back(HssItem{(int)a, c});
        }
      }
      // the one-barrier 1024-thread variant holds one workgroup per CU: used
      // when the level's large clusters all fit it and do not outnumber the
      // CUs (otherwise occupancy, or running with the global-memory ones in
      // one launch, matters more)
      if (items[1].size() > 256 || !items[2].empty()) {
        items[2].insert(items[2].end(), items[1].begin(), items[1].end());
        items[1].clear();
      }
      for (int sz = 0; sz < 3; ++sz) {
        if (items[sz].empty()) continue;
        launches.push_back({lev, sz, (long)all_items.size(), (long)items[sz].size()});
        all_items.insert(all_items.end(), items[sz].begin(), items[sz].end());
      }
    }
    HssItem *d_all = all_items.empty() ? nullptr : sg.put(all_items);
    // the small-cluster launch of a level is independent of its large-cluster
    // launches (different clusters, same inputs): when a level has both, the
    // small one runs on a side stream, forked from and joined back into st
    SideStream &side = side_stream();
    for (size_t a = 0; a < launches.size();) {
      size_t b = a;
      while (b < launches.size() && launches[b][0] == launches[a][0]) ++b;
      const bool fork = b - a > 1 && launches[a][1] == 0;
      if (fork) {
        HSSX_HIP(hipEventRecord(side.fork, st));
        HSSX_HIP(hipStreamWaitEvent(side.s, side.fork, 0));
      }
      for (size_t e = a; e < b; ++e) {
        const auto &l = launches[e];
        hipStream_t ls = fork && l[1] == 0 ? side.s : st;
        double cflops = 0;
        for (long q = l[2]; q < l[2] + l[3]; ++q) {
          const auto &it = all_items[q];
          cflops += compress_flops(cls[inst[it.inst].cl_off + it.cl], inst[it.inst]);
        }
        hipEvent_t pc = prof_begin(ls);
        launch_compress_level<T>((int)l[3], d_all + l[2], d_inst, d_cls, d_pool, d_ipool, d_rank,
                                 base, Y, Om, d_scr, id_tol, (int)l[1], ls);
        prof_end("compress_level", ls, pc, cflops);
      }
      if (fork) {
        HSSX_HIP(hipEventRecord(side.join, side.s));
        HSSX_HIP(hipStreamWaitEvent(st, side.join, 0));
      }
      a = b;
    }

    // ---- error estimate with r fresh probes (eq. 2.7), kXC columns per job
    gen_and_sample(active, true);
    std::vector<MatvecJob<T>> mj;
    long xh_total = 0;
    for (size_t a = 0; a < active.size(); ++a) {
      auto &t = tasks[active[a]];
      for (int c0 = 0; c0 < r; c0 += kXC) {
        MatvecJob<T> j{};
        j.inst = (int)a;
        j.X = Om + t.ooff + (long)(t.s + c0) * t.m;
        j.ldX = t.m;
        j.nc = std::min(kXC, r - c0);
        j.c0 = 0;
        j.out = nullptr;
        j.ldO = 0;
        j.Yref = Y + t.yoff + (long)(t.s + c0) * t.m;
        j.ldR = t.m;
        j.err2 = d_err + 2 * active[a];
        j.ref2 = d_err + 2 * active[a] + 1;
        j.woff = xh_total;
        xh_total += xh_of[a];
        mj.push_back(j);
      }
    }
    MatvecJob<T> *d_mj = sg.put(mj);
    cplx<T> *d_xh = ar.get<cplx<T>>(xh_total);
    HSSX_HIP(hipMemsetAsync(d_err, 0, 2 * tasks.size() * sizeof(double), st));
    hipEvent_t pm = prof_begin(st);
    launch_hss_matvec<T>((int)mj.size(), d_mj, d_inst, d_cls, d_pool, d_rank, d_xh, maxlev + 1,
                         max_width, max_ncl, st);
    prof_end("hss_matvec", st, pm, 0.0);
    std::vector<double> h_err(2 * tasks.size());
    std::vector<int> h_rank(cls.size());
    HSSX_HIP(hipMemcpyAsync(h_err.data(), d_err, h_err.size() * sizeof(double),
                            hipMemcpyDeviceToHost, st));
    HSSX_HIP(hipMemcpyAsync(h_rank.data(), d_rank, h_rank.size() * sizeof(int),
                            hipMemcpyDeviceToHost, st));
    HSSX_HIP(hipStreamSynchronize(st));

    // ---- decisions; expand the accepted instances into their targets
    std::vector<int> next;
    std::vector<MatvecJob<T>> ej;
    long xh2_total = 0;
    for (size_t a = 0; a < active.size(); ++a) {
      auto &t = tasks[active[a]];
      t.rounds += 1;
      double e2 = h_err[2 * active[a]], r2 = h_err[2 * active[a] + 1];
      t.est_prev = t.est;
      t.est = r2 > 0 ? std::sqrt(e2 / r2) : 0.0;
      int mr = 0;
      for (int c = 0; c < t.ct.count(); ++c) mr = std::max(mr, h_rank[inst[a].cl_off + c]);
      t.maxrank = mr;
      // growing needs room for the next round's probes: columns [s + r, s + 2r),
      // and local blocks of at most 2 (k + r) rows
      bool accept = t.est <= tol || t.k >= t.m || t.rounds >= o.max_rounds ||
                    t.s + 2 * r > t.cap || 2 * (t.k + r) > kMaxLocalRows;
      // complex64 fronts carry rounding noise of relative size ~ eps_fp32
      // sqrt(m): once the estimate sits within kStallSlack of tol and another
      // r columns no longer halve it, the rank is chasing that noise
      if (sizeof(T) == sizeof(float) && t.rounds >= 2 && t.est <= kStallSlack * tol &&
          t.est > 0.5 * t.est_prev)
        accept = true;
      if (!accept) {
        t.k += r;
        t.s += r;
        next.push_back(active[a]);
        continue;
      }
      t.done = true;
      // expansion H I in kXC-column blocks
      for (int c0 = 0; c0 < t.m; c0 += kXC) {
        MatvecJob<T> j{};
        j.inst = (int)a;
        j.X = nullptr;
        j.c0 = c0;
        j.nc = std::min(kXC, t.m - c0);
        j.out = t.target + (long)c0 * t.ldT;
        j.ldO = t.ldT;
        j.Yref = nullptr;
        j.woff = xh2_total;
        xh2_total += xh_of[a];
        ej.push_back(j);
      }
    }
    if (!ej.empty()) {
      MatvecJob<T> *d_ej = sg.put(ej);
      cplx<T> *d_xh2 = ar.get<cplx<T>>(xh2_total);
      hipEvent_t pm2 = prof_begin(st);
      launch_hss_matvec<T>((int)ej.size(), d_ej, d_inst, d_cls, d_pool, d_rank, d_xh2,
                           maxlev + 1, max_width, max_ncl, st);
      prof_end("hss_matvec", st, pm2, 0.0);
    }
    // the round's pools go back to the arena; later kernels that reuse the
    // memory are ordered after the expansion on the same stream
    ar.release(round_mark);
    active.swap(next);
  }
}

// Gauss-Jordan flops: 8 per complex multiply-add over the reduced rows
template <typename T> double elim_flops(const std::vector<ElimJob<T>> &jobs) {
  double f = 0;
  for (const auto &j : jobs)
    for (int p = 0; p < j.ne; ++p) f += 8.0 * (j.m - 1) * (double)(j.ncols - p - 1);
  return f;
}

// Gauss-Jordan elimination of a batch of jobs: fronts with few pivots run in
// one workgroup each; larger ones go panel by panel (32 columns) through the
// blocked sequence, all fronts of the batch advancing together.  The blocked
// path eliminates only the pivot rows [0, ne): they become
// [I | A_ii^-1 A_ib | A_ii^-1]; the remaining rows are then updated by one
// product per front, F(ne:m, ne:) -= F(ne:m, 0:ne) F(0:ne, ne:), which gives
// S = A_bb - A_bi A_ii^-1 A_ib and L = -A_bi A_ii^-1 (eqs. 3.2-3.5) with
// every entry accumulated once instead of once per panel.
// After the pivot rows of a front are eliminated: the non-pivot rows,
// F(ne:m, ne:ncols) -= F(ne:m, 0:ne) F(0:ne, ne:ncols), and R = -(A_ii^-1
// A_ib), the negated block F(0:ne, ne:m), as batched job lists
template <typename T> struct ProductListsT {
  std::vector<GemmJob<T>> gj;
  std::vector<AxpbyJob<T>> neg;
  int gm = 0, gn = 0, nm = 0, nn = 0;
};
template <typename T>
ProductListsT<T> product_lists_of(const std::vector<ElimJob<T>> &js) {
  ProductListsT<T> p;
  for (const auto &j : js) {
    if (j.m == j.ne || j.ne == 0) continue;
    const cplx<T> *Abi = j.ptr + j.ne, *Bx = j.ptr + (long)j.ne * j.ld;
    cplx<T> *C = j.ptr + j.ne + (long)j.ne * j.ld;
    p.gj.push_back(GemmJob<T>{Abi, Bx, C, j.ld, j.ld, j.ld, j.m - j.ne, j.ncols - j.ne, j.ne});
    p.gm = std::max(p.gm, j.m - j.ne);
    p.gn = std::max(p.gn, j.ncols - j.ne);
  }
  for (const auto &j : js) {
    if (!j.negate_r || j.m == j.ne) continue;
    cplx<T> *R = j.ptr + (long)j.ne * j.ld;
    p.neg.push_back(AxpbyJob<T>{R, R, nullptr, j.ld, j.ld, 0, j.ne, j.m - j.ne, (T)-2, (T)0});
    p.nm = std::max(p.nm, j.ne);
    p.nn = std::max(p.nn, j.m - j.ne);
  }
  return p;
}

template <typename T>
void eliminate_jobs(const std::vector<ElimJob<T>> &jobs, int *err, Staging &sg, Arena &ar) {
  using ProductLists = ProductListsT<T>;
  auto product_lists = [](const std::vector<ElimJob<T>> &js) { return product_lists_of<T>(js); };
  // panel width: the register-resident panel holds 32 complex64 or 16
  // complex128 columns per row
  constexpr int NB = sizeof(T) == sizeof(float) ? 32 : 16, kSmall = 64;
  const hipStream_t st = sg.stream();
  std::vector<ElimJob<T>> small, big;
  // single-workgroup elimination for fronts with few pivots and few rows;
  // the blocked path spreads the trailing update of larger fronts over many
  // workgroups
  // fronts with few pivots whose pivot rows fit in LDS are eliminated there
  // (pivot rows only; the others follow by the product below), the rest of
  // the few-pivot fronts in one workgroup from global memory
  constexpr size_t kLdsMax = 156 * 1024;   // of the 160 KiB per workgroup
  std::vector<ElimJob<T>> in_lds, rows_done;
  size_t lds = 0;
  for (const auto &j : jobs) {
    const size_t b = (size_t)j.ne * j.ncols * sizeof(cplx<T>);
    if (j.ne < kSmall && j.ne > 0 && b <= kLdsMax) {
      ElimJob<T> q = j;
      q.m = j.ne;
      q.negate_r = 0;
      in_lds.push_back(q);
      rows_done.push_back(j);
      lds = std::max(lds, b);
    } else {
      (j.ne < kSmall && j.m <= 128 ? small : big).push_back(j);
    }
  }
  // the few-pivot fronts are independent of the blocked elimination of the
  // large fronts until the product over the non-pivot rows: with large
  // fronts present they run on the side stream (forked after their job lists
  // are uploaded on st, joined before that product)
  const bool overlap = !big.empty() && (!in_lds.empty() || !small.empty());
  int *queue = nullptr;
  ElimJob<T> *d_order = nullptr, *d_small = nullptr;
  if (!in_lds.empty()) {
    // longest first: GJ work of the pivot rows, about ne^2 ncols
    std::vector<ElimJob<T>> order = in_lds;
    std::stable_sort(order.begin(), order.end(), [](const ElimJob<T> &a, const ElimJob<T> &b) {
      return (long)a.ne * a.ne * a.ncols > (long)b.ne * b.ne * b.ncols;
    });
    queue = sg.put(std::vector<int>{0});
    d_order = sg.put(order);
  }
  if (!small.empty()) d_small = sg.put(small);
  // products over the non-pivot rows and the negation of R for the fronts
  // eliminated in LDS, queued on the same stream right after them
  const ProductLists pr_done = product_lists(rows_done);
  GemmJob<T> *d_gd = pr_done.gj.empty() ? nullptr : sg.put(pr_done.gj);
  AxpbyJob<T> *d_nd = pr_done.neg.empty() ? nullptr : sg.put(pr_done.neg);
  SideStream *side = overlap ? &side_stream() : nullptr;
  hipStream_t fs = st;
  if (overlap) {
    HSSX_HIP(hipEventRecord(side->fork, st));
    HSSX_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    fs = side->s;
  }
  if (d_order) launch_eliminate<T>((int)in_lds.size(), d_order, err, fs, lds, queue);
  if (d_small) launch_eliminate<T>((int)small.size(), d_small, err, fs);
  if (d_gd) launch_gemm_sub<T>((int)pr_done.gj.size(), d_gd, pr_done.gm, pr_done.gn, fs);
  if (d_nd) launch_axpby<T>((int)pr_done.neg.size(), d_nd, pr_done.nm, pr_done.nn, fs);
  if (big.empty()) return;   // no fork without large fronts
  // scratch per job: pivots, G, Y, W
  long ysz = 0, wsz = 0;
  std::vector<long> yo, wo;
  int steps = 0;
  for (const auto &j : big) {
    yo.push_back(ysz);
    wo.push_back(wsz);
    ysz += (long)NB * j.ncols;
    wsz += (long)j.ne * NB;
    steps = std::max(steps, ceil_div(j.ne, NB));
  }
  const Arena::Mark mk0 = ar.mark();
  int *piv = ar.get<int>(std::max<size_t>(1, big.size()) * NB);
  cplx<T> *G = ar.get<cplx<T>>(std::max<size_t>(1, big.size()) * NB * NB);
  cplx<T> *Y = ar.get<cplx<T>>(std::max(1L, ysz));
  // the panel copy W is only read when a panel is too tall for registers
  int maxne = 0;
  for (const auto &j : big) maxne = std::max(maxne, j.ne);
  cplx<T> *W = maxne > 1536 ? ar.get<cplx<T>>(wsz) : nullptr;
  // every panel step's job list goes up in one upload
  std::vector<PanelJob<T>> all_pj;
  std::vector<std::array<int, 6>> step_cfg;   // offset, count, max m, cols, panel rows, nb
  for (int k = 0; k < steps; ++k) {
    const int off = (int)all_pj.size();
    int mm = 0, mc = 0, mp = 0, mnb = 0;
    for (size_t a = 0; a < big.size(); ++a) {
      const auto &j = big[a];
      int p0 = k * NB;
      if (p0 >= j.ne) continue;
      PanelJob<T> q;
      q.F = j.ptr;
      q.ld = j.ld;
      q.m = j.ne;
      q.ncols = j.ncols;
      q.ne = j.ne;
      q.p0 = p0;
      q.nb = std::min(NB, j.ne - p0);
      q.piv = piv + a * NB;
      q.G = G + a * NB * NB;
      q.Y = Y + yo[a];
      q.W = W ? W + wo[a] : nullptr;
      q.node = j.node;
      all_pj.push_back(q);
      mm = std::max(mm, j.ne);
      mc = std::max(mc, j.ncols - p0);
      mp = std::max(mp, j.ne - p0);
      mnb = std::max(mnb, q.nb);
    }
    step_cfg.push_back({off, (int)all_pj.size() - off, mm, mc, mp, mnb});
  }
  PanelJob<T> *d_pj = all_pj.empty() ? nullptr : sg.put(all_pj);
  for (const auto &c : step_cfg)
    launch_panel_step<T>(c[1], d_pj + c[0], c[2], c[3], c[4], c[5], err, st);
  // non-pivot rows and R of the large fronts
  const ProductLists pr_big = product_lists(big);
  if (!pr_big.gj.empty())
    launch_gemm_sub<T>((int)pr_big.gj.size(), sg.put(pr_big.gj), pr_big.gm, pr_big.gn, st);
  if (!pr_big.neg.empty())
    launch_axpby<T>((int)pr_big.neg.size(), sg.put(pr_big.neg), pr_big.nm, pr_big.nn, st);
  if (overlap) {
    HSSX_HIP(hipEventRecord(side->join, side->s));
    HSSX_HIP(hipStreamWaitEvent(st, side->join, 0));
  }
  // the panel scratch is released on return (stream-ordered reuse)
  ar.release(mk0);
}

template <typename T>
void factor_impl(hssx_fact_ &P, hipStream_t st, Staging &sg, Arena &ar) {
  hssx_op_ &A = *P.A;
  const Symbolic &sym = P.sym;
  cplx<T> *F = P.front.as<cplx<T>>();
  const FrontDesc *desc = P.desc.as<FrontDesc>();
  // default pivot threshold of the interpolative decomposition: 1e-2 tol,
  // but not below the working precision's noise level
  const double eps = sizeof(T) == sizeof(float) ? 1.1920929e-7 : 2.220446049250313e-16;
  const double id_tol =
      P.opts.id_rel_tol > 0 ? P.opts.id_rel_tol : std::max(1e-2 * P.tol, 4.0 * eps);
  int *err = ar.get<int>(1);
  int *d_err = sg.put(std::vector<int>{-1});
  HSSX_HIP(hipMemcpyAsync(err, d_err, sizeof(int), hipMemcpyDeviceToDevice, st));
  int kmax = 0, rounds_max = 0, ncomp = 0, rounds_sum = 0;
  double est_max = 0;
  // accepted rank cap k of each node's Schur-complement compression; a
  // parent's compressions start from its children's (Algorithm A.1 takes an
  // initial rank guess)
  std::vector<int> kfin(sym.nodes.size(), 0);
  auto record = [&](const CompressTask<T> &t) {
    kmax = std::max(kmax, t.maxrank);
    rounds_max = std::max(rounds_max, t.rounds);
    rounds_sum += t.rounds;
    est_max = std::max(est_max, t.est);
    P.node_rank[t.node] = std::max(P.node_rank[t.node], t.maxrank);
  };

  for (int d = sym.max_depth; d >= 0; --d) {
    const auto &nodes = P.depth_nodes[d];
    if (nodes.empty()) continue;
    const int cnt = (int)nodes.size();
    if (std::is_same<T, float>::value && d == 0) {
      // complex64 factor: the root fronts (top separators) are assembled
      // from the children's complex64 Schur blocks into complex128 storage
      // and eliminated in FP64
      c128 *F64 = P.front64.as<c128>();
      hipEvent_t pa = prof_begin(st);
      launch_front_assemble<double, T>(cnt, P.depth_dev[0].as<int>(), desc, P.src_gid.as<int>(),
                                       P.src_code.as<int>(),
                                       A.rowptr.as<int>(), A.col.as<int>(), A.val.as<c128>(), F,
                                       F64, st, P.depth_max_f[0]);
      prof_end("front_assemble", st, pa, P.asm_bytes[0]);
      std::vector<ElimJob<double>> rj;
      for (int k : nodes) {
        const FrontDesc &fd = P.h_desc[k];
        rj.push_back(ElimJob<double>{F64 + fd.foff, fd.f, fd.f, fd.f + fd.ni, fd.ni, 1, k});
      }
      hipEvent_t pe = prof_begin(st);
      eliminate_jobs<double>(rj, err, sg, ar);
      prof_end("front_eliminate", st, pe, elim_flops(rj));
      HSSX_HIP(hipStreamSynchronize(st));
      sg.recycle();
      continue;
    }
    hipEvent_t pa = prof_begin(st);
    launch_front_assemble<T, T>(cnt, P.depth_dev[d].as<int>(), desc, P.src_gid.as<int>(),
                                P.src_code.as<int>(), A.rowptr.as<int>(),
                                A.col.as<int>(), A.val.as<c128>(), F, F, st, P.depth_max_f[d]);
    prof_end("front_assemble", st, pa, P.asm_bytes[d]);

    // ---- HSS-arithmetic interiors: compress S~ and substitute it (Alg. 3.3)
    std::vector<int> hn;
    for (int k : nodes)
      if (P.arith[k] && sym.nodes[k].parent >= 0 && P.h_desc[k].ni > 0) hn.push_back(k);
    const Arena::Mark depth_mark = ar.mark();
    if (!hn.empty()) {
      long gsz = 0, hsz = 0;
      std::vector<long> goff, hoff;
      for (int k : hn) {
        int ni = P.h_desc[k].ni, p = sym.nodes[sym.nodes[k].lo].p0;
        goff.push_back(gsz);
        hoff.push_back(hsz);
        gsz += (long)ni * ni;
        hsz += (long)(ni - p) * (ni - p);
      }
      cplx<T> *G = ar.get<cplx<T>>(gsz);
      cplx<T> *H = ar.get<cplx<T>>(hsz);
      std::vector<AxpbyJob<T>> cp;
      std::vector<ElimJob<T>> ej;
      std::vector<CompressTask<T>> tasks;
      int mm = 0;
      for (size_t a = 0; a < hn.size(); ++a) {
        int k = hn[a];
        const FrontDesc &fd = P.h_desc[k];
        int ni = fd.ni, p = sym.nodes[sym.nodes[k].lo].p0;
        cplx<T> *g = G + goff[a];
        cp.push_back(AxpbyJob<T>{g, F + fd.foff, nullptr, ni, fd.f, 0, ni, ni, (T)1, (T)0});
        mm = std::max(mm, ni);
        ej.push_back(ElimJob<T>{g, ni, ni, ni, p, 0, k});
        if (ni - p > 0) {
          CompressTask<T> t;
          t.node = k;
          t.kind = 1;
          t.m = ni - p;
          t.k_init = kfin[sym.nodes[k].hi];
          t.ct = interior_subtree(sym.nodes[sym.nodes[k].hi]);
          t.S = g + p + (long)p * ni;
          t.ldS = ni;
          t.target = H + hoff[a];
          t.ldT = ni - p;
          tasks.push_back(std::move(t));
        }
      }
      // G := 0 then G += A_ii; eliminate mu's block: G(p:, p:) = S~
      HSSX_HIP(hipMemsetAsync(G, 0, gsz * sizeof(cplx<T>), st));
      launch_axpby<T>((int)cp.size(), sg.put(cp), mm, mm, st);
      hipEvent_t pe = prof_begin(st);
      eliminate_jobs<T>(ej, err, sg, ar);
      prof_end("front_eliminate", st, pe, elim_flops(ej));
      compress_batch<T>(tasks, P.opts, P.tol, id_tol, sg, ar);
      std::vector<AxpbyJob<T>> fix;
      int fm = 0;
      size_t ti = 0;
      for (size_t a = 0; a < hn.size(); ++a) {
        int k = hn[a];
        const FrontDesc &fd = P.h_desc[k];
        int ni = fd.ni, p = sym.nodes[sym.nodes[k].lo].p0;
        if (ni - p <= 0) continue;
        auto &t = tasks[ti++];
        record(t);
        // F(p:ni, p:ni) += S~_HSS - S~
        fix.push_back(AxpbyJob<T>{F + fd.foff + p + (long)p * fd.f, t.target,
                                  G + goff[a] + p + (long)p * ni, fd.f, ni - p,
                                  ni, ni - p, ni - p, (T)1, (T)-1});
        fm = std::max(fm, ni - p);
      }
      launch_axpby<T>((int)fix.size(), sg.put(fix), fm, fm, st);
    }

    // ---- eliminate all fronts of this depth
    std::vector<ElimJob<T>> jobs;
    for (int k : nodes) {
      const FrontDesc &fd = P.h_desc[k];
      jobs.push_back(ElimJob<T>{F + fd.foff, fd.f, fd.f, fd.f + fd.ni, fd.ni, 1, k});
    }
    hipEvent_t pe = prof_begin(st);
    eliminate_jobs<T>(jobs, err, sg, ar);
    prof_end("front_eliminate", st, pe, elim_flops(jobs));

    // ---- compress the Schur complements the parents will use in HSS form
    std::vector<CompressTask<T>> tasks;
    for (int k : nodes) {
      const FrontDesc &fd = P.h_desc[k];
      if (!P.comp[k] || fd.nb == 0) continue;
      CompressTask<T> t;
      t.node = k;
      t.kind = 0;
      t.m = fd.nb;
      const NDNode &nd = sym.nodes[k];
      if (!nd.leafnode()) t.k_init = std::max(kfin[nd.lo], kfin[nd.hi]);
      t.ct = nd.ct;
      t.S = F + fd.foff + fd.ni + (long)fd.ni * fd.f;
      t.ldS = fd.f;
      t.target = t.S;
      t.ldT = fd.f;
      tasks.push_back(std::move(t));
    }
    if (!tasks.empty()) {
      compress_batch<T>(tasks, P.opts, P.tol, id_tol, sg, ar);
      for (auto &t : tasks) {
        record(t);
        kfin[t.node] = t.k;
        ++ncomp;
      }
    }
    // everything launched for this depth is complete before its scratch
    // (G, H) and the staged descriptors are released
    HSSX_HIP(hipStreamSynchronize(st));
    sg.recycle();
    ar.release(depth_mark);
  }
  int bad = -1;
  HSSX_HIP(hipStreamSynchronize(st));
  HSSX_HIP(hipMemcpy(&bad, err, sizeof(int), hipMemcpyDeviceToHost));
  HSSX_CHECK(bad < 0, HSSX_ESINGULAR, "zero pivot in the dense block of tree node " + std::to_string(bad));
  P.stats.k_max = kmax;
  P.stats.max_rounds_used = rounds_max;
  P.stats.rounds_total = rounds_sum;
  P.stats.max_estimate = est_max;
  P.stats.n_compressed = ncomp;
}

}  // namespace

namespace {
std::mutex g_pool_mu;
std::map<int, std::vector<std::unique_ptr<Arena>>> g_arenas;
std::map<int, std::vector<std::unique_ptr<Staging>>> g_stagings;
}  // namespace

std::unique_ptr<Arena> acquire_arena(int device) {
  std::lock_guard<std::mutex> g(g_pool_mu);
  auto &v = g_arenas[device];
  if (v.empty()) return std::make_unique<Arena>();
  auto a = std::move(v.back());
  v.pop_back();
  return a;
}

void return_arena(int device, std::unique_ptr<Arena> a) {
  a->release(Arena::Mark{0, 0});
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_arenas[device].push_back(std::move(a));
}

std::unique_ptr<Staging> acquire_staging(int device, hipStream_t st) {
  std::unique_ptr<Staging> s;
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto &v = g_stagings[device];
    if (!v.empty()) {
      s = std::move(v.back());
      v.pop_back();
    }
  }
  if (!s) s = std::make_unique<Staging>(st);
  s->set_stream(st);
  return s;
}

void return_staging(int device, std::unique_ptr<Staging> s) {
  s->recycle();
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_stagings[device].push_back(std::move(s));
}

void factor_numeric(hssx_fact_ &P, hipStream_t st) {
  hipEvent_t e0, e1;
  HSSX_HIP(hipEventCreate(&e0));
  HSSX_HIP(hipEventCreate(&e1));
  HSSX_HIP(hipEventRecord(e0, st));
  // scratch arena and pinned staging are taken from per-device caches and
  // returned afterwards (also on error), so repeated factorizations reuse them
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  std::unique_ptr<Arena> ar = acquire_arena(dev);
  std::unique_ptr<Staging> sg = acquire_staging(dev, st);
  try {
    if (P.dtype == HSSX_C128) factor_impl<double>(P, st, *sg, *ar);
    else factor_impl<float>(P, st, *sg, *ar);
  } catch (...) {
    // an error between a fork onto the side stream and its join leaves work
    // there that st does not wait for: drain the device before the arena and
    // the staging areas are handed on
    (void)hipDeviceSynchronize();
    return_arena(dev, std::move(ar));
    return_staging(dev, std::move(sg));
    throw;
  }
  return_arena(dev, std::move(ar));
  return_staging(dev, std::move(sg));
  HSSX_HIP(hipEventRecord(e1, st));
  HSSX_HIP(hipEventSynchronize(e1));
  float ms = 0;
  HSSX_HIP(hipEventElapsedTime(&ms, e0, e1));
  P.stats.ms_numeric = ms;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
}

namespace {

// ---- apply tile autotuner: tile configuration per (factor precision,
// sweep, right-hand-side bucket, size bucket, node-count bucket), measured
// once per process on scratch vectors and shared by all factors
std::mutex g_tune_mu;
std::map<std::array<int, 5>, int> g_tuned;

int log2_bucket(long v) {
  int b = 0;
  while ((1L << b) < v) ++b;
  return b;
}

// launches one depth's up (or down) step with tile configuration cfg
void sweep_step(hssx_fact_ &P, int d, bool up, int trans, int nrhs, c128 *w, c128 *tb, int cfg,
                hipStream_t st) {
  const int n = P.A->n, cnt = (int)P.depth_nodes[d].size();
  const FrontDesc *desc = P.desc.as<FrontDesc>();
  const int *nodes = P.depth_dev[d].as<int>();
  const bool f64 = P.dtype == HSSX_C128 || d == 0;
  const c128 *pool64 = P.dtype == HSSX_C64 ? P.front64.as<c128>() : P.front.as<c128>();
  if (up) {
    if (f64)
      launch_apply_up<double>(cnt, nodes, desc, pool64, P.bpos.as<int>(), tb, w, n, nrhs, trans,
                              P.depth_max_ni[d], P.depth_max_f[d], cfg, st);
    else
      launch_apply_up<float>(cnt, nodes, desc, P.front.as<c64>(), P.bpos.as<int>(), tb, w, n,
                             nrhs, trans, P.depth_max_ni[d], P.depth_max_f[d], cfg, st);
  } else {
    if (f64)
      launch_apply_down<double>(cnt, nodes, desc, pool64, P.bpos.as<int>(), w, n, nrhs, trans,
                                P.depth_max_nb[d], P.depth_max_ni[d], cfg, st);
    else
      launch_apply_down<float>(cnt, nodes, desc, P.front.as<c64>(), P.bpos.as<int>(), w, n, nrhs,
                               trans, P.depth_max_nb[d], P.depth_max_ni[d], cfg, st);
  }
}

std::array<int, 5> tune_key(const hssx_fact_ &P, int d, bool up, int nrhs) {
  const bool f64 = P.dtype == HSSX_C128 || d == 0;
  const int size = up ? P.depth_max_f[d] : P.depth_max_ni[d];
  return {f64 ? 0 : 1, up ? 0 : 1, log2_bucket(nrhs), log2_bucket(size),
          log2_bucket((long)P.depth_nodes[d].size())};
}

// tile configuration of every depth and sweep for nrhs right-hand sides;
// missing entries of the process cache are measured (events, best of 2)
void tune_apply(hssx_fact_ &P, int nrhs, hipStream_t st) {
  if (P.cfg_up.count(nrhs)) return;
  const int D = P.sym.max_depth, n = P.A->n;
  std::vector<int> up(D + 1, 2), down(D + 1, 2);
  if (!P.opts.autotune) {
    P.cfg_up[nrhs] = up;
    P.cfg_down[nrhs] = down;
    return;
  }
  std::lock_guard<std::mutex> g(g_tune_mu);
  DevBuf x2, t2;
  hipEvent_t e0, e1;
  bool have_bufs = false;
  for (int d = 0; d <= D; ++d) {
    if (P.depth_nodes[d].empty()) continue;
    for (int u = 0; u < 2; ++u) {
      const auto key = tune_key(P, d, u == 0, nrhs);
      auto it = g_tuned.find(key);
      if (it != g_tuned.end()) {
        (u == 0 ? up : down)[d] = it->second;
        continue;
      }
      if (!have_bufs) {
        x2.alloc((size_t)n * nrhs * sizeof(c128));
        t2.alloc((size_t)n * nrhs * sizeof(c128));
        HSSX_HIP(hipMemsetAsync(x2.p, 0, x2.bytes, st));
        HSSX_HIP(hipMemsetAsync(t2.p, 0, t2.bytes, st));
        HSSX_HIP(hipEventCreate(&e0));
        HSSX_HIP(hipEventCreate(&e1));
        have_bufs = true;
      }
      int best = 2;
      float best_ms = 1e30f;
      for (int c = 0; c < kNumApplyCfgs; ++c) {
        sweep_step(P, d, u == 0, 0, nrhs, x2.as<c128>(), t2.as<c128>(), c, st);
        for (int rep = 0; rep < 2; ++rep) {
          HSSX_HIP(hipEventRecord(e0, st));
          sweep_step(P, d, u == 0, 0, nrhs, x2.as<c128>(), t2.as<c128>(), c, st);
          HSSX_HIP(hipEventRecord(e1, st));
          HSSX_HIP(hipEventSynchronize(e1));
          float ms = 0;
          HSSX_HIP(hipEventElapsedTime(&ms, e0, e1));
          if (ms < best_ms) { best_ms = ms; best = c; }
        }
      }
      g_tuned[key] = best;
      (u == 0 ? up : down)[d] = best;
    }
  }
  if (have_bufs) {
    HSSX_HIP(hipStreamSynchronize(st));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  P.cfg_up[nrhs] = up;
  P.cfg_down[nrhs] = down;
}

// Algorithm 3.1 on vectors in elimination order: up-sweep with the fused
// block solve depth by depth from the leaves, then the down-sweep
void sweeps(hssx_fact_ &P, int trans, int nrhs, c128 *w, c128 *tb, hipStream_t st) {
  const int D = P.sym.max_depth;
  const auto &cu = P.cfg_up.at(nrhs), &cd = P.cfg_down.at(nrhs);
  const bool prof = prof_on() && !P.capturing;
  for (int d = D; d >= 0; --d) {
    if (P.depth_nodes[d].empty()) continue;
    hipEvent_t pu = prof ? prof_begin(st) : nullptr;
    sweep_step(P, d, true, trans, nrhs, w, tb, cu[d], st);
    if (prof) prof_end("apply_up", st, pu, P.up_fbytes[d] + P.up_velems[d] * nrhs * sizeof(c128));
  }
  for (int d = 0; d <= D; ++d) {
    if (P.depth_nodes[d].empty()) continue;
    hipEvent_t pd = prof ? prof_begin(st) : nullptr;
    sweep_step(P, d, false, trans, nrhs, w, tb, cd[d], st);
    if (prof)
      prof_end("apply_down", st, pd, P.down_fbytes[d] + P.down_velems[d] * nrhs * sizeof(c128));
  }
}

}  // namespace

void destroy_graphs(hssx_fact_ &P) {
  for (auto &g : P.graphs) (void)hipGraphExecDestroy(g.exec);
  P.graphs.clear();
}

void apply(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y, long ldy,
           hipStream_t st) {
  const int n = P.A->n;
  if (P.work_cols < (size_t)nrhs) {
    HSSX_HIP(hipStreamSynchronize(st));
    destroy_graphs(P);   // they hold the old workspace's addresses
    P.work.alloc((size_t)2 * n * nrhs * sizeof(c128));
    P.work_cols = nrhs;
  }
  c128 *w = P.work.as<c128>();
  c128 *tb = w + (size_t)n * nrhs;
  tune_apply(P, nrhs, st);
  launch_permute(n, nrhs, P.perm.as<int>(), x, ldx, w, n, 0, st);
  if (P.opts.apply_graph) {
    // the sweeps on the internal workspace replayed as one graph per
    // (right-hand-side count, transpose)
    hipGraphExec_t exec = nullptr;
    for (auto &g : P.graphs)
      if (g.nrhs == nrhs && g.trans == trans) exec = g.exec;
    if (!exec) {
      if (!P.cap_stream) HSSX_HIP(hipStreamCreateWithFlags(&P.cap_stream, hipStreamNonBlocking));
      HSSX_HIP(hipStreamBeginCapture(P.cap_stream, hipStreamCaptureModeThreadLocal));
      hipGraph_t graph = nullptr;
      P.capturing = true;
      try {
        sweeps(P, trans, nrhs, w, tb, P.cap_stream);
      } catch (...) {
        P.capturing = false;
        (void)hipStreamEndCapture(P.cap_stream, &graph);
        if (graph) (void)hipGraphDestroy(graph);
        throw;
      }
      P.capturing = false;
      HSSX_HIP(hipStreamEndCapture(P.cap_stream, &graph));
      hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      HSSX_HIP(e);
      P.graphs.push_back(hssx_fact_::SweepGraph{nrhs, trans, exec});
    }
    hipEvent_t pg = prof_begin(st);
    HSSX_HIP(hipGraphLaunch(exec, st));
    double bytes = 0;
    for (int d = 0; d <= P.sym.max_depth; ++d)
      bytes += P.up_fbytes[d] + P.down_fbytes[d] +
               (P.up_velems[d] + P.down_velems[d]) * nrhs * sizeof(c128);
    prof_end("apply_graph", st, pg, bytes);
  } else {
    sweeps(P, trans, nrhs, w, tb, st);
  }
  launch_permute(n, nrhs, P.perm.as<int>(), w, n, y, ldy, 1, st);
}

}  // namespace hssx
