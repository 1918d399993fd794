// Numeric factorization P = LDR (Algorithm 3.4) and its application
// (Algorithm 3.1).
//
// Nodes are processed one tree depth at a time, deepest first; all nodes of
// a depth are independent (their boxes are disjoint).  Node classes (by
// height, the switching rule): dense (height <= h_sw, and the roots) and
// HSS-class (height > h_sw, not a root).  Per depth:
//   1. dense nodes: assemble the augmented fronts (eq. 3.2 at leaves,
//      eq. 3.4 above) and eliminate them by Gauss-Jordan (A_ii^-1, R, L, S);
//   2. HSS-class nodes (Sec. 3.3-3.5), from the children's Schur complements
//      in generator form: telescoping inverse of S_ii^mu; the inner Schur
//      complement S~ = S_ii^nu - A~(nu,mu) (S_ii^mu)^-1 A~(mu,nu) compressed
//      by Algorithm A.1 from products (telescoping products, sparse
//      couplings, telescoping solves) and entries (entry access to the HSS
//      forms); telescoping inverse of S~ (Alg. 3.3); low-rank Gauss
//      transforms A_ib = X_I Y_B^T, W = A_ii^-1 X_I, C = X_I^T W (eq. 3.7);
//   3. Schur complements of nodes whose parent uses HSS arithmetic are
//      compressed by Algorithm A.1: the dense S of a dense node, and
//      S(sigma) = A_bb - Y_B C Y_B^T of an HSS-class node from products and
//      entries without forming it (Sec. 3.5).  The generators are kept; a
//      dense parent (a root) gets the expansion in its children's blocks.
// The compressions of a depth are batched: all instances sample, compress
// level by level, and estimate together; only those whose estimate
// (eq. 2.7) misses the tolerance grow k <- k + r and go round again.
#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
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
  std::vector<ElimJob<T>> in_lds, rows_done, reg2;
  size_t lds = 0;
  for (const auto &j : jobs) {
    const size_t b = (size_t)j.ne * j.ncols * sizeof(cplx<T>);
    if (j.ne >= kSmall && j.ne <= 128 && j.m == j.ne && !j.negate_r &&
        j.ncols - j.m <= eliminate_reg_max_cols<T>(j.ne)) {
      // square blocks of 64-128 pivots: one register-resident workgroup each
      reg2.push_back(j);
    } else if (j.ne < kSmall && j.ne > 0 && b <= kLdsMax) {
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
    d_order = sg.put_const(order);
  }
  if (!small.empty()) d_small = sg.put_const(small);
  int *queue2 = nullptr;
  ElimJob<T> *d_reg2 = nullptr;
  int reg2_m = 0, reg2_w = 0;
  if (!reg2.empty()) {
    std::stable_sort(reg2.begin(), reg2.end(), [](const ElimJob<T> &a, const ElimJob<T> &b) {
      return (long)a.ne * a.ncols > (long)b.ne * b.ncols;
    });
    for (const auto &j : reg2) {
      reg2_m = std::max(reg2_m, j.ne);
      reg2_w = std::max(reg2_w, j.ncols - j.m);
    }
    queue2 = sg.put(std::vector<int>{0});
    d_reg2 = sg.put_const(reg2);
  }
  // products over the non-pivot rows and the negation of R for the fronts
  // eliminated in LDS, queued on the same stream right after them
  const ProductLists pr_done = product_lists(rows_done);
  GemmJob<T> *d_gd = pr_done.gj.empty() ? nullptr : sg.put_const(pr_done.gj);
  AxpbyJob<T> *d_nd = pr_done.neg.empty() ? nullptr : sg.put_const(pr_done.neg);
  SideStream *side = overlap ? &side_stream() : nullptr;
  hipStream_t fs = st;
  if (overlap) {
    HSSX_HIP(hipEventRecord(side->fork, st));
    HSSX_HIP(hipStreamWaitEvent(side->s, side->fork, 0));
    fs = side->s;
  }
  if (d_order) {
    // register-resident Gauss-Jordan when every block fits, else staged in LDS
    int max_m = 0, max_nc = 0;
    for (const auto &j : in_lds) {
      max_m = std::max(max_m, j.m);
      max_nc = std::max(max_nc, j.ncols - j.m);
    }
    if (!launch_eliminate_reg<T>((int)in_lds.size(), d_order, err, fs, max_m, max_nc, queue))
      launch_eliminate<T>((int)in_lds.size(), d_order, err, fs, lds, queue);
  }
  if (d_small) launch_eliminate<T>((int)small.size(), d_small, err, fs);
  if (d_reg2)
    HSSX_CHECK(launch_eliminate_reg<T>((int)reg2.size(), d_reg2, err, st, reg2_m, reg2_w, queue2),
               HSSX_EINVAL, "register elimination sizes");
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
  PanelJob<T> *d_pj = all_pj.empty() ? nullptr : sg.put_const(all_pj);
  for (const auto &c : step_cfg)
    launch_panel_step<T>(c[1], d_pj + c[0], c[2], c[3], c[4], c[5], err, st);
  // non-pivot rows and R of the large fronts
  const ProductLists pr_big = product_lists(big);
  if (!pr_big.gj.empty())
    launch_gemm_sub<T>((int)pr_big.gj.size(), sg.put_const(pr_big.gj), pr_big.gm, pr_big.gn, st);
  if (!pr_big.neg.empty())
    launch_axpby<T>((int)pr_big.neg.size(), sg.put_const(pr_big.neg), pr_big.nm, pr_big.nn, st);
  if (overlap) {
    HSSX_HIP(hipEventRecord(side->join, side->s));
    HSSX_HIP(hipStreamWaitEvent(st, side->join, 0));
  }
  // the panel scratch is released on return (stream-ordered reuse)
  ar.release(mk0);
}

template void eliminate_jobs<float>(const std::vector<ElimJob<float>> &, int *, Staging &, Arena &);
template void eliminate_jobs<double>(const std::vector<ElimJob<double>> &, int *, Staging &,
                                     Arena &);

namespace {

// One Algorithm A.1 call.  The operator is either a dense block (S, ldS) or
// structured (S null): entries then come from the entry operator eop
// (launch_entries, before each tree level) and samples from the depth's
// structured sampler (item sid).
template <typename T> struct CompressTask {
  int node = 0, kind = 0;
  int m = 0;
  int k_init = 0;   // initial rank guess (0: the option k0)
  ClusterTree ct;
  const cplx<T> *S = nullptr;
  int ldS = 0;
  int eop = -1, sid = -1;
  cplx<T> *target = nullptr;   // dense expansion of the result (or null)
  int ldT = 0;
  HssMat<T> *out = nullptr;    // generators of the result (or null)
  // state / results
  int k = 0, s = 0, rounds = 0, cap = 0;
  double est = 0, est_prev = 0;
  int maxrank = 0;
  bool done = false, above_tol = false;
  long ooff = 0, yoff = 0;
};

// samples of structured operators: Y (m x nc, ld ldY) = Op Omega (ld ldO)
template <typename T> struct SampleReq {
  int task;
  const double *Om;
  long ldO;
  cplx<T> *Y;
  long ldY;
  int nc;
};
template <typename T>
using StructSampler = std::function<void(Prog<T> &, const std::vector<SampleReq<T>> &,
                                         const std::vector<CompressTask<T>> &, const Alloc<T> &)>;

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

// nominal flops of one cluster's step of Algorithm A.1 (interpolative
// decomposition by column-pivoted QR: 4 (2 rows s k - (rows + s) k^2 +
// 2 k^3 / 3) for a complex rows x s block of rank k), plus the local
// samples, the interpolation matrix and the reduced sketch
inline double compress_flops(const HssCluster &c, const HssInstance &I) {
  const double s = I.s, rows = c.rows_cap, k = std::min<double>(c.k_cap, std::min<double>(rows, s));
  double f = 0;
  if (c.left < 0) f += 4.0 * rows * rows * s;                 // D Omega
  else f += 8.0 * rows * rows * s / 2;                        // B12 Om_r, B21 Om_l
  f += 4.0 * (2.0 * rows * s * k - (rows + s) * k * k + 2.0 * k * k * k / 3.0);
  f += 4.0 * (rows - k) * k * k + 8.0 * k * rows * s;         // T and U^T Omega
  return f;
}

// staged job-array bytes of one factorization before the staging area is
// reused from its start (after a stream synchronisation at a depth boundary)
constexpr size_t kStageCap = size_t(512) << 20;
// rows of one local sample block the compression kernel holds
constexpr int kMaxLocalRows = 1024;
// acceptance slack of a stalled complex64 estimate, relative to tol
constexpr double kStallSlack = 10.0;
// a complex64 round that keeps more than this fraction of the previous
// estimate makes no progress
constexpr double kNoProgress = 0.7;

struct CompressAcc {
  double flops = 0;
  int n_above_tol = 0;
};

template <typename T>
void compress_batch(std::vector<CompressTask<T>> &tasks, const hssx_factor_opts &o, double tol,
                    double id_tol, Staging &sg, Arena &ar, Arena &store, const hssx_op_ &A,
                    const std::vector<EntryOp<T>> &eops, const StructSampler<T> &sampler,
                    CompressAcc &acc) {
  if (tasks.empty()) return;
  const hipStream_t st = sg.stream();
  const int k0 = o.k0, r = o.r;
  const c128 *val = A.val.as<c128>();
  long osz = 0, ysz = 0;
  // sample columns one compression kernel holds
  constexpr int kMaxCols = 1024;
  for (auto &t : tasks) {
    // the initial rank guess stays below the capacity (s + r probes fit)
    t.k = std::max(1, std::min(std::min(std::max(k0, t.k_init), t.m), kMaxCols - 2 * r));
    t.s = t.k + r;
    // room for every round up to k >= m (s = k + r samples + r probes), at
    // most the kernel's capacity: a compression that reaches it stops there
    // (counted above tol when its estimate misses)
    t.cap = std::min(t.k + r * (o.max_rounds + 1), t.m + 3 * r);
    t.cap = std::min(kMaxCols, std::max(t.cap, t.s + r));
    t.ooff = osz;
    t.yoff = ysz;
    osz += (long)t.m * t.cap;
    ysz += (long)t.m * t.cap;
    t.rounds = 0;
    t.done = false;
    HSSX_CHECK(t.cap <= 1024, HSSX_EINVAL, "sample block wider than the compression kernel holds");
    HSSX_CHECK(t.m <= 1 << 24, HSSX_EINVAL, "compression size");
    HSSX_CHECK(t.S || (t.eop >= 0 && t.sid >= 0), HSSX_EINVAL, "compression without operator");
  }
  // sketches and samples live until the last round; each round's generator
  // pools are released once the round has been synchronised
  double *Om = ar.get<double>(osz);
  cplx<T> *Y = ar.get<cplx<T>>(ysz);
  double *d_err = ar.get<double>(2 * tasks.size());
  const EntryOp<T> *d_eops = eops.empty() ? nullptr : sg.put_const(eops);
  Alloc<T> scratch = [&](size_t n) { return ar.get<cplx<T>>(n); };

  auto gen_and_sample = [&](const std::vector<int> &ids, bool probe) {
    std::vector<GaussJob> gj;
    std::vector<SampleJob<T>> sj;
    std::vector<SampleReq<T>> sr;
    int mm = 0, mc = 0, gm = 0, gc = 0;
    for (int i : ids) {
      auto &t = tasks[i];
      int c0 = probe ? t.s : 0, nc = probe ? r : t.s;
      GaussJob g{Om + t.ooff, t.m, t.m, c0, nc, 0, (uint32_t)(4 * t.node + t.kind)};
      gj.push_back(g);
      gm = std::max(gm, t.m);
      gc = std::max(gc, nc);
      if (t.S) {
        SampleJob<T> s{t.S, Om + t.ooff + (long)c0 * t.m, Y + t.yoff + (long)c0 * t.m,
                       t.ldS, t.m, t.m, t.m, nc};
        sj.push_back(s);
        mm = std::max(mm, t.m);
        mc = std::max(mc, nc);
      } else {
        sr.push_back(SampleReq<T>{i, Om + t.ooff + (long)c0 * t.m, t.m,
                                  Y + t.yoff + (long)c0 * t.m, t.m, nc});
      }
    }
    GaussJob *dg = sg.put_const(gj);
    launch_gaussian((int)gj.size(), dg, o.seed, gm, gc, st);
    if (!sj.empty()) {
      SampleJob<T> *ds = sg.put_const(sj);
      double sflops = 0;
      for (const auto &q : sj) sflops += 4.0 * q.m * (double)q.m * q.nc;
      acc.flops += sflops;
      hipEvent_t ps = prof_begin(st);
      if constexpr (std::is_same<T, float>::value) {
        if (o.sample_bf16) launch_sample_bf16((int)sj.size(), ds, mm, mc, o.sample_bf16, st);
        else launch_sample<T>((int)sj.size(), ds, mm, mc, st);
      } else {
        launch_sample<T>((int)sj.size(), ds, mm, mc, st);
      }
      prof_end("sample", st, ps, sflops);
    }
    if (!sr.empty()) {
      Prog<T> p;
      sampler(p, sr, tasks, scratch);
      hipEvent_t ps = prof_begin(st);
      run_prog(p, sg, val, st);
      prof_end("sample_struct", st, ps, p.flops);
      acc.flops += p.flops;
    }
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
      h.pre = t.S ? 0 : 1;
      h.eop = t.S ? -1 : t.eop;
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
    // dense operators live in the front pool: the kernel adds soff to the
    // first dense task's S (structured instances never read it)
    const cplx<T> *base = nullptr;
    for (int i : active)
      if (tasks[i].S) { base = tasks[i].S; break; }
    for (size_t a = 0; a < active.size(); ++a)
      inst[a].soff = tasks[active[a]].S ? tasks[active[a]].S - base : 0;

    HssInstance *d_inst = sg.put_const(inst);
    HssCluster *d_cls = sg.put_const(cls);
    // generator pools live in the factor's storage: an accepted instance's
    // generators stay where the compression wrote them
    cplx<T> *d_pool = store.get<cplx<T>>(pool);
    int *d_ipool = ar.get<int>(ipool);
    int *d_rank = ar.get<int>(cls.size());
    long scratch_sz = 0;
    for (long v : lev_scr) scratch_sz = std::max(scratch_sz, v);
    cplx<T> *d_scr = ar.get<cplx<T>>(scratch_sz);
    HSSX_HIP(hipMemsetAsync(d_rank, 0, cls.size() * sizeof(int), st));

    // ---- bottom-up compression, one launch per cluster-tree level and size
    // class (clusters of at most 64 rows in small workgroups; the larger
    // ones in large workgroups, split by whether they fit the register path);
    // the entries of structured operators go into the pool right before
    // their level's launches
    std::vector<HssItem> all_items, ent_items;
    std::vector<std::array<long, 4>> launches;   // level, size class, offset, count
    std::vector<std::array<long, 2>> ent_of;     // per level: offset, count of entry items
    for (int lev = maxlev; lev >= 0; --lev) {
      std::vector<HssItem> items[7];
      const long e0 = (long)ent_items.size();
      for (size_t a = 0; a < active.size(); ++a) {
        for (int c = inst[a].lev_off[std::min(lev, inst[a].nlev)];
             c < inst[a].lev_off[std::min(lev + 1, inst[a].nlev)]; ++c) {
          const int rc = cls[inst[a].cl_off + c].rows_cap, sc = inst[a].s;
          int v;
          if (rc <= 64) v = sc <= 64 ? kCls256S64 : sc <= 128 ? kCls256S128 : kCls256;
          else if (rc <= kRegRows && sc <= kRegCols)
            v = rc > 128 ? kCls1024 : sc <= 64 ? kCls1024R128S64 : sc <= 128 ? kCls1024R128S128
                                                                             : kCls1024;
          else v = kClsGlobal;
          items[v].push_back(HssItem{(int)a, c});
          if (inst[a].pre) ent_items.push_back(HssItem{(int)a, c});
        }
      }
      ent_of.push_back({e0, (long)ent_items.size() - e0});
      // the one-barrier 1024-thread variants hold one workgroup per CU: used
      // when the level's large clusters all fit them and do not outnumber the
      // CUs (otherwise occupancy, or running with the global-memory ones in
      // one launch, matters more)
      const int big[3] = {kCls1024, kCls1024R128S64, kCls1024R128S128};
      size_t nbig = 0;
      for (int v : big) nbig += items[v].size();
      if (nbig > 256 || !items[kClsGlobal].empty())
        for (int v : big) {
          items[kClsGlobal].insert(items[kClsGlobal].end(), items[v].begin(), items[v].end());
          items[v].clear();
        }
      for (int sz = 0; sz < 7; ++sz) {
        if (items[sz].empty()) continue;
        launches.push_back({lev, sz, (long)all_items.size(), (long)items[sz].size()});
        all_items.insert(all_items.end(), items[sz].begin(), items[sz].end());
      }
    }
    HssItem *d_all = all_items.empty() ? nullptr : sg.put_const(all_items);
    HssItem *d_ent = ent_items.empty() ? nullptr : sg.put_const(ent_items);
    // the small-cluster launch of a level is independent of its large-cluster
    // launches (different clusters, same inputs): when a level has both, the
    // small one runs on a side stream, forked from and joined back into st
    SideStream &side = side_stream();
    for (size_t a = 0; a < launches.size();) {
      size_t b = a;
      while (b < launches.size() && launches[b][0] == launches[a][0]) ++b;
      const auto &eo = ent_of[maxlev - launches[a][0]];
      if (eo[1] > 0) {
        hipEvent_t pe = prof_begin(st);
        launch_entries<T>((int)eo[1], d_ent + eo[0], d_inst, d_cls, d_pool, d_ipool, d_rank,
                          d_eops, A.rowptr.as<int>(), A.col.as<int>(), val, st);
        prof_end("hss_entries", st, pe, 0.0);
      }
      // the 256-thread launches run on the side stream when the level also
      // has 1024-thread ones
      auto small = [](long v) { return v == kCls256 || v == kCls256S64 || v == kCls256S128; };
      bool any_small = false, any_big = false;
      for (size_t e = a; e < b; ++e) (small(launches[e][1]) ? any_small : any_big) = true;
      const bool fork = any_small && any_big;
      if (fork) {
        HSSX_HIP(hipEventRecord(side.fork, st));
        HSSX_HIP(hipStreamWaitEvent(side.s, side.fork, 0));
      }
      for (size_t e = a; e < b; ++e) {
        const auto &l = launches[e];
        hipStream_t ls = fork && small(l[1]) ? side.s : st;
        double cflops = 0;
        for (long q = l[2]; q < l[2] + l[3]; ++q) {
          const auto &it = all_items[q];
          cflops += compress_flops(cls[inst[it.inst].cl_off + it.cl], inst[it.inst]);
        }
        acc.flops += cflops;
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
    MatvecJob<T> *d_mj = sg.put_const(mj);
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

    // ---- decisions; the accepted instances are made symmetric, expanded
    // into their targets and kept in generator form
    std::vector<int> next, acc_ids;
    std::vector<MatvecJob<T>> ej;
    std::vector<SymJob<T>> sj;
    long xh2_total = 0, sym_max = 0;
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
      // complex64 operators carry rounding noise of relative size ~ eps_fp32
      // sqrt(m): once the estimate sits within kStallSlack of tol and another
      // r columns no longer halve it, the rank is chasing that noise.  Far
      // above tol the same holds when a round improves the estimate by less
      // than kNoProgress: the operator's entries and products then disagree
      // at that level (rounding of a telescoping inverse of ill-conditioned
      // blocks), and more rank cannot remove it
      if (sizeof(T) == sizeof(float) && t.rounds >= 2 &&
          ((t.est <= kStallSlack * tol && t.est > 0.5 * t.est_prev) ||
           t.est > kNoProgress * t.est_prev))
        accept = true;
      if (!accept) {
        t.k += r;
        t.s += r;
        next.push_back(active[a]);
        continue;
      }
      t.done = true;
      // stopped above the tolerance (round or capacity limit, or the
      // complex64 noise floor): counted and reported
      t.above_tol = t.est > tol && t.k < t.m;
      if (t.above_tol) ++acc.n_above_tol;
      acc_ids.push_back((int)a);
      cplx<T> *P0 = d_pool + inst[a].pool;
      for (int c = 0; c < t.ct.count(); ++c) {
        const HssCluster &C = cls[inst[a].cl_off + c];
        if (C.left < 0) {
          sj.push_back(SymJob<T>{P0 + C.D, P0 + C.D, C.size, C.size, C.size, C.size});
          sym_max = std::max(sym_max, (long)C.size * C.size);
        } else {
          const int kl = h_rank[inst[a].cl_off + C.left], kr = h_rank[inst[a].cl_off + C.right];
          if (kl && kr) {
            sj.push_back(SymJob<T>{P0 + C.B12, P0 + C.B21, kl, kr, kl, kr});
            sym_max = std::max(sym_max, (long)kl * kr);
          }
        }
      }
      if (!t.target) continue;
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
    if (!sj.empty()) launch_symmetrize<T>((int)sj.size(), sg.put_const(sj), sym_max, st);
    if (!ej.empty()) {
      MatvecJob<T> *d_ej = sg.put_const(ej);
      cplx<T> *d_xh2 = ar.get<cplx<T>>(xh2_total);
      hipEvent_t pm2 = prof_begin(st);
      launch_hss_matvec<T>((int)ej.size(), d_ej, d_inst, d_cls, d_pool, d_rank, d_xh2,
                           maxlev + 1, max_width, max_ncl, st);
      prof_end("hss_matvec", st, pm2, 0.0);
    }
    for (int a : acc_ids) {
      auto &t = tasks[active[a]];
      if (!t.out) continue;
      cplx<T> *dst = d_pool + inst[a].pool;
      HssMat<T> &H = *t.out;
      H.m = t.m;
      H.ct = t.ct;
      const int nc = t.ct.count();
      H.k.assign(nc, 0);
      H.U.assign(nc, nullptr);
      H.D.assign(nc, nullptr);
      H.B12.assign(nc, nullptr);
      H.B21.assign(nc, nullptr);
      for (int c = 0; c < nc; ++c) {
        const HssCluster &C = cls[inst[a].cl_off + c];
        H.k[c] = c == 0 ? 0 : h_rank[inst[a].cl_off + c];
        H.U[c] = dst + C.U;
        if (C.left < 0) H.D[c] = dst + C.D;
        else {
          H.B12[c] = dst + C.B12;
          H.B21[c] = dst + C.B21;
        }
      }
    }
    // the round's pools go back to the arena; later kernels that reuse the
    // memory are ordered after the expansion and the copies on the same stream
    ar.release(round_mark);
    active.swap(next);
  }
}

}  // namespace

namespace {

template <typename T> std::vector<HssNodeData<T>> &hdata(hssx_fact_ &P);
template <> std::vector<HssNodeData<float>> &hdata<float>(hssx_fact_ &P) { return P.h32; }
template <> std::vector<HssNodeData<double>> &hdata<double>(hssx_fact_ &P) { return P.h64; }

// Working state of one HSS-class node while its depth is factored.
template <typename T> struct HssLocal {
  int node = -1;
  const HssSym *hs = nullptr;
  HssNodeData<T> *nd = nullptr;
  const HssMat<T> *Smu = nullptr, *Snu = nullptr;
  Gen<T> gmu, gnu, gii_mu, gbb_mu, gii_nu, gbb_nu, xg;
  EntPrep<T> emu, enu, ex;
  EntView<T> vmu{}, vnu{}, vx{};
  cplx<T> *YC = nullptr;   // Y_B C (nb x r)
  cplx<T> *YCt = nullptr, *YBt = nullptr;   // (Y_B C)^T and Y_B^T (r x nb)
  int kmu = 0, knu = 0;    // columns of Y_B from mu's and nu's S_ib
};

// entry descriptors of many matrices in one upload
template <typename T>
std::vector<EntView<T>> upload_views(const std::vector<const EntPrep<T> *> &ep, Staging &sg) {
  std::vector<char> h;
  std::vector<size_t> oc, ol;
  auto put = [&](const void *src, size_t bytes) {
    const size_t off = (h.size() + 63) / 64 * 64;
    h.resize(off + std::max<size_t>(bytes, 1));
    if (bytes) std::memcpy(h.data() + off, src, bytes);
    return off;
  };
  for (const auto *e : ep) {
    oc.push_back(put(e->cl.data(), e->cl.size() * sizeof(EntCl<T>)));
    ol.push_back(put(e->leaf_of.data(), e->leaf_of.size() * sizeof(int)));
  }
  std::vector<EntView<T>> v(ep.size());
  if (ep.empty()) return v;
  const char *d = sg.put_const(h);
  for (size_t i = 0; i < ep.size(); ++i)
    v[i] = EntView<T>{(const EntCl<T> *)(d + oc[i]), (const int *)(d + ol[i])};
  return v;
}

// Algorithm 3.3 (with the index reading of Alg. 3.2 for the B21 block):
// Y = A_ii^-1 X for A_ii = [[S_ii^mu, A~(mu,nu)], [A~(nu,mu), S_ii^nu]],
//   X1 <- (S_ii^mu)^-1 X1;  X2 <- X2 - A~(nu,mu) X1;  X2 <- S~^-1 X2;
//   X1 <- X1 - (S_ii^mu)^-1 A~(mu,nu) X2,
// both inverses in telescoping HSS form.  X and Y must not overlap.
template <typename T> struct A33Item {
  const HssSym *hs;
  const HssNodeData<T> *nd;
  const cplx<T> *X;
  long ldx;
  cplx<T> *Y;
  long ldy;
  int nc;
};

template <typename T>
void alg33(Prog<T> &p, const std::vector<A33Item<T>> &items, const int *ip, const Alloc<T> &alloc) {
  const size_t n = items.size();
  std::vector<cplx<T> *> Z1(n, nullptr), R2(n, nullptr), Tm(n, nullptr), Z3(n, nullptr);
  std::vector<SolveItem<T>> s1, s4, s6;
  for (size_t a = 0; a < n; ++a) {
    const auto &it = items[a];
    const int pm = it.hs->pmu, pn = it.hs->pnu, nc = it.nc;
    if (pm) {
      Z1[a] = alloc((size_t)pm * nc);
      s1.push_back(SolveItem<T>{&it.nd->Hmu, it.X, it.ldx, Z1[a], pm, nc});
    }
    if (pn) {
      R2[a] = alloc((size_t)pn * nc);
      s4.push_back(SolveItem<T>{&it.nd->Hs, R2[a], pn, it.Y + pm, it.ldy, nc});
    }
    if (pm && pn) {
      Tm[a] = alloc((size_t)pm * nc);
      Z3[a] = alloc((size_t)pm * nc);
      s6.push_back(SolveItem<T>{&it.nd->Hmu, Tm[a], pm, Z3[a], pm, nc});
    }
  }
  gym_solve(p, s1, alloc);
  {
    Stage<T> &c = p.add(kCopy);
    for (size_t a = 0; a < n; ++a) {
      const auto &it = items[a];
      const int pm = it.hs->pmu, pn = it.hs->pnu;
      if (pn) c.copy.push_back(CopyJob<T>{it.X + pm, R2[a], (int)it.ldx, pn, pn, it.nc, 0, (T)1});
      if (pm) c.copy.push_back(CopyJob<T>{Z1[a], it.Y, pm, (int)it.ldy, pm, it.nc, 0, (T)1});
    }
  }
  {
    Stage<T> &s = p.add(kSpmm);
    for (size_t a = 0; a < n; ++a) {
      const auto &it = items[a];
      const HssSym &h = *it.hs;
      if (!h.pmu || !h.pnu) continue;
      s.sp.push_back(SpJob<T>{ip + h.inu_rp, ip + h.inu_cp, ip + h.inu_vi, h.pnu, it.nc, 1, Z1[a],
                              h.pmu, R2[a], h.pnu, (T)-1});
    }
  }
  gym_solve(p, s4, alloc);
  {
    Stage<T> &s = p.add(kSpmm);
    for (size_t a = 0; a < n; ++a) {
      const auto &it = items[a];
      const HssSym &h = *it.hs;
      if (!h.pmu || !h.pnu) continue;
      s.sp.push_back(SpJob<T>{ip + h.imu_rp, ip + h.imu_cp, ip + h.imu_vi, h.pmu, it.nc, 0,
                              it.Y + h.pmu, it.ldy, Tm[a], h.pmu, (T)1});
    }
  }
  gym_solve(p, s6, alloc);
  {
    Stage<T> &c = p.add(kCopy);
    for (size_t a = 0; a < n; ++a) {
      const auto &it = items[a];
      if (!Z3[a]) continue;
      c.copy.push_back(CopyJob<T>{Z3[a], it.Y, it.hs->pmu, (int)it.ldy, it.hs->pmu, it.nc, 4, (T)-1});
    }
  }
}

// Subtree roots of a child's cluster tree: [P0 | P1] split at the root when
// both parts exist (Fig. 4), else the whole tree is the one present part.
inline void child_roots(const NDNode &c, int &ii, int &bb, int &split) {
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

}  // namespace

namespace {

template <typename T>
void factor_impl(hssx_fact_ &P, hipStream_t st, Staging &sg, Arena &ar) {
  hssx_op_ &A = *P.A;
  const Symbolic &sym = P.sym;
  cplx<T> *F = P.front.as<cplx<T>>();
  const FrontDesc *desc = P.desc.as<FrontDesc>();
  const c128 *val = A.val.as<c128>();
  const int *ip = P.hsym_pool.as<int>();
  // default pivot threshold of the interpolative decomposition: 1e-2 tol,
  // but not below the working precision's noise level
  const double eps = sizeof(T) == sizeof(float) ? 1.1920929e-7 : 2.220446049250313e-16;
  const double id_tol =
      P.opts.id_rel_tol > 0 ? P.opts.id_rel_tol : std::max(1e-2 * P.tol, 4.0 * eps);
  int *err = ar.get<int>(1);
  int *d_err = sg.put_const(std::vector<int>{-1});
  HSSX_HIP(hipMemcpyAsync(err, d_err, sizeof(int), hipMemcpyDeviceToDevice, st));
  // storage of this factorization's HSS data (the previous one's is dropped:
  // every use of it was queued on this stream before)
  P.store.release(Arena::Mark{0, 0});
  auto &HD = hdata<T>(P);
  HD.clear();
  HD.resize(sym.nodes.size());
  Alloc<T> keep = [&](size_t n) { return P.store.get<cplx<T>>(n); };
  Alloc<T> scratch = [&](size_t n) { return ar.get<cplx<T>>(n); };
  // telescoping inverses of the HSS-class nodes; with wide_inverse a
  // complex64 factor computes them in complex128 (gym_factor_wide) and keeps
  // them in complex64
  auto gym_inverse = [&](std::vector<HssInv<T>> &out, const std::vector<const Gen<T> *> &in,
                         const std::vector<int> &nid, double &gf) {
    if constexpr (std::is_same<T, float>::value) {
      if (P.opts.wide_inverse) {
        Alloc<double> wide = [&](size_t n) { return ar.get<c128>(n); };
        gym_factor_wide(out, in, nid, keep, wide, err, sg, ar, val, st, &gf);
        return;
      }
    }
    gym_factor(out, in, nid, keep, scratch, err, sg, ar, val, st, &gf);
  };
  CompressAcc cacc;
  double flops = 0;
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
  auto dense_parent = [&](int k) {
    const int p = sym.nodes[k].parent;
    return p >= 0 && P.hss_idx[p] < 0;
  };

  for (int d = sym.max_depth; d >= 0; --d) {
    const auto &dn = P.dense_nodes[d], &hn = P.hss_nodes[d];
    if (dn.empty() && hn.empty()) continue;
    const Arena::Mark depth_mark = ar.mark();
    if (std::is_same<T, float>::value && d == 0) {
      // complex64 factor: the root fronts (top separators) are assembled
      // from the children's complex64 Schur blocks into complex128 storage
      // and eliminated in FP64
      c128 *F64 = P.front64.as<c128>();
      hipEvent_t pa = prof_begin(st);
      launch_front_assemble<double, T>((int)dn.size(), P.depth_dev[0].as<int>(), desc,
                                       P.src_gid.as<int>(), P.src_code.as<int>(),
                                       A.rowptr.as<int>(), A.col.as<int>(), val, F, F64, st,
                                       P.depth_max_f[0]);
      prof_end("front_assemble", st, pa, P.asm_bytes[0]);
      std::vector<ElimJob<double>> rj;
      for (int k : dn) {
        const FrontDesc &fd = P.h_desc[k];
        rj.push_back(ElimJob<double>{F64 + fd.foff, fd.f, fd.f, fd.f + fd.ni, fd.ni, 1, k});
      }
      hipEvent_t pe = prof_begin(st);
      eliminate_jobs<double>(rj, err, sg, ar);
      const double ef = elim_flops(rj);
      flops += ef;
      prof_end("front_eliminate", st, pe, ef);
      // stream order makes the depth's scratch reusable by the next one
      ar.release(depth_mark);
      continue;
    }
    // ---- dense fronts: assemble and eliminate
    if (!dn.empty()) {
      hipEvent_t pa = prof_begin(st);
      launch_front_assemble<T, T>((int)dn.size(), P.depth_dev[d].as<int>(), desc,
                                  P.src_gid.as<int>(), P.src_code.as<int>(), A.rowptr.as<int>(),
                                  A.col.as<int>(), val, F, F, st, P.depth_max_f[d]);
      prof_end("front_assemble", st, pa, P.asm_bytes[d]);
      std::vector<ElimJob<T>> jobs;
      for (int k : dn) {
        const FrontDesc &fd = P.h_desc[k];
        jobs.push_back(ElimJob<T>{F + fd.foff, fd.f, fd.f, fd.f + fd.ni, fd.ni, 1, k});
      }
      hipEvent_t pe = prof_begin(st);
      eliminate_jobs<T>(jobs, err, sg, ar);
      const double ef = elim_flops(jobs);
      flops += ef;
      prof_end("front_eliminate", st, pe, ef);
    }

    // ---- HSS-class nodes (Sec. 3.3-3.5)
    std::deque<HssLocal<T>> loc;
    for (int k : hn) {
      HssLocal<T> L;
      L.node = k;
      L.hs = &P.hsym[P.hss_idx[k]];
      L.nd = &HD[k];
      const HssSym &h = *L.hs;
      HSSX_CHECK(HD[h.mu].has_S && HD[h.nu].has_S, HSSX_EINVAL,
                 "HSS-class node without compressed children");
      L.Smu = &HD[h.mu].S;
      L.Snu = &HD[h.nu].S;
      loc.push_back(std::move(L));
    }
    for (auto &L : loc) {
      const HssSym &h = *L.hs;
      L.gmu = L.Smu->gen(0);
      L.gnu = L.Snu->gen(0);
      if (h.ii_mu >= 0) L.gii_mu = L.Smu->gen(h.ii_mu);
      if (h.bb_mu >= 0) L.gbb_mu = L.Smu->gen(h.bb_mu);
      if (h.ii_nu >= 0) L.gii_nu = L.Snu->gen(h.ii_nu);
      if (h.bb_nu >= 0) L.gbb_nu = L.Snu->gen(h.bb_nu);
    }
    std::vector<CompressTask<T>> stask;   // S(sigma) of the HSS-class nodes
    std::vector<EntryOp<T>> sops;
    if (!loc.empty()) {
      // (a) entry access to the children's Schur complements
      {
        Prog<T> p;
        std::vector<EntPrep<T>> ev(2 * loc.size());
        for (size_t a = 0; a < loc.size(); ++a) {
          ev[2 * a].g = &loc[a].gmu;
          ev[2 * a + 1].g = &loc[a].gnu;
        }
        entry_prep(p, ev, scratch);
        hipEvent_t pp = prof_begin(st);
        run_prog(p, sg, val, st);
        prof_end("hss_prep", st, pp, p.flops);
        flops += p.flops;
        std::vector<const EntPrep<T> *> eps;
        for (size_t a = 0; a < loc.size(); ++a) {
          loc[a].emu = std::move(ev[2 * a]);
          loc[a].enu = std::move(ev[2 * a + 1]);
          eps.push_back(&loc[a].emu);
          eps.push_back(&loc[a].enu);
        }
        const std::vector<EntView<T>> vs = upload_views(eps, sg);
        for (size_t a = 0; a < loc.size(); ++a) {
          loc[a].vmu = vs[2 * a];
          loc[a].vnu = vs[2 * a + 1];
        }
      }
      // (b) telescoping inverse of S_ii^mu (Alg. 3.3, first block)
      {
        std::vector<const Gen<T> *> in;
        std::vector<int> nid;
        std::vector<HssLocal<T> *> who;
        for (auto &L : loc)
          if (L.hs->pmu > 0) {
            in.push_back(&L.gii_mu);
            nid.push_back(L.node);
            who.push_back(&L);
          }
        std::vector<HssInv<T>> out;
        hipEvent_t pg = prof_begin(st);
        double gf = 0;
        gym_inverse(out, in, nid, gf);
        prof_end("hss_inverse", st, pg, gf);
        flops += gf;
        for (size_t i = 0; i < who.size(); ++i) who[i]->nd->Hmu = std::move(out[i]);
        // (S_ii^mu)^-1 in HSS form for the entries of S~
        Prog<T> p;
        std::vector<HssInv<T> *> hs;
        for (auto *L : who) hs.push_back(&L->nd->Hmu);
        gym_inverse_blocks(p, hs, scratch, scratch);
        std::vector<EntPrep<T>> ev(who.size());
        for (size_t i = 0; i < who.size(); ++i) {
          who[i]->xg = who[i]->nd->Hmu.inv_gen();
          ev[i].g = &who[i]->xg;
        }
        entry_prep(p, ev, scratch);
        hipEvent_t pp = prof_begin(st);
        run_prog(p, sg, val, st);
        prof_end("hss_prep", st, pp, p.flops);
        flops += p.flops;
        std::vector<const EntPrep<T> *> eps;
        for (size_t i = 0; i < who.size(); ++i) {
          who[i]->ex = std::move(ev[i]);
          eps.push_back(&who[i]->ex);
        }
        const std::vector<EntView<T>> vs = upload_views(eps, sg);
        for (size_t i = 0; i < who.size(); ++i) who[i]->vx = vs[i];
      }
      // (c) inner Schur complement S~ = S_ii^nu - A~(nu,mu) (S_ii^mu)^-1 A~(mu,nu),
      // compressed by Algorithm A.1 from products and entries
      {
        std::vector<CompressTask<T>> tasks;
        std::vector<EntryOp<T>> ops;
        for (size_t a = 0; a < loc.size(); ++a) {
          HssLocal<T> &L = loc[a];
          const HssSym &h = *L.hs;
          if (h.pnu == 0) continue;
          EntryOp<T> op{};
          op.kind = 1;
          op.H0 = h.pmu ? L.vx : L.vnu;
          op.H1 = L.vnu;
          op.rp = ip + h.inu_rp;
          op.cp = ip + h.inu_cp;
          op.vi = ip + h.inu_vi;
          CompressTask<T> t;
          t.node = L.node;
          t.kind = 1;
          t.m = h.pnu;
          t.k_init = kfin[h.nu];
          t.ct = interior_subtree(sym.nodes[h.nu]);
          t.eop = (int)ops.size();
          t.sid = (int)a;
          t.out = &L.nd->St;
          ops.push_back(op);
          tasks.push_back(std::move(t));
        }
        StructSampler<T> samp = [&](Prog<T> &p, const std::vector<SampleReq<T>> &req,
                                    const std::vector<CompressTask<T>> &ts, const Alloc<T> &al) {
          Stage<T> &g = p.add(kGrt);
          std::vector<MvItem<T>> mv;
          std::vector<SolveItem<T>> sv;
          std::vector<cplx<T> *> T1(req.size()), T2(req.size()), Oc(req.size());
          for (size_t q = 0; q < req.size(); ++q) {
            const HssLocal<T> &L = loc[ts[req[q].task].sid];
            const HssSym &h = *L.hs;
            const int nc = req[q].nc;
            Oc[q] = al((size_t)h.pnu * nc);
            g.grt.push_back(GatherJob<double, cplx<T>>{req[q].Om, Oc[q], req[q].ldO, h.pnu,
                                                        nullptr, nullptr, h.pnu, nc, 0, 1.0});
            mv.push_back(MvItem<T>{&L.gii_nu, Oc[q], h.pnu, req[q].Y, req[q].ldY, nc});
            if (h.pmu) {
              T1[q] = al((size_t)h.pmu * nc);
              T2[q] = al((size_t)h.pmu * nc);
              sv.push_back(SolveItem<T>{&L.nd->Hmu, T1[q], h.pmu, T2[q], h.pmu, nc});
            }
          }
          hss_matvec(p, mv, al);
          Stage<T> &s1 = p.add(kSpmm);
          for (size_t q = 0; q < req.size(); ++q) {
            const HssSym &h = *loc[ts[req[q].task].sid].hs;
            if (!h.pmu) continue;
            s1.sp.push_back(SpJob<T>{ip + h.imu_rp, ip + h.imu_cp, ip + h.imu_vi, h.pmu,
                                     req[q].nc, 0, Oc[q], h.pnu, T1[q], h.pmu, (T)1});
          }
          gym_solve(p, sv, al);
          Stage<T> &s2 = p.add(kSpmm);
          for (size_t q = 0; q < req.size(); ++q) {
            const HssSym &h = *loc[ts[req[q].task].sid].hs;
            if (!h.pmu) continue;
            s2.sp.push_back(SpJob<T>{ip + h.inu_rp, ip + h.inu_cp, ip + h.inu_vi, h.pnu,
                                     req[q].nc, 1, T2[q], h.pmu, req[q].Y, req[q].ldY, (T)-1});
          }
        };
        compress_batch<T>(tasks, P.opts, P.tol, id_tol, sg, ar, P.store, A, ops, samp, cacc);
        for (auto &t : tasks) record(t);
      }
      // (d) telescoping inverse of S~
      {
        std::vector<Gen<T>> gs;
        std::vector<HssLocal<T> *> who;
        std::vector<int> nid;
        for (auto &L : loc)
          if (L.hs->pnu > 0) {
            who.push_back(&L);
            nid.push_back(L.node);
          }
        gs.reserve(who.size());
        std::vector<const Gen<T> *> in;
        for (auto *L : who) {
          gs.push_back(L->nd->St.gen(0));
          in.push_back(&gs.back());
        }
        std::vector<HssInv<T>> out;
        hipEvent_t pg = prof_begin(st);
        double gf = 0;
        gym_inverse(out, in, nid, gf);
        prof_end("hss_inverse", st, pg, gf);
        flops += gf;
        for (size_t i = 0; i < who.size(); ++i) who[i]->nd->Hs = std::move(out[i]);
      }
      // (e) low-rank Gauss transforms (eq. 3.7): A_ib = X_I Y_B^T exactly,
      // from the children's top-level generators and the few couplings of A
      // across the children; W = A_ii^-1 X_I (Alg. 3.3), C = X_I^T W
      {
        Prog<T> p;
        Stage<T> &z = p.add(kCopy);
        Stage<T> &c = p.add(kCopy);
        Stage<T> &g = p.add(kGtt);
        Stage<T> &f = p.add(kFill);
        std::vector<cplx<T> *> XI(loc.size());
        for (size_t a = 0; a < loc.size(); ++a) {
          HssLocal<T> &L = loc[a];
          const HssSym &h = *L.hs;
          L.kmu = h.split_mu ? L.Smu->k[h.bb_mu] : 0;
          L.knu = h.split_nu ? L.Snu->k[h.bb_nu] : 0;
          const int r = L.kmu + L.knu + h.ncr;
          L.nd->r = r;
          XI[a] = scratch((size_t)std::max(1, h.ni * r));
          L.nd->W = keep((size_t)std::max(1, h.ni * r));
          L.nd->YB = keep((size_t)std::max(1, h.nb * r));
          if (!r) continue;
          z.copy.push_back(CopyJob<T>{nullptr, XI[a], 0, h.ni, h.ni, r, 3, (T)1});
          z.copy.push_back(CopyJob<T>{nullptr, L.nd->YB, 0, h.nb, h.nb, r, 3, (T)1});
          // S_ib of a child = (full P0 basis) B12 (full P1 basis)^T: X_I takes
          // the first product, Y_B the P1 basis at sigma's boundary positions
          if (L.kmu) {
            const int m1 = h.mmu - h.pmu;
            cplx<T> *Ub = scratch((size_t)m1 * L.kmu);
            c.copy.push_back(CopyJob<T>{L.emu.UB[h.ii_mu], XI[a], L.kmu, h.ni, h.pmu, L.kmu, 1, (T)1});
            c.copy.push_back(CopyJob<T>{L.emu.Uf[h.bb_mu], Ub, L.kmu, m1, m1, L.kmu, 1, (T)1});
            g.gtt.push_back(GatherJob<cplx<T>, cplx<T>>{Ub, L.nd->YB, m1, h.nb, ip + h.smu, nullptr,
                                                        h.nb, L.kmu, 0, 1.0});
          }
          if (L.knu) {
            const int m1 = h.mnu - h.pnu;
            cplx<T> *Ub = scratch((size_t)m1 * L.knu);
            c.copy.push_back(CopyJob<T>{L.enu.UB[h.ii_nu], XI[a] + h.pmu + (long)L.kmu * h.ni,
                                        L.knu, h.ni, h.pnu, L.knu, 1, (T)1});
            c.copy.push_back(CopyJob<T>{L.enu.Uf[h.bb_nu], Ub, L.knu, m1, m1, L.knu, 1, (T)1});
            g.gtt.push_back(GatherJob<cplx<T>, cplx<T>>{Ub, L.nd->YB + (long)L.kmu * h.nb, m1,
                                                        h.nb, ip + h.snu, nullptr, h.nb, L.knu, 0,
                                                        1.0});
          }
          if (h.ncr) {
            f.fill.push_back(FillJob<T>{ip + h.ib_ri, ip + h.ib_ci, ip + h.ib_vi, h.nib, h.ni,
                                        L.kmu + L.knu, XI[a]});
            f.fill.push_back(FillJob<T>{ip + h.yb_ri, ip + h.yb_ci, ip + h.yb_vi, h.ncr, h.nb,
                                        L.kmu + L.knu, L.nd->YB});
          }
        }
        std::vector<A33Item<T>> it;
        std::vector<cplx<T> *> Cm(loc.size());
        for (size_t a = 0; a < loc.size(); ++a) {
          HssLocal<T> &L = loc[a];
          const int r = L.nd->r;
          if (!r) continue;
          it.push_back(A33Item<T>{L.hs, L.nd, XI[a], L.hs->ni, L.nd->W, L.hs->ni, r});
          Cm[a] = scratch((size_t)r * r);
          L.YC = scratch((size_t)L.hs->nb * r);
          L.YCt = scratch((size_t)L.hs->nb * r);
        }
        alg33(p, it, ip, scratch);
        Stage<T> &s1 = p.add(kGemm);
        for (size_t a = 0; a < loc.size(); ++a) {
          HssLocal<T> &L = loc[a];
          const int r = L.nd->r, ni = L.hs->ni;
          if (!r) continue;
          p.gemm_job(s1, XI[a], ni, 1, L.nd->W, ni, 0, Cm[a], r, r, r, ni, (T)1, 0);
        }
        // (Y_B C)^T = C^T Y_B^T and Y_B^T (r x nb): contiguous rows for the
        // low-rank term of single entries
        Stage<T> &s2 = p.add(kGemm);
        Stage<T> &s3 = p.add(kCopy);
        for (size_t a = 0; a < loc.size(); ++a) {
          HssLocal<T> &L = loc[a];
          const int r = L.nd->r, nb = L.hs->nb;
          if (!r || !nb) continue;
          L.YBt = scratch((size_t)r * nb);
          p.gemm_job(s2, L.nd->YB, nb, 0, Cm[a], r, 0, L.YC, nb, nb, r, r, (T)1, 0);
          p.gemm_job(s2, Cm[a], r, 1, L.nd->YB, nb, 1, L.YCt, r, r, nb, r, (T)1, 0);
          s3.copy.push_back(CopyJob<T>{L.nd->YB, L.YBt, nb, r, r, nb, 1, (T)1});
        }
        hipEvent_t pp = prof_begin(st);
        run_prog(p, sg, val, st);
        prof_end("hss_gauss", st, pp, p.flops);
        flops += p.flops;
      }
      // entry operators of S(sigma) = A_bb - Y_B C Y_B^T (Sec. 3.5)
      for (size_t a = 0; a < loc.size(); ++a) {
        HssLocal<T> &L = loc[a];
        const HssSym &h = *L.hs;
        if (h.nb == 0) continue;
        EntryOp<T> op{};
        op.kind = 0;
        op.H0 = L.vmu;
        op.H1 = L.vnu;
        op.bchild = ip + h.bchild;
        op.bcpos = ip + h.bcpos;
        op.gid = ip + h.gid;
        op.YC = L.YCt;
        op.YB = L.YBt;
        op.r = L.nd->r;
        CompressTask<T> t;
        t.node = L.node;
        t.kind = 0;
        t.m = h.nb;
        t.k_init = std::max(kfin[h.mu], kfin[h.nu]);
        t.ct = sym.nodes[L.node].ct;
        t.eop = (int)sops.size();
        t.sid = (int)a;
        t.out = &L.nd->S;
        if (dense_parent(L.node)) {
          const FrontDesc &fd = P.h_desc[L.node];
          t.target = F + fd.foff + fd.ni + (long)fd.ni * fd.f;
          t.ldT = fd.f;
        }
        sops.push_back(op);
        stask.push_back(std::move(t));
      }
    }

    // ---- compress the Schur complements the parents use in HSS form:
    // dense ones of the dense-class nodes, structured ones of the HSS-class
    // nodes ("form S directly in HSS form via Algorithm A.1")
    std::vector<CompressTask<T>> tasks;
    for (int k : dn) {
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
      if (dense_parent(k)) {
        t.target = const_cast<cplx<T> *>(t.S);
        t.ldT = fd.f;
      }
      t.out = &HD[k].S;
      tasks.push_back(std::move(t));
    }
    for (auto &t : stask) tasks.push_back(std::move(t));
    if (!tasks.empty()) {
      StructSampler<T> samp = [&](Prog<T> &p, const std::vector<SampleReq<T>> &req,
                                  const std::vector<CompressTask<T>> &ts, const Alloc<T> &al) {
        // S(sigma) Omega = A_bb Omega - Y_B (C (Y_B^T Omega)), A_bb Omega from
        // the children's S_bb (telescoping products) and the couplings of A
        Stage<T> &g = p.add(kGrt);
        std::vector<MvItem<T>> mv;
        const size_t nq = req.size();
        std::vector<cplx<T> *> Ym(nq, nullptr), Yn(nq, nullptr), Oc(nq), Tq(nq);
        for (size_t q = 0; q < nq; ++q) {
          const HssLocal<T> &L = loc[ts[req[q].task].sid];
          const HssSym &h = *L.hs;
          const int nc = req[q].nc;
          Oc[q] = al((size_t)h.nb * nc);
          g.grt.push_back(GatherJob<double, cplx<T>>{req[q].Om, Oc[q], req[q].ldO, h.nb, nullptr,
                                                      nullptr, h.nb, nc, 0, 1.0});
          if (h.bb_mu >= 0) {
            const int m1 = h.mmu - h.pmu;
            cplx<T> *X = al((size_t)m1 * nc);
            Ym[q] = al((size_t)m1 * nc);
            g.grt.push_back(GatherJob<double, cplx<T>>{req[q].Om, X, req[q].ldO, m1, ip + h.p1mu,
                                                        nullptr, m1, nc, 0, 1.0});
            mv.push_back(MvItem<T>{&L.gbb_mu, X, m1, Ym[q], m1, nc});
          }
          if (h.bb_nu >= 0) {
            const int m1 = h.mnu - h.pnu;
            cplx<T> *X = al((size_t)m1 * nc);
            Yn[q] = al((size_t)m1 * nc);
            g.grt.push_back(GatherJob<double, cplx<T>>{req[q].Om, X, req[q].ldO, m1, ip + h.p1nu,
                                                        nullptr, m1, nc, 0, 1.0});
            mv.push_back(MvItem<T>{&L.gbb_nu, X, m1, Yn[q], m1, nc});
          }
          Tq[q] = al((size_t)std::max(1, L.nd->r) * nc);
        }
        hss_matvec(p, mv, al);
        Stage<T> &g1 = p.add(kGtt);
        Stage<T> &g2 = p.add(kGtt);
        Stage<T> &sp = p.add(kSpmm);
        Stage<T> &m1 = p.add(kGemm);
        for (size_t q = 0; q < nq; ++q) {
          const HssLocal<T> &L = loc[ts[req[q].task].sid];
          const HssSym &h = *L.hs;
          const int nc = req[q].nc;
          g1.gtt.push_back(GatherJob<cplx<T>, cplx<T>>{Ym[q] ? Ym[q] : Oc[q],
                                                       req[q].Y, std::max(1, h.mmu - h.pmu),
                                                       req[q].ldY, ip + h.smu, nullptr, h.nb, nc,
                                                       0, 1.0});
          if (Yn[q])
            g2.gtt.push_back(GatherJob<cplx<T>, cplx<T>>{Yn[q], req[q].Y, h.mnu - h.pnu,
                                                         req[q].ldY, ip + h.snu, nullptr, h.nb,
                                                         nc, 1, 1.0});
          sp.sp.push_back(SpJob<T>{ip + h.bb_rp, ip + h.bb_cp, ip + h.bb_vi, h.nb, nc, 1, Oc[q],
                                   h.nb, req[q].Y, req[q].ldY, (T)1});
          if (L.nd->r)
            p.gemm_job(m1, L.nd->YB, h.nb, 1, Oc[q], h.nb, 0, Tq[q], L.nd->r, L.nd->r, nc, h.nb,
                       (T)1, 0);
        }
        Stage<T> &m2 = p.add(kGemm);
        for (size_t q = 0; q < nq; ++q) {
          const HssLocal<T> &L = loc[ts[req[q].task].sid];
          if (!L.nd->r) continue;
          p.gemm_job(m2, L.YC, L.hs->nb, 0, Tq[q], L.nd->r, 0, req[q].Y, (int)req[q].ldY,
                     L.hs->nb, req[q].nc, L.nd->r, (T)-1, 1);
        }
      };
      compress_batch<T>(tasks, P.opts, P.tol, id_tol, sg, ar, P.store, A, sops, samp, cacc);
      for (auto &t : tasks) {
        record(t);
        kfin[t.node] = t.k;
        HD[t.node].has_S = true;
        ++ncomp;
      }
    }
    // the next depth's launches follow this depth's on the same stream (the
    // side stream of the compressions is joined back), so its scratch is
    // reused without waiting; the staged descriptors stay (positions keep
    // advancing within a factorization, so a repeated one finds its arrays
    // where it left them)
    ar.release(depth_mark);
    // large forests: once the staged arrays pass kStageCap the stream is
    // drained and staging starts again at its first position (every staged
    // array serves one depth; positions stay deterministic, so a repeated
    // factorization still finds its unchanged arrays in place)
    if (sg.used() > kStageCap) {
      HSSX_HIP(hipStreamSynchronize(st));
      sg.synced();
      sg.recycle();
    }
  }
  int bad = -1;
  HSSX_HIP(hipStreamSynchronize(st));
  sg.synced();
  HSSX_HIP(hipMemcpy(&bad, err, sizeof(int), hipMemcpyDeviceToHost));
  HSSX_CHECK(bad < 0, HSSX_ESINGULAR, "zero pivot in a dense block of tree node " + std::to_string(bad));
  // bytes the apply reads: dense blocks of the dense-class nodes, telescoping
  // inverses and Gauss-transform generators of the HSS-class nodes
  double fb = 0;
  const size_t esz = sizeof(cplx<T>);
  for (size_t k = 0; k < sym.nodes.size(); ++k) {
    const FrontDesc &q = P.h_desc[k];
    if (P.hss_idx[k] < 0) {
      const size_t e = std::is_same<T, float>::value && sym.nodes[k].parent < 0 ? sizeof(c128) : esz;
      fb += ((double)q.ni * q.ni + 2.0 * q.ni * q.nb) * e;
    } else {
      const HssNodeData<T> &nd = HD[k];
      fb += nd.Hmu.bytes() + nd.Hs.bytes() + (double)(q.ni + q.nb) * nd.r * esz;
    }
  }
  P.stats.factor_bytes = fb;
  P.stats.factor_flops = flops + cacc.flops;
  P.stats.k_max = kmax;
  P.stats.max_rounds_used = rounds_max;
  P.stats.rounds_total = rounds_sum;
  P.stats.max_estimate = est_max;
  P.stats.n_compressed = ncomp;
  P.stats.n_above_tol = cacc.n_above_tol;
  HSSX_CHECK(!P.opts.strict_tol || cacc.n_above_tol == 0, HSSX_ERANKCAP,
             std::to_string(cacc.n_above_tol) +
                 " compressions stopped above tol (largest estimate " + std::to_string(est_max) + ")");
}

}  // namespace

void drop_hss_plans(hssx_fact_ &P);

namespace {
std::mutex g_pool_mu;
std::map<int, std::vector<std::unique_ptr<Arena>>> g_arenas;
std::map<int, std::vector<std::unique_ptr<Staging>>> g_stagings;
}  // namespace

// Calls under a context take their arena and staging area from the
// context's own pools (freed through its allocator by hssx_destroy)
std::unique_ptr<Arena> acquire_arena(int device) {
  if (hssx_ctx_ *c = alloc_scope()) {
    std::lock_guard<std::mutex> g(c->mu);
    if (c->arenas.empty()) return std::make_unique<Arena>();
    auto a = std::move(c->arenas.back());
    c->arenas.pop_back();
    return a;
  }
  std::lock_guard<std::mutex> g(g_pool_mu);
  auto &v = g_arenas[device];
  if (v.empty()) return std::make_unique<Arena>();
  auto a = std::move(v.back());
  v.pop_back();
  return a;
}

void return_arena(int device, std::unique_ptr<Arena> a) {
  a->release(Arena::Mark{0, 0});
  if (hssx_ctx_ *c = alloc_scope()) {
    std::lock_guard<std::mutex> g(c->mu);
    c->arenas.push_back(std::move(a));
    return;
  }
  std::lock_guard<std::mutex> g(g_pool_mu);
  g_arenas[device].push_back(std::move(a));
}

std::unique_ptr<Staging> acquire_staging(int device, hipStream_t st) {
  std::unique_ptr<Staging> s;
  if (hssx_ctx_ *c = alloc_scope()) {
    std::lock_guard<std::mutex> g(c->mu);
    if (!c->stagings.empty()) {
      s = std::move(c->stagings.back());
      c->stagings.pop_back();
    }
  } else {
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
  if (hssx_ctx_ *c = alloc_scope()) {
    std::lock_guard<std::mutex> g(c->mu);
    c->stagings.push_back(std::move(s));
    return;
  }
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
  if (!P.hsym.empty()) {
    // the HSS apply programs and graphs hold the previous factor's ranks
    // and addresses
    HSSX_HIP(hipStreamSynchronize(st));
    destroy_graphs(P);
    drop_hss_plans(P);
  }
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
  const int n = P.A->n, cnt = (int)P.dense_nodes[d].size();
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
          log2_bucket((long)P.dense_nodes[d].size())};
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
    if (P.dense_nodes[d].empty()) continue;
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

// Apply program of the HSS-class nodes of every depth for nrhs columns of
// the workspace w (elimination order, ld n).  Up-step of node sigma
// (Alg. 3.1 with the block solve fused, as for the dense nodes):
//   t = w(I);  w(B) += L t = -Y_B (W^T t);  w(I) = A_ii^-1 t (Alg. 3.3);
// down-step:  w(I) += R w(B) = -W (Y_B^T w(B)).
// The approximate A_ii, L and R are symmetric and transposed (L = R^T), so
// the transposed apply runs the same programs.
template <typename T>
void build_hss_progs(hssx_fact_ &P, int nrhs, c128 *w, const Alloc<T> &al,
                     std::vector<Prog<T>> &ups, std::vector<Prog<T>> &downs, double &fbytes) {
  auto &HD = hdata<T>(P);
  const int n = P.A->n, D = P.sym.max_depth;
  const int *ip = P.hsym_pool.as<int>();
  const int *bpos = P.bpos.as<int>();
  ups.assign(D + 1, Prog<T>{});
  downs.assign(D + 1, Prog<T>{});
  fbytes = 0;
  for (int d = 0; d <= D; ++d) {
    const auto &hn = P.hss_nodes[d];
    if (hn.empty()) continue;
    Prog<T> up, dn;
    Stage<T> &g0 = up.add(kGwt);
    Stage<T> &m0 = up.add(kGemm);
    std::vector<A33Item<T>> it;
    std::vector<cplx<T> *> u(hn.size()), z(hn.size()), wb(hn.size()), xb(hn.size()), v(hn.size()),
        q(hn.size());
    for (size_t a = 0; a < hn.size(); ++a) {
      const int k = hn[a];
      const HssSym &h = P.hsym[P.hss_idx[k]];
      const HssNodeData<T> &nd = HD[k];
      const FrontDesc &fd = P.h_desc[k];
      const int r = nd.r;
      fbytes += nd.Hmu.bytes() + nd.Hs.bytes() + (double)(h.ni + h.nb) * r * sizeof(cplx<T>);
      cplx<T> *t = al((size_t)h.ni * nrhs);
      z[a] = al((size_t)h.ni * nrhs);
      g0.gwt.push_back(GatherJob<c128, cplx<T>>{w + fd.ioff, t, n, h.ni, nullptr, nullptr, h.ni,
                                                 nrhs, 0, 1.0});
      if (r) {
        u[a] = al((size_t)r * nrhs);
        wb[a] = al((size_t)std::max(1, h.nb) * nrhs);
        up.gemm_job(m0, nd.W, h.ni, 1, t, h.ni, 0, u[a], r, r, nrhs, h.ni, (T)1, 0);
      }
      it.push_back(A33Item<T>{&h, &nd, t, h.ni, z[a], h.ni, nrhs});
    }
    alg33(up, it, ip, al);
    Stage<T> &m1 = up.add(kGemm);
    Stage<T> &s1 = up.add(kGtw);
    for (size_t a = 0; a < hn.size(); ++a) {
      const int k = hn[a];
      const HssSym &h = P.hsym[P.hss_idx[k]];
      const HssNodeData<T> &nd = HD[k];
      const FrontDesc &fd = P.h_desc[k];
      if (nd.r && h.nb) {
        up.gemm_job(m1, nd.YB, h.nb, 0, u[a], nd.r, 0, wb[a], h.nb, h.nb, nrhs, nd.r, (T)-1, 0);
        s1.gtw.push_back(GatherJob<cplx<T>, c128>{wb[a], w, h.nb, n, nullptr, bpos + fd.bpos_off,
                                                   h.nb, nrhs, 1, 1.0});
      }
      s1.gtw.push_back(GatherJob<cplx<T>, c128>{z[a], w + fd.ioff, h.ni, n, nullptr, nullptr,
                                                 h.ni, nrhs, 0, 1.0});
    }
    Stage<T> &g2 = dn.add(kGwt);
    Stage<T> &m2 = dn.add(kGemm);
    Stage<T> &m3 = dn.add(kGemm);
    Stage<T> &s2 = dn.add(kGtw);
    for (size_t a = 0; a < hn.size(); ++a) {
      const int k = hn[a];
      const HssSym &h = P.hsym[P.hss_idx[k]];
      const HssNodeData<T> &nd = HD[k];
      const FrontDesc &fd = P.h_desc[k];
      if (!nd.r || !h.nb) continue;
      xb[a] = al((size_t)h.nb * nrhs);
      v[a] = al((size_t)nd.r * nrhs);
      q[a] = al((size_t)h.ni * nrhs);
      g2.gwt.push_back(GatherJob<c128, cplx<T>>{w, xb[a], n, h.nb, bpos + fd.bpos_off, nullptr,
                                                 h.nb, nrhs, 0, 1.0});
      dn.gemm_job(m2, nd.YB, h.nb, 1, xb[a], h.nb, 0, v[a], nd.r, nd.r, nrhs, h.nb, (T)1, 0);
      dn.gemm_job(m3, nd.W, h.ni, 0, v[a], nd.r, 0, q[a], h.ni, h.ni, nrhs, nd.r, (T)-1, 0);
      s2.gtw.push_back(GatherJob<cplx<T>, c128>{q[a], w + fd.ioff, h.ni, n, nullptr, nullptr,
                                                 h.ni, nrhs, 1, 1.0});
    }
    ups[d] = std::move(up);
    downs[d] = std::move(dn);
  }
}

template <typename T>
void build_hss_plan(hssx_fact_ &P, int nrhs, c128 *w, HssApplyPlan<T> &pl) {
  pl.mem = std::make_unique<Arena>();
  Arena &mem = *pl.mem;
  Alloc<T> al = [&](size_t k) { return mem.get<cplx<T>>(k); };
  std::vector<Prog<T>> ups, downs;
  build_hss_progs<T>(P, nrhs, w, al, ups, downs, pl.fbytes);
  const int D = P.sym.max_depth;
  pl.up.resize(D + 1);
  pl.down.resize(D + 1);
  for (int d = 0; d <= D; ++d) {
    pl.up[d].build(std::move(ups[d]));
    pl.down[d].build(std::move(downs[d]));
  }
}

template <typename T> std::map<int, HssApplyPlan<T>> &plans_of(hssx_fact_ &P);
template <> std::map<int, HssApplyPlan<float>> &plans_of<float>(hssx_fact_ &P) { return P.plans32; }
template <> std::map<int, HssApplyPlan<double>> &plans_of<double>(hssx_fact_ &P) { return P.plans64; }

void ensure_hss_plan(hssx_fact_ &P, int nrhs, c128 *w) {
  if (P.hsym.empty()) return;
  if (P.dtype == HSSX_C64) {
    if (!P.plans32.count(nrhs)) build_hss_plan<float>(P, nrhs, w, P.plans32[nrhs]);
  } else {
    if (!P.plans64.count(nrhs)) build_hss_plan<double>(P, nrhs, w, P.plans64[nrhs]);
  }
}

void hss_step(hssx_fact_ &P, int d, bool up, int nrhs, hipStream_t st) {
  if (P.hsym.empty() || P.hss_nodes[d].empty()) return;
  const c128 *val = P.A->val.as<c128>();
  if (P.dtype == HSSX_C64) {
    const auto &pl = P.plans32.at(nrhs);
    (up ? pl.up : pl.down)[d].launch(val, st);
  } else {
    const auto &pl = P.plans64.at(nrhs);
    (up ? pl.up : pl.down)[d].launch(val, st);
  }
}

// Algorithm 3.1 on vectors in elimination order: up-sweep with the fused
// block solve depth by depth from the leaves, then the down-sweep
using HssLauncher = std::function<void(int, bool)>;

void sweeps(hssx_fact_ &P, int trans, int nrhs, c128 *w, c128 *tb, hipStream_t st,
            const std::vector<int> &cu, const std::vector<int> &cd, const HssLauncher &hss) {
  const int D = P.sym.max_depth;
  const bool prof = prof_on() && !P.capturing;
  for (int d = D; d >= 0; --d) {
    if (!P.dense_nodes[d].empty()) {
      hipEvent_t pu = prof ? prof_begin(st) : nullptr;
      sweep_step(P, d, true, trans, nrhs, w, tb, cu[d], st);
      if (prof) prof_end("apply_up", st, pu, P.up_fbytes[d] + P.up_velems[d] * nrhs * sizeof(c128));
    }
    if (!P.hss_nodes[d].empty()) {
      hipEvent_t ph = prof ? prof_begin(st) : nullptr;
      hss(d, true);
      if (prof) prof_end("apply_hss", st, ph, 0.0);
    }
  }
  for (int d = 0; d <= D; ++d) {
    if (!P.dense_nodes[d].empty()) {
      hipEvent_t pd = prof ? prof_begin(st) : nullptr;
      sweep_step(P, d, false, trans, nrhs, w, tb, cd[d], st);
      if (prof)
        prof_end("apply_down", st, pd, P.down_fbytes[d] + P.down_velems[d] * nrhs * sizeof(c128));
    }
    if (!P.hss_nodes[d].empty()) {
      hipEvent_t ph = prof ? prof_begin(st) : nullptr;
      hss(d, false);
      if (prof) prof_end("apply_hss", st, ph, 0.0);
    }
  }
}

}  // namespace

void destroy_graphs(hssx_fact_ &P) {
  for (auto &g : P.graphs) (void)hipGraphExecDestroy(g.exec);
  P.graphs.clear();
}

void drop_hss_plans(hssx_fact_ &P) {
  P.plans32.clear();
  P.plans64.clear();
}

void apply(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y, long ldy,
           hipStream_t st) {
  const int n = P.A->n;
  if (P.work_cols < (size_t)nrhs) {
    HSSX_HIP(hipStreamSynchronize(st));
    destroy_graphs(P);   // they and the HSS programs hold the old workspace's addresses
    drop_hss_plans(P);
    P.work.alloc((size_t)2 * n * nrhs * sizeof(c128));
    P.work_cols = nrhs;
  }
  c128 *w = P.work.as<c128>();
  c128 *tb = w + (size_t)n * nrhs;
  tune_apply(P, nrhs, st);
  ensure_hss_plan(P, nrhs, w);
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
        sweeps(P, trans, nrhs, w, tb, P.cap_stream, P.cfg_up.at(nrhs), P.cfg_down.at(nrhs),
               [&](int d, bool up) { hss_step(P, d, up, nrhs, P.cap_stream); });
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
    sweeps(P, trans, nrhs, w, tb, st, P.cfg_up.at(nrhs), P.cfg_down.at(nrhs),
           [&](int d, bool up) { hss_step(P, d, up, nrhs, st); });
  }
  launch_permute(n, nrhs, P.perm.as<int>(), w, n, y, ldy, 1, st);
}

namespace {

template <typename T> bool expand_t(hssx_fact_ &P, int node, std::vector<c128> &out) {
  auto &HD = hdata<T>(P);
  if ((size_t)node >= HD.size() || !HD[node].has_S) return false;
  const HssMat<T> &H = HD[node].S;
  const int m = H.m;
  int dev = 0;
  HSSX_HIP(hipGetDevice(&dev));
  hipStream_t st = nullptr;
  std::unique_ptr<Arena> ar = acquire_arena(dev);
  std::unique_ptr<Staging> sg = acquire_staging(dev, st);
  try {
    Alloc<T> al = [&](size_t n) { return ar->get<cplx<T>>(n); };
    cplx<T> *X = al((size_t)m * m), *Y = al((size_t)m * m);
    Prog<T> p;
    p.add(kCopy).copy.push_back(CopyJob<T>{nullptr, X, 0, m, m, m, 2, (T)1});
    const Gen<T> g = H.gen(0);
    hss_matvec(p, std::vector<MvItem<T>>{MvItem<T>{&g, X, m, Y, m, m}}, al);
    run_prog(p, *sg, nullptr, st);
    std::vector<cplx<T>> h((size_t)m * m);
    HSSX_HIP(hipMemcpyAsync(h.data(), Y, h.size() * sizeof(cplx<T>), hipMemcpyDeviceToHost, st));
    HSSX_HIP(hipStreamSynchronize(st));
    out.resize(h.size());
    for (size_t e = 0; e < h.size(); ++e) out[e] = mk((double)h[e].re, (double)h[e].im);
  } catch (...) {
    (void)hipDeviceSynchronize();
    return_arena(dev, std::move(ar));
    return_staging(dev, std::move(sg));
    throw;
  }
  return_arena(dev, std::move(ar));
  return_staging(dev, std::move(sg));
  return true;
}

}  // namespace

// the compressed Schur complement of a node, expanded (false when the node
// kept none)
bool expand_schur(hssx_fact_ &P, int node, std::vector<c128> &out) {
  return P.dtype == HSSX_C64 ? expand_t<float>(P, node, out) : expand_t<double>(P, node, out);
}

namespace {

template <typename T>
void apply_ws_t(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y, long ldy,
                hipStream_t st, char *ws, size_t ws_bytes) {
  const int n = P.A->n, D = P.sym.max_depth;
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = (off + 255) / 256 * 256;
    HSSX_CHECK(o + bytes <= ws_bytes, HSSX_EINVAL,
               "apply workspace exceeds the allocation-free entry point's maximum (" +
                   std::to_string(ws_bytes >> 20) + " MiB)");
    off = o + bytes;
    return ws + o;
  };
  c128 *w = reinterpret_cast<c128 *>(take((size_t)n * nrhs * sizeof(c128)));
  c128 *tb = reinterpret_cast<c128 *>(take((size_t)n * nrhs * sizeof(c128)));
  // programs of the HSS-class nodes: scratch and job arrays in the workspace
  std::vector<Prog<T>> ups, downs;
  double fb = 0;
  Alloc<T> al = [&](size_t k) {
    return reinterpret_cast<cplx<T> *>(take(std::max<size_t>(k, 1) * sizeof(cplx<T>)));
  };
  if (!P.hsym.empty()) build_hss_progs<T>(P, nrhs, w, al, ups, downs, fb);
  std::vector<ProgBlob<T>> bu(D + 1), bd(D + 1);
  std::vector<char> h;
  std::vector<size_t> ou(D + 1, 0), od(D + 1, 0);
  auto append = [&](const std::vector<char> &v) {
    const size_t o = (h.size() + 255) / 256 * 256;
    h.resize(o + std::max<size_t>(v.size(), 1));
    if (!v.empty()) std::memcpy(h.data() + o, v.data(), v.size());
    return o;
  };
  for (int d = 0; d <= D && !P.hsym.empty(); ++d) {
    bu[d].build(ups[d].st);
    bd[d].build(downs[d].st);
    ou[d] = append(bu[d].h);
    od[d] = append(bd[d].h);
  }
  char *jobs = h.empty() ? nullptr : take(h.size());
  if (jobs) HSSX_HIP(hipMemcpyAsync(jobs, h.data(), h.size(), hipMemcpyHostToDevice, st));
  // default tile shapes (the autotuner would allocate its trial vectors)
  const std::vector<int> cfg(D + 1, 2);
  const c128 *val = P.A->val.as<c128>();
  launch_permute(n, nrhs, P.perm.as<int>(), x, ldx, w, n, 0, st);
  sweeps(P, trans, nrhs, w, tb, st, cfg, cfg, [&](int d, bool up) {
    if (up) bu[d].launch(ups[d].st, jobs + ou[d], val, st);
    else bd[d].launch(downs[d].st, jobs + od[d], val, st);
  });
  launch_permute(n, nrhs, P.perm.as<int>(), w, n, y, ldy, 1, st);
  // the job image is host memory of this call
  HSSX_HIP(hipStreamSynchronize(st));
}

}  // namespace

void apply_workspace(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y,
                     long ldy, hipStream_t st, char *ws, size_t ws_bytes) {
  if (P.dtype == HSSX_C64) apply_ws_t<float>(P, trans, nrhs, x, ldx, y, ldy, st, ws, ws_bytes);
  else apply_ws_t<double>(P, trans, nrhs, x, ldx, y, ldy, st, ws, ws_bytes);
}

}  // namespace hssx
