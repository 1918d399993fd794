// HSS arithmetic on the device, driven by host-built job lists (Sec. 2.2,
// Sec. 3.3-3.5).
//
// A compressed symmetric matrix is kept in generator form (HssMat): per
// cluster of its binary cluster tree a basis U (leaf: |I_c| x k_c; internal:
// (k_l + k_r) x k_c, the transfer matrix of eq. 2.3), per leaf its diagonal
// block D, per internal cluster the sibling couplings B12, B21.  On it:
//
//  * hss_matvec: the telescoping product y = H x (eqs. 2.5-2.6);
//  * gym_factor / gym_solve: the telescoping inverse.  With H = D + U H' U^T
//    on one level (D, U block diagonal over the clusters of the level, H'
//    the matrix on the concatenated skeletons), the inverse is
//        H^-1 = E (H' + Dh)^-1 E^T + G,   Dh = (U^T D^-1 U)^-1,
//        E = D^-1 U Dh,                   G = D^-1 - E U^T D^-1,
//    and H' + Dh is again of this form one level up, its diagonal blocks
//    being [[Dh_l, B12], [B21, Dh_r]]; at the root that block is inverted.
//    This is the direct HSS solver of Gillman, Young and Martinsson (2012),
//    one of the "ULV-style" HSS factorizations the paper applies; every step
//    is a small dense product or inverse per cluster;
//  * inverse_view: H^-1 in HSS form for entry access: bases E, couplings and
//    leaf blocks from W_c = G_c + E_c W_p(c, c) E_c^T (top-down, W_root = G_root);
//  * entry_prep: full bases and basis-times-coupling blocks, so that one
//    entry costs one dot product of length k (EntCl, hss_entry).
// All operations on many matrices of one tree depth go into the same
// launches: each builder appends stages (one launch each) to a program.
#pragma once

#include <cstring>
#include <deque>
#include <functional>
#include <vector>

#include "hssops.h"
#include "prof.h"
#include "symbolic.h"

namespace hssx {

template <typename T>
void eliminate_jobs(const std::vector<ElimJob<T>> &jobs, int *err, Staging &sg, Arena &ar);

// ---------------------------------------------------------------- programs
enum StageKind { kGemm, kCopy, kSpmm, kGtt, kGwt, kGtw, kGrt, kFill, kSym };

template <typename T> struct Stage {
  StageKind kind = kGemm;
  std::vector<BgJob<T>> gemm;
  std::vector<CopyJob<T>> copy;
  std::vector<SpJob<T>> sp;
  std::vector<GatherJob<cplx<T>, cplx<T>>> gtt;
  std::vector<GatherJob<c128, cplx<T>>> gwt;
  std::vector<GatherJob<cplx<T>, c128>> gtw;
  std::vector<GatherJob<double, cplx<T>>> grt;
  std::vector<FillJob<T>> fill;
  std::vector<SymJob<T>> sym;
  size_t size() const {
    switch (kind) {
      case kGemm: return gemm.size();
      case kCopy: return copy.size();
      case kSpmm: return sp.size();
      case kGtt: return gtt.size();
      case kGwt: return gwt.size();
      case kGtw: return gtw.size();
      case kGrt: return grt.size();
      case kFill: return fill.size();
      default: return sym.size();
    }
  }
};

// stages in launch order (a deque: references to earlier stages stay valid
// while later ones are added)
template <typename T> struct Prog {
  std::deque<Stage<T>> st;
  double flops = 0;   // 8 per complex multiply-add of the products
  Stage<T> &add(StageKind k) {
    st.emplace_back();
    st.back().kind = k;
    return st.back();
  }
  void gemm_job(Stage<T> &s, const cplx<T> *A, int lda, int ta, const cplx<T> *B, int ldb, int tb,
                cplx<T> *C, int ldc, int M, int N, int K, T ar, int beta) {
    if (M <= 0 || N <= 0) return;
    s.gemm.push_back(BgJob<T>{A, B, C, lda, ldb, ldc, M, N, K, ta, tb, beta, ar, (T)0});
    flops += 8.0 * M * N * K;
  }
  void append(Prog &&o) {
    for (auto &s : o.st) st.push_back(std::move(s));
    flops += o.flops;
  }
};

template <typename T> inline std::vector<BgTask<T>> gemm_tasks(const std::vector<BgJob<T>> &jobs) {
  std::vector<BgTask<T>> t;
  for (size_t j = 0; j < jobs.size(); ++j)
    for (int a = 0; a < (jobs[j].M + 31) / 32; ++a)
      for (int b = 0; b < (jobs[j].N + 31) / 32; ++b) t.push_back(BgTask<T>{jobs[j], a, b});
  return t;
}

template <typename J> inline long job_elems(const J &j) { return (long)j.nrows * j.nc; }
template <typename T> inline long job_elems(const CopyJob<T> &j) { return (long)j.m * j.n; }
template <typename T> inline long job_elems(const SymJob<T> &j) { return (long)j.m * j.n; }
template <typename T> inline long job_elems(const FillJob<T> &j) { return j.cnt; }
template <typename V> inline long max_elems(const V &v) {
  long m = 0;
  for (const auto &j : v) m = std::max(m, job_elems(j));
  return m;
}

// one stage from device job arrays
template <typename T>
inline void launch_stage(const Stage<T> &s, const void *jobs, int ntiles, long me,
                         const c128 *val, hipStream_t st) {
  const int n = (int)s.size();
  switch (s.kind) {
    case kGemm: {
      hipEvent_t pe = prof_begin(st);
      launch_bgemm<T>(ntiles, (const BgTask<T> *)jobs, st);
      if (pe) {
        double fl = 0;
        for (const BgJob<T> &g : s.gemm) fl += 8.0 * g.M * g.N * g.K;
        prof_end("bgemm", st, pe, fl);
      }
      break;
    }
    case kCopy: launch_copy<T>(n, (const CopyJob<T> *)jobs, me, st); break;
    case kSpmm: launch_spmm<T>(n, (const SpJob<T> *)jobs, val, me, st); break;
    case kGtt: launch_gather<cplx<T>, cplx<T>>(n, (const GatherJob<cplx<T>, cplx<T>> *)jobs, me, st); break;
    case kGwt: launch_gather<c128, cplx<T>>(n, (const GatherJob<c128, cplx<T>> *)jobs, me, st); break;
    case kGtw: launch_gather<cplx<T>, c128>(n, (const GatherJob<cplx<T>, c128> *)jobs, me, st); break;
    case kGrt: launch_gather<double, cplx<T>>(n, (const GatherJob<double, cplx<T>> *)jobs, me, st); break;
    case kFill: launch_fill_coo<T>(n, (const FillJob<T> *)jobs, val, (int)me, st); break;
    default: launch_symmetrize<T>(n, (const SymJob<T> *)jobs, me, st); break;
  }
}

template <typename T> inline long stage_elems(const Stage<T> &s) {
  switch (s.kind) {
    case kCopy: return max_elems(s.copy);
    case kSpmm: return max_elems(s.sp);
    case kGtt: return max_elems(s.gtt);
    case kGwt: return max_elems(s.gwt);
    case kGtw: return max_elems(s.gtw);
    case kGrt: return max_elems(s.grt);
    case kFill: return max_elems(s.fill);
    case kSym: return max_elems(s.sym);
    default: return 0;
  }
}

// host image of a program's job arrays (one upload): per stage the offset
// of its jobs and of its tile list
template <typename T> struct ProgBlob {
  std::vector<char> h;
  std::vector<size_t> jobs;
  std::vector<int> ntiles;
  std::vector<long> me;
  size_t put(const void *src, size_t bytes) {
    const size_t off = (h.size() + 255) / 256 * 256;
    h.resize(off + std::max<size_t>(bytes, 1));
    if (bytes) std::memcpy(h.data() + off, src, bytes);
    return off;
  }
  template <typename V> size_t putv(const V &v) { return put(v.data(), v.size() * sizeof(v[0])); }
  template <typename Q> void build(const Q &stages) {
    for (const Stage<T> &s : stages) {
      size_t j = 0;
      int nt = 0;
      switch (s.kind) {
        case kGemm: {
          std::vector<BgTask<T>> tl = gemm_tasks(s.gemm);
          j = putv(tl);
          nt = (int)tl.size();
          break;
        }
        case kCopy: j = putv(s.copy); break;
        case kSpmm: j = putv(s.sp); break;
        case kGtt: j = putv(s.gtt); break;
        case kGwt: j = putv(s.gwt); break;
        case kGtw: j = putv(s.gtw); break;
        case kGrt: j = putv(s.grt); break;
        case kFill: j = putv(s.fill); break;
        default: j = putv(s.sym); break;
      }
      jobs.push_back(j);
      ntiles.push_back(nt);
      me.push_back(stage_elems(s));
    }
  }
  template <typename Q>
  void launch(const Q &stages, const char *base, const c128 *val, hipStream_t st) const {
    size_t i = 0;
    for (const Stage<T> &s : stages) {
      const size_t q = i++;
      if (s.size() == 0 || (s.kind == kGemm && ntiles[q] == 0)) continue;
      launch_stage(s, base + jobs[q], ntiles[q], me[q], val, st);
    }
  }
};

// run a program now: all its job arrays go up through the staging area in
// one copy
template <typename T>
inline void run_prog(const Prog<T> &p, Staging &sg, const c128 *val, hipStream_t st) {
  if (p.st.empty()) return;
  ProgBlob<T> b;
  b.build(p.st);
  const char *d = sg.put_const(b.h);
  b.launch(p.st, d, val, st);
}

// A program kept on the device for replay (the apply runs the same launches
// for every vector block of a given width).
template <typename T> struct Plan {
  std::vector<Stage<T>> st;   // job lists (host copies; sizes and kinds)
  ProgBlob<T> b;
  DevBuf blob;
  void build(Prog<T> &&p) {
    st.assign(std::make_move_iterator(p.st.begin()), std::make_move_iterator(p.st.end()));
    b = ProgBlob<T>{};
    b.build(st);
    blob.alloc(std::max<size_t>(b.h.size(), 256));
    if (!b.h.empty()) HSSX_HIP(hipMemcpy(blob.p, b.h.data(), b.h.size(), hipMemcpyHostToDevice));
    b.h.clear();
    b.h.shrink_to_fit();
  }
  void launch(const c128 *val, hipStream_t s) const {
    b.launch(st, static_cast<const char *>(blob.p), val, s);
  }
  bool empty() const { return st.empty(); }
};

// ---------------------------------------------------------------- trees
inline std::vector<std::vector<int>> sub_levels(const ClusterTree &ct, int root) {
  std::vector<std::vector<int>> lev;
  if (root < 0 || root >= ct.count()) return lev;
  lev.push_back({root});
  for (size_t l = 0; l < lev.size(); ++l) {
    std::vector<int> nxt;
    for (int c : lev[l])
      if (!ct.leaf(c)) {
        nxt.push_back(ct.left[c]);
        nxt.push_back(ct.right[c]);
      }
    if (nxt.empty()) break;
    lev.push_back(std::move(nxt));
  }
  return lev;
}

inline std::vector<int> parents_of(const ClusterTree &ct) {
  std::vector<int> p(ct.count(), -1);
  for (int c = 0; c < ct.count(); ++c)
    if (!ct.leaf(c)) p[ct.left[c]] = p[ct.right[c]] = c;
  return p;
}

// Generators of a symmetric nested-basis HSS matrix, restricted to the
// subtree rooted at `root` (its positions start at ct->start[root]).
template <typename T> struct Gen {
  const ClusterTree *ct = nullptr;
  int root = 0;
  std::vector<int> k;   // basis columns per cluster
  std::vector<const cplx<T> *> U, D, B12, B21;
  std::vector<int> ldU, ldD, ldB12, ldB21;
  int base() const { return ct->start[root]; }
  int m() const { return ct->size[root]; }
  int rowsU(int c) const { return ct->leaf(c) ? ct->size[c] : k[ct->left[c]] + k[ct->right[c]]; }
  // row offset of child c inside its parent's stacked skeleton block
  int off(int c, int p) const { return ct->left[p] == c ? 0 : k[ct->left[p]]; }
};

// A compressed matrix in generator form (pointers into factor storage).
template <typename T> struct HssMat {
  int m = 0;
  ClusterTree ct;
  std::vector<int> k;
  std::vector<cplx<T> *> U, D, B12, B21;
  int maxrank() const {
    int r = 0;
    for (int c = 1; c < ct.count(); ++c) r = std::max(r, k[c]);
    return r;
  }
  Gen<T> gen(int root = 0) const {
    Gen<T> g;
    g.ct = &ct;
    g.root = root;
    g.k = k;
    const int n = ct.count();
    g.U.resize(n); g.D.resize(n); g.B12.resize(n); g.B21.resize(n);
    g.ldU.resize(n); g.ldD.resize(n); g.ldB12.resize(n); g.ldB21.resize(n);
    for (int c = 0; c < n; ++c) {
      g.U[c] = U[c];
      g.ldU[c] = std::max(1, g.rowsU(c));
      g.D[c] = D[c];
      g.ldD[c] = std::max(1, ct.size[c]);
      g.B12[c] = B12[c];
      g.B21[c] = B21[c];
      if (!ct.leaf(c)) {
        g.ldB12[c] = std::max(1, k[ct.left[c]]);
        g.ldB21[c] = std::max(1, k[ct.right[c]]);
      } else {
        g.ldB12[c] = g.ldB21[c] = 1;
      }
    }
    return g;
  }
  // device bytes of the generators
  double bytes() const {
    double b = 0;
    for (int c = 0; c < ct.count(); ++c) {
      if (c) b += (double)(ct.leaf(c) ? ct.size[c] : k[ct.left[c]] + k[ct.right[c]]) * k[c];
      if (ct.leaf(c)) b += (double)ct.size[c] * ct.size[c];
      else b += 2.0 * k[ct.left[c]] * k[ct.right[c]];
    }
    return b * sizeof(cplx<T>);
  }
};

// Telescoping inverse of a Gen's subtree.
template <typename T> struct HssInv {
  const ClusterTree *ct = nullptr;
  int root = -1, base = 0;
  std::vector<std::vector<int>> lev;
  std::vector<int> k, mc, par;          // per cluster id of ct
  std::vector<cplx<T> *> E, G, W;       // E: mc x k, G and W: mc x mc
  bool empty() const { return lev.empty(); }
  int m() const { return empty() ? 0 : ct->size[root]; }
  int off(int c) const {
    const int p = par[c];
    return ct->left[p] == c ? 0 : k[ct->left[p]];
  }
  double bytes() const {
    double b = 0;
    for (const auto &l : lev)
      for (int c : l) b += (double)mc[c] * (mc[c] + (c == root ? 0 : k[c]));
    return b * sizeof(cplx<T>);
  }
  // generators of H^-1 (bases E, blocks of W), valid once W is filled
  Gen<T> inv_gen() const {
    Gen<T> g;
    g.ct = ct;
    g.root = root;
    g.k = k;
    const int n = ct->count();
    g.U.assign(n, nullptr); g.D.assign(n, nullptr); g.B12.assign(n, nullptr);
    g.B21.assign(n, nullptr);
    g.ldU.assign(n, 1); g.ldD.assign(n, 1); g.ldB12.assign(n, 1); g.ldB21.assign(n, 1);
    for (const auto &l : lev)
      for (int c : l) {
        g.U[c] = E[c];
        g.ldU[c] = std::max(1, mc[c]);
        if (ct->leaf(c)) {
          g.D[c] = W[c];
          g.ldD[c] = std::max(1, mc[c]);
        } else {
          const int kl = k[ct->left[c]];
          g.B12[c] = W[c] + (long)kl * mc[c];
          g.B21[c] = W[c] + kl;
          g.ldB12[c] = g.ldB21[c] = std::max(1, mc[c]);
        }
      }
    return g;
  }
};

// allocator for device scratch or storage
template <typename T> using Alloc = std::function<cplx<T> *(size_t)>;

// ---------------------------------------------------------------- matvec
template <typename T> struct MvItem {
  const Gen<T> *g;
  const cplx<T> *X;
  long ldx;
  cplx<T> *Y;
  long ldy;
  int nc;
};

// y = H x for every item (telescoping product over each subtree)
template <typename T>
void hss_matvec(Prog<T> &p, const std::vector<MvItem<T>> &items, const Alloc<T> &alloc) {
  struct W {
    std::vector<std::vector<int>> lev;
    std::vector<int> par;
    std::vector<cplx<T> *> XS, YS;
  };
  std::vector<W> w(items.size());
  int maxL = 0;
  for (size_t a = 0; a < items.size(); ++a) {
    const Gen<T> &g = *items[a].g;
    w[a].lev = sub_levels(*g.ct, g.root);
    w[a].par = parents_of(*g.ct);
    w[a].XS.assign(g.ct->count(), nullptr);
    w[a].YS.assign(g.ct->count(), nullptr);
    for (const auto &l : w[a].lev)
      for (int c : l)
        if (!g.ct->leaf(c)) {
          const size_t e = (size_t)std::max(1, g.rowsU(c)) * items[a].nc;
          w[a].XS[c] = alloc(e);
          w[a].YS[c] = alloc(e);
        }
    maxL = std::max(maxL, (int)w[a].lev.size() - 1);
  }
  auto xin = [&](size_t a, int c, const cplx<T> *&ptr, int &ld) {
    const Gen<T> &g = *items[a].g;
    if (g.ct->leaf(c)) {
      ptr = items[a].X + (g.ct->start[c] - g.base());
      ld = (int)items[a].ldx;
    } else {
      ptr = w[a].XS[c];
      ld = std::max(1, g.rowsU(c));
    }
  };
  for (int L = maxL; L >= 1; --L) {   // up-sweep: x_c = U_c^T x(c)
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      if (L >= (int)w[a].lev.size()) continue;
      const Gen<T> &g = *items[a].g;
      for (int c : w[a].lev[L]) {
        const int pp = w[a].par[c];
        const cplx<T> *in;
        int ld;
        xin(a, c, in, ld);
        p.gemm_job(s, g.U[c], g.ldU[c], 1, in, ld, 0, w[a].XS[pp] + g.off(c, pp),
                   std::max(1, g.rowsU(pp)), g.k[c], items[a].nc, g.rowsU(c), (T)1, 0);
      }
    }
  }
  {   // sibling couplings
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      const Gen<T> &g = *items[a].g;
      for (const auto &l : w[a].lev)
        for (int c : l) {
          if (g.ct->leaf(c)) continue;
          const int kl = g.k[g.ct->left[c]], kr = g.k[g.ct->right[c]], mc = std::max(1, kl + kr);
          p.gemm_job(s, g.B12[c], g.ldB12[c], 0, w[a].XS[c] + kl, mc, 0, w[a].YS[c], mc, kl,
                     items[a].nc, kr, (T)1, 0);
          p.gemm_job(s, g.B21[c], g.ldB21[c], 0, w[a].XS[c], mc, 0, w[a].YS[c] + kl, mc, kr,
                     items[a].nc, kl, (T)1, 0);
        }
    }
  }
  for (int L = 1; L <= maxL; ++L) {   // down-sweep over internal clusters
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      if (L >= (int)w[a].lev.size()) continue;
      const Gen<T> &g = *items[a].g;
      for (int c : w[a].lev[L]) {
        if (g.ct->leaf(c)) continue;
        const int pp = w[a].par[c];
        p.gemm_job(s, g.U[c], g.ldU[c], 0, w[a].YS[pp] + g.off(c, pp), std::max(1, g.rowsU(pp)),
                   0, w[a].YS[c], std::max(1, g.rowsU(c)), g.rowsU(c), items[a].nc, g.k[c], (T)1,
                   1);
      }
    }
  }
  Stage<T> &sd = p.add(kGemm);   // leaves: y = D x, then y += U y_c
  for (size_t a = 0; a < items.size(); ++a) {
    const Gen<T> &g = *items[a].g;
    for (const auto &l : w[a].lev)
      for (int c : l) {
        if (!g.ct->leaf(c)) continue;
        const int o = g.ct->start[c] - g.base(), sz = g.ct->size[c];
        p.gemm_job(sd, g.D[c], g.ldD[c], 0, items[a].X + o, (int)items[a].ldx, 0, items[a].Y + o,
                   (int)items[a].ldy, sz, items[a].nc, sz, (T)1, 0);
      }
  }
  Stage<T> &su = p.add(kGemm);
  for (size_t a = 0; a < items.size(); ++a) {
    const Gen<T> &g = *items[a].g;
    for (const auto &l : w[a].lev)
      for (int c : l) {
        if (!g.ct->leaf(c) || c == g.root) continue;
        const int pp = w[a].par[c], o = g.ct->start[c] - g.base(), sz = g.ct->size[c];
        p.gemm_job(su, g.U[c], g.ldU[c], 0, w[a].YS[pp] + g.off(c, pp), std::max(1, g.rowsU(pp)),
                   0, items[a].Y + o, (int)items[a].ldy, sz, items[a].nc, g.k[c], (T)1, 1);
      }
  }
}

// ---------------------------------------------------------------- GYM factor
// Telescoping inverses of the given subtrees (bottom-up, one round of
// launches per tree level across all of them).  E, G live in `store`;
// the augmented blocks are scratch.  node[i] names inverse i on a zero pivot.
template <typename T>
void gym_factor(std::vector<HssInv<T>> &out, const std::vector<const Gen<T> *> &in,
                const std::vector<int> &node, const Alloc<T> &store, const Alloc<T> &scratch,
                int *err, Staging &sg, Arena &ar, const c128 *val, hipStream_t st,
                double *flops) {
  const size_t n = in.size();
  out.assign(n, HssInv<T>{});
  std::vector<std::vector<cplx<T> *>> aug(n), maug(n);
  int maxL = -1;
  for (size_t i = 0; i < n; ++i) {
    const Gen<T> &g = *in[i];
    HssInv<T> &h = out[i];
    h.ct = g.ct;
    h.root = g.root;
    h.base = g.base();
    h.lev = sub_levels(*g.ct, g.root);
    h.par = parents_of(*g.ct);
    const int nc = g.ct->count();
    h.k.assign(nc, 0);
    h.mc.assign(nc, 0);
    h.E.assign(nc, nullptr);
    h.G.assign(nc, nullptr);
    h.W.assign(nc, nullptr);
    aug[i].assign(nc, nullptr);
    maug[i].assign(nc, nullptr);
    for (const auto &l : h.lev)
      for (int c : l) h.k[c] = c == g.root ? 0 : g.k[c];
    for (const auto &l : h.lev)
      for (int c : l) {
        h.mc[c] = g.ct->leaf(c) ? g.ct->size[c] : h.k[g.ct->left[c]] + h.k[g.ct->right[c]];
        const size_t m = h.mc[c], k = h.k[c];
        h.E[c] = store(std::max<size_t>(1, m * k));
        h.G[c] = store(std::max<size_t>(1, m * m));
        aug[i][c] = scratch(std::max<size_t>(1, m * (2 * m + k)));
        maug[i][c] = scratch(std::max<size_t>(1, 2 * k * k));
      }
    maxL = std::max(maxL, (int)h.lev.size() - 1);
  }
  for (int L = maxL; L >= 0; --L) {
    Prog<T> p;
    Stage<T> &cp = p.add(kCopy);
    std::vector<ElimJob<T>> ej, mj;
    for (size_t i = 0; i < n; ++i) {
      HssInv<T> &h = out[i];
      const Gen<T> &g = *in[i];
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const int m = h.mc[c], k = h.k[c];
        if (m == 0) continue;
        cplx<T> *A = aug[i][c];
        if (g.ct->leaf(c)) {
          cp.copy.push_back(CopyJob<T>{g.D[c], A, g.ldD[c], m, m, m, 0, (T)1});
        } else {
          const int l = g.ct->left[c], r = g.ct->right[c], kl = h.k[l], kr = h.k[r];
          if (kl) cp.copy.push_back(CopyJob<T>{maug[i][l] + (long)kl * kl, A, kl, m, kl, kl, 0, (T)1});
          if (kr)
            cp.copy.push_back(CopyJob<T>{maug[i][r] + (long)kr * kr, A + kl + (long)kl * m, kr, m, kr,
                                         kr, 0, (T)1});
          if (kl && kr) {
            cp.copy.push_back(CopyJob<T>{g.B12[c], A + (long)kl * m, g.ldB12[c], m, kl, kr, 0, (T)1});
            cp.copy.push_back(CopyJob<T>{g.B21[c], A + kl, g.ldB21[c], m, kr, kl, 0, (T)1});
          }
        }
        if (k) {
          cp.copy.push_back(CopyJob<T>{g.U[c], A + (long)m * m, g.ldU[c], m, m, k, 0, (T)1});
          cp.copy.push_back(CopyJob<T>{nullptr, maug[i][c] + (long)k * k, 0, k, k, k, 2, (T)1});
        }
        cp.copy.push_back(CopyJob<T>{nullptr, A + (long)(m + k) * m, 0, m, m, m, 2, (T)1});
        ej.push_back(ElimJob<T>{A, m, m, 2 * m + k, m, 0, node[i]});
        if (k) mj.push_back(ElimJob<T>{maug[i][c], k, k, 2 * k, k, 0, node[i]});
      }
    }
    run_prog(p, sg, val, st);
    if (!ej.empty()) eliminate_jobs<T>(ej, err, sg, ar);
    for (const auto &j : ej)
      *flops += 8.0 * j.m * (double)j.m * j.ncols;
    // M = U^T Z, Dh = M^-1, E = Z Dh, G = D^-1 - E Z^T
    Prog<T> q;
    Stage<T> &sm = q.add(kGemm);
    for (size_t i = 0; i < n; ++i) {
      HssInv<T> &h = out[i];
      const Gen<T> &g = *in[i];
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const int m = h.mc[c], k = h.k[c];
        if (!m || !k) continue;
        q.gemm_job(sm, g.U[c], g.ldU[c], 1, aug[i][c] + (long)m * m, m, 0, maug[i][c], k, k, k, m,
                   (T)1, 0);
      }
    }
    run_prog(q, sg, val, st);
    if (!mj.empty()) eliminate_jobs<T>(mj, err, sg, ar);
    for (const auto &j : mj) *flops += 8.0 * j.m * (double)j.m * j.ncols;
    Prog<T> r;
    Stage<T> &se = r.add(kGemm);
    Stage<T> &sgc = r.add(kCopy);
    for (size_t i = 0; i < n; ++i) {
      HssInv<T> &h = out[i];
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const int m = h.mc[c], k = h.k[c];
        if (!m) continue;
        const cplx<T> *Z = aug[i][c] + (long)m * m, *Dinv = aug[i][c] + (long)(m + k) * m;
        if (k) r.gemm_job(se, Z, m, 0, maug[i][c] + (long)k * k, k, 0, h.E[c], m, m, k, k, (T)1, 0);
        sgc.copy.push_back(CopyJob<T>{Dinv, h.G[c], m, m, m, m, 0, (T)1});
      }
    }
    Stage<T> &sg2 = r.add(kGemm);
    for (size_t i = 0; i < n; ++i) {
      HssInv<T> &h = out[i];
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const int m = h.mc[c], k = h.k[c];
        if (!m || !k) continue;
        r.gemm_job(sg2, h.E[c], m, 0, aug[i][c] + (long)m * m, m, 1, h.G[c], m, m, m, k, (T)-1, 1);
      }
    }
    run_prog(r, sg, val, st);
    *flops += p.flops + q.flops + r.flops;
  }
}

// ---------------------------------------------------------------- GYM solve
template <typename T> struct SolveItem {
  const HssInv<T> *h;
  const cplx<T> *X;
  long ldx;
  cplx<T> *Y;   // must not overlap X
  long ldy;
  int nc;
};

template <typename T>
void gym_solve(Prog<T> &p, const std::vector<SolveItem<T>> &items, const Alloc<T> &alloc) {
  std::vector<std::vector<cplx<T> *>> BS(items.size()), YS(items.size());
  int maxL = -1;
  for (size_t a = 0; a < items.size(); ++a) {
    const HssInv<T> &h = *items[a].h;
    if (h.empty()) continue;
    BS[a].assign(h.ct->count(), nullptr);
    YS[a].assign(h.ct->count(), nullptr);
    for (const auto &l : h.lev)
      for (int c : l)
        if (!h.ct->leaf(c)) {
          BS[a][c] = alloc((size_t)std::max(1, h.mc[c]) * items[a].nc);
          YS[a][c] = alloc((size_t)std::max(1, h.mc[c]) * items[a].nc);
        }
    maxL = std::max(maxL, (int)h.lev.size() - 1);
  }
  auto leaf_x = [&](size_t a, int c) {
    const HssInv<T> &h = *items[a].h;
    return items[a].X + (h.ct->start[c] - h.base);
  };
  for (int L = maxL; L >= 1; --L) {   // b_c = E_c^T beta_c into the parent's stack
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      const HssInv<T> &h = *items[a].h;
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const bool lf = h.ct->leaf(c);
        const int pp = h.par[c];
        p.gemm_job(s, h.E[c], std::max(1, h.mc[c]), 1, lf ? leaf_x(a, c) : BS[a][c],
                   lf ? (int)items[a].ldx : std::max(1, h.mc[c]), 0, BS[a][pp] + h.off(c),
                   std::max(1, h.mc[pp]), h.k[c], items[a].nc, h.mc[c], (T)1, 0);
      }
    }
  }
  {   // root block
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      const HssInv<T> &h = *items[a].h;
      if (h.empty()) continue;
      const int c = h.root, m = h.mc[c];
      if (h.ct->leaf(c))
        p.gemm_job(s, h.G[c], std::max(1, m), 0, items[a].X, (int)items[a].ldx, 0, items[a].Y,
                   (int)items[a].ldy, m, items[a].nc, m, (T)1, 0);
      else
        p.gemm_job(s, h.G[c], std::max(1, m), 0, BS[a][c], std::max(1, m), 0, YS[a][c],
                   std::max(1, m), m, items[a].nc, m, (T)1, 0);
    }
  }
  for (int L = 1; L <= maxL; ++L) {   // x_c = E_c y_c + G_c beta_c
    Stage<T> &s1 = p.add(kGemm);
    Stage<T> &s2 = p.add(kGemm);
    for (size_t a = 0; a < items.size(); ++a) {
      const HssInv<T> &h = *items[a].h;
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const bool lf = h.ct->leaf(c);
        const int pp = h.par[c], m = h.mc[c];
        cplx<T> *dst = lf ? items[a].Y + (h.ct->start[c] - h.base) : YS[a][c];
        const int ldd = lf ? (int)items[a].ldy : std::max(1, m);
        p.gemm_job(s1, h.E[c], std::max(1, m), 0, YS[a][pp] + h.off(c), std::max(1, h.mc[pp]), 0,
                   dst, ldd, m, items[a].nc, h.k[c], (T)1, 0);
        p.gemm_job(s2, h.G[c], std::max(1, m), 0, lf ? leaf_x(a, c) : BS[a][c],
                   lf ? (int)items[a].ldx : std::max(1, m), 0, dst, ldd, m, items[a].nc, m, (T)1,
                   1);
      }
    }
  }
}

// Telescoping inverses of complex64 generators computed in complex128 and
// stored in complex64.  On indefinite Schur complements the leaf blocks D
// and the reduced blocks U^T D^-1 U can be nearly singular; in single
// precision their inverses, and G = D^-1 - E Z^T formed from them, then carry
// errors far above the rounding level, which the compressions built on these
// inverses cannot get below.  The generators are widened once, the levels run
// as in gym_factor<double> (scratch from wide), and E, G are rounded once.
inline void gym_factor_wide(std::vector<HssInv<float>> &out,
                            const std::vector<const Gen<float> *> &in, const std::vector<int> &node,
                            const Alloc<float> &store, const Alloc<double> &wide, int *err,
                            Staging &sg, Arena &ar, const c128 *val, hipStream_t st,
                            double *flops) {
  const size_t n = in.size();
  std::vector<Gen<double>> gd(n);
  Prog<float> up;
  Stage<float> &sw = up.add(kGtw);
  auto widen = [&](const cplx<float> *src, int ld, int rows, int cols) -> const c128 * {
    if (!src || rows <= 0 || cols <= 0) return nullptr;
    c128 *d = wide((size_t)rows * cols);
    sw.gtw.push_back(GatherJob<cplx<float>, c128>{src, d, ld, rows, nullptr, nullptr, rows, cols, 0,
                                                  1.0});
    return d;
  };
  for (size_t i = 0; i < n; ++i) {
    const Gen<float> &g = *in[i];
    Gen<double> &h = gd[i];
    h.ct = g.ct;
    h.root = g.root;
    h.k = g.k;
    const int nc = g.ct->count();
    h.U.assign(nc, nullptr); h.D.assign(nc, nullptr); h.B12.assign(nc, nullptr);
    h.B21.assign(nc, nullptr);
    h.ldU.assign(nc, 1); h.ldD.assign(nc, 1); h.ldB12.assign(nc, 1); h.ldB21.assign(nc, 1);
    for (const auto &l : sub_levels(*g.ct, g.root))
      for (int c : l) {
        const int rows = g.rowsU(c), k = c == g.root ? 0 : g.k[c];
        if (k) {
          h.U[c] = widen(g.U[c], g.ldU[c], rows, k);
          h.ldU[c] = std::max(1, rows);
        }
        if (g.ct->leaf(c)) {
          const int sz = g.ct->size[c];
          h.D[c] = widen(g.D[c], g.ldD[c], sz, sz);
          h.ldD[c] = std::max(1, sz);
        } else {
          const int kl = g.k[g.ct->left[c]], kr = g.k[g.ct->right[c]];
          h.B12[c] = widen(g.B12[c], g.ldB12[c], kl, kr);
          h.B21[c] = widen(g.B21[c], g.ldB21[c], kr, kl);
          h.ldB12[c] = std::max(1, kl);
          h.ldB21[c] = std::max(1, kr);
        }
      }
  }
  run_prog(up, sg, val, st);
  std::vector<const Gen<double> *> gp;
  for (auto &h : gd) gp.push_back(&h);
  std::vector<HssInv<double>> od;
  gym_factor<double>(od, gp, node, wide, wide, err, sg, ar, val, st, flops);
  // the same structure in complex64 storage
  out.assign(n, HssInv<float>{});
  Prog<float> down;
  Stage<float> &sn = down.add(kGwt);
  for (size_t i = 0; i < n; ++i) {
    const HssInv<double> &w = od[i];
    HssInv<float> &h = out[i];
    h.ct = w.ct;
    h.root = w.root;
    h.base = w.base;
    h.lev = w.lev;
    h.k = w.k;
    h.mc = w.mc;
    h.par = w.par;
    const int nc = w.ct->count();
    h.E.assign(nc, nullptr);
    h.G.assign(nc, nullptr);
    h.W.assign(nc, nullptr);
    for (const auto &l : w.lev)
      for (int c : l) {
        const int m = w.mc[c], k = w.k[c];
        h.E[c] = store(std::max<size_t>(1, (size_t)m * k));
        h.G[c] = store(std::max<size_t>(1, (size_t)m * m));
        if (m && k)
          sn.gwt.push_back(GatherJob<c128, cplx<float>>{w.E[c], h.E[c], m, m, nullptr, nullptr, m,
                                                        k, 0, 1.0});
        if (m)
          sn.gwt.push_back(GatherJob<c128, cplx<float>>{w.G[c], h.G[c], m, m, nullptr, nullptr, m,
                                                        m, 0, 1.0});
      }
  }
  run_prog(down, sg, val, st);
}

// W_c = G_c + E_c W_p(c, c) E_c^T top-down (W_root = G_root): H^-1 in HSS
// form with bases E (inverse_view)
template <typename T>
void gym_inverse_blocks(Prog<T> &p, std::vector<HssInv<T> *> &hs, const Alloc<T> &store,
                        const Alloc<T> &scratch) {
  int maxL = -1;
  std::vector<std::vector<cplx<T> *>> T1(hs.size());
  for (size_t a = 0; a < hs.size(); ++a) {
    HssInv<T> &h = *hs[a];
    if (h.empty()) continue;
    T1[a].assign(h.ct->count(), nullptr);
    h.W[h.root] = h.G[h.root];
    for (size_t L = 1; L < h.lev.size(); ++L)
      for (int c : h.lev[L]) {
        const size_t m = h.mc[c];
        h.W[c] = store(std::max<size_t>(1, m * m));
        T1[a][c] = scratch(std::max<size_t>(1, m * h.k[c]));
      }
    maxL = std::max(maxL, (int)h.lev.size() - 1);
  }
  for (int L = 1; L <= maxL; ++L) {
    Stage<T> &s1 = p.add(kGemm);
    Stage<T> &s2 = p.add(kCopy);
    Stage<T> &s3 = p.add(kGemm);
    for (size_t a = 0; a < hs.size(); ++a) {
      HssInv<T> &h = *hs[a];
      if (L >= (int)h.lev.size()) continue;
      for (int c : h.lev[L]) {
        const int pp = h.par[c], m = h.mc[c], k = h.k[c], o = h.off(c), mp = std::max(1, h.mc[pp]);
        p.gemm_job(s1, h.E[c], std::max(1, m), 0, h.W[pp] + o + (long)o * mp, mp, 0, T1[a][c],
                   std::max(1, m), m, k, k, (T)1, 0);
        s2.copy.push_back(CopyJob<T>{h.G[c], h.W[c], std::max(1, m), std::max(1, m), m, m, 0, (T)1});
        p.gemm_job(s3, T1[a][c], std::max(1, m), 0, h.E[c], std::max(1, m), 1, h.W[c],
                   std::max(1, m), m, m, k, (T)1, 1);
      }
    }
  }
}

// ---------------------------------------------------------------- entries
// Transposed full bases Uf^T and coupling products (Uf B)^T of a generator
// set, and the per-cluster entry descriptors (positions relative to the
// subtree).
template <typename T> struct EntPrep {
  const Gen<T> *g = nullptr;
  std::vector<cplx<T> *> Uf, UB;   // k_c x size_c and k_sibling x size_c
  std::vector<EntCl<T>> cl;
  std::vector<int> leaf_of;
};

template <typename T>
void entry_prep(Prog<T> &p, std::vector<EntPrep<T>> &ep, const Alloc<T> &scratch) {
  int maxL = -1;
  std::vector<std::vector<std::vector<int>>> lev(ep.size());
  std::vector<std::vector<int>> par(ep.size());
  Stage<T> &cp = p.add(kCopy);
  for (size_t a = 0; a < ep.size(); ++a) {
    const Gen<T> &g = *ep[a].g;
    lev[a] = sub_levels(*g.ct, g.root);
    par[a] = parents_of(*g.ct);
    const int n = g.ct->count();
    ep[a].Uf.assign(n, nullptr);
    ep[a].UB.assign(n, nullptr);
    for (const auto &l : lev[a])
      for (int c : l) {
        if (c == g.root) continue;
        const int pp = par[a][c], sz = g.ct->size[c];
        const int sib = g.ct->left[pp] == c ? g.ct->right[pp] : g.ct->left[pp];
        ep[a].Uf[c] = scratch((size_t)std::max(1, sz * g.k[c]));
        ep[a].UB[c] = scratch((size_t)std::max(1, sz * g.k[sib]));
        if (g.ct->leaf(c) && g.k[c])
          cp.copy.push_back(CopyJob<T>{g.U[c], ep[a].Uf[c], g.ldU[c], g.k[c], g.k[c], sz, 1, (T)1});
      }
    maxL = std::max(maxL, (int)lev[a].size() - 1);
  }
  for (int L = maxL; L >= 1; --L) {
    Stage<T> &s = p.add(kGemm);
    for (size_t a = 0; a < ep.size(); ++a) {
      const Gen<T> &g = *ep[a].g;
      if (L >= (int)lev[a].size()) continue;
      for (int c : lev[a][L]) {
        if (g.ct->leaf(c)) continue;
        const int l = g.ct->left[c], r = g.ct->right[c], sl = g.ct->size[l];
        const int kc = g.k[c], kl = g.k[l], kr = g.k[r];
        p.gemm_job(s, g.U[c], g.ldU[c], 1, ep[a].Uf[l], std::max(1, kl), 0, ep[a].Uf[c],
                   std::max(1, kc), kc, sl, kl, (T)1, 0);
        p.gemm_job(s, g.U[c] + kl, g.ldU[c], 1, ep[a].Uf[r], std::max(1, kr), 0,
                   ep[a].Uf[c] + (long)sl * kc, std::max(1, kc), kc, g.ct->size[r], kr, (T)1, 0);
      }
    }
  }
  Stage<T> &s = p.add(kGemm);
  for (size_t a = 0; a < ep.size(); ++a) {
    const Gen<T> &g = *ep[a].g;
    for (const auto &l : lev[a])
      for (int c : l) {
        if (g.ct->leaf(c)) continue;
        const int lc = g.ct->left[c], rc = g.ct->right[c];
        const int kl = g.k[lc], kr = g.k[rc], sl = g.ct->size[lc], sr = g.ct->size[rc];
        p.gemm_job(s, g.B12[c], g.ldB12[c], 1, ep[a].Uf[lc], std::max(1, kl), 0, ep[a].UB[lc],
                   std::max(1, kr), kr, sl, kl, (T)1, 0);
        p.gemm_job(s, g.B21[c], g.ldB21[c], 1, ep[a].Uf[rc], std::max(1, kr), 0, ep[a].UB[rc],
                   std::max(1, kl), kl, sr, kr, (T)1, 0);
      }
  }
  // descriptors (ids of the full tree; only the subtree's entries are used)
  for (size_t a = 0; a < ep.size(); ++a) {
    const Gen<T> &g = *ep[a].g;
    const int n = g.ct->count(), base = g.base();
    ep[a].cl.assign(n, EntCl<T>{});
    ep[a].leaf_of.assign(std::max(1, g.m()), 0);
    for (size_t L = 0; L < lev[a].size(); ++L)
      for (int c : lev[a][L]) {
        EntCl<T> &e = ep[a].cl[c];
        e.start = g.ct->start[c] - base;
        e.size = g.ct->size[c];
        e.left = g.ct->left[c];
        e.right = g.ct->right[c];
        e.parent = c == g.root ? -1 : par[a][c];
        e.level = (int)L;
        e.k = c == g.root ? 0 : g.k[c];
        e.ldD = g.ldD[c];
        e.D = g.D[c];
        e.Uf = ep[a].Uf[c];
        e.UB = ep[a].UB[c];
        if (g.ct->leaf(c))
          for (int q = 0; q < e.size; ++q) ep[a].leaf_of[e.start + q] = c;
      }
  }
}

}  // namespace hssx
