// Box nested dissection and cluster trees (host, integer-only).
//
// Rules: a box [x0,x1) x [y0,y1) of grid nodes is a leaf when nx*ny <=
// leaf_dofs; otherwise it is cut across its longer side (x on ties) at
// x0 + nx/2 (y0 + ny/2) into (low, high).  Nodes are numbered in post-order
// (Sec. 3.1, Fig. 1).  Bd(sigma) holds the box's grid nodes with a stencil
// neighbour outside the box; the P1 stencil couples (i,j) to (i+-1,j),
// (i,j+-1), (i+1,j+1) and (i-1,j-1) (shared triangles of the SW-NE split).
// Leaf I = box \ Bd in id order; non-leaf I = [P0(lo) ; P0(hi)] (eq. 3.4
// layout); B = Bd(sigma) ordered by its cluster tree whose root separates
// P0 = Bd \ Bd(parent) from P1 = Bd n Bd(parent) (Fig. 4); each part is
// bisected geometrically (axis of larger extent, x on ties; order by axis
// coordinate then the other coordinate; split at count/2) down to <= beta.
// Vector problems (dofs unknowns per node) apply the same rules on nodes with
// sizes counted in DOFs; every node's components stay consecutive.
// Discontinuous Galerkin meshes (Sec. 3.3, Fig. 5 left) use boxes of cells and
// whole triangles as the units: cell (i,j) holds the lower triangle 2 c and
// the upper triangle 2 c + 1 (c = j N + i); the lower one meets the upper one
// of its own cell, of cell (i,j-1) across its south edge and of cell (i+1,j)
// across its east edge.  Cluster coordinates are the triangle centroids in
// units of h/3: (3i+2, 3j+1) lower, (3i+1, 3j+2) upper.
#include "symbolic.h"

#include <algorithm>
#include <atomic>
#include <functional>
#include <memory>
#include <thread>

namespace hssx {

namespace {

struct CNode {
  std::unique_ptr<CNode> l, r;
  int start = 0, stop = 0;  // range in the leaf order
};

// Integer unit coordinates (both below M): grid nodes, or triangle
// centroids in thirds of a cell.
struct Coords {
  int N, mesh;
  int M() const { return mesh == kMeshDG ? 3 * N : N; }
  void operator()(int u, long &x, long &y) const {
    if (mesh == kMeshDG) {
      const int c = u >> 1, t = u & 1;
      x = 3L * (c % N) + 2 - t;
      y = 3L * (c / N) + 1 + t;
    } else {
      x = u % N;
      y = u / N;
    }
  }
};

// Geometric bisection of ids[0, n) in place; the final array is the leaf
// order (in-order concatenation of the leaves), node ranges are offsets.
std::unique_ptr<CNode> bisect(int *ids, int n, int offset, const Coords &cc, int beta,
                              std::vector<long> &key) {
  auto node = std::make_unique<CNode>();
  node->start = offset;
  node->stop = offset + n;
  if (n <= beta) return node;
  const long M = cc.M();
  long xmin = M, xmax = -1, ymin = M, ymax = -1;
  for (int k = 0; k < n; ++k) {
    long x, y;
    cc(ids[k], x, y);
    xmin = std::min(xmin, x); xmax = std::max(xmax, x);
    ymin = std::min(ymin, y); ymax = std::max(ymax, y);
  }
  const bool by_x = (xmax - xmin) >= (ymax - ymin);
  // order by the split axis, then the other coordinate, then the id
  key.resize(n);
  for (int k = 0; k < n; ++k) {
    long x, y;
    cc(ids[k], x, y);
    key[k] = by_x ? ((x * M + y) << 32 | (unsigned)ids[k]) : ((y * M + x) << 32 | (unsigned)ids[k]);
  }
  std::sort(key.begin(), key.begin() + n);
  for (int k = 0; k < n; ++k) ids[k] = (int)(key[k] & 0xffffffffL);
  const int h = n / 2;
  node->l = bisect(ids, h, offset, cc, beta, key);
  node->r = bisect(ids + h, n - h, offset + h, cc, beta, key);
  return node;
}

// Level-order cluster tree + leaf order of the given parts.
void make_cluster_tree(const std::vector<int> &P0, const std::vector<int> &P1,
                       const Coords &cc, int beta, ClusterTree &ct, std::vector<int> &order) {
  ct = ClusterTree();
  order.clear();
  if (P0.empty() && P1.empty()) return;
  order = P0;
  order.insert(order.end(), P1.begin(), P1.end());
  std::vector<long> key;
  std::unique_ptr<CNode> root;
  const int n0 = (int)P0.size(), n1 = (int)P1.size();
  if (n0 && n1) {
    root = std::make_unique<CNode>();
    root->start = 0;
    root->stop = n0 + n1;
    root->l = bisect(order.data(), n0, 0, cc, beta, key);
    root->r = bisect(order.data() + n0, n1, n0, cc, beta, key);
  } else {
    root = bisect(order.data(), n0 + n1, 0, cc, beta, key);
  }
  // breadth-first numbering
  std::vector<std::pair<const CNode *, int>> q{{root.get(), 0}};
  for (size_t k = 0; k < q.size(); ++k) {
    const CNode *t = q[k].first;
    if (t->l) {
      q.push_back({t->l.get(), q[k].second + 1});
      q.push_back({t->r.get(), q[k].second + 1});
    }
  }
  int nc = (int)q.size();
  ct.start.resize(nc); ct.size.resize(nc); ct.left.assign(nc, -1);
  ct.right.assign(nc, -1); ct.level.resize(nc);
  for (int k = 0, child = 1; k < nc; ++k) {
    ct.start[k] = q[k].first->start;
    ct.size[k] = q[k].first->stop - q[k].first->start;
    ct.level[k] = q[k].second;
    if (q[k].first->l) {
      // children of the k-th node were appended in order; locate them
      for (int j = child; j < nc; ++j)
        if (q[j].first == q[k].first->l.get()) { ct.left[k] = j; ct.right[k] = j + 1; child = j + 2; break; }
    }
  }
}

// fn(k) for k in [0, n) on up to `threads` host threads
template <typename F> void parallel_for(int n, int threads, F fn) {
  threads = std::max(1, std::min(threads, n / 64));
  if (threads <= 1) {
    for (int k = 0; k < n; ++k) fn(k);
    return;
  }
  std::atomic<int> next{0};
  auto work = [&] {
    for (int k; (k = next.fetch_add(64)) < n;)
      for (int j = k; j < std::min(n, k + 64); ++j) fn(j);
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < threads; ++t) pool.emplace_back(work);
  work();
  for (auto &t : pool) t.join();
}

}  // namespace

Symbolic build_symbolic(int N, int leaf_dofs, int beta, int threads, int dofs, int mesh) {
  Symbolic s;
  s.N = N;
  s.leaf_dofs = leaf_dofs;
  s.beta = beta;
  s.dofs = dofs;
  s.mesh = mesh;
  auto &nodes = s.nodes;
  const bool dg = mesh == kMeshDG;
  const int per_cell = dg ? 2 : 1;   // units per box cell
  // boxes and clusters are formed on units with sizes counted in DOFs:
  // nx ny per_cell dofs > leaf_dofs  <=>  nx ny > leaf_dofs / (per_cell dofs)
  const int leaf_nodes = leaf_dofs / (per_cell * dofs);
  beta = beta / dofs;
  const Coords cc{N, mesh};

  std::function<int(int, int, int, int, int)> rec = [&](int x0, int x1, int y0, int y1, int depth) {
    NDNode b;
    b.x0 = x0; b.x1 = x1; b.y0 = y0; b.y1 = y1; b.depth = depth;
    int nx = x1 - x0, ny = y1 - y0;
    if ((long)nx * ny > leaf_nodes) {
      int lo, hi;
      if (nx >= ny) {
        int xm = x0 + nx / 2;
        lo = rec(x0, xm, y0, y1, depth + 1);
        hi = rec(xm, x1, y0, y1, depth + 1);
      } else {
        int ym = y0 + ny / 2;
        lo = rec(x0, x1, y0, ym, depth + 1);
        hi = rec(x0, x1, ym, y1, depth + 1);
      }
      b.lo = lo; b.hi = hi;
      b.height = 1 + std::max(nodes[lo].height, nodes[hi].height);
    }
    nodes.push_back(std::move(b));
    int k = (int)nodes.size() - 1;
    if (nodes[k].lo >= 0) { nodes[nodes[k].lo].parent = k; nodes[nodes[k].hi].parent = k; }
    s.max_depth = std::max(s.max_depth, depth);
    return k;
  };
  rec(0, N, 0, N, 0);

  static const int dx[6] = {1, -1, 0, 0, 1, -1};
  static const int dy[6] = {0, 0, 1, -1, 1, -1};
  // face neighbours of the lower (t = 0: south, east) and upper (t = 1:
  // north, west) triangle of a cell, as cell offsets
  static const int fx[2][2] = {{0, 1}, {0, -1}}, fy[2][2] = {{-1, 0}, {1, 0}};
  const int nn = (int)nodes.size();
  // a unit with a neighbour outside the box lies in a border cell, so only
  // border cells are tested (row-major, so the ids come out sorted)
  parallel_for(nn, threads, [&](int k) {
    auto &b = nodes[k];
    auto outside = [&](int u, int v) {
      return u >= 0 && v >= 0 && u < N && v < N && (u < b.x0 || u >= b.x1 || v < b.y0 || v >= b.y1);
    };
    for (int y = b.y0; y < b.y1; ++y)
      for (int x = b.x0; x < b.x1; x = (y == b.y0 || y == b.y1 - 1 || x == b.x1 - 1) ? x + 1 : b.x1 - 1) {
        if (dg) {
          for (int t = 0; t < 2; ++t)
            if (outside(x + fx[t][0], y + fy[t][0]) || outside(x + fx[t][1], y + fy[t][1]))
              b.bd.push_back(2 * (y * N + x) + t);
          continue;
        }
        bool out = false;
        for (int d = 0; d < 6 && !out; ++d) out = outside(x + dx[d], y + dy[d]);
        if (out) b.bd.push_back(y * N + x);     // row-major scan = sorted ids
      }
  });

  parallel_for(nn, threads, [&](int k) {
    auto &b = nodes[k];
    if (b.parent < 0) return;
    const auto &pbd = nodes[b.parent].bd;
    std::vector<int> P0, P1;
    for (int v : b.bd)
      (std::binary_search(pbd.begin(), pbd.end(), v) ? P1 : P0).push_back(v);
    make_cluster_tree(P0, P1, cc, beta, b.ct, b.B);
    b.p0 = (int)P0.size();
  });

  parallel_for(nn, threads, [&](int k) {
    auto &b = nodes[k];
    if (b.leafnode()) {
      for (int y = b.y0; y < b.y1; ++y)
        for (int x = b.x0; x < b.x1; ++x)
          for (int t = 0; t < per_cell; ++t) {
            int v = per_cell * (y * N + x) + t;
            if (!std::binary_search(b.bd.begin(), b.bd.end(), v)) b.I.push_back(v);
          }
    } else {
      const auto &mu = nodes[b.lo], &nu = nodes[b.hi];
      b.I.assign(mu.B.begin(), mu.B.begin() + mu.p0);
      b.I.insert(b.I.end(), nu.B.begin(), nu.B.begin() + nu.p0);
    }
  });

  // unit lists -> DOF lists (DOF id = dofs * unit + component)
  if (dofs > 1) {
    parallel_for(nn, threads, [&](int k) {
      auto &b = nodes[k];
      auto ex = [dofs](std::vector<int> &v) {
        std::vector<int> o;
        o.reserve(v.size() * dofs);
        for (int x : v)
          for (int c = 0; c < dofs; ++c) o.push_back(dofs * x + c);
        v.swap(o);
      };
      ex(b.I);
      ex(b.B);
      b.p0 *= dofs;
      for (auto &x : b.ct.start) x *= dofs;
      for (auto &x : b.ct.size) x *= dofs;
    });
  }
  for (auto &b : nodes) std::vector<int>().swap(b.bd);   // only needed above
  const size_t n = (size_t)N * N * per_cell * dofs;
  s.perm.reserve(n);
  for (auto &b : nodes) {
    b.offset = (int)s.perm.size();
    s.perm.insert(s.perm.end(), b.I.begin(), b.I.end());
  }
  s.iperm.assign(n, -1);
  for (size_t k = 0; k < s.perm.size(); ++k) s.iperm[s.perm[k]] = (int)k;
  s.part_nodes = {0, (int)nodes.size()};
  return s;
}

Symbolic merge_forest(std::vector<Symbolic> &&parts, const std::vector<int> &dof_off) {
  Symbolic f;
  if (parts.empty()) return f;
  f.leaf_dofs = parts[0].leaf_dofs;
  f.beta = parts[0].beta;
  const int n = dof_off.back();
  size_t total = 0;
  for (const auto &s : parts) total += s.nodes.size();
  f.nodes.reserve(total);
  f.perm.reserve(n);
  f.iperm.assign(n, -1);
  f.part_nodes.push_back(0);
  for (size_t q = 0; q < parts.size(); ++q) {
    Symbolic &s = parts[q];
    const int base = (int)f.nodes.size(), o = dof_off[q];
    auto shift = [o](std::vector<int> &v) { for (int &x : v) x += o; };
    for (NDNode &nd : s.nodes) {
      if (nd.lo >= 0) { nd.lo += base; nd.hi += base; }
      if (nd.parent >= 0) nd.parent += base;
      shift(nd.bd);
      shift(nd.I);
      shift(nd.B);
      nd.offset += o;
      f.nodes.push_back(std::move(nd));
    }
    for (int v : s.perm) f.perm.push_back(v + o);
    for (size_t k = 0; k < s.iperm.size(); ++k) f.iperm[k + o] = s.iperm[k] + o;
    f.max_depth = std::max(f.max_depth, s.max_depth);
    f.part_nodes.push_back((int)f.nodes.size());
    Symbolic().nodes.swap(s.nodes);   // release the part's storage
  }
  return f;
}

ClusterTree interior_subtree(const NDNode &nd) {
  const ClusterTree &ct = nd.ct;
  if (ct.count() == 0 || nd.p0 == 0) return ClusterTree();   // no P0 part
  if (nd.p0 == (int)nd.B.size()) return ct;                  // no P1 part
  ClusterTree out;
  std::vector<std::pair<int, int>> q{{ct.left[0], 0}};
  for (size_t k = 0; k < q.size(); ++k) {
    int c = q[k].first;
    if (ct.left[c] >= 0) {
      q.push_back({ct.left[c], q[k].second + 1});
      q.push_back({ct.right[c], q[k].second + 1});
    }
  }
  int nc = (int)q.size();
  out.start.resize(nc); out.size.resize(nc); out.left.assign(nc, -1);
  out.right.assign(nc, -1); out.level.resize(nc);
  std::vector<int> num(ct.count(), -1);
  for (int k = 0; k < nc; ++k) num[q[k].first] = k;
  int base = ct.start[ct.left[0]];
  for (int k = 0; k < nc; ++k) {
    int c = q[k].first;
    out.start[k] = ct.start[c] - base;
    out.size[k] = ct.size[c];
    out.level[k] = q[k].second;
    if (ct.left[c] >= 0) { out.left[k] = num[ct.left[c]]; out.right[k] = num[ct.right[c]]; }
  }
  return out;
}

}  // namespace hssx
