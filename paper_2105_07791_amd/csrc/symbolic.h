// Symbolic analysis: box nested dissection, elimination tree, cluster trees.
// Integer-only host code (Sec. 3.1 Def. 3.1, Fig. 3; Sec. 3.2 Fig. 4).
#pragma once

#include <vector>

namespace hssx {

// Binary cluster tree over the positions of an ordered DOF list, in level
// order (Def. 2.1 with contiguous clusters).
struct ClusterTree {
  std::vector<int> start, size, left, right, level;
  int count() const { return (int)start.size(); }
  bool leaf(int c) const { return left[c] < 0; }
  int depth() const {
    int d = 0;
    for (int l : level) d = l > d ? l : d;
    return d;
  }
};

struct NDNode {
  int x0, x1, y0, y1;        // half-open box of grid nodes (CG) or cells (DG)
  int lo = -1, hi = -1;      // children (post-order ids), -1 for leaves
  int parent = -1;
  int depth = 0, height = 0;
  std::vector<int> bd;       // Bd(sigma), sorted node ids
  std::vector<int> I;        // interior DOFs, elimination order
  std::vector<int> B;        // boundary DOFs, cluster-tree leaf order
  int p0 = 0;                // first p0 entries of B face the parent's I
  ClusterTree ct;            // cluster tree over B
  int offset = 0;            // first position of I in the permutation
  bool leafnode() const { return lo < 0; }
};

// meshes: continuous (units are the N x N grid nodes) or discontinuous
// (units are the two triangles of each of N x N cells)
constexpr int kMeshCG = 0, kMeshDG = 1;

struct Symbolic {
  int N = 0, leaf_dofs = 0, beta = 0, dofs = 1, mesh = kMeshCG;
  std::vector<NDNode> nodes;   // post-order; root last
  std::vector<int> perm;       // perm[k] = node id eliminated at position k
  std::vector<int> iperm;      // iperm[node id] = position
  int max_depth = 0;
  // forests: nodes of part q are [part_nodes[q], part_nodes[q+1])
  std::vector<int> part_nodes;
};

// threads: host threads for the per-node work (boundary sets, cluster
// trees, interiors); the result does not depend on it.  dofs: unknowns per
// unit (1 scalar, 2 for the elastic operator, 6 for P2 triangles); I, B, perm
// and the cluster ranges are then DOF lists (DOF id = dofs * unit + c).
// mesh: kMeshCG (N grid nodes per side) or kMeshDG (N cells per side).
Symbolic build_symbolic(int N, int leaf_dofs, int beta, int threads = 1, int dofs = 1,
                        int mesh = kMeshCG);

// Forest of independent problems: the trees of `parts` side by side, with
// node ids, DOF ids and permutation positions shifted so that part p's DOFs
// are [dof_off[p], dof_off[p+1]) of one block-diagonal system.  Every tree
// keeps its own depths, so depth 0 holds all roots.
Symbolic merge_forest(std::vector<Symbolic> &&parts, const std::vector<int> &dof_off);

// Cluster tree of the P0 block of a node's boundary: the left subtree of the
// top split, the whole tree when the node has no P1 part, empty without P0.  Positions are
// relative to the subtree's first position (which is 0).
ClusterTree interior_subtree(const NDNode &nd);

}  // namespace hssx
