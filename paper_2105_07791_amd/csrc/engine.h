// Handles behind the C ABI and the host drivers that sequence the kernels.
#pragma once

#include <map>
#include <memory>

#include "common.h"
#include "kernels.h"
#include "prof.h"
#include "symbolic.h"

struct hssx_op_ {
  int device = 0;
  int N = 0;          // grid side (0 for a batch of problems)
  double omega = 0;
  int n = 0;
  int dofs = 1;       // unknowns per unit (2: elastic node, 6: P2 triangle)
  int mesh = 0;       // hssx::kMeshCG (grid nodes) or hssx::kMeshDG (triangles)
  int row_max = 7;    // longest CSR row (7 scalar P1, 14 elastic, 24 SIPG-P2)
  // the structured assemblers' patterns are functions of (mesh, dofs, grid
  // sides of the parts): operators with equal keys have equal patterns
  std::vector<long> pattern_key() const {
    std::vector<long> k{device, mesh, dofs, n, nnz};
    k.insert(k.end(), part_N.begin(), part_N.end());
    return k;
  }
  long nnz = 0;
  hssx::DevBuf rowptr, col, val, mval, s;
  std::vector<int> h_rowptr, h_col;
  // A batch of independent problems is one block-diagonal operator: part p
  // owns rows [part_off[p], part_off[p+1]) and is the grid of side part_N[p]
  // at frequency part_omega[p].  A single problem is the batch of one.
  std::vector<int> part_N, part_off;
  std::vector<double> part_omega;
  hssx::DevBuf part_off_dev, row_part_dev;   // row_part_dev only for batches
  hssx::Segs segs() const {
    return hssx::Segs{(int)part_N.size(), part_off_dev.as<int>(),
                      part_N.size() > 1 ? row_part_dev.as<int>() : nullptr};
  }
};

struct hssx_fact_ {
  hssx_op_ *A = nullptr;      // operator the factor was built from (not owned)
  std::vector<long> pattern;  // its pattern key (checked by hssx_refactor)
  hssx_dtype dtype = HSSX_C128;
  double tol = 0;
  int leaf = 0;
  hssx_factor_opts opts{};
  hssx::Symbolic sym;
  std::vector<int> arith, comp; // per node: HSS arithmetic, compressed S
  std::vector<hssx::FrontDesc> h_desc;
  hssx::DevBuf desc, bpos, src_gid, src_code, perm, front;
  // complex64 factors keep the roots (top separators) in complex128: their
  // fronts live in front64, at the roots' foff
  hssx::DevBuf front64;
  // per depth (index = depth): nodes, and the largest |I|, |B|, front size
  std::vector<std::vector<int>> depth_nodes;
  std::vector<hssx::DevBuf> depth_dev;
  std::vector<int> depth_max_ni, depth_max_nb, depth_max_f;
  // per depth: factor bytes and vector elements (per rhs) the apply moves
  std::vector<double> up_fbytes, up_velems, down_fbytes, down_velems, asm_bytes;
  hssx_factor_stats stats{};
  std::vector<int> node_rank;   // largest compressed rank per node (stats)
  hssx::DevBuf work;            // apply workspace (elimination-order vectors)
  size_t work_cols = 0;
  // apply: tile configuration per depth (by right-hand-side count) and the
  // sweeps captured as graphs (by right-hand-side count and transpose)
  std::map<int, std::vector<int>> cfg_up, cfg_down;
  struct SweepGraph {
    int nrhs, trans;
    hipGraphExec_t exec;
  };
  std::vector<SweepGraph> graphs;
  hipStream_t cap_stream = nullptr;
  bool capturing = false;
  ~hssx_fact_();
};

namespace hssx {

void factor_numeric(hssx_fact_ &P, hipStream_t st);
void destroy_graphs(hssx_fact_ &P);
void apply(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y, long ldy,
           hipStream_t st);
void gmres(hssx_op_ &A, hssx_fact_ *P, int trans, int nrhs, const c128 *b, long ldb, c128 *x,
           long ldx, const hssx_gmres_opts &o, hssx_gmres_stats *stats, hipStream_t st);

}  // namespace hssx
