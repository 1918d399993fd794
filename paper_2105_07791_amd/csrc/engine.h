// Handles behind the C ABI and the host drivers that sequence the kernels.
#pragma once

#include <memory>

#include "common.h"
#include "kernels.h"
#include "prof.h"
#include "symbolic.h"

struct hssx_op_ {
  int device = 0;
  int N = 0;
  double omega = 0;
  int n = 0;
  long nnz = 0;
  hssx::DevBuf rowptr, col, val, mval, s;
  std::vector<int> h_rowptr, h_col;
};

struct hssx_fact_ {
  hssx_op_ *A = nullptr;      // operator the factor was built from (not owned)
  hssx_dtype dtype = HSSX_C128;
  double tol = 0;
  int leaf = 0;
  hssx_factor_opts opts{};
  hssx::Symbolic sym;
  std::vector<int> arith, comp; // per node: HSS arithmetic, compressed S
  std::vector<hssx::FrontDesc> h_desc;
  hssx::DevBuf desc, bpos, src_gid, src_child, src_pos, perm, front;
  // complex64 factors keep the root (top separator) in complex128: its front
  // lives in front64 and desc64 is the descriptor table with the root at 0
  hssx::DevBuf front64, desc64;
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
};

namespace hssx {

void factor_numeric(hssx_fact_ &P, hipStream_t st);
void apply(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y, long ldy,
           hipStream_t st);
void gmres(hssx_op_ &A, hssx_fact_ *P, int trans, int nrhs, const c128 *b, long ldb, c128 *x,
           long ldx, const hssx_gmres_opts &o, hssx_gmres_stats *stats, hipStream_t st);

}  // namespace hssx
