// Handles behind the C ABI and the host drivers that sequence the kernels.
#pragma once

#include <atomic>
#include <map>
#include <memory>
#include <mutex>

#include "common.h"
#include "hss_arith.h"
#include "kernels.h"
#include "prof.h"
#include "symbolic.h"

namespace hssx {

// Index maps of one HSS-class node sigma (children mu, nu), built once per
// analysis; the int arrays live in one device pool at the listed offsets.
// Positions: sigma's interior I = [P0(mu); P0(nu)] (pmu + pnu), sigma's
// boundary B in its cluster-tree order (nb), a child's boundary in its own
// cluster-tree order (P0 first).
struct HssSym {
  int node = -1, mu = -1, nu = -1;
  int pmu = 0, pnu = 0, ni = 0, nb = 0, mmu = 0, mnu = 0;
  int ii_mu = -1, bb_mu = -1, ii_nu = -1, bb_nu = -1;   // subtree roots in the children's trees
  int split_mu = 0, split_nu = 0;                       // child's tree splits [P0 | P1] at its root
  long bchild = 0, bcpos = 0, gid = 0;                  // per B position: child, child position, DOF
  long p1mu = 0, p1nu = 0;                              // child's P1 row -> B position
  long smu = 0, snu = 0;                                // B position -> child's P1 row or -1
  long bb_rp = 0, bb_cp = 0, bb_vi = 0;                 // couplings of the children inside B
  long inu_rp = 0, inu_cp = 0, inu_vi = 0;              // A~(nu,mu): rows P0(nu), columns P0(mu)
  long imu_rp = 0, imu_cp = 0, imu_vi = 0;              // A~(mu,nu)
  long ib_ri = 0, ib_ci = 0, ib_vi = 0;                 // A_ib couplings across the children (COO)
  long yb_ri = 0, yb_ci = 0, yb_vi = 0;                 // unit entries of those columns in Y_B
  int nib = 0, ncr = 0;                                 // COO entries, coupling columns
};

// Factor data of the HSS arithmetic for one precision.
template <typename T> struct HssNodeData {
  HssMat<T> S;          // S(sigma) in generator form (when its parent uses HSS arithmetic)
  bool has_S = false;
  HssMat<T> St;         // inner Schur complement S~ (Alg. 3.3)
  HssInv<T> Hmu, Hs;    // telescoping inverses of S_ii^mu and S~
  cplx<T> *W = nullptr, *YB = nullptr;   // R = -W Y_B^T, L = -Y_B W^T (eq. 3.7)
  int r = 0;
};

// Apply program of the HSS-class nodes for one right-hand-side count: per
// depth the up-step (block solve of Alg. 3.3 and the L update) and the
// down-step (R update); scratch in its own arena.
template <typename T> struct HssApplyPlan {
  std::vector<Plan<T>> up, down;
  std::unique_ptr<Arena> mem;
  double fbytes = 0;
};

}  // namespace hssx

// A context: the device allocator the caller hands in (hssx_create), and
// the scratch arenas and staging areas of the calls made on its handles,
// all freed through that allocator by hssx_destroy.
struct hssx_ctx_ {
  int device = 0;
  hssx_allocator a{};
  std::atomic<long> live_bytes{0}, allocs{0}, frees{0};
  std::mutex mu;
  std::vector<std::unique_ptr<hssx::Arena>> arenas;
  std::vector<std::unique_ptr<hssx::Staging>> stagings;
};

struct hssx_op_ {
  int device = 0;
  hssx_ctx_ *ctx = nullptr;   // context it was created under (or null)
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
  hssx_ctx_ *ctx = nullptr;   // context it was created under (or null)
  int device = 0;             // device of its buffers (A may be gone at destroy)
  std::vector<long> pattern;  // its pattern key (checked by hssx_refactor)
  hssx_dtype dtype = HSSX_C128;
  double tol = 0;
  int leaf = 0;
  hssx_factor_opts opts{};
  hssx::Symbolic sym;
  std::vector<int> arith, comp; // per node: HSS arithmetic, compressed S
  // HSS-class nodes (HSS arithmetic, not the root): their maps, and the
  // factor data of both precisions (only the factor's is filled)
  std::vector<int> hss_idx;                 // node -> index into hsym or -1
  std::vector<hssx::HssSym> hsym;
  hssx::DevBuf hsym_pool;
  std::vector<hssx::HssNodeData<float>> h32;
  std::vector<hssx::HssNodeData<double>> h64;
  hssx::Arena store;                        // device storage of the HSS factor data
  std::map<int, hssx::HssApplyPlan<float>> plans32;
  std::map<int, hssx::HssApplyPlan<double>> plans64;
  std::vector<hssx::FrontDesc> h_desc;
  hssx::DevBuf desc, bpos, src_gid, src_code, perm, front;
  // complex64 factors keep the roots (top separators) in complex128: their
  // fronts live in front64, at the roots' foff
  hssx::DevBuf front64;
  // per depth (index = depth): nodes, and the largest |I|, |B|, front size;
  // depth_dev lists the nodes with dense fronts, hss_nodes the others
  std::vector<std::vector<int>> depth_nodes, dense_nodes, hss_nodes;
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
bool expand_schur(hssx_fact_ &P, int node, std::vector<c128> &out);
// the allocation-free apply's workspace on the current device (its address,
// looked up once per device, and its size)
char *noalloc_workspace(size_t *bytes);
// Algorithm 3.1 with every device buffer taken from the caller's workspace
// (no device allocation); synchronises st before returning
void apply_workspace(hssx_fact_ &P, int trans, int nrhs, const c128 *x, long ldx, c128 *y,
                     long ldy, hipStream_t st, char *ws, size_t ws_bytes);
// hssx_hss_eval's work (one caller-given HSS matrix)
void hss_eval(hssx_dtype dtype, int m, int ncl, const int32_t *tree, const int32_t *rank,
              const double *gens, int op, int nrhs, const void *x_dev, void *y_dev, long nij,
              const int32_t *ij, double *vals, hipStream_t st);
void gmres(hssx_op_ &A, hssx_fact_ *P, int trans, int nrhs, const c128 *b, long ldb, c128 *x,
           long ldx, const hssx_gmres_opts &o, hssx_gmres_stats *stats, hipStream_t st);

}  // namespace hssx
