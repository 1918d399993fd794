// Adaptive randomized HSS compression (Sec. 2.3, Appendix A, Algorithm A.1)
// for complex symmetric operators (V = U, transposes, no conjugates).
//
// gaussian: Omega(i, j) = Box-Muller(Philox4x32-10(ctr = (i, j, 0, 0),
//           key = (seed, instance))), u = (word + 0.5) 2^-32, using the first
//           two output words: g = sqrt(-2 ln u1) cos(2 pi u2).
// sample:   Y = S Omega (complex operator times real sketch).
// compress_level: one workgroup per cluster of the current tree level.  A
//           leaf removes its diagonal block, S_loc = Y(I, :) - D Omega(I, :),
//           D = S(I, I); an internal cluster stacks the children's reduced
//           samples minus the sibling coupling, S_loc = [Sr_l - B12 Om_r;
//           Sr_r - B21 Om_l], B12 = S(sk_l, sk_r), B21 = S(sk_r, sk_l).  The
//           interpolative decomposition S_loc ~ U S_loc(J, :) comes from a
//           pivoted Gram-Schmidt QR of S_loc^T (pivot = largest remaining row
//           norm, lowest row index on ties; one projection per pivot: the
//           rounding it leaves along the pivot direction is far below the
//           ID threshold of at least 4 unit roundoffs;
//           for complex64 and blocks up to 256 x 192 the rows stay in
//           registers, 16 lanes per row), rank =
//           min(k, rows, s) reduced to the pivots above id_tol * first pivot;
//           T = R11^-1 R12, U(J, :) = I, U(rest, :) = T^T.  The cluster keeps
//           Om_c = U^T Om_loc, Sr_c = S_loc(J, :), skeleton I_loc(J).  The
//           root only reads its B blocks.
// hss_matvec: telescoping product (eqs. 2.5-2.6), one launch per tree level
//           and phase, one workgroup per (job, cluster); used both for the
//           error estimate of eq. 2.7 and to expand the compressed matrix
//           column block by column block.
#include "common.h"
#include "kernels.h"

namespace hssx {

namespace {

constexpr int kTPR = 4;          // lanes per row in the global-memory pivoted QR
constexpr int kPasses = 1;       // projections per pivot step
// Workgroup sizes of the compression kernel: NT = 1024 for clusters of more
// than 64 rows, 256 below.  The register-resident pivoted QR (complex64)
// uses RT lanes per row, NT / RT row slots, RPT rows per slot and RSEG
// columns per lane: rows <= NT / RT * RPT, sample columns <= RT * RSEG.
// register tiles of the pivoted Gram-Schmidt: RT lanes per row, RPT rows
// per lane group, RSEG column segments of RT entries each (capacity
// NT / RT * RPT rows by RT * RSEG columns); the defaults are the largest
// tiles, smaller ones are chosen per launch so that a step's instruction
// stream follows the block's size
template <int NT> struct CCfg;
template <> struct CCfg<1024> { static constexpr int RT = 16, RPT = 4, RSEG = 12; };
template <> struct CCfg<256> { static constexpr int RT = 8, RPT = 2, RSEG = 24; };
constexpr int kMaxRows = 1024;   // rows of one local sample block (LDS index arrays)
constexpr int kMaxS = 1024;      // sample columns held in LDS for the projector

__device__ __forceinline__ void philox(uint32_t c[4], uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint32_t hi0 = __umulhi(M0, c[0]), lo0 = M0 * c[0];
    uint32_t hi1 = __umulhi(M1, c[2]), lo1 = M1 * c[2];
    uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
  }
}

__global__ void gaussian_kernel(const GaussJob *__restrict__ jobs, uint32_t seed) {
  const GaussJob jb = jobs[blockIdx.z];
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  int jj = blockIdx.y;
  if (i >= jb.m || jj >= jb.nc) return;
  uint32_t c[4] = {(uint32_t)i, (uint32_t)(jb.c0 + jj), 0u, 0u};
  philox(c, seed, jb.key1);
  double u1 = ((double)c[0] + 0.5) * 0x1p-32;
  double u2 = ((double)c[1] + 0.5) * 0x1p-32;
  double g = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
  jb.out[i + (long)(jb.c0 + jj - jb.cbase) * jb.ld] = g;
}

// Sampling on the matrix cores in the factor's real precision: the
// complex-times-real product in its real view, Yr (2m x nc) = Sr (2m x m)
// Omega (m x nc) with the re/im parts of S as interleaved rows, computed
// transposed (D = Yr^T = Omega^T Sr^T) so that each output register of a lane
// group holds 16 consecutive rows of one column of Y and the stores are
// coalesced.  Four wavefronts cover a 64 x 64 tile of Yr as 2 x 2 blocks of
// 32 x 32 and read their operands straight from global memory (the waves of a
// tile share them through the vector L1).  One step of the K loop takes 16
// sketch rows: lane group g feeds rows 4 g .. 4 g + 3 to the four 16x16x4
// products (any split of the rows over the products gives the same sum).
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
template <typename T> struct SampleMma;
template <> struct SampleMma<float> {
  using V = floatx4;
  __device__ static V fma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // row of D held by register r of lane group g
  __device__ static int drow(int g, int r) { return 4 * g + r; }
};
template <> struct SampleMma<double> {
  using V = doublex4;
  __device__ static V fma(double a, double b, V c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static int drow(int g, int r) { return g + 4 * r; }
};

template <typename T>
__global__ __launch_bounds__(256) void sample_kernel(const SampleJob<T> *__restrict__ jobs) {
  using M = SampleMma<T>;
  const SampleJob<T> jb = jobs[blockIdx.z];
  const int R = 2 * jb.m, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = blockIdx.x * 64 + 32 * (w & 1), wc = blockIdx.y * 64 + 32 * (w >> 1);
  if (wr >= R || wc >= jb.nc) return;   // no barriers below: waves leave alone
  const int q = lane & 15, g = lane >> 4;
  const T *Sr = reinterpret_cast<const T *>(jb.S);
  const long ldS = 2L * jb.ldS;
  int ri[2], cj[2];
  bool rok[2], cok[2];
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    ri[b] = wr + 16 * b + q;
    rok[b] = ri[b] < R;
    cj[b] = wc + 16 * b + q;
    cok[b] = cj[b] < jb.nc;
  }
  typename M::V d[2][2];
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int bi = 0; bi < 2; ++bi) d[bc][bi] = typename M::V{0, 0, 0, 0};
  for (int k0 = 0; k0 < jb.m; k0 += 16) {
    T a[2][4], o[2][4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int k = k0 + 4 * g + u;
      const bool kok = k < jb.m;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        a[b][u] = (rok[b] && kok) ? Sr[ri[b] + (long)k * ldS] : T(0);
        o[b][u] = (cok[b] && kok) ? (T)jb.Om[k + (long)cj[b] * jb.ldO] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int bc = 0; bc < 2; ++bc)
#pragma unroll
        for (int bi = 0; bi < 2; ++bi) d[bc][bi] = M::fma(o[bc][u], a[bi][u], d[bc][bi]);
  }
  // lane (q, g), register r: Yr row wr + 16 bi + q, column wc + 16 bc + drow(g, r)
  T *Yr = reinterpret_cast<T *>(jb.Y);
  const long ldY = 2L * jb.ldY;
#pragma unroll
  for (int bc = 0; bc < 2; ++bc)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int j = wc + 16 * bc + M::drow(g, r);
      if (j >= jb.nc) continue;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
        if (rok[bi]) Yr[ri[bi] + (long)j * ldY] = d[bc][bi][r];
    }
}

// bf16 sampling (complex64 only): the complex-times-real product in its real
// view, Y_r (2m x nc) = S_r (2m x m) Omega (m x nc) with the re/im parts of S
// as interleaved rows, on the 16x16x16 bf16 matrix cores with fp32
// accumulation.  SPLIT = 1: operands rounded to bf16 (nearest even) on load.
// SPLIT = 2: each operand is split into a bf16 head and a bf16 tail
// (x ~ hi + lo) and the product keeps hi*hi + hi*lo + lo*hi (three matrix-core
// products, about 16 significant bits).  One wavefront per 16 x 16 output
// tile; four wavefronts per workgroup stack their tiles over rows.
typedef short bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned bf16_bits(float f) {
  unsigned u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

template <int SPLIT>
__global__ __launch_bounds__(256) void sample_bf16_kernel(const SampleJob<float> *__restrict__ jobs) {
  const SampleJob<float> jb = jobs[blockIdx.z];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int R = 2 * jb.m;                               // real rows
  const int row0 = (blockIdx.x * 4 + wave) * 16, col0 = blockIdx.y * 16;
  if (row0 >= R || col0 >= jb.nc) return;
  const float *Sr = reinterpret_cast<const float *>(jb.S);
  const long ldS = 2L * jb.ldS;
  const int ai = row0 + lane % 16, bj = col0 + lane % 16, kq = 4 * (lane / 16);
  floatx4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < jb.m; k0 += 16) {
    bf16x4 ah, bh, al, bl;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + kq + q;
      const float a = (ai < R && k < jb.m) ? Sr[ai + (long)k * ldS] : 0.f;
      const float b = (bj < jb.nc && k < jb.m) ? (float)jb.Om[k + (long)bj * jb.ldO] : 0.f;
      const unsigned ha = bf16_bits(a), hb = bf16_bits(b);
      ah[q] = (short)ha;
      bh[q] = (short)hb;
      if (SPLIT == 2) {
        al[q] = (short)bf16_bits(a - __uint_as_float(ha << 16));
        bl[q] = (short)bf16_bits(b - __uint_as_float(hb << 16));
      }
    }
    if (SPLIT == 2) {
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, bh, acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bl, acc, 0, 0, 0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bh, acc, 0, 0, 0);
  }
  float *Yr = reinterpret_cast<float *>(jb.Y);
  const long ldY = 2L * jb.ldY;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = row0 + kq + q, j = col0 + lane % 16;
    if (i < R && j < jb.nc) Yr[i + (long)j * ldY] = acc[q];
  }
}

// Block-wide argmax with one barrier: wavefront maxima go to LDS slot set
// `par` (alternate between calls), then every thread reduces all of them in
// the same order, so all threads agree without a second barrier.  Ties keep
// the smaller index.
template <int NT, typename T>
__device__ void block_argmax_1b(T &v, int &idx, T (*sv)[NT / 64], int (*si)[NT / 64], int par) {
  wave_argmax(v, idx);
  if ((threadIdx.x & 63) == 0) { sv[par][threadIdx.x / 64] = v; si[par][threadIdx.x / 64] = idx; }
  lds_barrier();
  v = sv[par][0];
  idx = si[par][0];
#pragma unroll
  for (int k = 1; k < NT / 64; ++k)
    if (sv[par][k] > v || (sv[par][k] == v && si[par][k] < idx)) { v = sv[par][k]; idx = si[par][k]; }
}

template <int NT, typename T>
__device__ void block_argmax(T &v, int &idx, T *sv, int *si) {
  for (int off = 32; off > 0; off >>= 1) {
    T ov = __shfl_xor(v, off);
    int oi = __shfl_xor(idx, off);
    if (ov > v || (ov == v && oi < idx)) { v = ov; idx = oi; }
  }
  int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) { sv[w] = v; si[w] = idx; }
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 1; k < NT / 64; ++k)
      if (sv[k] > sv[0] || (sv[k] == sv[0] && si[k] < si[0])) { sv[0] = sv[k]; si[0] = si[k]; }
  __syncthreads();
  v = sv[0];
  idx = si[0];
  __syncthreads();
}

// Small dense products inside one NT-thread workgroup: C (M x N) =
// op(A) B, or C = C0 - op(A) B, with op(A) = A (M x K, ld lda) or A^T (A
// stored K x M).  (NT/32 RU) x 128 output tiles, each thread an RU x 4 block
// (RU = 4 for complex64, 2 for complex128); K in chunks of 16 staged through
// LDS (As, Bs: 16 x 128 each).  Every thread of the workgroup must call it
// (it synchronises).
template <typename T, int NT, bool TA, bool SUB>
__device__ void wg_gemm(int M, int N, int K, const cplx<T> *__restrict__ A, long lda,
                        const cplx<T> *__restrict__ B, long ldb, const cplx<T> *C0, long ldc0,
                        cplx<T> *C, long ldc, cplx<T> (*As)[128], cplx<T> (*Bs)[128]) {
  constexpr int RU = sizeof(T) == sizeof(float) ? 4 : 2, TY = NT / 32, TM = TY * RU;
  static_assert((16 * TM) % NT == 0 && (16 * 128) % NT == 0, "staging loads per thread");
  const int tid = threadIdx.x, tx = tid % 32, ty = tid / 32;
  for (int i0 = 0; i0 < M; i0 += TM)
    for (int j0 = 0; j0 < N; j0 += 128) {
      cplx<T> acc[RU][4];
#pragma unroll
      for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[u][v] = czero<T>();
      for (int k0 = 0; k0 < K; k0 += 16) {
        // the chunk's global loads all go out before its LDS writes, so they
        // are not waited out one by one
        constexpr int kA = 16 * TM / NT, kB = 16 * 128 / NT;
        cplx<T> ra[kA], rb[kB];
#pragma unroll
        for (int u = 0; u < kA; ++u) {
          const int e = tid + NT * u;
          int kk, i;
          if (TA) { kk = e % 16; i = e / 16; }
          else { i = e % TM; kk = e / TM; }
          const int gi = i0 + i, gk = k0 + kk;
          ra[u] = czero<T>();
          if (gi < M && gk < K) ra[u] = TA ? A[gk + (long)gi * lda] : A[gi + (long)gk * lda];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int e = tid + NT * u;
          const int kk = e % 16, j = e / 16, gk = k0 + kk, gj = j0 + j;
          rb[u] = (gk < K && gj < N) ? B[gk + (long)gj * ldb] : czero<T>();
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < kA; ++u) {
          const int e = tid + NT * u;
          if (TA) As[e % 16][e / 16] = ra[u];
          else As[e / TM][e % TM] = ra[u];
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int e = tid + NT * u;
          Bs[e % 16][e / 16] = rb[u];
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 16; ++kk) {
          cplx<T> a[RU], b[4];
#pragma unroll
          for (int u = 0; u < RU; ++u) a[u] = As[kk][ty + TY * u];
#pragma unroll
          for (int v = 0; v < 4; ++v) b[v] = Bs[kk][tx + 32 * v];
#pragma unroll
          for (int u = 0; u < RU; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) cfma(acc[u][v], a[u], b[v]);
        }
      }
      if (SUB) {
        // C0 read completely before the first store of C
        cplx<T> c0v[RU][4];
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int gi = i0 + ty + TY * u, gj = j0 + tx + 32 * v;
            c0v[u][v] = (gi < M && gj < N) ? C0[gi + (long)gj * ldc0] : czero<T>();
          }
#pragma unroll
        for (int u = 0; u < RU; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = c0v[u][v] - acc[u][v];
      }
#pragma unroll
      for (int u = 0; u < RU; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int gi = i0 + ty + TY * u, gj = j0 + tx + 32 * v;
          if (gi < M && gj < N) C[gi + (long)gj * ldc] = acc[u][v];
        }
    }
  __syncthreads();
}

// Interpolation coefficients T = R11^-1 R12 of the pivoted QR, written as
// U(row, b) for every non-pivot row: R(b, row) = Rm[b + row * ldr] (pivot
// index b, original row), R11(b, a) = R(b, perm[a]).  kG lanes per column
// hold its kXU-strided entries in registers; back substitution over a, the
// new entry broadcast to the column's lanes by a shuffle.  rk <= kG * kXU.
// When R11 fits the LDS area Rs (kRsCap entries) it is staged there first,
// Rs[b + a * rk] = R11(b, a), so the back substitution reads no global
// memory.  Every thread of the workgroup calls it.
constexpr int kG = 32, kXU = 6, kRsCap = 2 * 16 * 128;
template <typename T, int NT, bool STAGED>
__device__ void interp_coeffs_t(int rows, int rk, const int *perm,
                                const cplx<T> *__restrict__ Rm, long ldr,
                                cplx<T> *__restrict__ U, const cplx<T> *Rs) {
  const int tid = threadIdx.x, sub = tid % kG, col = tid / kG;
  const int base = (tid % 64) & ~(kG - 1);
  const int nc = rows - rk;
  constexpr bool staged = STAGED;
  // R11(b, a); rows b >= rk (lanes past the rank) read as zero
  auto r11 = [&](int b, int a, long pa) -> cplx<T> {
    if constexpr (STAGED) return b < rk ? Rs[b + a * rk] : czero<T>();
    else return Rm[b + pa];
  };
  for (int c0 = 0; c0 < nc; c0 += NT / kG) {
    const int ci = c0 + col;
    const bool act = ci < nc;
    const long pr = act ? (long)perm[rk + ci] * ldr : 0;
    cplx<T> x[kXU];
#pragma unroll
    for (int u = 0; u < kXU; ++u) {
      const int b = sub + kG * u;
      x[u] = (act && b < rk) ? Rm[b + pr] : czero<T>();
    }
#pragma unroll
    for (int u = kXU - 1; u >= 0; --u) {
      for (int la = kG - 1; la >= 0; --la) {
        const int a = u * kG + la;
        if (a >= rk) continue;
        const long pa = staged ? 0 : (long)perm[a] * ldr;
        cplx<T> v = x[u] * cinv(r11(a, a, pa));
        v.re = __shfl(v.re, base + la);
        v.im = __shfl(v.im, base + la);
        if (sub == la) x[u] = v;
#pragma unroll
        for (int w = 0; w < u; ++w) cfms(x[w], r11(sub + kG * w, a, pa), v);
        if (sub < la) cfms(x[u], r11(sub + kG * u, a, pa), v);
      }
    }
    if (act) {
      const int row = perm[rk + ci];
#pragma unroll
      for (int u = 0; u < kXU; ++u) {
        const int b = sub + kG * u;
        if (b < rk) U[row + (long)b * rows] = x[u];
      }
    }
  }
}

template <typename T, int NT>
__device__ void interp_coeffs(int rows, int rk, const int *perm, const cplx<T> *__restrict__ Rm,
                              long ldr, cplx<T> *__restrict__ U, cplx<T> *Rs) {
  if (rk * rk <= kRsCap) {
    for (int e = threadIdx.x; e < rk * rk; e += NT) Rs[e] = Rm[e % rk + (long)perm[e / rk] * ldr];
    __syncthreads();
    interp_coeffs_t<T, NT, true>(rows, rk, perm, Rm, ldr, U, Rs);
  } else {
    interp_coeffs_t<T, NT, false>(rows, rk, perm, Rm, ldr, U, Rs);
  }
}

// perm[t..rows) = the rows i < rows with sel[i] == 0, ascending (rows <= NT):
// per-wavefront ballots and counts, one exclusive offset per wavefront.
// Every thread calls it; wcnt holds NT / 64 ints of LDS.
template <int NT>
__device__ void append_unselected(int rows, int t, const unsigned char *sel, int *perm,
                                  int *wcnt) {
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const bool un = tid < rows && !sel[tid];
  const unsigned long long m = __ballot(un);
  if (lane == 0) wcnt[wv] = __popcll(m);
  __syncthreads();
  int off = t;
  for (int k = 0; k < wv; ++k) off += wcnt[k];
  if (un) perm[off + __popcll(m & ((1ull << lane) - 1))] = tid;
  __syncthreads();
}

// ONEB: the register path takes one barrier per pivot (each wavefront's best
// row staged in LDS: in the product staging area for 256 threads, in a
// buffer of its own for 1024); else two (pivot row broadcast after the
// maxima).  The 1024-thread one-barrier variant is launched only for
// clusters that fit the register path, since its buffer costs occupancy.
template <typename T, int NT, bool ONEB, int RPT = CCfg<NT>::RPT, int RSEG = CCfg<NT>::RSEG>
__global__ __launch_bounds__(NT) void compress_level_kernel(
    const HssItem *__restrict__ items, const HssInstance *__restrict__ insts,
    const HssCluster *__restrict__ cls, cplx<T> *__restrict__ pool, int *__restrict__ ipool,
    int *__restrict__ rank, const cplx<T> *__restrict__ front, const cplx<T> *__restrict__ Yall,
    const double *__restrict__ Omall, cplx<T> *__restrict__ scratch, double id_tol) {
  __shared__ int I_loc[kMaxRows];
  __shared__ int perm[kMaxRows];
  __shared__ cplx<T> q[kMaxS];
  __shared__ T sv[NT / 64];
  __shared__ int si[NT / 64];
  __shared__ unsigned char sel[kMaxRows];
  __shared__ int s_rank;
  constexpr int kRT = CCfg<NT>::RT, kRS = NT / kRT, kRPT = RPT, kRSEG = RSEG;
  // register path: pivot rows (two-barrier steps, 1024 threads) or each
  // wavefront's best row (one-barrier steps, 256 threads; held in the
  // product staging area As, idle during the ID), and the wavefront maxima,
  // double-buffered by step parity
  __shared__ cplx<T> qb[2][kRT * kRSEG];
  constexpr int kOwnCand = (ONEB && NT != 256 && sizeof(T) == sizeof(float)) ? kRT * kRSEG : 1;
  static_assert(NT != 1024 || (kRS * kRPT <= kRegRows && kRT * kRSEG <= kRegCols),
                "host size classes must not exceed the register-path capacity");
  __shared__ cplx<T> own_cand[2][NT / 64][kOwnCand];
  __shared__ T sv2[2][NT / 64];
  __shared__ int si2[2][NT / 64];
  // product staging areas, contiguous so that the interpolation step can
  // hold R11 in both
  __shared__ cplx<T> ABs[2][16][128];
  auto &As = ABs[0];
  auto &Bs = ABs[1];
  const HssItem it = items[blockIdx.x];
  const HssInstance I = insts[it.inst];
  const int cg = I.cl_off + it.cl;
  const HssCluster C = cls[cg];
  const int tid = threadIdx.x;
  const int s = I.s;
  cplx<T> *P = pool + I.pool;
  int *IP = ipool + I.ipool;
  const cplx<T> *S = front + I.soff;
  const long ldS = I.ldS;
  const cplx<T> *Y = Yall + I.yoff;
  const double *Om = Omall + I.ooff;
  const long ldY = I.ldY, ldO = I.m;
  cplx<T> *Sloc = scratch + I.woff + C.W;
  const int rcap = C.rows_cap;
  cplx<T> *Wm = Sloc + (long)rcap * s;
  cplx<T> *Oloc = Wm + (long)rcap * s;
  cplx<T> *Rm = Oloc + (long)rcap * s;           // k_cap x rows_cap (by original row)

  int rows;
  const bool leaf = C.left < 0;
  if (leaf) {
    rows = C.size;
    for (int i = tid; i < rows; i += NT) I_loc[i] = C.start + i;
    __syncthreads();
    cplx<T> *D = P + C.D;
    // D = S(I, I) and Om_loc = Om(I, :) (the real sketch as complex), copied
    // in batches of loads ahead of their stores; then S_loc = Y(I, :) - D Om_loc
    // (an instance whose operator is not formed has D in the pool already)
    for (int e0 = I.pre ? rows * rows : tid; e0 < rows * rows; e0 += NT * 8) {
      cplx<T> v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + NT * u;
        v[u] = e < rows * rows ? S[(C.start + e % rows) + (long)(C.start + e / rows) * ldS]
                               : czero<T>();
      }
#pragma unroll
      for (int u = 0; u < 8; ++u)
        if (e0 + NT * u < rows * rows) D[e0 + NT * u] = v[u];
    }
    for (int e0 = tid; e0 < rows * s; e0 += NT * 8) {
      double w[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + NT * u;
        w[u] = e < rows * s ? Om[(C.start + e % rows) + (long)(e / rows) * ldO] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int e = e0 + NT * u;
        if (e < rows * s) Oloc[e % rows + (long)(e / rows) * rcap] = mk((T)w[u], (T)0);
      }
    }
    __syncthreads();
    wg_gemm<T, NT, false, true>(rows, s, rows, D, rows, Oloc, rcap, Y + C.start, ldY, Sloc, rcap,
                                As, Bs);
  } else {
    const HssCluster L = cls[I.cl_off + C.left], R = cls[I.cl_off + C.right];
    const int kl = rank[I.cl_off + C.left], kr = rank[I.cl_off + C.right];
    rows = kl + kr;
    const int *skl = IP + L.sk, *skr = IP + R.sk;
    for (int i = tid; i < rows; i += NT) I_loc[i] = i < kl ? skl[i] : skr[i - kl];
    cplx<T> *B12 = P + C.B12, *B21 = P + C.B21;
    // B12 = S(sk_l, sk_r), B21 = S(sk_r, sk_l): skeleton indices, then the
    // entries, then the stores, eight elements per lane at a time
    auto gather = [&](cplx<T> *Bd, const int *ra, const int *cb, int na, int nb) {
      for (int e0 = tid; e0 < na * nb; e0 += NT * 8) {
        int ia[8], ib[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + NT * u;
          const bool ok = e < na * nb;
          ia[u] = ok ? ra[e % na] : 0;
          ib[u] = ok ? cb[e / na] : 0;
        }
        cplx<T> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          v[u] = e0 + NT * u < na * nb ? S[ia[u] + (long)ib[u] * ldS] : czero<T>();
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (e0 + NT * u < na * nb) Bd[e0 + NT * u] = v[u];
      }
    };
    if (!I.pre) {
      gather(B12, skl, skr, kl, kr);
      gather(B21, skr, skl, kr, kl);
    }
    __syncthreads();
    if (it.cl != 0) {
      const cplx<T> *Srl = P + L.Sr, *Srr = P + R.Sr, *Oml = P + L.Om, *Omr = P + R.Om;
      for (int e0 = tid; e0 < rows * s; e0 += NT * 8) {
        cplx<T> v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + NT * u, i = e % rows, j = e / rows;
          v[u] = e >= rows * s ? czero<T>()
                 : i < kl      ? Oml[i + (long)j * kl]
                               : Omr[(i - kl) + (long)j * kr];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int e = e0 + NT * u;
          if (e < rows * s) Oloc[e % rows + (long)(e / rows) * rcap] = v[u];
        }
      }
      // S_loc = [Sr_l - B12 Om_r ; Sr_r - B21 Om_l]
      wg_gemm<T, NT, false, true>(kl, s, kr, B12, kl, Omr, kr, Srl, kl, Sloc, rcap, As, Bs);
      wg_gemm<T, NT, false, true>(kr, s, kl, B21, kr, Oml, kl, Srr, kr, Sloc + kl, rcap, As, Bs);
    }
  }
  __syncthreads();
  if (it.cl == 0) {                 // root: generators B (or D) only
    if (tid == 0) rank[cg] = 0;
    return;
  }

  // ---- interpolative decomposition of S_loc (rows x s)
  int kmax = I.k < rows ? I.k : rows;
  kmax = kmax < s ? kmax : s;
  kmax = kmax < C.k_cap ? kmax : C.k_cap;
  T first = (T)0;
  int t = 0;
  bool reg_done = false;
  if constexpr (sizeof(T) == sizeof(float)) {
    if (rows <= kRS * kRPT && s <= kRT * kRSEG) {
      // Register-resident pivoted Gram-Schmidt: each row stays with its 8
      // lanes for the whole decomposition; pivots are marked, not moved.
      const int sub = tid % kRT, slot = tid / kRT;
      cplx<T> w[kRPT][kRSEG];
#pragma unroll
      for (int r = 0; r < kRPT; ++r) {
        const int row = slot + kRS * r;
#pragma unroll
        for (int c = 0; c < kRSEG; ++c) {
          const int j = sub + kRT * c;
          w[r][c] = (row < rows && j < s) ? Sloc[row + (long)j * rcap] : czero<T>();
        }
      }
      if constexpr (ONEB) {
      constexpr int kC = kRT * kRSEG;
      static_assert(NT != 256 || 2 * (NT / 64) * kC <= 16 * 128,
                    "candidate rows exceed the staging area");
      static_assert(NT == 256 || kOwnCand == kC, "one-barrier steps need the candidate buffer");
      cplx<T>(*cand)[NT / 64][kC] =
          NT == 256 ? reinterpret_cast<cplx<T>(*)[NT / 64][kC]>(&As[0][0])
                    : reinterpret_cast<cplx<T>(*)[NT / 64][kC]>(&own_cand[0][0][0]);
      // one barrier per pivot: every wavefront stages its best row (owner
      // lanes) and its maximum in LDS before the barrier, so after it all
      // threads pick the winner and read the pivot row without a second one;
      // LDS buffers alternate between steps, picked rows are register flags
      bool pk[kRPT];
#pragma unroll
      for (int r = 0; r < kRPT; ++r) pk[r] = false;
      const int wv = tid / 64;
      __syncthreads();
      for (; t < kmax; ++t) {
        const int par = t & 1;
        T best = (T)-1;
        int bi = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < kRPT; ++r) {
          if (kRS * r >= rows) continue;
          const int row = slot + kRS * r;
          T nrm = 0;
#pragma unroll
          for (int c = 0; c < kRSEG; ++c) nrm += abs2(w[r][c]);
          nrm = group_sum<kRT>(nrm);
          if (row < rows && !pk[r] && (nrm > best || (nrm == best && row < bi))) {
            best = nrm;
            bi = row;
          }
        }
        wave_argmax(best, bi);
        if (bi != 0x7fffffff && slot == bi % kRS) {
          const int ro = bi / kRS;
#pragma unroll
          for (int r = 0; r < kRPT; ++r)
            if (r == ro) {
#pragma unroll
              for (int c = 0; c < kRSEG; ++c) cand[par][wv][sub + kRT * c] = w[r][c];
            }
        }
        if ((tid & 63) == 0) { sv2[par][wv] = best; si2[par][wv] = bi; }
        lds_barrier();
        // all wavefront maxima loaded before the first comparison
        T vv[NT / 64];
        int iv[NT / 64];
#pragma unroll
        for (int k = 0; k < NT / 64; ++k) {
          vv[k] = sv2[par][k];
          iv[k] = si2[par][k];
        }
        T v = vv[0];
        int vi = iv[0], ww = 0;
#pragma unroll
        for (int k = 1; k < NT / 64; ++k)
          if (vv[k] > v || (vv[k] == v && iv[k] < vi)) {
            v = vv[k];
            vi = iv[k];
            ww = k;
          }
        const T pn = sqrt(v);
        if (t == 0) first = pn;
        if (!(pn > (T)0) || pn <= (T)id_tol * first) break;
        const T inv = (T)1 / pn;
        // pivot row p = cand * pn: q = p / pn is applied as inv * cand
        const cplx<T> *qr = cand[par][ww];
        if (slot == vi % kRS) {
          const int ro = vi / kRS;
#pragma unroll
          for (int r = 0; r < kRPT; ++r)
            if (r == ro) pk[r] = true;
        }
        if (tid == 0) {
          perm[t] = vi;
          Rm[t + (long)vi * C.k_cap] = mk(pn, (T)0);
        }
        // this lane's entries of the pivot row, loaded once per step
        cplx<T> qv[kRSEG];
#pragma unroll
        for (int c = 0; c < kRSEG; ++c) qv[c] = qr[sub + kRT * c];
#pragma unroll
        for (int r = 0; r < kRPT; ++r) {
          if (kRS * r >= rows) continue;
          const int row = slot + kRS * r;
          const bool act = row < rows && !pk[r];
          cplx<T> rr = czero<T>();
          for (int pass = 0; pass < kPasses; ++pass) {
            cplx<T> d = czero<T>();
#pragma unroll
            for (int c = 0; c < kRSEG; ++c) cfma(d, conj(qv[c]), w[r][c]);
            d.re = inv * group_sum<kRT>(d.re);
            d.im = inv * group_sum<kRT>(d.im);
            // no lane guards: entries past s are zero in w and in the
            // candidate rows, rows past the block stay zero, and a picked
            // row (projected onto itself) is never read again
            const cplx<T> dq = inv * d;
#pragma unroll
            for (int c = 0; c < kRSEG; ++c) cfms(w[r][c], dq, qv[c]);
            rr = rr + d;
          }
          if (act && sub == 0) Rm[t + (long)row * C.k_cap] = rr;
        }
      }
      __syncthreads();
      // the unselected rows follow the pivots in ascending order
      for (int i = tid; i < rows; i += NT) sel[i] = 0;
      __syncthreads();
      for (int a = tid; a < t; a += NT) sel[perm[a]] = 1;
      __syncthreads();
      append_unselected<NT>(rows, t, sel, perm, si);
      } else {
      for (int i = tid; i < rows; i += NT) sel[i] = 0;
      __syncthreads();
      // two barriers per pivot: after the wavefront maxima and after the
      // pivot row; LDS buffers alternate between steps
      for (; t < kmax; ++t) {
        const int par = t & 1;
        cplx<T> *q = qb[par];
        T best = (T)-1;
        int bi = 0x7fffffff;
#pragma unroll
        for (int r = 0; r < kRPT; ++r) {
          if (kRS * r >= rows) continue;
          const int row = slot + kRS * r;
          T nrm = 0;
#pragma unroll
          for (int c = 0; c < kRSEG; ++c) {
            if (kRT * c >= s) continue;
            nrm += abs2(w[r][c]);
          }
          nrm = group_sum<kRT>(nrm);
          if (row < rows && !sel[row] && (nrm > best || (nrm == best && row < bi))) {
            best = nrm;
            bi = row;
          }
        }
        block_argmax_1b<NT>(best, bi, sv2, si2, par);
        const T pn = sqrt(best);
        if (t == 0) first = pn;
        if (!(pn > (T)0) || pn <= (T)id_tol * first) break;
        const T inv = (T)1 / pn;
        if (slot == bi % kRS) {
          const int ro = bi / kRS;
#pragma unroll
          for (int r = 0; r < kRPT; ++r)
            if (r == ro) {
#pragma unroll
              for (int c = 0; c < kRSEG; ++c) {
                if (kRT * c >= s) continue;
                const int j = sub + kRT * c;
                if (j < s) q[j] = inv * w[r][c];
              }
            }
        }
        if (tid == 0) {
          perm[t] = bi;
          sel[bi] = 1;
          Rm[t + (long)bi * C.k_cap] = mk(pn, (T)0);
        }
        // LDS-only barrier: the R coefficients go to global memory and are
        // read after the loop's closing full barrier
        lds_barrier();
#pragma unroll
        for (int r = 0; r < kRPT; ++r) {
          if (kRS * r >= rows) continue;
          const int row = slot + kRS * r;
          const bool act = row < rows && !sel[row];
          cplx<T> rr = czero<T>();
          for (int pass = 0; pass < kPasses; ++pass) {
            cplx<T> d = czero<T>();
#pragma unroll
            for (int c = 0; c < kRSEG; ++c) {
              if (kRT * c >= s) continue;
              const int j = sub + kRT * c;
              if (j < s) cfma(d, conj(q[j]), w[r][c]);
            }
            d.re = group_sum<kRT>(d.re);
            d.im = group_sum<kRT>(d.im);
            if (act) {
#pragma unroll
              for (int c = 0; c < kRSEG; ++c) {
                if (kRT * c >= s) continue;
                const int j = sub + kRT * c;
                if (j < s) cfms(w[r][c], d, q[j]);
              }
            }
            rr = rr + d;
          }
          if (act && sub == 0) Rm[t + (long)row * C.k_cap] = rr;
        }
      }
      __syncthreads();
      // the unselected rows follow the pivots in ascending order
      append_unselected<NT>(rows, t, sel, perm, si);
      }
      reg_done = true;
    }
  }
  if (!reg_done) {
  // copies and row sweeps below take kGB elements per lane per batch, all
  // loads of a batch before its stores: the pointers may alias, so a store
  // between two loads would make each load wait for the previous one
  constexpr int kGB = 8;
  for (int e0 = tid; e0 < rows * s; e0 += NT * kGB) {
    cplx<T> v[kGB];
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int e = e0 + NT * u;
      v[u] = e < rows * s ? Sloc[e % rows + (long)(e / rows) * rcap] : czero<T>();
    }
#pragma unroll
    for (int u = 0; u < kGB; ++u) {
      const int e = e0 + NT * u;
      if (e < rows * s) Wm[e % rows + (long)(e / rows) * rcap] = v[u];
    }
  }
  for (int i = tid; i < rows; i += NT) perm[i] = i;
  __syncthreads();
  const int sub = tid % kTPR, slot = tid / kTPR, nslot = NT / kTPR;
  // residual row norms (kTPR lanes per row, reduced by shuffles), indexed by
  // original row; after the first they come from the projection pass, which
  // sums the updated entries, so each pivot reads the block twice, not three
  // times.  They live in the product staging area As, idle during the ID
  // (16 x 128 complex >= kMaxRows reals).
  T *rnorm = reinterpret_cast<T *>(&As[0][0]);
  for (int pp0 = 0; pp0 < rows; pp0 += nslot) {
    const int pp = pp0 + slot;
    T nrm = 0;
    if (pp < rows)
      for (int j0 = sub; j0 < s; j0 += kTPR * kGB) {
        cplx<T> v[kGB];
#pragma unroll
        for (int u = 0; u < kGB; ++u) {
          const int j = j0 + kTPR * u;
          v[u] = j < s ? Wm[pp + (long)j * rcap] : czero<T>();
        }
#pragma unroll
        for (int u = 0; u < kGB; ++u)
          if (j0 + kTPR * u < s) nrm += abs2(v[u]);
      }
    for (int o = 1; o < kTPR; o <<= 1) nrm += __shfl_xor(nrm, o);
    if (pp < rows && sub == 0) rnorm[pp] = nrm;
  }
  __syncthreads();
  for (; t < kmax; ++t) {
    T best = (T)-1;
    int bi = 0x7fffffff;
    for (int pp = t + tid; pp < rows; pp += NT) {
      const T nrm = rnorm[perm[pp]];
      if (nrm > best || (nrm == best && pp < bi)) { best = nrm; bi = pp; }
    }
    block_argmax<NT>(best, bi, sv, si);
    T pn = sqrt(best);
    if (t == 0) first = pn;
    if (!(pn > (T)0) || pn <= (T)id_tol * first) break;
    if (tid == 0 && bi != t) {
      int a = perm[t];
      perm[t] = perm[bi];
      perm[bi] = a;
    }
    __syncthreads();
    const int prow = perm[t];
    T inv = (T)1 / pn;
    for (int j = tid; j < s; j += NT) q[j] = inv * Wm[prow + (long)j * rcap];
    if (tid == 0) Rm[t + (long)prow * C.k_cap] = mk(pn, (T)0);
    __syncthreads();
    for (int pp0 = t + 1; pp0 < rows; pp0 += nslot) {
      const int pp = pp0 + slot;
      const bool act = pp < rows;
      const int row = act ? perm[pp] : 0;
      cplx<T> rr = czero<T>();
      for (int pass = 0; pass < kPasses; ++pass) {
        cplx<T> d = czero<T>();
        if (act)
          for (int j0 = sub; j0 < s; j0 += kTPR * kGB) {
            cplx<T> v[kGB];
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
              const int j = j0 + kTPR * u;
              v[u] = j < s ? Wm[row + (long)j * rcap] : czero<T>();
            }
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
              const int j = j0 + kTPR * u;
              if (j < s) cfma(d, conj(q[j]), v[u]);
            }
          }
        for (int o = 1; o < kTPR; o <<= 1) {
          d.re += __shfl_xor(d.re, o);
          d.im += __shfl_xor(d.im, o);
        }
        T nrm = 0;
        if (act)
          for (int j0 = sub; j0 < s; j0 += kTPR * kGB) {
            cplx<T> v[kGB];
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
              const int j = j0 + kTPR * u;
              v[u] = j < s ? Wm[row + (long)j * rcap] : czero<T>();
            }
#pragma unroll
            for (int u = 0; u < kGB; ++u) {
              const int j = j0 + kTPR * u;
              if (j < s) {
                cfms(v[u], d, q[j]);
                Wm[row + (long)j * rcap] = v[u];
                nrm += abs2(v[u]);
              }
            }
          }
        for (int o = 1; o < kTPR; o <<= 1) nrm += __shfl_xor(nrm, o);
        if (act && sub == 0) rnorm[row] = nrm;
        rr = rr + d;
      }
      if (act && sub == 0) Rm[t + (long)row * C.k_cap] = rr;
    }
    __syncthreads();
  }
  }  // global-memory pivoted QR
  const int rk = t;
  if (tid == 0) s_rank = rk;
  __syncthreads();

  // U (rows x rk): identity rows at the skeleton, T^T = (R11^-1 R12)^T elsewhere
  cplx<T> *U = P + C.U;
  for (int e = tid; e < rows * rk; e += NT) U[e] = czero<T>();
  __syncthreads();
  for (int a = tid; a < rk; a += NT) U[perm[a] + (long)a * rows] = mk((T)1, (T)0);
  if (rk <= kG * kXU) {
    interp_coeffs<T, NT>(rows, rk, perm, Rm, C.k_cap, U, &ABs[0][0][0]);
  } else {
    for (int c2 = tid; c2 < rows - rk; c2 += NT) {
      int row = perm[rk + c2];
      // back substitution, solution written straight into U(row, :)
      for (int a = rk - 1; a >= 0; --a) {
        cplx<T> v = Rm[a + (long)row * C.k_cap];
        for (int b = a + 1; b < rk; ++b)
          cfms(v, Rm[a + (long)perm[b] * C.k_cap], U[row + (long)b * rows]);
        U[row + (long)a * rows] = v * cinv(Rm[a + (long)perm[a] * C.k_cap]);
      }
    }
  }
  __syncthreads();
  int *sk = IP + C.sk;
  for (int a = tid; a < rk; a += NT) sk[a] = I_loc[perm[a]];
  cplx<T> *Omc = P + C.Om, *Src = P + C.Sr;
  for (int e0 = tid; e0 < rk * s; e0 += NT * 8) {
    cplx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + NT * u;
      v[u] = e < rk * s ? Sloc[perm[e % rk] + (long)(e / rk) * rcap] : czero<T>();
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + NT * u;
      if (e < rk * s) Src[e % rk + (long)(e / rk) * rk] = v[u];
    }
  }
  // Om_c = U^T Om_loc
  wg_gemm<T, NT, true, false>(rk, s, rows, U, rows, Oloc, rcap, nullptr, 0, Omc, rk, As, Bs);
  if (tid == 0) rank[cg] = rk;
}

// ---------------------------------------------------------------- matvec
// Telescoping product out = H X (eqs. 2.5-2.6) for a batch of jobs (one
// instance, up to kXC columns each), one launch per tree level and phase:
// up-sweep xh_c = U_c^T [X rows | children's xh], sibling couplings
// yh_l = B12 xh_r, yh_r = B21 xh_l, down-sweep [yh_l; yh_r] += U_c yh_c, and
// the leaves out = D X + U yh.  Every (job, cluster) pair is one workgroup.
constexpr int kMT = 256;

// out(M x nc) = op(A) X for one workgroup: A(m, k) from aload, X(k, j) from
// xin, results handed to put(m, j, value).  64 output rows at a time, K in
// chunks of 32; A and X tiles staged through LDS.  TA selects the loading
// order (k fastest when A is stored K x M).
template <typename T, bool TA, typename AF, typename XF, typename PF>
__device__ void mv_block(int M, int K, int nc, AF aload, XF xin, PF put, cplx<T> (*As)[65],
                         cplx<T> (*Xs)[kXC]) {
  static_assert((32 * 64) % kMT == 0 && (32 * kXC) % kMT == 0, "staging loads per thread");
  const int tid = threadIdx.x, jj = tid % kXC, ab = tid / kXC;
  for (int a0 = 0; a0 < M; a0 += 64) {
    cplx<T> acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = czero<T>();
    for (int i0 = 0; i0 < K; i0 += 32) {
      // the chunk's global loads all go out before its LDS writes
      constexpr int kA = 32 * 64 / kMT, kX = 32 * kXC / kMT;
      cplx<T> ra[kA], rx[kX];
#pragma unroll
      for (int u = 0; u < kA; ++u) {
        const int e = tid + kMT * u;
        int ii, aa;
        if (TA) { ii = e % 32; aa = e / 32; }
        else { aa = e % 64; ii = e / 64; }
        const int gi = i0 + ii, ga = a0 + aa;
        ra[u] = (gi < K && ga < M) ? aload(ga, gi) : czero<T>();
      }
#pragma unroll
      for (int u = 0; u < kX; ++u) {
        const int e = tid + kMT * u;
        const int ii = e % 32, j = e / 32, gi = i0 + ii;
        rx[u] = (gi < K && j < nc) ? xin(gi, j) : czero<T>();
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kA; ++u) {
        const int e = tid + kMT * u;
        if (TA) As[e % 32][e / 32] = ra[u];
        else As[e / 64][e % 64] = ra[u];
      }
#pragma unroll
      for (int u = 0; u < kX; ++u) {
        const int e = tid + kMT * u;
        Xs[e % 32][e / 32] = rx[u];
      }
      __syncthreads();
#pragma unroll 8
      for (int ii = 0; ii < 32; ++ii) {
        const cplx<T> x = Xs[ii][jj];
#pragma unroll
        for (int u = 0; u < 4; ++u) cfma(acc[u], As[ii][ab + 16 * u], x);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int a = a0 + ab + 16 * u;
      if (a < M && jj < nc) put(a, jj, acc[u]);
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kMT) void mv_up_kernel(int lev, const MatvecJob<T> *__restrict__ jobs,
                                                    const HssInstance *__restrict__ insts,
                                                    const HssCluster *__restrict__ cls,
                                                    const cplx<T> *__restrict__ pool,
                                                    const int *__restrict__ rank,
                                                    cplx<T> *__restrict__ scratch) {
  __shared__ cplx<T> As[32][65];
  __shared__ cplx<T> Xs[32][kXC];
  const MatvecJob<T> jb = jobs[blockIdx.x];
  const HssInstance &I = insts[jb.inst];
  if (lev >= I.nlev) return;
  const int c = I.lev_off[lev] + blockIdx.y;
  if (c >= I.lev_off[lev + 1]) return;
  const HssCluster cc = cls[I.cl_off + c];
  const int k = rank[I.cl_off + c], nc = jb.nc;
  cplx<T> *W = scratch + jb.woff;
  cplx<T> *xh = W + cc.XH;
  // identity columns outside a cluster make its up-sweep vector zero; it is
  // not stored, its readers (the parent here, mv_couple_kernel) test for it
  auto outside = [&](const HssCluster &h) {
    return !jb.X && (h.start + h.size <= jb.c0 || h.start >= jb.c0 + nc);
  };
  if (outside(cc)) return;
  const cplx<T> *U = pool + I.pool + cc.U;
  auto put = [&](int a, int j, cplx<T> v) { xh[a + (long)j * k] = v; };
  if (cc.left < 0) {
    const int rows = cc.size;
    auto aload = [&](int a, int i) { return U[i + (long)a * rows]; };
    auto xin = [&](int i, int j) {
      const int gi = cc.start + i;
      const T v = jb.X ? (T)jb.X[gi + (long)j * jb.ldX] : (T)(gi == jb.c0 + j ? 1 : 0);
      return mk(v, (T)0);
    };
    mv_block<T, true>(k, rows, nc, aload, xin, put, As, Xs);
  } else {
    const int kl = rank[I.cl_off + cc.left], kr = rank[I.cl_off + cc.right], rows = kl + kr;
    const HssCluster L = cls[I.cl_off + cc.left], R = cls[I.cl_off + cc.right];
    const bool lz = outside(L), rz = outside(R);
    const cplx<T> *xl = W + L.XH, *xr = W + R.XH;
    auto aload = [&](int a, int i) { return U[i + (long)a * rows]; };
    auto xin = [&](int i, int j) {
      if (i < kl) return lz ? czero<T>() : xl[i + (long)j * kl];
      return rz ? czero<T>() : xr[(i - kl) + (long)j * kr];
    };
    mv_block<T, true>(k, rows, nc, aload, xin, put, As, Xs);
  }
}

template <typename T>
__global__ __launch_bounds__(kMT) void mv_couple_kernel(const MatvecJob<T> *__restrict__ jobs,
                                                        const HssInstance *__restrict__ insts,
                                                        const HssCluster *__restrict__ cls,
                                                        const cplx<T> *__restrict__ pool,
                                                        const int *__restrict__ rank,
                                                        cplx<T> *__restrict__ scratch) {
  __shared__ cplx<T> As[32][65];
  __shared__ cplx<T> Xs[32][kXC];
  const MatvecJob<T> jb = jobs[blockIdx.x];
  const HssInstance &I = insts[jb.inst];
  const int c = blockIdx.y;
  if (c >= I.ncl) return;
  const HssCluster cc = cls[I.cl_off + c];
  if (cc.left < 0) return;
  const int kl = rank[I.cl_off + cc.left], kr = rank[I.cl_off + cc.right], nc = jb.nc;
  const HssCluster L = cls[I.cl_off + cc.left], R = cls[I.cl_off + cc.right];
  const cplx<T> *B12 = pool + I.pool + cc.B12, *B21 = pool + I.pool + cc.B21;
  cplx<T> *W = scratch + jb.woff;
  cplx<T> *yl = W + L.XH + (long)L.k_cap * kXC, *yr = W + R.XH + (long)R.k_cap * kXC;
  const cplx<T> *xl = W + L.XH, *xr = W + R.XH;
  // identity columns outside a child give it a zero up-sweep vector (see
  // mv_up_kernel), so the sibling's coupling product is zero
  auto outside = [&](const HssCluster &h) {
    return !jb.X && (h.start + h.size <= jb.c0 || h.start >= jb.c0 + nc);
  };
  if (outside(R)) {
    for (int e = threadIdx.x; e < kl * nc; e += kMT) yl[e] = czero<T>();
  } else {
    mv_block<T, false>(
        kl, kr, nc, [&](int a, int b) { return B12[a + (long)b * kl]; },
        [&](int b, int j) { return xr[b + (long)j * kr]; },
        [&](int a, int j, cplx<T> v) { yl[a + (long)j * kl] = v; }, As, Xs);
  }
  if (outside(L)) {
    for (int e = threadIdx.x; e < kr * nc; e += kMT) yr[e] = czero<T>();
  } else {
    mv_block<T, false>(
        kr, kl, nc, [&](int a, int b) { return B21[a + (long)b * kr]; },
        [&](int b, int j) { return xl[b + (long)j * kl]; },
        [&](int a, int j, cplx<T> v) { yr[a + (long)j * kr] = v; }, As, Xs);
  }
}

template <typename T>
__global__ __launch_bounds__(kMT) void mv_down_kernel(int lev, const MatvecJob<T> *__restrict__ jobs,
                                                      const HssInstance *__restrict__ insts,
                                                      const HssCluster *__restrict__ cls,
                                                      const cplx<T> *__restrict__ pool,
                                                      const int *__restrict__ rank,
                                                      cplx<T> *__restrict__ scratch) {
  __shared__ cplx<T> As[32][65];
  __shared__ cplx<T> Xs[32][kXC];
  const MatvecJob<T> jb = jobs[blockIdx.x];
  const HssInstance &I = insts[jb.inst];
  if (lev >= I.nlev) return;
  const int c = I.lev_off[lev] + blockIdx.y;
  if (c >= I.lev_off[lev + 1]) return;
  const HssCluster cc = cls[I.cl_off + c];
  if (cc.left < 0) return;
  const int k = rank[I.cl_off + c], kl = rank[I.cl_off + cc.left],
            kr = rank[I.cl_off + cc.right], rows = kl + kr, nc = jb.nc;
  const cplx<T> *U = pool + I.pool + cc.U;
  cplx<T> *W = scratch + jb.woff;
  const cplx<T> *yh = W + cc.XH + (long)cc.k_cap * kXC;
  const HssCluster L = cls[I.cl_off + cc.left], R = cls[I.cl_off + cc.right];
  cplx<T> *yl = W + L.XH + (long)L.k_cap * kXC, *yr = W + R.XH + (long)R.k_cap * kXC;
  mv_block<T, false>(
      rows, k, nc, [&](int i, int a) { return U[i + (long)a * rows]; },
      [&](int a, int j) { return yh[a + (long)j * k]; },
      [&](int i, int j, cplx<T> v) {
        if (i < kl) yl[i + (long)j * kl] = yl[i + (long)j * kl] + v;
        else yr[(i - kl) + (long)j * kr] = yr[(i - kl) + (long)j * kr] + v;
      },
      As, Xs);
}

template <typename T>
__global__ __launch_bounds__(kMT) void mv_leaf_kernel(const MatvecJob<T> *__restrict__ jobs,
                                                      const HssInstance *__restrict__ insts,
                                                      const HssCluster *__restrict__ cls,
                                                      const cplx<T> *__restrict__ pool,
                                                      const int *__restrict__ rank,
                                                      cplx<T> *__restrict__ scratch) {
  __shared__ cplx<T> As[32][65];
  __shared__ cplx<T> Xs[32][kXC];
  __shared__ double red[2][kMT];
  const MatvecJob<T> jb = jobs[blockIdx.x];
  const HssInstance &I = insts[jb.inst];
  const int c = blockIdx.y;
  if (c >= I.ncl) return;
  const HssCluster cc = cls[I.cl_off + c];
  if (cc.left >= 0) return;
  const int k = c == 0 ? 0 : rank[I.cl_off + c], rows = cc.size, nc = jb.nc;
  const cplx<T> *U = pool + I.pool + cc.U, *D = pool + I.pool + cc.D;
  const cplx<T> *yh = scratch + jb.woff + cc.XH + (long)cc.k_cap * kXC;
  double e2 = 0.0, r2 = 0.0;
  // out = [D U] [X rows; yh]; identity columns outside the leaf make its X
  // rows zero, and the product starts at the U block (lo = rows)
  const int lo = (!jb.X && (cc.start + rows <= jb.c0 || cc.start >= jb.c0 + nc)) ? rows : 0;
  mv_block<T, false>(
      rows, rows + k - lo, nc,
      [&](int i, int l) {
        l += lo;
        return l < rows ? D[i + (long)l * rows] : U[i + (long)(l - rows) * rows];
      },
      [&](int l, int j) {
        l += lo;
        if (l >= rows) return yh[(l - rows) + (long)j * k];
        const int gl = cc.start + l;
        const T v = jb.X ? (T)jb.X[gl + (long)j * jb.ldX] : (T)(gl == jb.c0 + j ? 1 : 0);
        return mk(v, (T)0);
      },
      [&](int i, int j, cplx<T> v) {
        const long gi = cc.start + i;
        if (jb.Yref) {
          const cplx<T> y = jb.Yref[gi + (long)j * jb.ldR];
          e2 += (double)abs2(y - v);
          r2 += (double)abs2(y);
        } else {
          jb.out[gi + (long)j * jb.ldO] = v;
        }
      },
      As, Xs);
  if (jb.Yref) {
    const int tid = threadIdx.x;
    red[0][tid] = e2;
    red[1][tid] = r2;
    __syncthreads();
    for (int w = kMT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        red[0][tid] += red[0][tid + w];
        red[1][tid] += red[1][tid + w];
      }
      __syncthreads();
    }
    if (tid == 0) {
      atomicAdd(jb.err2, red[0][0]);
      atomicAdd(jb.ref2, red[1][0]);
    }
  }
}

}  // namespace

void launch_gaussian(int count, const GaussJob *jobs, uint32_t seed, int max_m, int max_nc,
                     hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_nc <= 0) return;
  hipLaunchKernelGGL(gaussian_kernel, dim3(ceil_div(max_m, 256), max_nc, count), dim3(256), 0,
                     st, jobs, seed);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_sample(int count, const SampleJob<T> *jobs, int max_m, int max_nc, hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_nc <= 0) return;
  hipLaunchKernelGGL(sample_kernel<T>, dim3(ceil_div(2L * max_m, 64), ceil_div(max_nc, 64), count),
                     dim3(256), 0, st, jobs);
  HSSX_HIP(hipGetLastError());
}

void launch_sample_bf16(int count, const SampleJob<float> *jobs, int max_m, int max_nc, int split,
                        hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_nc <= 0) return;
  const dim3 grid(ceil_div(2L * max_m, 64), ceil_div(max_nc, 16), count);
  if (split == 2) hipLaunchKernelGGL(sample_bf16_kernel<2>, grid, dim3(256), 0, st, jobs);
  else hipLaunchKernelGGL(sample_bf16_kernel<1>, grid, dim3(256), 0, st, jobs);
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_compress_level(int count, const HssItem *items, const HssInstance *inst,
                           const HssCluster *cl, cplx<T> *pool, int *ipool, int *rank,
                           const cplx<T> *front, const cplx<T> *Y, const double *Om,
                           cplx<T> *scratch, double id_tol, int size_class, hipStream_t st) {
  if (count <= 0) return;
  constexpr bool kF32 = sizeof(T) == sizeof(float);
  // the register path exists for complex64 only: complex128 takes the
  // general kernels for every class
  if (!kF32) size_class = size_class == kCls256S64 || size_class == kCls256S128 ? kCls256
                          : size_class == kCls1024R128S64 || size_class == kCls1024R128S128
                              ? kCls1024
                              : size_class;
#define HSSX_CL(NT, ONEB, ...)                                                              \
  hipLaunchKernelGGL((compress_level_kernel<T, NT, ONEB, ##__VA_ARGS__>), dim3(count), dim3(NT), \
                     0, st, items, inst, cl, pool, ipool, rank, front, Y, Om, scratch, id_tol)
  switch (size_class) {
    case kCls256: HSSX_CL(256, kF32); break;
    case kCls1024: if (kF32) HSSX_CL(1024, kF32); else HSSX_CL(1024, false); break;
    case kCls256S64: if constexpr (kF32) HSSX_CL(256, true, 2, 8); break;
    case kCls256S128: if constexpr (kF32) HSSX_CL(256, true, 2, 16); break;
    case kCls1024R128S64: if constexpr (kF32) HSSX_CL(1024, true, 2, 4); break;
    case kCls1024R128S128: if constexpr (kF32) HSSX_CL(1024, true, 2, 8); break;
    default: HSSX_CL(1024, false); break;
  }
#undef HSSX_CL
  HSSX_HIP(hipGetLastError());
}

template <typename T>
void launch_hss_matvec(int count, const MatvecJob<T> *jobs, const HssInstance *inst,
                       const HssCluster *cl, const cplx<T> *pool, const int *rank,
                       cplx<T> *scratch, int nlev, int max_width, int max_ncl, hipStream_t st) {
  if (count <= 0) return;
  for (int lev = nlev - 1; lev >= 1; --lev)
    hipLaunchKernelGGL(mv_up_kernel<T>, dim3(count, max_width), dim3(kMT), 0, st, lev, jobs, inst,
                       cl, pool, rank, scratch);
  hipLaunchKernelGGL(mv_couple_kernel<T>, dim3(count, max_ncl), dim3(kMT), 0, st, jobs, inst, cl,
                     pool, rank, scratch);
  for (int lev = 1; lev < nlev; ++lev)
    hipLaunchKernelGGL(mv_down_kernel<T>, dim3(count, max_width), dim3(kMT), 0, st, lev, jobs,
                       inst, cl, pool, rank, scratch);
  hipLaunchKernelGGL(mv_leaf_kernel<T>, dim3(count, max_ncl), dim3(kMT), 0, st, jobs, inst, cl,
                     pool, rank, scratch);
  HSSX_HIP(hipGetLastError());
}

#define HSSX_INST(T)                                                                          \
  template void launch_sample<T>(int, const SampleJob<T> *, int, int, hipStream_t);          \
  template void launch_compress_level<T>(int, const HssItem *, const HssInstance *,           \
                                         const HssCluster *, cplx<T> *, int *, int *,         \
                                         const cplx<T> *, const cplx<T> *, const double *,    \
                                         cplx<T> *, double, int, hipStream_t);                \
  template void launch_hss_matvec<T>(int, const MatvecJob<T> *, const HssInstance *,          \
                                     const HssCluster *, const cplx<T> *, const int *,        \
                                     cplx<T> *, int, int, int, hipStream_t);
HSSX_INST(double)
HSSX_INST(float)
#undef HSSX_INST

}  // namespace hssx
