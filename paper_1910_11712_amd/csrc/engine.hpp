// Moment engine: device descriptors and kernel launchers shared by the
// single-problem call, the batched plan and the server.
#pragma once

#include <vector>

#include "common.hpp"
#include "fn_device.hpp"
#include "lu.hpp"

namespace nep {

constexpr int kMaxTerms = 16;
constexpr int kBandMax = 64;  // widest half-bandwidth kept in band form
constexpr int kLowRankMax = 96;  // largest rank kept in factored form
constexpr int kMaxMoments = 32;  // 2K
constexpr int kSolveBlk = 64;    // triangular-solve block rows
constexpr int kResidRealTM = 64, kResidRealTQ = 64;  // real-term residual tile: rows x real columns
constexpr int kResidBigTM = 128, kResidBigTQ = 128;  // the same when the big tiles still fill the device
constexpr int kFallbackSweeps = 2;  // FP64 refinement sweeps after an FP64 re-solve
constexpr int kNormStride = 64;  // per-node stride of the column-norm arrays (L <= 64)
// Default stopping tolerance of the refinement (normwise backward error per
// probe column).  1e-15 rather than 1e-14: the residual a stopped solve
// leaves, mapped through T(z_j)^{-1}, lies along the eigenvectors of the
// eigenvalues near the node, so it moves the extracted eigenvalues instead of
// averaging out; at 1e-14 it moved them by up to a few 1e-11 (and lifted
// noise singular values above the rank threshold), at 1e-15 by ~1e-11, the
// level of the plain FP64 path.
constexpr double kDefaultRefineTol = 1e-15;

// Per-problem descriptor (device resident).
struct ProbDesc {
  int n, ell, N, L, KK;   // KK = 2K moments
  int a_cplx;             // 1 if any A_i is complex
  int node0;              // global index of node 0 of this problem
  int ld;                 // factor leading dimension
  long long offT0;        // factor block of node 0 (elements)
  long long strideT;      // between consecutive nodes
  long long offW0;        // solve work (n*L per node)
  long long offY;         // Y / R blocks: n x N*L complex, row-major
  int offRow0;            // row maps: offRow0 + j*n
  int kind;               // contour kind
  c128 c;                 // contour centre
  double rho, v;
  const void* A[kMaxTerms];        // device row-major A_i (double or c128)
  const double* normA;             // device, ell inf-norms
  const FnNode* fn_nodes;
  const c128* fn_coef;
  int fn_root[kMaxTerms];
  int a_is_cplx[kMaxTerms];
  int a_is_diag[kMaxTerms];        // diagonal A_i: residual applies d_r f_i y_r
  const c128* Adiag[kMaxTerms];
  int a_bw[kMaxTerms];             // real banded A_i (half-bandwidth, 0: not banded): the
                                   // real-term residual runs over the band's k only
  int a_lr[kMaxTerms];             // real low-rank A_i = G H^T (rank, 0: not factored):
  const double* LrG[kMaxTerms];    // the real-term residual applies G (H^T Y), with
  c128* LrZ[kMaxTerms];            // Z = H^T Y (rank x N*L) formed before it
  const c128* V;          // caller probes, column-major n x L
  c128* S;                // caller moments, column-major n x L x KK
  const c128* zpts;       // explicit points (N, device) instead of the contour's
                          // nodes, or nullptr
  long long s_stride;     // elements between consecutive moment blocks of S (>= n*L)
  int active;             // 0: the problem sits out this pass on resident factors (its
                          // nodes count as converged, its V and S are not touched)
  const c128* fpts;       // with zpts: given coefficients in place of f_i(z_j), at
                          // fpts[j*ell + i] (device), or nullptr
};

// Per-node arrays (global node index g).
struct NodeArrays {
  c128* z;        // nodes
  c128* zeta;     // (z - c)/rho
  c128* w;        // quadrature weights
  c128* fz;       // f_i(z_g) at [g*kMaxTerms + i]
  double* fnorm;  // sum_i |f_i(z_g)| ||A_i||_inf
  c128* mcoef;    // w_g zeta_g^p at [g*kMaxMoments + p]
  int* prob;      // problem of node g
  int* jnode;     // node index within the problem
  int* bad;       // 1 if some f_i is not holomorphic at z_g
};

// Per-node refinement state.
struct IrState {
  unsigned long long* rnorm;  // max |R| per (g, c) at g*kNormStride + c, double bits
  unsigned long long* ynorm;  // max |Y| per (g, c)
  double* vnorm;              // max |V| per (problem, c), index prob*64 + c
  double* rho;                // last scaled residual per node
  int* conv;                  // 1 when converged (skip further work)
  int* stalled;               // 1 when the residual stopped decreasing
  int* sweeps;                // sweeps run per node
  int* counters;              // [0] unconverged, [1] bad fn, [2] spare, [3] first bad node
};

// Launch tables of a batch (host copies; uploaded into one device buffer).
struct Table {
  int off = 0, cnt = 0, total = 0;  // prefix at off (cnt+1 ints), sum = total
};

struct SolvePlan {
  int nmat = 0;     // matrices (sorted order)
  int lg = 4;       // right-hand columns per group
  int groups = 1;   // column groups per matrix
  int rpt = 1;      // rows per thread of the 512-thread solve groups (n <= 512 * rpt)
  int nbig = 0;     // matrices of more than 512 rows (the first nbig in sorted order)
  int nmid = 0;     // then matrices of 257..512 rows; the rest have at most 256
  // the large matrices as paired 256-thread groups (complex FP32, lg <= 8,
  // rpt <= 2): -1 when they make 2048 groups or more, 0 never, 1 always
  int paired = -1;
  // complex FP32: the first nblk matrices (at least kSolveBlockedMinN rows)
  // take the blocked solve (solve_blk.hip) over big blocks of nbk rows, with
  // right-hand sides in the work buffer W (npad x L complex FP32 per matrix,
  // npad the largest n rounded up to 64); the rest take k_trsv
  int nblk = 0, nbk = 256, npad = 0, L = 0;
  c64* W = nullptr;
};
constexpr int kSolveBlockedMinN = 1024;

// Column-group widths the solve is built for (4, 8, 16) that fit the plan:
// fewer than 2L columns (a wider group would be more than half empty) and
// within the register budget of the accumulators.
bool solve_lg_fits(const SolvePlan& sp, int lg, int L, int prec);
void solve_set_lg(SolvePlan& sp, int lg, int L);

struct ProblemTables {
  Table assemble;  // element tiles per problem
  Table resid;       // residual GEMM tiles per problem with complex terms (64 x 64)
  Table resid_real;  // residual GEMM tiles per problem with real terms only (kResidRealTM x kResidRealTQ,
                     // or kResidBigTM x kResidBigTQ with resid_big)
  int resid_big = 0;
  Table moments;   // n*L tiles per problem
};

void build_prefix(std::vector<int>& buf, Table& t, const std::vector<int>& counts);

// Kernel launchers (all asynchronous on st).
hipError_t launch_coef(const ProbDesc* pd, const NodeArrays& na, int nnodes, IrState ir, hipStream_t st);
template <typename P>
hipError_t launch_assemble(const ProbDesc* pd, const int* prefix, const Table& t, const NodeArrays& na,
                           cx<P>* T, const int* skip, hipStream_t st);
hipError_t launch_moments(const ProbDesc* pd, const int* prefix, const Table& t, const NodeArrays& na,
                          const c128* Y, hipStream_t st);
hipError_t launch_vnorm(const ProbDesc* pd, int nprob, int L, IrState ir, hipStream_t st);  // L: columns (max over problems)

template <typename P>
hipError_t solve_run(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                     const cx<P>* T, const int* rows, const cx<P>* Dinv, const long long* dinv_off,
                     const c128* R, c128* Y, bool refine, const int* conv, IrState ir, hipStream_t st);
// Blocked solve of the first sp.nblk matrices (solve_blk.hip).
hipError_t solve_blocked(const SolvePlan& sp, const ProbDesc* pd, const MatDesc* md, const NodeArrays& na,
                         const c64* T, const int* rows, const c64* Dinv, const long long* dinv_off,
                         const c128* R, c128* Y, bool refine, const int* conv, IrState ir, hipStream_t st);
void SolvePlan_build(SolvePlan& sp, std::vector<int>& buf, const std::vector<MatDesc>& sorted, int L, int prec,
                     std::vector<long long>& dinv_off, long long& dinv_elems);
hipError_t solve_configure();

// One low-rank term of one problem: Z = H^T Y (rank x N*L) for the residual.
struct LrJob {
  const double* H;  // n x r row-major
  c128* Z;          // r x NL row-major
  long long offY;   // the problem's Y block
  int n, r, NL;
  c128* Zp;         // S partial sums of Z (S x r x NL), used when S > 1
  int S, srows;     // the sum over s cut into S ranges of srows rows
};
hipError_t resid_run(const ProbDesc* pd, const int* prefix, const Table& t, const Table& tr, int resid_big, const NodeArrays& na,
                     const c128* Y, c128* R, IrState ir, int nnodes, hipStream_t st, const LrJob* lr = nullptr,
                     int nlr = 0);
// status read-back block (see k_gather_status) and its size
size_t status_bytes(int G);
hipError_t gather_status(IrState ir, const int* info, const int* bad, int G, void* out, hipStream_t st);
// smallest pivot modulus per node into the status block (after rho)
template <typename P>
hipError_t min_pivot(const MatDesc* md, int nmat, const cx<P>* T, const int* rows, int G, void* status,
                     hipStream_t st);
hipError_t ir_control(const ProbDesc* pd, const NodeArrays& na, IrState ir, int nnodes, int sweep, double tol,
                      hipStream_t st);
hipError_t ir_reset(IrState ir, int nnodes, hipStream_t st);
hipError_t engine_configure();

}  // namespace nep
